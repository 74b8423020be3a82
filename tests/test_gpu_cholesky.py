"""The library's FP32 Cholesky solve on its own, against numpy in FP64 (GPU)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2007_08576_amd import tt
    tt.lib()
    return tt


@pytest.mark.parametrize("n", [1, 7, 64, 72, 128, 200, 384, 700, 2400])
def test_cholesky_solve_random_spd(T, n):
    rng = np.random.default_rng(n)
    B = rng.normal(size=(n, n))
    A = B @ B.T / n + np.eye(n)  # condition number ~ 5
    b = rng.normal(size=n)
    x, fail = T.debug_cholesky_solve(A, b)
    assert not fail
    want = np.linalg.solve(A, b)
    err = np.linalg.norm(x - want) / np.linalg.norm(want)
    print(f"n={n}: rel err {err:.2e}", flush=True)
    assert err < 1e-5


def test_cholesky_flags_indefinite(T):
    rng = np.random.default_rng(3)
    A = np.eye(100)
    A[50, 50] = -1.0
    _, fail = T.debug_cholesky_solve(A, rng.normal(size=100))
    assert fail


def _spd(n, cond, seed):
    """SPD matrix with eigenvalues spread log-uniformly over [1/cond, 1] (random orthogonal basis)."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.logspace(0.0, -np.log10(cond), n)
    return (Q * ev) @ Q.T


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("n", [64, 200, 700])
def test_cholesky_16bit_refined(T, prec, n):
    """16-bit tile products + 2 refinement steps reach the FP32 bar on a well-conditioned system."""
    p = T.TT_BF16_IR if prec == "bf16" else T.TT_FP16_IR
    rng = np.random.default_rng(n + 7)
    B = rng.normal(size=(n, n))
    A = B @ B.T / n + np.eye(n)
    b = rng.normal(size=n)
    x, fail = T.debug_cholesky_solve(A, b, precision=p, ir_iters=2)
    assert not fail
    want = np.linalg.solve(A, b)
    err = np.linalg.norm(x - want) / np.linalg.norm(want)
    print(f"{prec} n={n}: rel err {err:.2e}", flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_cholesky_refinement_converges(T, prec):
    """On a condition-1e3 system the refinement error shrinks step by step to the FP32 level."""
    p = T.TT_BF16_IR if prec == "bf16" else T.TT_FP16_IR
    n = 384
    A = _spd(n, 1e3, 11)
    b = np.random.default_rng(12).normal(size=n)
    want = np.linalg.solve(A, b)
    errs = []
    for it in (0, 1, 2, 4, 8):
        x, fail = T.debug_cholesky_solve(A, b, precision=p, ir_iters=it)
        assert not fail
        errs.append(np.linalg.norm(x - want) / np.linalg.norm(want))
    x32, _ = T.debug_cholesky_solve(A, b)
    e32 = np.linalg.norm(x32 - want) / np.linalg.norm(want)
    print(f"{prec}: errors by refinement steps 0,1,2,4,8: {['%.1e' % e for e in errs]}; FP32 {e32:.1e}", flush=True)
    assert errs[1] < errs[0] and errs[2] < errs[1]
    assert errs[-1] < max(10 * e32, 1e-5)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n", [200, 700])
def test_cholesky_repeatable(T, prec, n):
    """Every tile of the factorisation is summed in a fixed order whichever workgroup computes it and
    whenever its inputs arrive, so solves of one system agree bit for bit from run to run; a task
    that read a tile unordered with a write of it would show here as differences between runs."""
    p = T.TT_BF16_IR if prec == "bf16" else T.TT_FP32
    rng = np.random.default_rng(n + 29)
    B = rng.normal(size=(n, n))
    A = B @ B.T / n + np.eye(n)
    b = rng.normal(size=n)
    ref, fail = T.debug_cholesky_solve(A, b, precision=p, ir_iters=2)
    assert not fail
    for rep in range(12):
        x, fail = T.debug_cholesky_solve(A, b, precision=p, ir_iters=2)
        assert not fail
        assert np.array_equal(x, ref), f"run {rep + 1} differs from the first"
