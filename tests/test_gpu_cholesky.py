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
