"""The allocation-free solve (tt_cholesky_solve_noalloc) against the allocating diagnostic solve it
is a variant of (tt_debug_cholesky_solve_ex, FP32): the same kernels on the same inputs, so the
solutions agree bit for bit, on two calls in a row, the second one smaller (the static workspace
keeps the first call's contents, which the second must not depend on). GPU."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _spd(rng, n):
    B = rng.normal(size=(n, n)) / np.sqrt(n)
    return (B @ B.T + np.eye(n) * (1.0 + rng.uniform(size=n))).astype(np.float32)


def test_noalloc_solve_matches_the_allocating_solve():
    import torch
    from paper_2007_08576_amd import tt
    tt.lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(77)
    stream = torch.cuda.current_stream()
    for n in (1000, 333):
        A = _spd(rng, n)
        b = rng.normal(size=n).astype(np.float32)
        x_ref, fail = tt.debug_cholesky_solve(A, b)
        assert not fail
        dA = torch.from_numpy(A).to(dev)
        db = torch.from_numpy(b).to(dev)
        dx = torch.full((n,), float("nan"), dtype=torch.float32, device=dev)
        status = torch.full((2,), -1, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        tt.cholesky_solve_noalloc(n, dA, db, dx, status, hip_stream=stream.cuda_stream)
        torch.cuda.synchronize()
        assert status.cpu().tolist() == [0, 0]
        x = dx.cpu().numpy()
        assert np.array_equal(x, x_ref), f"n = {n}: max difference {np.abs(x - x_ref).max()}"
        # and it solves the system
        r = A.astype(np.float64) @ x.astype(np.float64) - b
        assert np.linalg.norm(r) <= 1e-4 * np.linalg.norm(b)


def test_noalloc_solve_rejects_sizes_beyond_its_workspace():
    import torch
    from paper_2007_08576_amd import tt
    dev = torch.device("cuda:0")
    n = tt.lib() and 1025
    dA = torch.zeros((n, n), dtype=torch.float32, device=dev)
    db = torch.zeros(n, dtype=torch.float32, device=dev)
    dx = torch.zeros(n, dtype=torch.float32, device=dev)
    st = torch.zeros(2, dtype=torch.int32, device=dev)
    for bad in (0, 1025):
        with pytest.raises(tt.TTError) as e:
            tt.cholesky_solve_noalloc(bad, dA, db, dx, st)
        assert e.value.code == tt.TT_EINVAL
    with pytest.raises(tt.TTError) as e:
        tt.cholesky_solve_noalloc(10, dA, None, dx, st)
    assert e.value.code == tt.TT_EINVAL
