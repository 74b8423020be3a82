"""Tuning and the autotuner (tt_set_tuning / tt_autotune): launch shapes that leave the solve as it
is. The factorisation's launch width and the rows + ARAP fusion change nothing bit for bit; the
ARAP workgroup size only reorders FP32 sums (vertices within 1e-4 mm); the autotuner returns one of
its candidates with a measured time and leaves the stream exactly as it found it (GPU)."""
import numpy as np
import pytest

from paper_2007_08576_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2007_08576_amd import tt
    tt.lib()
    sc = synth.make_sequence(seed=51, M=2400, N=70, K1=300, width=192, height=144, n_frames=4, max_step_mm=3.0,
                             name="tune")
    dev = torch.device("cuda:0")
    frames = [tuple(torch.from_numpy(a).to(dev) for a in (f.depth, f.feat_xyz, f.feat_desc))
              for f in (sc.frame(t) for t in (1, 2, 3))]
    torch.cuda.synchronize()
    return tt, torch, sc, frames


def _track(tt, torch, sc, frames, tuning=None, autotune=False, graph=0):
    dev = torch.device("cuda:0")
    s = tt.Stream(tt.default_params(num_control_points=sc.num_control_points, seed=9, graph=graph),
                  tt.intrinsics(sc.intr.width, sc.intr.height, sc.intr.fx, sc.intr.fy, sc.intr.cx, sc.intr.cy))
    s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    if tuning is not None:
        s.set_tuning(**tuning)
    ov = torch.zeros((sc.pts.shape[0], 3), dtype=torch.float32, device=dev)
    oq = torch.zeros((sc.num_control_points, 8), dtype=torch.float32, device=dev)
    out, best = [], None
    for k, d in enumerate(frames):
        if autotune and k == 1:  # tuned in the middle of a sequence, on the frame about to be tracked
            best = s.autotune(d[0], d[1], d[2], d[1].shape[0], reps=2)
        s.track_frame_device(d[0], d[1], d[2], d[1].shape[0], ov, oq)
        s.sync()
        out.append((ov.cpu().numpy().copy(), oq.cpu().numpy().copy()))
    tun = s.get_tuning()
    s.destroy()
    return out, best, tun


def test_launch_width_and_fusion_change_nothing(env):
    tt, torch, sc, frames = env
    ref, _, _ = _track(tt, torch, sc, frames)
    for t in ({"chol_grid_pct": 25}, {"chol_grid_pct": 50}, {"chol_grid_pct": 100, "fuse_rows_arap": 0},
              {"chol_grid_pct": 400, "fuse_rows_arap": 1}):
        got, _, _ = _track(tt, torch, sc, frames, tuning=t)
        for k in range(len(frames)):
            assert np.array_equal(got[k][0], ref[k][0]) and np.array_equal(got[k][1], ref[k][1]), (t, k)


def test_arap_workgroup_size_only_reorders_sums(env):
    tt, torch, sc, frames = env
    ref, _, _ = _track(tt, torch, sc, frames)
    got, _, _ = _track(tt, torch, sc, frames, tuning={"arap_threads": 128, "fuse_rows_arap": 0})
    for k in range(len(frames)):
        rms = float(np.sqrt(((got[k][0].astype(np.float64) - ref[k][0]) ** 2).sum(1).mean()))
        assert rms <= 1e-4, (k, rms)


def test_autotune_picks_a_candidate_and_restores_the_stream(env):
    tt, torch, sc, frames = env
    got, best, tun = _track(tt, torch, sc, frames, autotune=True)
    assert best["frame_ms"] > 0
    assert best["chol_grid_pct"] in (50, 100, 200)
    assert (best["arap_threads"], best["fuse_rows_arap"]) in ((256, 1), (256, 0), (128, 0))
    assert {k: tun[k] for k in ("chol_grid_pct", "arap_threads", "fuse_rows_arap")} == \
        {k: best[k] for k in ("chol_grid_pct", "arap_threads", "fuse_rows_arap")}
    # the same frames with that tuning set from the start: identical, so the tuner's trial frames
    # left neither the warps nor the frame counter changed
    ref, _, _ = _track(tt, torch, sc, frames, tuning={k: best[k] for k in ("chol_grid_pct", "arap_threads",
                                                                            "fuse_rows_arap")})
    for k in range(len(frames)):
        assert np.array_equal(got[k][0], ref[k][0]) and np.array_equal(got[k][1], ref[k][1]), k


def test_tuning_validation_and_graph_recapture(env):
    tt, torch, sc, frames = env
    s = tt.Stream(tt.default_params(num_control_points=sc.num_control_points, seed=9),
                  tt.intrinsics(sc.intr.width, sc.intr.height, sc.intr.fx, sc.intr.fy, sc.intr.cx, sc.intr.cy))
    for bad in ({"chol_grid_pct": 10}, {"arap_threads": 192}, {"arap_threads": 128, "fuse_rows_arap": 1},
                {"fuse_rows_arap": 2}):
        with pytest.raises(tt.TTError):
            s.set_tuning(**bad)
    s.destroy()
    # graph replay with a tuning change in the middle of the sequence: the graphs are recaptured
    ref, _, _ = _track(tt, torch, sc, frames, tuning={"chol_grid_pct": 100})
    got, _, _ = _track(tt, torch, sc, frames, tuning={"chol_grid_pct": 100}, graph=1)
    for k in range(len(frames)):
        assert np.array_equal(got[k][0], ref[k][0]), k
