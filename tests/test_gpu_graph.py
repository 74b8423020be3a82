"""Graph replay of the LM iterations (tt_params.graph = 1): each frame's LM set-up and iterations are
captured once per front-buffer parity and replayed on later frames. The kernels and their arguments
are those of the kernel-by-kernel launches (the solve epochs live on the device), so the frames
must come out bit for bit the same. GPU."""
import numpy as np
import pytest

from paper_2007_08576_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2007_08576_amd import tt
    tt.lib()
    return tt, torch


def _stream(tt, sc, graph, **kw):
    s = tt.Stream(tt.default_params(num_control_points=sc.num_control_points, seed=3, graph=graph, **kw),
                  tt.intrinsics(sc.intr.width, sc.intr.height, sc.intr.fx, sc.intr.fy, sc.intr.cx, sc.intr.cy))
    s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    return s


def _run(tt, torch, sc, frames, graph, set_state_at=None, **kw):
    dev = torch.device("cuda:0")
    s = _stream(tt, sc, graph, **kw)
    ov = torch.zeros((sc.pts.shape[0], 3), dtype=torch.float32, device=dev)
    oq = torch.zeros((sc.num_control_points, 8), dtype=torch.float32, device=dev)
    ready = torch.cuda.Event()
    ready.record()
    out = []
    for k, d in enumerate(frames):
        if set_state_at is not None and k == set_state_at:
            s.set_state(np.tile(np.r_[1.0, 0, 0, 0, 0, 0, 0, 0], (sc.num_control_points, 1)), 0)
        s.track_frame_device(d[0], d[1], d[2], d[1].shape[0], ov, oq, inputs_ready=ready)
        s.sync()
        out.append((ov.cpu().numpy().copy(), oq.cpu().numpy().copy(), s.frame_log()))
    s.destroy()
    return out


def _dev_frames(torch, sc, ts):
    dev = torch.device("cuda:0")
    fr = [tuple(torch.from_numpy(a).to(dev) for a in (f.depth, f.feat_xyz, f.feat_desc)) for f in (sc.frame(t) for t in ts)]
    torch.cuda.synchronize()
    return fr


def _same(a, b):
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x[0], y[0]), f"frame {k}: vertices differ"
        assert np.array_equal(x[1], y[1]), f"frame {k}: warps differ"
        for key in ("cost_old", "accepted", "lambda"):
            assert np.array_equal(np.asarray(x[2][key], np.float64), np.asarray(y[2][key], np.float64),
                                  equal_nan=True), f"frame {k}: {key} differs"


@pytest.mark.parametrize("form", ["fp32", "bf16_ir", "node"])
def test_graph_replay_equals_kernel_launches_on_a_sequence(env, form):
    tt, torch = env
    sc = synth.make_sequence(seed=31, M=2400, N=60, K1=300, width=192, height=144, n_frames=6, max_step_mm=3.0,
                             name="graphseq")
    kw = dict(bf16_ir=dict(precision=tt.TT_BF16_IR), node=dict(solver=tt.TT_SOLVE_NODE), fp32={})[form]
    frames = _dev_frames(torch, sc, (1, 2, 3, 4, 5))  # both front-buffer parities, replayed twice or more
    _same(_run(tt, torch, sc, frames, 0, **kw), _run(tt, torch, sc, frames, 1, **kw))


def test_graph_replay_with_teacher_forcing_and_config2(env):
    tt, torch = env
    sc = synth.make_config2(seed=2, n_frames=4)
    frames = _dev_frames(torch, sc, (1, 2, 3))
    _same(_run(tt, torch, sc, frames, 0, set_state_at=2), _run(tt, torch, sc, frames, 1, set_state_at=2))


def test_graph_is_recaptured_after_a_new_template_and_skipped_when_timed(env):
    tt, torch = env
    dev = torch.device("cuda:0")
    a = synth.make_sequence(seed=32, M=1500, N=40, K1=200, width=160, height=120, n_frames=3, name="ga")
    # the same number of control points (a stream parameter), a different template of another size
    b = synth.make_sequence(seed=33, M=1800, N=40, K1=250, width=160, height=120, n_frames=3, name="gb")
    fa = _dev_frames(torch, a, (1, 2))
    fb = _dev_frames(torch, b, (1, 2))
    # one graph-mode stream given template a, then template b: its frames of b equal a fresh stream's
    s = _stream(tt, a, 1)
    ov = torch.zeros((b.pts.shape[0], 3), dtype=torch.float32, device=dev)
    oq = torch.zeros((b.num_control_points, 8), dtype=torch.float32, device=dev)
    for d in fa:
        s.track_frame_device(d[0], d[1], d[2], d[1].shape[0], None, None)
    s.sync()
    s.set_template(b.pts, b.feat_xyz, b.feat_desc)
    got = []
    for d in fb:
        s.track_frame_device(d[0], d[1], d[2], d[1].shape[0], ov, oq)
        s.sync()
        got.append((ov.cpu().numpy().copy(), oq.cpu().numpy().copy(), s.frame_log()))
    # stage timers on: the frames run kernel by kernel (the timers count every stage call)
    s.set_timing(True)
    s.set_template(b.pts, b.feat_xyz, b.feat_desc)
    timed = []
    for d in fb:
        s.track_frame_device(d[0], d[1], d[2], d[1].shape[0], ov, oq)
        s.sync()
        timed.append((ov.cpu().numpy().copy(), oq.cpu().numpy().copy(), s.frame_log()))
    ms, n = s.get_timing()
    assert n[tt.STAGES.index("factor")] == 2 * s.params.lm_iters
    s.destroy()
    ref = _run(tt, torch, b, fb, 0)
    _same(ref, got)
    _same(ref, timed)
