"""The serving loop (tt_server_*): frames of many streams batched at LM-iteration boundaries give
each stream the result it gets when tracked alone, bit for bit; streams are admitted against one HBM
budget (an open that does not fit waits until a close releases bytes); a stream the server owns
refuses the single-stream calls (GPU).
"""
import threading
import time

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


def _scenes():
    # uneven sizes: control points, image sizes and feature counts differ between streams
    return [synth.make_sequence(seed=41, M=1500, N=40, K1=200, width=160, height=120, n_frames=4,
                                max_step_mm=3.0, name="srvA"),
            synth.make_sequence(seed=42, M=2400, N=70, K1=350, width=192, height=144, n_frames=4,
                                max_step_mm=3.0, name="srvB"),
            synth.make_sequence(seed=43, M=1200, N=25, K1=150, width=128, height=96, n_frames=4,
                                max_step_mm=3.0, name="srvC"),
            synth.make_sequence(seed=44, M=3000, N=100, K1=400, width=192, height=144, n_frames=4,
                                max_step_mm=3.0, name="srvD")]


def _params(tt, sc, q):
    kw = {}
    if q == 1:
        kw["precision"] = tt.TT_BF16_IR
    if q == 2:
        kw["solver"] = tt.TT_SOLVE_NODE
    return tt.default_params(num_control_points=sc.num_control_points, seed=7, **kw)


def _intr(tt, sc):
    return tt.intrinsics(sc.intr.width, sc.intr.height, sc.intr.fx, sc.intr.fy, sc.intr.cx, sc.intr.cy)


def _dev_frames(torch, sc, ts, dev):
    out = [tuple(torch.from_numpy(a).to(dev) for a in (f.depth, f.feat_xyz, f.feat_desc))
           for f in (sc.frame(t) for t in ts)]
    torch.cuda.synchronize()
    return out


def _alone(tt, torch, sc, q, frames, dev):
    s = tt.Stream(_params(tt, sc, q), _intr(tt, sc))
    s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    ov = torch.zeros((sc.pts.shape[0], 3), dtype=torch.float32, device=dev)
    oq = torch.zeros((sc.num_control_points, 8), dtype=torch.float32, device=dev)
    res = []
    for d in frames:
        s.track_frame_device(d[0], d[1], d[2], d[1].shape[0], ov, oq)
        s.sync()
        res.append((ov.cpu().numpy().copy(), oq.cpu().numpy().copy()))
    s.destroy()
    return res


def test_served_frames_equal_alone_with_staggered_arrivals(env):
    tt, torch = env
    dev = torch.device("cuda:0")
    scenes = _scenes()
    ts = (1, 2, 3)
    frames = [_dev_frames(torch, sc, ts, dev) for sc in scenes]
    ref = [_alone(tt, torch, sc, q, frames[q], dev) for q, sc in enumerate(scenes)]
    sv = tt.Server()
    streams = [sv.open(_params(tt, sc, q), _intr(tt, sc), sc.pts, sc.feat_xyz, sc.feat_desc, K2max=512)
               for q, sc in enumerate(scenes)]
    outs = [[(torch.zeros((sc.pts.shape[0], 3), dtype=torch.float32, device=dev),
              torch.zeros((sc.num_control_points, 8), dtype=torch.float32, device=dev)) for _ in ts]
            for sc in scenes]
    tickets = []
    # every stream's frames queued at once, but the streams arrive one after another: later frames
    # join rounds that are already running
    for q in range(len(scenes)):
        for k in range(len(ts)):
            d = frames[q][k]
            ov, oq = outs[q][k]
            tickets.append(sv.submit(streams[q], d[0], d[1], d[2], d[1].shape[0], ov, oq))
        time.sleep(0.002)
    lats = [sv.wait(t, 60.0) for t in tickets]
    st = sv.stats()
    for q in range(len(scenes)):
        for k in range(len(ts)):
            ov, oq = outs[q][k]
            assert np.array_equal(ov.cpu().numpy(), ref[q][k][0]), f"stream {q} frame {k}: vertices differ"
            assert np.array_equal(oq.cpu().numpy(), ref[q][k][1]), f"stream {q} frame {k}: warps differ"
    assert all(v > 0 for v in lats)
    assert st["frames_done"] == st["frames_submitted"] == len(tickets)
    # frames of different streams shared rounds (more than one frame per round on average)
    assert st["frame_iterations"] > st["rounds"]
    for s in streams:
        sv.close(s)
    assert sv.stats()["streams_open"] == 0 and sv.stats()["reserved_bytes"] == 0
    sv.destroy()


def test_open_waits_for_budget_then_is_admitted(env):
    tt, torch = env
    dev = torch.device("cuda:0")
    a, b = _scenes()[0], _scenes()[1]
    # the bytes each stream holds, from an unlimited server
    probe = tt.Server()
    sa = probe.open(_params(tt, a, 0), _intr(tt, a), a.pts, a.feat_xyz, a.feat_desc, K2max=512)
    bytes_a = probe.stats()["reserved_bytes"]
    sb = probe.open(_params(tt, b, 0), _intr(tt, b), b.pts, b.feat_xyz, b.feat_desc, K2max=512)
    bytes_b = probe.stats()["reserved_bytes"] - bytes_a
    probe.close(sa)
    probe.close(sb)
    probe.destroy()
    assert bytes_a > 0 and bytes_b > 0
    # room for either stream alone, not for both
    sv = tt.Server(hbm_budget_bytes=max(bytes_a, bytes_b) + min(bytes_a, bytes_b) // 2)
    sa = sv.open(_params(tt, a, 0), _intr(tt, a), a.pts, a.feat_xyz, a.feat_desc, K2max=512)
    # no room and no wait: refused at once
    t0 = time.time()
    with pytest.raises(tt.TTError) as ei:
        sv.open(_params(tt, b, 0), _intr(tt, b), b.pts, b.feat_xyz, b.feat_desc, K2max=512, wait_s=0.0)
    assert ei.value.code == tt.TT_EBUSY and time.time() - t0 < 5.0
    got = {}

    def opener():
        try:
            got["s"] = sv.open(_params(tt, b, 0), _intr(tt, b), b.pts, b.feat_xyz, b.feat_desc, K2max=512,
                               wait_s=60.0)
        except Exception as e:  # reported below
            got["e"] = e

    th = threading.Thread(target=opener)
    th.start()
    time.sleep(0.5)
    assert th.is_alive(), "the open should wait while the budget is full"
    assert sv.stats()["opens_waiting"] == 1
    # a frame of the admitted stream still runs meanwhile
    fa = _dev_frames(torch, a, (1,), dev)[0]
    ova = torch.zeros((a.pts.shape[0], 3), dtype=torch.float32, device=dev)
    sv.wait(sv.submit(sa, fa[0], fa[1], fa[2], fa[1].shape[0], ova, None), 60.0)
    sv.close(sa)
    th.join(60.0)
    assert not th.is_alive() and "e" not in got, got.get("e")
    sb = got["s"]
    assert sv.stats()["streams_open"] == 1
    # the admitted stream tracks as it does alone
    fb = _dev_frames(torch, b, (1, 2), dev)
    ref = _alone(tt, torch, b, 0, fb, dev)
    ov = torch.zeros((b.pts.shape[0], 3), dtype=torch.float32, device=dev)
    for k, d in enumerate(fb):
        sv.wait(sv.submit(sb, d[0], d[1], d[2], d[1].shape[0], ov, None), 60.0)
        assert np.array_equal(ov.cpu().numpy(), ref[k][0])
    # a stream that could not fit even in an empty server is refused outright
    small = tt.Server(hbm_budget_bytes=min(bytes_a, bytes_b) // 4)
    with pytest.raises(tt.TTError) as ei:
        small.open(_params(tt, a, 0), _intr(tt, a), a.pts, a.feat_xyz, a.feat_desc, K2max=512, wait_s=1.0)
    assert ei.value.code == tt.TT_ENOMEM
    small.destroy()
    sv.destroy()


def test_owned_stream_refuses_single_stream_calls(env):
    tt, torch = env
    dev = torch.device("cuda:0")
    a = _scenes()[2]
    sv = tt.Server()
    s = sv.open(_params(tt, a, 0), _intr(tt, a), a.pts, a.feat_xyz, a.feat_desc, K2max=256)
    d = _dev_frames(torch, a, (1,), dev)[0]
    L = tt.lib()
    assert L.tt_track_frame_device(s.h, d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), d[1].shape[0],
                                   None, None) == tt.TT_EBUSY
    assert L.tt_destroy(s.h) == tt.TT_EBUSY
    # more features than the stream was opened for
    big = torch.zeros((600, 32), dtype=torch.uint8, device=dev)
    bxyz = torch.zeros((600, 3), dtype=torch.float32, device=dev)
    with pytest.raises(tt.TTError):
        sv.submit(s, d[0], bxyz, big, 600)
    sv.close(s)
    sv.destroy()


def test_config4_served_equals_alone_with_rounds_ahead(env):
    """The 16-stream serving mix (control points 123-772, uneven images and feature counts) through
    the serving loop with three rounds queued ahead of the device, so that the per-round argument
    tables of the multi-system launches cycle through their ring of slots many times, and with the
    streams arriving one after another (frames entering and frames continuing share rounds); in FP32
    and in the binary16 form with one refinement step: every frame equals the stream's result when
    tracked alone, bit for bit."""
    tt, torch = env
    dev = torch.device("cuda:0")
    scenes = synth.make_config4(seed=4, n_streams=16, n_frames=300)
    ts = (1, 2, 3)
    frames = [_dev_frames(torch, sc, ts, dev) for sc in scenes]
    for prec, ir in ((tt.TT_FP32, 2), (tt.TT_FP16_IR, 1)):
        def params(sc):
            return tt.default_params(num_control_points=sc.num_control_points, seed=4, precision=prec, ir_iters=ir)

        ref = []
        for q, sc in enumerate(scenes):
            s = tt.Stream(params(sc), _intr(tt, sc))
            s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
            ov = torch.zeros((sc.pts.shape[0], 3), dtype=torch.float32, device=dev)
            oq = torch.zeros((sc.num_control_points, 8), dtype=torch.float32, device=dev)
            r = []
            for d in frames[q]:
                s.track_frame_device(d[0], d[1], d[2], d[1].shape[0], ov, oq)
                s.sync()
                r.append((ov.cpu().numpy().copy(), oq.cpu().numpy().copy()))
            s.destroy()
            ref.append(r)
        sv = tt.Server(max_rounds_ahead=3)
        streams = [sv.open(params(sc), _intr(tt, sc), sc.pts, sc.feat_xyz, sc.feat_desc,
                           K2max=max(d[1].shape[0] for d in frames[q])) for q, sc in enumerate(scenes)]
        outs = [[(torch.zeros((sc.pts.shape[0], 3), dtype=torch.float32, device=dev),
                  torch.zeros((sc.num_control_points, 8), dtype=torch.float32, device=dev)) for _ in ts]
                for sc in scenes]
        tickets = []
        for q in range(len(scenes)):
            for k in range(len(ts)):
                d = frames[q][k]
                ov, oq = outs[q][k]
                tickets.append(sv.submit(streams[q], d[0], d[1], d[2], d[1].shape[0], ov, oq))
            time.sleep(0.001)
        for t in tickets:
            sv.wait(t, 60.0)
        st = sv.stats()
        assert st["frames_done"] == len(tickets) and st["frame_iterations"] > st["rounds"]
        for q in range(len(scenes)):
            for k in range(len(ts)):
                ov, oq = outs[q][k]
                assert np.array_equal(ov.cpu().numpy(), ref[q][k][0]), f"precision {prec}: stream {q} frame {k}"
                assert np.array_equal(oq.cpu().numpy(), ref[q][k][1]), f"precision {prec}: stream {q} frame {k}"
        for s in streams:
            sv.close(s)
        sv.destroy()
