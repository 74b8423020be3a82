"""Parity of the uniform ORB front end (FAST-9 response, neighbour suppression, orientation,
rotated binary descriptors, depth back-projection) with the oracle (GPU). All of it is integer
work except the orientation bin (FP64 from integer moments) and the back-projection, so the bar is
bit-exact: keypoints, their order, descriptors, bins, counts and the float32 3D points.
"""
import math

import numpy as np
import pytest

from paper_2007_08576_amd import synth
from tests import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2007_08576_amd import tt
    tt.lib()
    return tt


def _intr(mod, K):
    return mod.intrinsics(K.width, K.height, K.fx, K.fy, K.cx, K.cy)


def _both(O, T, img, depth=None, K=None, **kw):
    pat = synth.orb_pattern(0)
    o = O.orb_detect(img, pat, depth, _intr(O, K) if K is not None else None, **kw)
    det = T.Orb(T.orb_params(**kw), img.shape[1], img.shape[0], pat)
    g = det.detect(img, depth, _intr(T, K) if K is not None else None)
    det.destroy()
    return o, g


def _same(o, g, xyz=False):
    assert o["total"] == g["total"]
    assert np.array_equal(o["kp"], g["kp"])
    assert np.array_equal(o["angle_bin"], g["angle_bin"])
    assert np.array_equal(o["desc"], g["desc"])
    if xyz:
        assert np.array_equal(o["xyz"].view(np.uint32), g["xyz"].view(np.uint32))


def test_orb_hand_built_images(O, T):
    img = np.full((64, 64), 40, np.uint8)
    for u, v, val in ((30, 30, 200), (31, 30, 250), (20, 40, 200), (40, 22, 200), (41, 23, 200)):
        img[v, u] = val
    for r in (0, 1, 3):
        o, g = _both(O, T, img, nms_radius=r)
        _same(o, g)
    u = np.arange(64)[None, :] - 32.0
    v = np.arange(64)[:, None] - 32.0
    for b in (0, 7, 19):
        phi = math.radians(12.0 * b)
        ramp = np.clip(np.floor(100 + 2.5 * (u * math.cos(phi) + v * math.sin(phi)) + 0.5), 0, 255).astype(np.uint8)
        ramp[32, 32] = 255
        o, g = _both(O, T, ramp, fast_threshold=40)
        _same(o, g)
        assert len(g["kp"]) >= 1


def test_orb_config2_images_bit_exact(O, T):
    sc = synth.make_config2(seed=2, n_frames=300)
    for t in (0, 1):
        depth, img = sc.image(t)
        o, g = _both(O, T, img, depth, sc.intr)
        print(f"frame {t}: {len(g['kp'])} keypoints ({g['total']} kept), "
              f"{np.isfinite(g['xyz'][:, 2]).mean():.3f} with depth", flush=True)
        assert len(g["kp"]) > 1000
        _same(o, g, xyz=True)


def test_orb_cap_ragged_and_tiny_images(O, T):
    sc = synth.make_small_sequence(seed=12, M=500, N=8, K1=40, width=333, height=251, n_frames=1,
                                   max_step_mm=2.0)
    depth, img = sc.image(1)
    o, g = _both(O, T, img, depth, sc.intr)
    _same(o, g, xyz=True)
    o, g = _both(O, T, img, depth, sc.intr, max_features=50)
    _same(o, g, xyz=True)
    assert len(g["kp"]) == 50 and g["total"] > 50
    o, g = _both(O, T, img[:30, :30].copy(), max_features=16)
    assert g["total"] == 0 and len(g["kp"]) == 0
    _same(o, g)
    o, g = _both(O, T, img, max_features=0)
    assert len(g["kp"]) == 0 and g["total"] == o["total"] > 0


def test_orb_device_path_matches_host_path(T):
    import torch
    sc = synth.make_config2(seed=2, n_frames=300)
    depth, img = sc.image(1)
    pat = synth.orb_pattern(0)
    p = T.orb_params()
    det = T.Orb(p, img.shape[1], img.shape[0], pat)
    K = _intr(T, sc.intr)
    h = det.detect(img, depth, K)
    dev = torch.device("cuda:0")
    di, dd = torch.from_numpy(img).to(dev), torch.from_numpy(depth).to(dev)
    mx = p.max_features
    kp = torch.zeros((mx, 2), dtype=torch.int32, device=dev)
    xyz = torch.zeros((mx, 3), dtype=torch.float32, device=dev)
    desc = torch.zeros((mx, 32), dtype=torch.uint8, device=dev)
    ang = torch.zeros(mx, dtype=torch.int32, device=dev)
    cnt = torch.zeros(2, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    for _ in range(2):  # twice: nothing carries over between detections
        det.detect_device(di, dd, K, kp, xyz, desc, ang, cnt)
    torch.cuda.synchronize()
    n = int(cnt[0])
    assert n == len(h["kp"]) and int(cnt[1]) == h["total"]
    assert np.array_equal(kp[:n].cpu().numpy(), h["kp"])
    assert np.array_equal(desc[:n].cpu().numpy(), h["desc"])
    assert np.array_equal(ang[:n].cpu().numpy(), h["angle_bin"])
    det.destroy()


def test_tracking_with_detected_features(O, T):
    """Template features from the textured template image, frame features from frame 1, both
    detected on the GPU; the GPU and the oracle track the frame from the same features within
    0.01 mm RMS, and most features match their own surface point."""
    sc = synth.make_small_sequence(seed=12, M=4000, N=40, K1=40, width=192, height=144, n_frames=2,
                                   max_step_mm=2.0)
    pat = synth.orb_pattern(0)
    det = T.Orb(T.orb_params(), 192, 144, pat)
    K = _intr(T, sc.intr)
    d0, i0 = sc.image(0)
    d1, i1 = sc.image(1)
    a = det.detect(i0, d0, K)
    b = det.detect(i1, d1, K)
    keep = np.isfinite(a["xyz"]).all(1)
    fx, fd = a["xyz"][keep], a["desc"][keep]
    so = O.Stream(O.default_params(num_control_points=40, seed=3), _intr(O, sc.intr))
    sg = T.Stream(T.default_params(num_control_points=40, seed=3), K)
    so.set_template(sc.pts, fx, fd)
    sg.set_template(sc.pts, fx, fd)
    vo, _, do = so.track_frame(d1, b["xyz"], b["desc"], debug=True)
    vg, _, dg = sg.track_frame(d1, b["xyz"], b["desc"], debug=True)
    rms = float(np.sqrt(((vo - vg) ** 2).sum(1).mean()))
    truth = float(np.sqrt(((vg - sc.frame(1).gt_vertices) ** 2).sum(1).mean()))
    print(f"{len(fx)} template / {len(b['kp'])} frame features, {int(dg['preselected'].sum())} pre-selected, "
          f"rms vs oracle {rms:.2e} mm, vs truth {truth:.3f} mm", flush=True)
    assert np.array_equal(do["match_idx"], dg["match_idx"])
    assert rms <= 0.01
    det.destroy()


def test_orb_bad_arguments(T):
    pat = synth.orb_pattern(0)
    for kw in (dict(fast_threshold=-1), dict(nms_radius=17), dict(max_features=-1)):
        with pytest.raises(T.TTError) as e:
            T.Orb(T.orb_params(**kw), 64, 64, pat)
        assert e.value.code == T.TT_EINVAL
    bad = pat.copy()
    bad[0, 0] = 14
    with pytest.raises(T.TTError):
        T.Orb(T.orb_params(), 64, 64, bad)
    det = T.Orb(T.orb_params(), 64, 64, pat)
    with pytest.raises(T.TTError):  # depth without intrinsics
        det.detect(np.zeros((64, 64), np.uint8), np.ones((64, 64), np.float32), None)
    det.destroy()
