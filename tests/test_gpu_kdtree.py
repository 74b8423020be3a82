"""Closest-point association through the device kd-tree (assoc_kdtree; the search the paper's
re-projection replaces, Sec. 2). The kd-tree search is exact for float32 squared distances, so at
the identity its correspondences equal a brute-force float32 nearest-point search bit for bit;
against the FP64 oracle they may differ only where two frame points are equally near to within
float32 rounding, and the vertices stay within the 0.01 mm bar. GPU."""
import numpy as np
import pytest

from paper_2007_08576_amd import synth

pytestmark = pytest.mark.gpu

RMS_TOL_MM = 0.01


@pytest.fixture(scope="module")
def T():
    from paper_2007_08576_amd import tt
    tt.lib()
    return tt


def _intr(mod, K):
    return mod.intrinsics(K.width, K.height, K.fx, K.fy, K.cx, K.cy)


def _rms(a, b):
    return float(np.sqrt(((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2).sum(1).mean()))


def _frame_points(O, depth, K):
    """Pixels with a normal and their back-projections ((u - cx) / fx z, (v - cy) / fy z, z), FP64."""
    _, val = O.normal_map(depth, _intr(O, K))
    valid = np.flatnonzero(val.reshape(-1))
    u, v = valid % K.width, valid // K.width
    z = depth.reshape(-1)[valid].astype(np.float64)
    return valid, np.stack([(u - K.cx) / K.fx * z, (v - K.cy) / K.fy * z, z], axis=1)


def _brute_fp32(q64, valid, pts):
    """Nearest frame point of each query by float32 squared distance (dx^2 + dy^2) + dz^2, ties to the
    lower pixel index (the pixels are in increasing order, and argmin takes the first minimum)."""
    q = q64.astype(np.float32)
    out = np.empty(len(pts), np.int64)
    for c0 in range(0, len(pts), 256):
        p = pts[c0:c0 + 256].astype(np.float32)
        dx = q[None, :, 0] - p[:, None, 0]
        dy = q[None, :, 1] - p[:, None, 1]
        dz = q[None, :, 2] - p[:, None, 2]
        d2 = (dx * dx + dy * dy) + dz * dz
        out[c0:c0 + 256] = valid[np.argmin(d2, axis=1)]
    return out


def test_kd_search_equals_fp32_brute_force_at_the_identity(O, T):
    for sc in (synth.make_config1(1),
               synth.make_sequence(seed=61, M=2500, N=40, K1=200, width=160, height=120, n_frames=2, name="kd")):
        fr = sc.frame(1)
        s = T.Stream(T.default_params(num_control_points=sc.num_control_points, seed=1, assoc_kdtree=1),
                     _intr(T, sc.intr))
        s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
        _, _, dg = s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
        s.destroy()
        valid, q = _frame_points(O, fr.depth, sc.intr)
        ref = _brute_fp32(q, valid, sc.pts)
        assert np.array_equal(dg["corr0"], ref), int((dg["corr0"] != ref).sum())


def test_kd_association_against_the_oracle(O, T):
    sc = synth.make_config1(1)
    fr = sc.frame(1)
    so = O.Stream(O.default_params(num_control_points=sc.num_control_points, seed=1, assoc_kdtree=1),
                  _intr(O, sc.intr))
    sg = T.Stream(T.default_params(num_control_points=sc.num_control_points, seed=1, assoc_kdtree=1),
                  _intr(T, sc.intr))
    so.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    sg.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    vo, _, do = so.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    vg, _, dg = sg.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    sg.destroy()
    # correspondences: equal, except where the two pixels' points are equally near in FP64 to within
    # float32 rounding of the coordinates (1e-4 mm on these 80 mm distances)
    diff = np.flatnonzero(do["corr0"] != dg["corr0"])
    valid, q = _frame_points(O, fr.depth, sc.intr)
    qa = np.full((sc.intr.width * sc.intr.height, 3), np.nan)
    qa[valid] = q
    for j in diff:
        d_o = np.linalg.norm(qa[do["corr0"][j]] - sc.pts[j])
        d_g = np.linalg.norm(qa[dg["corr0"][j]] - sc.pts[j])
        assert abs(d_g - d_o) <= 1e-4, (j, d_o, d_g)
    assert len(diff) <= len(sc.pts) // 100
    rms = _rms(vg, vo)
    print(f"kd association: {len(diff)} near-tie correspondences differ, vertex rms vs oracle {rms:.2e} mm", flush=True)
    assert rms <= RMS_TOL_MM


def test_kd_sequence_against_the_oracle_and_graph_replay(O, T):
    import torch
    sc = synth.make_sequence(seed=62, M=2000, N=36, K1=180, width=128, height=96, n_frames=3, max_step_mm=3.0,
                             name="kdseq")
    so = O.Stream(O.default_params(num_control_points=sc.num_control_points, seed=3, assoc_kdtree=1),
                  _intr(O, sc.intr))
    so.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    vos = [so.track_frame(f.depth, f.feat_xyz, f.feat_desc)[0] for f in (sc.frame(1), sc.frame(2))]
    dev = torch.device("cuda:0")
    frames = [tuple(torch.from_numpy(a).to(dev) for a in (f.depth, f.feat_xyz, f.feat_desc))
              for f in (sc.frame(1), sc.frame(2))]
    torch.cuda.synchronize()
    outs = {}
    for graph in (0, 1):
        s = T.Stream(T.default_params(num_control_points=sc.num_control_points, seed=3, assoc_kdtree=1, graph=graph),
                     _intr(T, sc.intr))
        s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
        ov = torch.zeros((sc.pts.shape[0], 3), dtype=torch.float32, device=dev)
        res = []
        for d in frames:
            s.track_frame_device(d[0], d[1], d[2], d[1].shape[0], ov, None)
            s.sync()
            res.append(ov.cpu().numpy().copy())
        s.destroy()
        outs[graph] = res
    for k in range(2):
        assert np.array_equal(outs[0][k], outs[1][k]), k
        assert _rms(outs[0][k], vos[k]) <= RMS_TOL_MM, (k, _rms(outs[0][k], vos[k]))


def test_kd_option_validation(T):
    import ctypes as C
    p = T.default_params(num_control_points=8, assoc_kdtree=1, assoc_zbuffer=1)
    h = C.c_void_p()
    K = T.intrinsics(16, 12, 10.0, 10.0, 8.0, 6.0)
    assert T.lib().tt_create_stream(C.byref(p), C.byref(K), None, C.byref(h)) == T.TT_EINVAL
