"""Parity of the sparse ARAP graph (each control point linked to its k nearest, the alternative to
the dense connection of Sec. 2.2) with the FP64 oracle (GPU). Bars as for the dense connection:
template tables to FP64 rounding, normal equations within 1e-5 relative at iteration 0, vertices
within 0.01 mm RMS after the frame's LM iterations from the same initial warps.
"""
import numpy as np
import pytest

from paper_2007_08576_amd import synth

pytestmark = pytest.mark.gpu

RMS_TOL_MM = 0.01
NE_TOL = 1e-5


@pytest.fixture(scope="module")
def T():
    from paper_2007_08576_amd import tt
    tt.lib()
    return tt


def _intr(mod, K):
    return mod.intrinsics(K.width, K.height, K.fx, K.fy, K.cx, K.cy)


def _pair(O, T, sc, **kw):
    so = O.Stream(O.default_params(num_control_points=sc.num_control_points, **kw), _intr(O, sc.intr))
    sg = T.Stream(T.default_params(num_control_points=sc.num_control_points, **kw), _intr(T, sc.intr))
    so.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    sg.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    return so, sg


def _rms(a, b):
    return float(np.sqrt(((np.asarray(a) - np.asarray(b)) ** 2).sum(1).mean()))


@pytest.mark.parametrize("k", [1, 8])
def test_config1_sparse_arap(O, T, k):
    sc = synth.make_config1(1)
    fr = sc.frame(1)
    so, sg = _pair(O, T, sc, seed=1, arap_knn=k)
    io, ig = so.template_info(), sg.template_info()
    assert abs(io["s_arap"] - ig["s_arap"]) <= 1e-9 * io["s_arap"]
    vo, qo, do = so.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    vg, qg, dg = sg.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    ea = np.linalg.norm(do["A0"] - dg["A0"]) / np.linalg.norm(do["A0"])
    eg = np.linalg.norm(do["g0"] - dg["g0"]) / np.linalg.norm(do["g0"])
    print(f"config 1 arap_knn={k}: |dA|/|A| {ea:.2e}, |dg|/|g| {eg:.2e}, vertex rms {_rms(vo, vg):.2e} mm",
          flush=True)
    assert abs(do["w_arap"] - dg["w_arap"]) <= 1e-6 * do["w_arap"]
    assert ea < NE_TOL and eg < NE_TOL
    # node-pair blocks that are exactly zero in the oracle (off the graph, no shared blend set) are
    # exactly zero here too
    N = so.N
    Bo = do["A0"].reshape(N, 6, N, 6).transpose(0, 2, 1, 3).reshape(N, N, 36)
    Bg = dg["A0"].reshape(N, 6, N, 6).transpose(0, 2, 1, 3).reshape(N, N, 36)
    zero = ~Bo.any(-1)
    assert zero.any() and not Bg[zero].any()
    # the accept decisions agree wherever the oracle's cost change is clear of the FP32 rounding
    # of the GPU's residuals; near convergence the change is at that level and either is right
    clear = np.abs(do["cost_new"] - do["cost_old"]) > 1e-5 * do["cost_old"]
    assert clear[:2].all()
    assert np.array_equal(do["accepted"][clear], dg["accepted"][clear])
    assert _rms(vo, vg) <= RMS_TOL_MM


def test_every_neighbour_equals_dense_on_gpu(T):
    """k = N - 1 keeps every pair: the same arithmetic as the dense connection, bit for bit."""
    sc = synth.make_small_sequence(seed=11, M=1500, N=20, K1=150, width=128, height=96, n_frames=1,
                                   max_step_mm=3.0)
    fr = sc.frame(1)
    out = []
    for k in (0, 19):
        s = T.Stream(T.default_params(num_control_points=20, seed=5, arap_knn=k), _intr(T, sc.intr))
        s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
        out.append(s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc))
        s.destroy()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_sparse_arap_sequence_teacher_forced(O, T):
    sc = synth.make_small_sequence(seed=11, M=2500, N=45, K1=300, width=160, height=120, n_frames=3,
                                   max_step_mm=3.0)
    so, sg = _pair(O, T, sc, seed=5, arap_knn=4)
    for t in range(1, 4):
        fr = sc.frame(t)
        dq, f = so.get_state()
        sg.set_state(dq, f)
        vo, qo, do = so.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
        vg, qg, dg = sg.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
        ea = np.linalg.norm(do["A0"] - dg["A0"]) / np.linalg.norm(do["A0"])
        print(f"frame {t}: |dA|/|A| {ea:.2e}, rms {_rms(vo, vg):.2e} mm", flush=True)
        assert ea < 1e-4
        assert _rms(vo, vg) <= RMS_TOL_MM


def test_config2_full_size_sparse_arap(O, T):
    sc = synth.make_config2(seed=2, n_frames=300)
    fr = sc.frame(1)
    so, sg = _pair(O, T, sc, seed=2, arap_knn=8)
    vg, qg, dg = sg.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    vo, qo, do = so.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    ea = np.linalg.norm(do["A0"] - dg["A0"]) / np.linalg.norm(do["A0"])
    eg = np.linalg.norm(do["g0"] - dg["g0"]) / np.linalg.norm(do["g0"])
    print(f"config 2 arap_knn=8: |dA|/|A| {ea:.2e}, |dg|/|g| {eg:.2e}, vertex rms {_rms(vo, vg):.2e} mm",
          flush=True)
    assert ea < NE_TOL and eg < NE_TOL
    assert _rms(vo, vg) <= RMS_TOL_MM


def test_bad_arap_knn_rejected(T):
    for k in (-1, 33):
        with pytest.raises(T.TTError) as e:
            T.Stream(T.default_params(num_control_points=4, arap_knn=k), T.intrinsics(16, 16, 20.0, 20.0, 8.0, 8.0))
        assert e.value.code == T.TT_EINVAL
