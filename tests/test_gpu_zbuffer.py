"""Parity of the z-buffered projective association (only the template point nearest the camera
takes a pixel) with the FP64 oracle (GPU). The pixel and the visibility decision are integers:
bit-exact wherever the two sides' vertices coincide (the identity warps of a first frame); floating
point as for the plain association (normal equations 1e-5 relative, vertices 0.01 mm RMS).
"""
import numpy as np
import pytest

from paper_2007_08576_amd import synth
from tests import scenes

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
    so = O.Stream(O.default_params(num_control_points=sc.num_control_points, assoc_zbuffer=1, **kw),
                  _intr(O, sc.intr))
    sg = T.Stream(T.default_params(num_control_points=sc.num_control_points, assoc_zbuffer=1, **kw),
                  _intr(T, sc.intr))
    so.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    sg.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    return so, sg


def _rms(a, b):
    return float(np.sqrt(((np.asarray(a) - np.asarray(b)) ** 2).sum(1).mean()))


def test_two_layers_hidden_layer_has_no_pixel(O, T):
    K, depth, pts, nb, nf = scenes.two_layer_scene()
    rng = np.random.default_rng(34)
    desc = rng.integers(0, 256, (4, 32), dtype=np.uint8)
    fi = np.arange(nb, nb + 4)
    out = []
    for mod in (O, T):
        s = mod.Stream(mod.default_params(num_control_points=8, lm_iters=3, assoc_zbuffer=1), _intr(mod, K))
        s.set_template(pts, pts[fi], desc)
        out.append(s.track_frame(depth, pts[fi], desc, debug=True))
    co, cg = out[0][2]["corr0"], out[1][2]["corr0"]
    assert np.array_equal(co, cg)
    assert (cg[:nb] == -1).all() and (cg[nb:nb + nf] >= 0).all() and cg[-1] == -1
    assert _rms(out[0][0], out[1][0]) <= RMS_TOL_MM


def test_config1_zbuffer(O, T):
    sc = synth.make_config1(1)
    fr = sc.frame(1)
    so, sg = _pair(O, T, sc, seed=1)
    vo, qo, do = so.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    vg, qg, dg = sg.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    ea = np.linalg.norm(do["A0"] - dg["A0"]) / np.linalg.norm(do["A0"])
    print(f"config 1 z-buffer: |dA|/|A| {ea:.2e}, vertex rms {_rms(vo, vg):.2e} mm", flush=True)
    assert np.array_equal(do["corr0"], dg["corr0"])
    assert ea < NE_TOL
    assert _rms(vo, vg) <= RMS_TOL_MM


def test_stressed_frames_zbuffer_teacher_forced(O, T):
    """Stressed frames (camera 10 deg / 20 mm away, 30 % of the pixels occluded, 60 % outlier
    matches) of a reduced stream, from the oracle's state before each frame."""
    st = synth.Stress()
    sc = synth.make_sequence(seed=77, M=2000, N=48, K1=300, width=160, height=120, n_frames=40,
                             max_step_mm=3.0, name="s5", stress=st)
    t1 = next(t for t in range(2, 40) if synth.stressed_frame(77, "s5", t, st.prob)
              and not synth.stressed_frame(77, "s5", t + 1, st.prob))
    so, sg = _pair(O, T, sc, seed=7)
    for t in (t1 - 1, t1, t1 + 1):
        fr = sc.frame(t)
        dq, f = so.get_state()
        sg.set_state(dq, f)
        vo, qo, do = so.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
        vg, qg, dg = sg.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
        same = (do["corr0"] == dg["corr0"]).mean()
        print(f"frame {t} stressed={fr.stressed}: corr agree {same:.5f}, rms {_rms(vo, vg):.2e} mm", flush=True)
        assert same > 0.995
        assert _rms(vo, vg) <= RMS_TOL_MM


def test_config2_full_size_zbuffer(O, T):
    sc = synth.make_config2(seed=2, n_frames=300)
    fr = sc.frame(1)
    so, sg = _pair(O, T, sc, seed=2)
    vg, qg, dg = sg.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    vo, qo, do = so.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    ea = np.linalg.norm(do["A0"] - dg["A0"]) / np.linalg.norm(do["A0"])
    print(f"config 2 z-buffer: |dA|/|A| {ea:.2e}, vertex rms {_rms(vo, vg):.2e} mm", flush=True)
    assert np.array_equal(do["corr0"], dg["corr0"])
    assert ea < NE_TOL
    assert _rms(vo, vg) <= RMS_TOL_MM


def test_bad_zbuffer_flag_rejected(T):
    with pytest.raises(T.TTError) as e:
        T.Stream(T.default_params(num_control_points=4, assoc_zbuffer=2), T.intrinsics(16, 16, 20.0, 20.0, 8.0, 8.0))
    assert e.value.code == T.TT_EINVAL
