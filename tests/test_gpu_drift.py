"""Drift over a long warm-started sequence (GPU): 300 frames of a small deforming sequence tracked in
order by the library and by the oracle, each side warm-started from its own previous frame, with no
teacher forcing. The FP32 path must stay within the vertex bar of the FP64 one (0.01 mm RMS) at
every frame: rounding differences do not accumulate from frame to frame. Both are also reported
against the generator's ground truth."""
import numpy as np
import pytest

from paper_2007_08576_amd import synth

pytestmark = pytest.mark.gpu

RMS_TOL_MM = 0.01
FRAMES = 300


def _rms(a, b):
    return float(np.sqrt(((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2).sum(1).mean()))


def test_300_warm_started_frames_stay_within_the_vertex_bar(O):
    from paper_2007_08576_amd import tt
    sc = synth.make_sequence(seed=71, M=2000, N=40, K1=200, width=128, height=96, n_frames=FRAMES,
                             max_step_mm=3.0, name="drift")
    K = sc.intr
    g = tt.Stream(tt.default_params(num_control_points=sc.num_control_points, seed=1),
                  tt.intrinsics(K.width, K.height, K.fx, K.fy, K.cx, K.cy))
    o = O.Stream(O.default_params(num_control_points=sc.num_control_points, seed=1),
                 O.intrinsics(K.width, K.height, K.fx, K.fy, K.cx, K.cy))
    g.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    o.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    worst, worst_t, truth_g, truth_o = 0.0, 0, [], []
    for t in range(1, FRAMES + 1):
        fr = sc.frame(t)
        vg = g.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc)[0]
        vo = o.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc)[0]
        d = _rms(vg, vo)
        if d > worst:
            worst, worst_t = d, t
        truth_g.append(_rms(vg, fr.gt_vertices))
        truth_o.append(_rms(vo, fr.gt_vertices))
        assert d <= RMS_TOL_MM, (t, d)
    g.destroy()
    o.close()
    print(f"drift over {FRAMES} frames: GPU vs oracle worst {worst:.2e} mm (frame {worst_t}); truth rms mean "
          f"{np.mean(truth_g):.3f} mm (GPU), {np.mean(truth_o):.3f} mm (oracle)", flush=True)
