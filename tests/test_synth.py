"""Checks of the seeded synthetic workload generator (CPU only)."""
import numpy as np

from paper_2007_08576_amd import synth


def test_config1_template_is_the_height_field():
    sc = synth.make_config1(1)
    K = sc.intr
    P = sc.pts.astype(np.float64)
    u = K.fx * P[:, 0] / P[:, 2] + K.cx
    v = K.fy * P[:, 1] / P[:, 2] + K.cy
    assert np.allclose(u, np.round(u), atol=1e-3) and np.allclose(v, np.round(v), atol=1e-3)
    z = 80 + 6 * np.sin(np.round(u) / 15) * np.cos(np.round(v) / 20)
    assert np.allclose(P[:, 2], z, atol=1e-4)
    assert len(sc.pts) == 3000 and len(sc.feat_xyz) == 400
    pix = np.round(v) * K.width + np.round(u)
    assert np.all(np.diff(pix) > 0)  # raster order, no repeats


def test_config1_features_outliers_and_bit_flips():
    sc = synth.make_config1(1)
    fr = sc.frame(1)
    assert (fr.inlier_of < 0).sum() == 100 and (fr.inlier_of >= 0).sum() == 300
    inl = fr.inlier_of >= 0
    d = np.unpackbits(fr.feat_desc[inl] ^ sc.feat_desc[fr.inlier_of[inl]], axis=1).sum(1)
    assert np.all(d == 8)
    # exact mode: inlier positions are the warped template features
    ok = np.isfinite(fr.feat_xyz[:, 0])
    assert ok.all()
    assert fr.depth.shape == (96, 128) and (fr.depth > 0).mean() > 0.9


def test_determinism_and_seed_sensitivity():
    a = synth.make_config1(1).frame(1)
    b = synth.make_config1(1).frame(1)
    c = synth.make_config1(2).frame(1)
    assert np.array_equal(a.depth, b.depth) and np.array_equal(a.feat_desc, b.feat_desc)
    assert not np.array_equal(a.feat_desc, c.feat_desc)


def test_render_depth_of_a_plane():
    K = synth.Intrinsics(40, 30, 50.0, 50.0, 20.0, 15.0)
    depth = np.full((30, 40), 100.0, np.float32)
    P = synth.backproject_grid(depth, K)
    P = P + np.array([3.0, -2.0, 5.0])  # shifted plane z = 105
    out = synth.render_depth(P, K)
    cov = out > 0
    assert cov.mean() > 0.7
    assert np.allclose(out[cov], 105.0, atol=1e-4)


def test_sequence_step_is_scaled_to_the_stated_maximum():
    sc = synth.make_small_sequence(seed=3, n_frames=6, max_step_mm=3.0)
    prev = sc.pts.astype(np.float64)
    steps = []
    for t in range(1, 7):
        g = sc.frame(t).gt_vertices
        steps.append(np.linalg.norm(g - prev, axis=1).max())
        prev = g
    assert max(steps) <= 3.0 + 1e-9 and max(steps) > 2.999


def test_rng_uniform_range_and_choice():
    r = synth.Rng(5, "x")
    u = r.uniform(10000)
    assert u.min() >= 0 and u.max() < 1 and abs(u.mean() - 0.5) < 0.02
    c = synth.Rng(5, "y").choice(100, 30)
    assert len(set(c.tolist())) == 30


def test_blob_mask_is_exact_and_seeded():
    m = synth.blob_mask(synth.Rng(3, "t"), 160, 120, 0.3, 8)
    assert m.shape == (120, 160) and m.sum() == round(0.3 * 160 * 120)
    assert np.array_equal(m, synth.blob_mask(synth.Rng(3, "t"), 160, 120, 0.3, 8))
    assert not np.array_equal(m, synth.blob_mask(synth.Rng(4, "t"), 160, 120, 0.3, 8))


def test_stressed_frames_config5_recipe():
    """A fifth of the frames are stressed; a stressed frame has 60 % outliers, at least 30 % of its
    pixels invalid, and sees the scene from the second camera pose (10 deg about an axis through
    the template centroid, then 20 mm)."""
    n = 2000
    frac = np.mean([synth.stressed_frame(9, "x", t, 0.2) for t in range(1, n + 1)])
    assert abs(frac - 0.2) < 4 * np.sqrt(0.2 * 0.8 / n)
    st = synth.Stress()
    sc = synth.make_sequence(seed=77, M=2000, N=48, K1=300, width=160, height=120, n_frames=40,
                             max_step_mm=3.0, name="s5", stress=st)
    t = next(t for t in range(2, 41) if synth.stressed_frame(77, "s5", t, st.prob))
    fr = sc.frame(t)
    assert fr.stressed
    assert (fr.inlier_of < 0).sum() == round(0.6 * 300)
    assert (fr.depth == 0).mean() >= 0.3
    # the same frame without stress differs by the camera's rigid motion only
    plain = synth.make_sequence(seed=77, M=2000, N=48, K1=300, width=160, height=120, n_frames=40,
                                max_step_mm=3.0, name="s5").frame(t)
    assert not plain.stressed and (plain.inlier_of < 0).sum() == round(0.3 * 300)
    P, Q = plain.gt_vertices, fr.gt_vertices
    Pc, Qc = P - P.mean(0), Q - Q.mean(0)
    U, _, Vt = np.linalg.svd(Qc.T @ Pc)
    R = U @ np.diag([1, 1, np.linalg.det(U @ Vt)]) @ Vt
    assert np.allclose(Pc @ R.T, Qc, atol=1e-9)
    ang = np.degrees(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1)))
    assert abs(ang - st.angle_deg) < 1e-6
    c = sc.pts.astype(np.float64).mean(0)
    shift = (Q - ((P - c) @ R.T + c)).mean(0)
    assert abs(np.linalg.norm(shift) - st.shift_mm) < 1e-6


def test_config5_stream_sizes():
    sc = synth.config5_stream(5, 0, n_frames=3)
    assert 200 <= sc.num_control_points <= 1500 and sc.pts.shape[0] == 640 * 480 // 10
    assert sc.intr.width == 640 and sc.feat_xyz.shape[0] == 2000


def test_textured_images_follow_the_depth_and_are_reproducible():
    sc = synth.make_small_sequence(seed=12, M=500, N=8, K1=40, width=160, height=120, n_frames=2,
                                   max_step_mm=2.0)
    d0, i0 = sc.image(0)
    d1, i1 = sc.image(1)
    assert i0.dtype == np.uint8 and i0.shape == (120, 160)
    assert np.array_equal(d1, sc.frame(1).depth)  # the same raster as the frame's depth
    assert np.array_equal(i1, sc.image(1)[1])
    assert i0.std() > 10 and not np.array_equal(i0, i1)
    # background (no surface) is black
    assert (i1[d1 == 0] == 0).all()


def test_orb_pattern_recipe():
    p = synth.orb_pattern(0)
    assert p.shape == (256, 4) and p.dtype == np.int8
    r2 = p[:, 0].astype(int) ** 2 + p[:, 1].astype(int) ** 2
    assert (r2 <= 169).all() and ((p[:, 2].astype(int) ** 2 + p[:, 3].astype(int) ** 2) <= 169).all()
    assert np.array_equal(p, synth.orb_pattern(0)) and not np.array_equal(p, synth.orb_pattern(1))
    assert 4.0 < np.abs(p.astype(float)).mean() < 6.0
