"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks one step of the oracle against something other than the oracle itself: a
published test vector, brute force on tiny inputs, a closed form, an invariant, or a library
routine (numpy) for a special case.
"""
import math
import os

import numpy as np
import pytest

from paper_2007_08576_amd import synth
from tests import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _intr(O, K):
    return O.intrinsics(K.width, K.height, K.fx, K.fy, K.cx, K.cy)


# ------------------------------------------------------------------------------------------------
# paper constants and the sampler

def test_default_params_match_paper_constants(O):
    p = O.default_params()
    rows = [l.split()[:2] for l in open(os.path.join(GOLDEN, "paper_constants.txt")) if not l.startswith("#")]
    fixed = {k: float(v) for k, v in rows}
    assert p.w_orb == fixed["w_orb"]
    assert p.w_angle == fixed["w_angle"]
    assert p.w_rotation == fixed["w_rotation"]
    assert p.ransac_iters == fixed["ransac_iters"]
    assert p.ransac_refs == fixed["ransac_refs"]


def test_splitmix64_published_vectors(O):
    want = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if not l.startswith("#")]
    got = [int(x) for x in O.splitmix64(0, len(want))]
    assert got == want


# ------------------------------------------------------------------------------------------------
# Hamming matching (Sec. 2.1): brute force

def _popcount_bytes(x):
    return np.unpackbits(x, axis=-1).sum(-1)


def test_hamming_brute_force_and_ties(O):
    rng = np.random.default_rng(5)
    d1 = rng.integers(0, 256, (37, 32), dtype=np.uint8)
    d2 = rng.integers(0, 256, (53, 32), dtype=np.uint8)
    d2[40] = d2[7]  # duplicate: ties must go to the lower index
    d1[3] = d2[7]
    idx, dist = O.hamming_match(d1, d2)
    D = _popcount_bytes(d1[:, None, :] ^ d2[None, :, :])
    assert np.array_equal(dist, D.min(1))
    assert np.array_equal(idx, D.argmin(1))  # argmin returns the first minimum
    assert idx[3] == 7 and dist[3] == 0


def test_hamming_special_distances(O):
    rng = np.random.default_rng(6)
    x = rng.integers(0, 256, (1, 32), dtype=np.uint8)
    _, d = O.hamming_match(x, x)
    assert d[0] == 0
    _, d = O.hamming_match(x, ~x)
    assert d[0] == 256
    y = synth.flip_bits(x, synth.Rng(1, "t"), 8)
    _, d = O.hamming_match(x, y)
    assert d[0] == 8


def test_hamming_empty_frame(O):
    x = np.zeros((4, 32), np.uint8)
    idx, dist = O.hamming_match(x, np.zeros((0, 32), np.uint8))
    assert np.all(idx == -1) and np.all(dist == 256)


# ------------------------------------------------------------------------------------------------
# rotation fit of Eq. (3)

def test_rotation_fit_recovers_noise_free_rotation(O):
    rng = np.random.default_rng(7)
    for _ in range(20):
        R = scenes.quat_to_matrix(rng.normal(size=4))
        S1 = rng.normal(size=(30, 3)) * 20
        S2 = S1 @ R.T
        M = S2.T @ S1
        Rf, sig, deg = O.rotation_fit(M)
        assert not deg
        assert np.abs(Rf - R).max() < 1e-12


def test_rotation_fit_matches_numpy_svd(O):
    rng = np.random.default_rng(8)
    for _ in range(50):
        M = rng.normal(size=(3, 3))
        U, s, Vt = np.linalg.svd(M)
        d = np.sign(np.linalg.det(U @ Vt))
        Rref = U @ np.diag([1, 1, d]) @ Vt
        Rf, sig, deg = O.rotation_fit(M)
        assert not deg
        assert np.abs(Rf - Rref).max() < 1e-10
        assert np.allclose(sig, s, rtol=1e-12, atol=1e-12)
        assert abs(np.linalg.det(Rf) - 1) < 1e-12


def test_rotation_fit_degenerate(O):
    a = np.array([1.0, 2.0, 3.0])
    b = np.array([0.5, -1.0, 2.0])
    _, _, deg = O.rotation_fit(np.outer(a, b))  # rank 1: one match does not fix R
    assert deg
    _, _, deg = O.rotation_fit(np.zeros((3, 3)))
    assert deg


# ------------------------------------------------------------------------------------------------
# 1-point RANSAC + reweighting (Sec. 2.1, Eqs. (2)-(4))

def _planted_matches(rng, n_in, n_out, H, noise=0.0):
    o1 = rng.uniform(-40, 40, size=(n_in + n_out, 3))
    R = scenes.quat_to_matrix(rng.normal(size=4))
    t = rng.normal(size=3) * 10
    o2 = o1 @ R.T + t
    o2[:n_in] += noise * rng.normal(size=(n_in, 3))
    # outliers displaced far beyond 5H
    o2[n_in:] += rng.normal(size=(n_out, 3)) / np.sqrt(3) * 0 + \
        (rng.uniform(20 * H, 40 * H, size=(n_out, 1)) * _unit(rng, n_out))
    return o1, o2


def _unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_preselect_exhaustive_planted_inliers(O):
    rng = np.random.default_rng(9)
    H = 3.0
    o1, o2 = _planted_matches(rng, 30, 12, H)
    usable = np.ones(42, np.uint8)
    r = O.preselect(o1, o2, usable, H, refs=0, iters=10)
    assert r["n"] == 42
    assert np.array_equal(r["preselected"], np.r_[np.ones(30), np.zeros(12)].astype(np.uint8))
    # every inlier reference fits the rigid motion exactly: all inliers at weight 1
    assert np.all(r["hyp_kept"][:30] == 1) and np.all(r["hyp_kept"][30:42] == 0)
    assert np.allclose(r["wstar"][:30], 1.0)
    assert np.all(r["hyp_nin"][:30] == 30)


def test_preselect_no_outliers_keeps_everything(O):
    rng = np.random.default_rng(10)
    o1, o2 = _planted_matches(rng, 25, 0, 3.0)
    r = O.preselect(o1, o2, np.ones(25, np.uint8), 3.0, refs=0, iters=10)
    assert np.all(r["hyp_kept"][:25] == 1)
    assert np.allclose(r["wstar"], 1.0) and r["preselected"].all()
    assert np.allclose(r["hyp_W"][:25], 25.0)


def test_preselect_weight_formula_at_one_reference(O):
    """With one inlier reference and exact rigid inliers, Eq. (4) gives w_k = min(H/d_k, 1)
    for an outlier displaced by a known distance from its rigid image."""
    rng = np.random.default_rng(11)
    H = 3.0
    o1 = rng.uniform(-30, 30, size=(12, 3))
    o2 = o1.copy()  # identity motion
    shift = np.array([0.0, 0.0, 10.0 * H])
    o2[11] += shift  # one outlier at distance 30 = 10 H from its image
    usable = np.ones(12, np.uint8)
    r = O.preselect(o1, o2, usable, H, refs=0, iters=10)
    # with reference k0 = 0 the fitted rotation stays close to identity and the outlier keeps
    # d = |shift| up to the tiny rotation the weighted fit allows
    assert r["hyp_kept"][0] == 1
    assert abs(r["wstar"][11] - 0.1) < 2e-3
    assert r["preselected"][:11].all() and not r["preselected"][11]


def test_preselect_unusable_and_degenerate(O):
    rng = np.random.default_rng(12)
    o1, o2 = _planted_matches(rng, 10, 0, 3.0)
    usable = np.zeros(10, np.uint8)
    r = O.preselect(o1, o2, usable, 3.0, refs=30)
    assert r["n"] == 0 and not r["preselected"].any() and np.all(r["wstar"] == 0)
    usable[4] = 1  # a single usable match cannot fix a rotation
    r = O.preselect(o1, o2, usable, 3.0, refs=30)
    assert r["n"] == 1 and r["hyp_kept"][0] == 2 and not r["preselected"].any()


def test_preselect_sampler_is_partial_fisher_yates(O):
    """The drawn references follow the partial Fisher-Yates shuffle of the usable list driven by
    SplitMix64 seeded with seed + golden * (frame + 1)."""
    rng = np.random.default_rng(13)
    K = 90
    o1, o2 = _planted_matches(rng, 60, 30, 3.0)
    usable = (rng.uniform(size=K) > 0.2).astype(np.uint8)
    seed, frame = 1234567, 5
    r = O.preselect(o1, o2, usable, 3.0, refs=30, iters=2, seed=seed, frame=frame)
    U = list(np.flatnonzero(usable))
    st = (seed + 0x9E3779B97F4A7C15 * (frame + 1)) & 0xFFFFFFFFFFFFFFFF
    draws = O.splitmix64(st, 30)
    for i in range(30):
        j = i + int(draws[i]) % (len(U) - i)
        U[i], U[j] = U[j], U[i]
    assert list(r["hyp_k0"][:30]) == U[:30]
    assert len(set(U[:30])) == 30


# ------------------------------------------------------------------------------------------------
# target normals

def test_normals_of_a_plane_and_validity(O):
    K = synth.Intrinsics(40, 30, 50.0, 55.0, 19.5, 14.0)
    n_true = np.array([0.3, -0.2, -1.0])
    n_true /= np.linalg.norm(n_true)
    d = -90.0  # plane n.X = d, in front of the camera
    u = np.arange(40)[None, :]
    v = np.arange(30)[:, None]
    ray = np.stack([(u - K.cx) / K.fx + 0 * v, (v - K.cy) / K.fy + 0 * u, np.ones((30, 40))], -1)
    depth = (d / (ray @ n_true)).astype(np.float32)
    depth[10, 10] = np.nan
    depth[20, 5] = -1.0
    nrm, val = O.normal_map(depth, _intr(O, K))
    bad = np.zeros((30, 40), bool)
    bad[0, :] = bad[-1, :] = bad[:, 0] = bad[:, -1] = True
    for (a, b) in [(10, 10), (20, 5)]:
        bad[a, b] = True
        for (da, db) in [(-1, 0), (1, 0), (0, -1), (0, 1)]:
            bad[a + da, b + db] = True
    assert np.array_equal(val.astype(bool), ~bad)
    got = nrm[~bad]
    assert np.abs(got - n_true).max() < 1e-5  # float32 depth rounding
    assert np.all(nrm[bad] == 0)


# ------------------------------------------------------------------------------------------------
# dual-quaternion blending (Sec. 2, after DynamicFusion)

def test_dqb_identity_is_exact(O):
    rng = np.random.default_rng(14)
    dq = np.tile(np.r_[1.0, 0, 0, 0, 0, 0, 0, 0], (6, 1))
    for _ in range(20):
        p = rng.uniform(-100, 100, 3)
        nodes = rng.choice(6, 4, replace=False).astype(np.int32)
        a = rng.uniform(0.1, 1, 4)
        a /= a.sum()
        assert np.array_equal(O.dqb(dq, nodes, a, p), p)


def test_dqb_common_rigid_and_sign_invariance(O):
    rng = np.random.default_rng(15)
    W = scenes.random_dq(rng, 1, 30.0, 10.0)[0]
    R, t = scenes.dq_rt(W)
    dq = np.tile(W, (5, 1))
    dq[2] *= -1  # antipodal representation of the same transform
    for _ in range(10):
        p = rng.uniform(-50, 50, 3)
        a = rng.uniform(0.1, 1, 4)
        a /= a.sum()
        v = O.dqb(dq, np.array([0, 2, 3, 4], np.int32), a, p)
        assert np.abs(v - (R @ p + t)).max() < 1e-12
    q = W[:4]
    assert np.abs(O.dq_transform(O.dq_from_rt(q, t), np.array([1.0, 2.0, 3.0])) -
                  (R @ np.array([1.0, 2.0, 3.0]) + t)).max() < 1e-12


# ------------------------------------------------------------------------------------------------
# template set-up: farthest-point sampling, blend neighbours and weights

def _small_scene(seed=21, N=6, M=300, K1=24, width=64, height=48):
    return synth.make_small_sequence(seed=seed, M=M, N=N, K1=K1, width=width, height=height,
                                     n_frames=1, max_step_mm=2.0)


def test_fps_knn_alpha_brute_force(O):
    sc = _small_scene(N=10)
    s = O.Stream(O.default_params(num_control_points=10), _intr(O, sc.intr))
    s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    info = s.template_info()
    P = sc.pts.astype(np.float64)
    idx = info["node_idx"]
    assert idx[0] == 0 and len(set(idx)) == 10
    for i in range(1, 10):
        dmin = ((P[:, None, :] - P[None, idx[:i], :]) ** 2).sum(-1).min(1)
        assert dmin[idx[i]] == dmin.max()
        assert idx[i] == np.flatnonzero(dmin == dmin.max())[0]
    C = P[idx]
    Dn = np.sqrt(((C[:, None] - C[None]) ** 2).sum(-1)) + np.diag(np.full(10, np.inf))
    sbar = Dn.min(1).mean()
    assert abs(info["sbar"] - sbar) < 1e-12 * sbar
    for X, knn, al in [(P, info["knn_pts"], info["alpha_pts"]),
                       (sc.feat_xyz.astype(np.float64), info["knn_feat"], info["alpha_feat"])]:
        D = ((X[:, None, :] - C[None, :, :]) ** 2).sum(-1)
        order = np.argsort(D, axis=1, kind="stable")[:, :4]
        assert np.array_equal(knn, order)
        g = np.exp(-np.take_along_axis(D, order, 1) / (2 * sbar ** 2))
        assert np.allclose(al, g / g.sum(1, keepdims=True), rtol=1e-12, atol=1e-15)
    sa = 2 * sbar
    Wp = np.exp(-((C[:, None] - C[None]) ** 2).sum(-1) / (2 * sa ** 2))
    assert abs(info["s_arap"] - (Wp.sum() - 10)) < 1e-10 * info["s_arap"]


def test_template_errors(O):
    sc = _small_scene()
    p = O.default_params(num_control_points=400)
    s = O.Stream(p, _intr(O, sc.intr))
    with pytest.raises(O.OracleError):
        s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)  # N > M
    s = O.Stream(O.default_params(num_control_points=3), _intr(O, sc.intr))
    dup = np.tile(sc.pts[:1], (5, 1))
    with pytest.raises(O.OracleError):
        s.set_template(dup, sc.feat_xyz, sc.feat_desc)  # fewer distinct points than nodes
    bad = sc.pts.copy()
    bad[3, 1] = np.nan
    with pytest.raises(O.OracleError):
        s.set_template(bad, sc.feat_xyz, sc.feat_desc)


# ------------------------------------------------------------------------------------------------
# residuals, Jacobians and normal equations of Eq. (1)

def _frame_ready_stream(O, N=6, seed=21):
    sc = _small_scene(seed=seed, N=N)
    fr = sc.frame(1)
    s = O.Stream(O.default_params(num_control_points=N, seed=3), _intr(O, sc.intr))
    s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    s.frame_begin(fr.depth, fr.feat_xyz, fr.feat_desc)
    return s, sc, fr


def test_jacobian_matches_central_differences(O):
    s, sc, fr = _frame_ready_stream(O)
    rng = np.random.default_rng(16)
    dq = scenes.random_dq(rng, s.N, 4.0, 1.5)
    r, J, wa = s.residuals(dq, jacobian=True)
    assert wa > 0
    n = 6 * s.N
    Jfd = np.zeros_like(J)
    h = 1e-6
    for c in range(n):
        e = np.zeros(n)
        e[c] = h
        rp, _ = s.residuals(s.apply_increment(dq, e), dq_assoc=dq, w_arap=wa)
        rm, _ = s.residuals(s.apply_increment(dq, -e), dq_assoc=dq, w_arap=wa)
        Jfd[:, c] = (rp - rm) / (2 * h)
    rows_icp = slice(0, s.M)
    rows_orb = slice(s.M, s.M + 3 * s.K1)
    rows_arap = slice(s.M + 3 * s.K1, None)
    for sl in (rows_icp, rows_orb, rows_arap):
        assert np.abs(J[sl]).max() > 0
        err = np.linalg.norm(J[sl] - Jfd[sl]) / np.linalg.norm(J[sl])
        assert err < 1e-6, err


def test_jacobian_closed_form_at_common_rigid_state(O):
    """At a common rigid state the blend stays rigid to first order under one node's increment:
    dv/d(omega_i, tau_i) = alpha_i [-[v - p_i]x, I]."""
    s, sc, fr = _frame_ready_stream(O)
    rng = np.random.default_rng(17)
    W = scenes.random_dq(rng, 1, 10.0, 3.0)[0]
    dq = np.tile(W, (s.N, 1))
    R, t = scenes.dq_rt(W)
    r, J, wa = s.residuals(dq, jacobian=True)
    info = s.template_info()
    C = sc.pts.astype(np.float64)[info["node_idx"]]
    pos = C @ R.T + t
    # feature rows carry sqrt(w_orb w_k) (DQB(o1) - o2)
    _, _, dbg = None, None, None
    P = sc.feat_xyz.astype(np.float64)
    checked = 0
    for k in range(s.K1):
        rows = slice(s.M + 3 * k, s.M + 3 * k + 3)
        if not np.any(J[rows]):
            continue
        v = R @ P[k] + t
        sw = None
        for slot in range(4):
            i = info["knn_feat"][k, slot]
            a = info["alpha_feat"][k, slot]
            d = v - pos[i]
            blk = np.hstack([-np.array([[0, -d[2], d[1]], [d[2], 0, -d[0]], [-d[1], d[0], 0]]), np.eye(3)]) * a
            got = J[rows, 6 * i:6 * i + 6]
            if sw is None:
                sw = got[0, 3] / blk[0, 3]
            assert np.abs(got - sw * blk).max() < 1e-9 * max(1.0, np.abs(got).max())
        checked += 1
    assert checked > 5


def test_arap_zero_under_common_rigid_motion(O):
    s, sc, fr = _frame_ready_stream(O)
    rng = np.random.default_rng(18)
    W = scenes.random_dq(rng, 1, 25.0, 8.0)[0]
    dq = np.tile(W, (s.N, 1))
    r, wa = s.residuals(dq)
    assert wa > 0
    assert np.abs(r[s.M + 3 * s.K1:]).max() < 1e-12


def test_arap_two_node_closed_forms(O):
    """Two nodes: a rotation of node a by theta about an axis normal to the rest offset, about
    its own position, gives chordal angle residual 2 sin(theta/2) and rotation residual
    2 sin(theta/4) (both times the square-root weights); a stretch gives the length change."""
    K = synth.Intrinsics(8, 8, 10.0, 10.0, 4.0, 4.0)
    pts = np.array([[0.0, 0.0, 100.0], [10.0, 0.0, 100.0], [5.0, 1.0, 100.0]], np.float32)
    p = O.default_params(num_control_points=2)
    s = O.Stream(p, _intr(O, K))
    s.set_template(pts, np.zeros((0, 3), np.float32), np.zeros((0, 32), np.uint8))
    s.frame_begin(np.zeros((8, 8), np.float32), np.zeros((0, 3), np.float32), np.zeros((0, 32), np.uint8))
    info = s.template_info()
    assert list(info["node_idx"]) == [0, 1]
    wab = math.exp(-100.0 / (2 * (2 * info["sbar"]) ** 2))
    theta = 0.3
    q = np.array([math.cos(theta / 2), 0, 0, math.sin(theta / 2)])  # about z, normal to e0 = x
    c0 = pts[0].astype(np.float64)
    tq = c0 - scenes.quat_to_matrix(q) @ c0  # rotate about node 0's own position
    dq = np.zeros((2, 8))
    dq[0, :4] = q
    dq[0, 4:] = 0.5 * scenes.quat_mul(np.r_[0.0, tq], q)
    dq[1, 0] = 1.0
    w_arap = 2.0
    r, _ = s.residuals(dq, w_arap=w_arap)
    rows = r[s.M:].reshape(2, 8)  # ordered pairs (0,1) and (1,0)
    sl, sa, sr = (math.sqrt(w_arap * wab), math.sqrt(w_arap * wab * 20.0), math.sqrt(w_arap * wab * 100.0))
    assert abs(rows[0, 0]) < 1e-12  # length unchanged
    assert abs(np.linalg.norm(rows[0, 1:4]) - sa * 2 * math.sin(theta / 2)) < 1e-12
    assert abs(np.linalg.norm(rows[0, 4:8]) - sr * 2 * math.sin(theta / 4)) < 1e-12
    assert abs(np.linalg.norm(rows[1, 1:4])) < 1e-12  # node 1 is not rotated: its angle term is 0
    # stretch: move node 1 by 2 mm along e0
    dq2 = np.zeros((2, 8))
    dq2[:, 0] = 1.0
    dq2[1, 4:] = 0.5 * np.r_[0.0, 2.0, 0.0, 0.0]
    r, _ = s.residuals(dq2, w_arap=w_arap)
    rows = r[s.M:].reshape(2, 8)
    assert abs(rows[0, 0] - sl * 2.0) < 1e-12 and abs(rows[1, 0] - sl * 2.0) < 1e-12


def test_normal_equations_equal_dense_products(O):
    s, sc, fr = _frame_ready_stream(O)
    rng = np.random.default_rng(19)
    dq = scenes.random_dq(rng, s.N, 3.0, 1.0)
    r, J, wa = s.residuals(dq, jacobian=True)
    A, g = s.normal_equations(dq, w_arap=wa)
    assert np.abs(A - J.T @ J).max() < 1e-9 * np.abs(A).max()
    assert np.abs(g - J.T @ r).max() < 1e-9 * np.abs(g).max()
    # and the finite-difference Jacobian gives the same normal matrix to FD accuracy
    n = 6 * s.N
    Jfd = np.zeros_like(J)
    h = 1e-6
    for c in range(n):
        e = np.zeros(n)
        e[c] = h
        rp, _ = s.residuals(s.apply_increment(dq, e), dq_assoc=dq, w_arap=wa)
        rm, _ = s.residuals(s.apply_increment(dq, -e), dq_assoc=dq, w_arap=wa)
        Jfd[:, c] = (rp - rm) / (2 * h)
    assert np.linalg.norm(A - Jfd.T @ Jfd) < 1e-6 * np.linalg.norm(A)


# ------------------------------------------------------------------------------------------------
# Cholesky

def test_cholesky_against_numpy(O):
    rng = np.random.default_rng(20)
    B = rng.normal(size=(40, 40))
    A = B @ B.T + 40 * np.eye(40)
    L, rc = O.cholesky(A)
    assert rc == 0
    assert np.abs(L - np.linalg.cholesky(A)).max() < 1e-12 * np.abs(L).max()
    b = rng.normal(size=40)
    x = O.cholesky_solve(L, b)
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) < 1e-12
    A[5, 5] = -1.0
    _, rc = O.cholesky(A)
    assert rc > 0


# ------------------------------------------------------------------------------------------------
# Levenberg-Marquardt end to end

def test_lm_no_deformation_returns_identity_exactly(O):
    """Target = template on a plane whose depths and back-projections are exact: every residual
    is exactly 0 in FP64, so the step is 0 and the warps stay the identity bit for bit."""
    K, depth, P = scenes.dyadic_plane()
    pts = P[2:-2, 2:-2].reshape(-1, 3).astype(np.float32)
    rng = np.random.default_rng(22)
    fi = rng.choice(len(pts), 12, replace=False)
    desc = rng.integers(0, 256, (12, 32), dtype=np.uint8)
    s = O.Stream(O.default_params(num_control_points=8), _intr(O, K))
    s.set_template(pts, pts[fi], desc)
    v, dq, dbg = s.track_frame(depth, pts[fi], desc, debug=True)
    ident = np.tile(np.r_[1.0, 0, 0, 0, 0, 0, 0, 0], (8, 1))
    assert np.array_equal(dq, ident)
    assert np.array_equal(v, pts.astype(np.float64))
    assert np.all(dbg["cost_old"] == 0.0)
    assert (dbg["corr0"] >= 0).sum() == len(pts)


def test_lm_recovers_rigid_motion_from_features_exactly(O):
    """Features only (all depth invalid), exact o2 = G(o1) for a rigid G on a Pythagorean
    lattice: zero ARAP cost forces a common rigid motion and the 25 features fix it."""
    pts, feats, R, t = scenes.lattice_scene()
    o2 = feats @ R.T + t
    assert np.array_equal(o2.astype(np.float32).astype(np.float64), o2)
    K = synth.Intrinsics(16, 16, 20.0, 20.0, 8.0, 8.0)
    rng = np.random.default_rng(23)
    desc = rng.integers(0, 256, (25, 32), dtype=np.uint8)
    p = O.default_params(num_control_points=12, lm_iters=10)
    s = O.Stream(p, _intr(O, K))
    s.set_template(pts.astype(np.float32), feats.astype(np.float32), desc)
    v, dq, dbg = s.track_frame(np.zeros((16, 16), np.float32), o2.astype(np.float32), desc, debug=True)
    assert dbg["preselected"].all()
    want = pts @ R.T + t
    assert np.abs(v - want).max() < 1e-9
    for i in range(s.N):
        Ri, ti = scenes.dq_rt(dq[i])
        assert np.abs(Ri - R).max() < 1e-12 and np.abs(ti - t).max() < 1e-9


def test_lm_recovers_rigid_motion_with_icp_on_a_plane(O):
    """ICP + features on a tilted plane moved rigidly; point-to-plane is exact for a plane, so
    the only error left is the float32 rounding of the rendered target depth (~1e-5 mm)."""
    K = synth.Intrinsics(64, 48, 70.0, 70.0, 32.0, 24.0)
    u = np.arange(64)[None, :]
    v = np.arange(48)[:, None]
    n0 = np.array([0.2, -0.1, -1.0])
    n0 /= np.linalg.norm(n0)
    d0 = -100.0
    ray = np.stack([(u - K.cx) / K.fx + 0 * v, (v - K.cy) / K.fy + 0 * u, np.ones((48, 64))], -1)
    depth0 = d0 / (ray @ n0)
    P0 = ray * depth0[..., None]
    pts = P0[4:-4:2, 4:-4:2].reshape(-1, 3)
    rng = np.random.default_rng(24)
    R = scenes.quat_to_matrix(np.r_[1.0, 0.02, -0.015, 0.01])
    t = np.array([1.0, -0.5, 0.8])
    n1 = R @ n0
    d1 = d0 + n1 @ t
    depth1 = (d1 / (ray @ n1)).astype(np.float32)
    fi = rng.choice(len(pts), 30, replace=False)
    desc = rng.integers(0, 256, (30, 32), dtype=np.uint8)
    o1 = pts[fi].astype(np.float32)
    o2 = (o1.astype(np.float64) @ R.T + t).astype(np.float32)
    s = O.Stream(O.default_params(num_control_points=10), _intr(O, K))
    s.set_template(pts.astype(np.float32), o1, desc)
    vtx, dq, dbg = s.track_frame(depth1, o2, desc, debug=True)
    want = pts.astype(np.float32).astype(np.float64) @ R.T + t
    assert (dbg["corr0"] >= 0).mean() > 0.9
    assert np.sqrt(((vtx - want) ** 2).sum(1).mean()) < 1e-4


def test_lm_step_rule_and_cost_bookkeeping(O):
    """Accepted steps lower the frozen-weight cost; lambda moves by exactly x0.1 / x10."""
    sc = synth.make_config1(1)
    fr = sc.frame(1)
    s = O.Stream(O.default_params(num_control_points=64, seed=1), _intr(O, sc.intr))
    s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    v, dq, d = s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    lam = d["lambda"]
    for t in range(len(lam) - 1):
        if d["accepted"][t]:
            assert d["cost_new"][t] < d["cost_old"][t]
            assert lam[t + 1] == max(lam[t] / 10, 1e-10)
        else:
            assert lam[t + 1] == min(lam[t] * 10, 1e10)
    # tracking improves on the identity
    rms = np.sqrt(((v - fr.gt_vertices) ** 2).sum(1).mean())
    rms0 = np.sqrt(((sc.pts - fr.gt_vertices) ** 2).sum(1).mean())
    assert rms < 0.25 * rms0


def test_frame_counter_and_state_roundtrip(O):
    sc = _small_scene()
    fr = sc.frame(1)
    s = O.Stream(O.default_params(num_control_points=6, lm_iters=2), _intr(O, sc.intr))
    s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    dq0, f0 = s.get_state()
    assert f0 == 0
    s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc)
    dq1, f1 = s.get_state()
    assert f1 == 1
    s.set_state(dq0, 0)
    s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc)
    dq2, _ = s.get_state()
    assert np.array_equal(dq1, dq2)  # deterministic replay


# ------------------------------------------------------------------------------------------------
# further pins (each one guards a step that the tests above leave free)

def test_preselect_keeps_a_second_locally_rigid_cluster(O):
    """Sec. 2.1's premise: deformation is locally rigid. Two clusters share a rotation but the
    second one is displaced by a further 40 mm; each cluster fits its own references exactly.
    The second cluster's hypotheses score 0.55-0.9 of the best one, above the keep ratio of 1/2,
    so both clusters are pre-selected; the far outliers are not."""
    rng = np.random.default_rng(30)
    H = 3.0
    A = rng.uniform(-10, 10, size=(30, 3))
    B = rng.uniform(-10, 10, size=(16, 3)) + np.array([100.0, 0, 0])
    R = scenes.quat_to_matrix(np.r_[1.0, 0.1, -0.05, 0.0])
    o1 = np.vstack([A, B, rng.uniform(-50, 50, size=(4, 3))])
    o2 = np.vstack([A @ R.T, B @ R.T + np.array([0.0, 40.0, 0.0]),
                    rng.uniform(-50, 50, size=(4, 3)) + 300])
    r = O.preselect(o1, o2, np.ones(50, np.uint8), H, refs=0, iters=10)
    assert np.array_equal(r["preselected"], np.r_[np.ones(46), np.zeros(4)].astype(np.uint8))
    assert r["hyp_W"][:30].max() == r["hyp_W"].max()
    ratio = r["hyp_W"][30:46] / r["hyp_W"].max()
    assert np.all(r["hyp_kept"][:46] == 1) and np.all(r["hyp_kept"][46:] == 0)
    assert np.all((ratio > 0.5) & (ratio < 0.95)), ratio


def test_fps_ties_go_to_lowest_index(O):
    """On an integer lattice many squared distances tie exactly; the brute-force rule is:
    next node = the lowest index attaining the largest distance to the chosen set."""
    g = np.arange(6, dtype=np.float64)
    X, Y = np.meshgrid(g, g)
    pts = np.stack([X.ravel(), Y.ravel(), np.full(36, 50.0)], 1)
    K = synth.Intrinsics(8, 8, 10.0, 10.0, 4.0, 4.0)
    s = O.Stream(O.default_params(num_control_points=9), _intr(O, K))
    s.set_template(pts.astype(np.float32), np.zeros((0, 3), np.float32), np.zeros((0, 32), np.uint8))
    idx = s.template_info()["node_idx"]
    chosen = [0]
    for i in range(1, 9):
        dmin = ((pts[:, None, :] - pts[None, chosen, :]) ** 2).sum(-1).min(1)
        chosen.append(int(np.flatnonzero(dmin == dmin.max())[0]))
    assert list(idx) == chosen
    ties = sum(int((((pts[:, None, :] - pts[None, chosen[:i], :]) ** 2).sum(-1).min(1) ==
                    (((pts[:, None, :] - pts[None, chosen[:i], :]) ** 2).sum(-1).min(1)).max()).sum() > 1)
               for i in range(1, 9))
    assert ties >= 3


def test_projective_association_is_nearest_pixel(O):
    """Sec. 2's re-projection: a template point corresponds to the pixel whose centre is nearest
    to its projection (brute force over all pixel centres)."""
    K = synth.Intrinsics(24, 20, 30.0, 33.0, 11.5, 9.25)
    depth = np.full((20, 24), 100.0, np.float32)
    rng = np.random.default_rng(31)
    uv = np.stack([rng.uniform(1.5, 21.5, 400), rng.uniform(1.5, 17.5, 400)], 1)
    z = rng.uniform(60, 140, 400)
    pts = np.stack([(uv[:, 0] - K.cx) / K.fx * z, (uv[:, 1] - K.cy) / K.fy * z, z], 1).astype(np.float32)
    s = O.Stream(O.default_params(num_control_points=5, lm_iters=1), _intr(O, K))
    s.set_template(pts, np.zeros((0, 3), np.float32), np.zeros((0, 32), np.uint8))
    _, _, dbg = s.track_frame(depth, np.zeros((0, 3), np.float32), np.zeros((0, 32), np.uint8), debug=True)
    P = pts.astype(np.float64)
    pu = K.fx * P[:, 0] / P[:, 2] + K.cx
    pv = K.fy * P[:, 1] / P[:, 2] + K.cy
    cu, cv = np.meshgrid(np.arange(24), np.arange(20))
    d2 = (pu[:, None] - cu.ravel()[None]) ** 2 + (pv[:, None] - cv.ravel()[None]) ** 2
    want = d2.argmin(1)
    amb = np.sort(d2, 1)[:, 1] - np.sort(d2, 1)[:, 0] < 1e-9
    got = dbg["corr0"]
    assert np.all((got == want) | amb)
    # the point-to-plane residual against the fronto-parallel target is z - 100 along n = -z
    assert np.allclose(dbg["r0"], -(P[:, 2] - 100.0), atol=1e-9)


def test_tukey_weights_on_known_residuals(O):
    """Tukey's biweight (Sec. 2): weight (1 - (r/c)^2)^2 inside |r| < c, 0 outside."""
    K = synth.Intrinsics(24, 20, 30.0, 30.0, 12.0, 10.0)
    depth = np.full((20, 24), 100.0, np.float32)
    dz = np.linspace(-7.0, 7.0, 57)
    uv = np.stack([np.tile(np.arange(4, 19), 4)[:57], np.repeat(np.arange(4, 8), 15)[:57]], 1).astype(np.float64)
    z = 100.0 + dz
    pts = np.stack([(uv[:, 0] - K.cx) / K.fx * z, (uv[:, 1] - K.cy) / K.fy * z, z], 1).astype(np.float32)
    s = O.Stream(O.default_params(num_control_points=4, lm_iters=1, tukey_c=5.0), _intr(O, K))
    s.set_template(pts, np.zeros((0, 3), np.float32), np.zeros((0, 32), np.uint8))
    _, _, dbg = s.track_frame(depth, np.zeros((0, 3), np.float32), np.zeros((0, 32), np.uint8), debug=True)
    r = -(pts[:, 2].astype(np.float64) - 100.0)
    want = np.where(np.abs(r) < 5.0, (1 - (r / 5.0) ** 2) ** 2, 0.0)
    assert np.all(dbg["corr0"] >= 0)
    assert np.allclose(dbg["omega0"], want, atol=1e-12)


def test_orb_weights_of_preselected_and_other_matches(O):
    """Sec. 2.1, last paragraph: pre-selected matches keep their pre-selection weight; the
    others get w = clamp(1 - d/(5H), 0, 1) of their current distance d."""
    pts, feats, R, t = scenes.lattice_scene(n_side=25, f_half=4)
    nf = len(feats)
    o2 = feats.copy()
    H = 3.0
    o2[3] += np.array([0, 0, 3.0 * H])    # w* = H/d = 1/3 -> not pre-selected, ramp 1 - 0.6
    o2[7] += np.array([0, 4.0 * H, 0])    # ramp 1 - 0.8
    o2[11] += np.array([6.0 * H, 0, 0])   # ramp clamps to 0
    o2[15] += np.array([0, 1.5 * H, 0])   # w* = 1/1.5 -> pre-selected with that weight
    K = synth.Intrinsics(16, 16, 20.0, 20.0, 8.0, 8.0)
    desc = np.random.default_rng(32).integers(0, 256, (nf, 32), dtype=np.uint8)
    s = O.Stream(O.default_params(num_control_points=12, lm_iters=1, H=H), _intr(O, K))
    s.set_template(pts.astype(np.float32), feats.astype(np.float32), desc)
    _, _, dbg = s.track_frame(np.zeros((16, 16), np.float32), o2.astype(np.float32), desc, debug=True)
    pre = dbg["preselected"].astype(bool)
    assert not pre[3] and not pre[7] and not pre[11] and pre[15]
    w = dbg["orbw0"]
    assert abs(w[3] - 0.4) < 1e-9 and abs(w[7] - 0.2) < 1e-9 and w[11] == 0.0
    # the weighted rotation fit leans slightly towards the displaced matches, so w* is near 1/1.5
    assert abs(w[15] - 1 / 1.5) < 0.05 and w[15] == dbg["wstar"][15]
    others = np.setdiff1d(np.arange(nf), [3, 7, 11, 15])
    assert np.allclose(w[others], 1.0)


def test_increment_is_exact_rotation_about_the_node(O):
    """A node-centred increment (omega, tau) maps the node's warp W to x -> Exp(omega)(W(x) - p)
    + p + tau with p = W(p^0); Exp by Rodrigues' formula."""
    sc = _small_scene()
    s = O.Stream(O.default_params(num_control_points=6), _intr(O, sc.intr))
    s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    rng = np.random.default_rng(33)
    dq = scenes.random_dq(rng, 6, 20.0, 5.0)
    delta = rng.normal(size=36) * 0.3
    out = s.apply_increment(dq, delta)
    info = s.template_info()
    C = sc.pts.astype(np.float64)[info["node_idx"]]
    for i in range(6):
        R, t = scenes.dq_rt(dq[i])
        p = R @ C[i] + t
        om, tau = delta[6 * i:6 * i + 3], delta[6 * i + 3:6 * i + 6]
        th = np.linalg.norm(om)
        k = om / th
        Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
        Rw = np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * Kx @ Kx
        R2, t2 = scenes.dq_rt(out[i])
        x = rng.normal(size=3) * 30
        assert np.abs((R2 @ x + t2) - (Rw @ (R @ x + t - p) + p + tau)).max() < 1e-10
        assert out[i, 0] >= 0 and abs(np.linalg.norm(out[i, :4]) - 1) < 1e-14


def test_dqb_is_invariant_to_antipodal_node_representations(O):
    rng = np.random.default_rng(34)
    dq = scenes.random_dq(rng, 4, 25.0, 5.0)
    nodes = np.arange(4, dtype=np.int32)
    a = np.array([0.4, 0.3, 0.2, 0.1])
    for _ in range(5):
        p = rng.uniform(-50, 50, 3)
        v = O.dqb(dq, nodes, a, p)
        for j in range(4):
            d2 = dq.copy()
            d2[j] *= -1
            assert np.abs(O.dqb(d2, nodes, a, p) - v).max() < 1e-11


def test_dynamic_arap_weight_bookkeeping(O):
    """Dynamic ARAP weight (Sec. 2, after Eq. (1)): lambda_arap times the summed ICP and ORB
    weights over the summed pair weights. (A reading; this checks the bookkeeping only.)"""
    sc = synth.make_config1(1)
    fr = sc.frame(1)
    s = O.Stream(O.default_params(num_control_points=64, seed=1, lm_iters=1, lambda_arap=1.5), _intr(O, sc.intr))
    s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    _, _, d = s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    want = 1.5 * (d["omega0"].sum() + 10.0 * d["orbw0"].sum()) / s.template_info()["s_arap"]
    assert abs(d["w_arap"] - want) < 1e-12 * want


# ------------------------------------------------------------------------------------------------
# per-node solve (the literal reading of Sec. 2: each node warp is updated on its own)

def test_node_solver_step_is_each_nodes_damped_least_squares(O):
    """Rebuild the iteration-0 step of the per-node solver from a central-difference Jacobian,
    node by node: numpy's least squares on [J_i; sqrt(lambda diag(J_i^T J_i) + eps)] against
    [-r; 0], with eps = 1e-12 max diag(J^T J). The oracle's step comes from its analytic blocks
    and its own Cholesky; a wrong block index, a transposed block or a dropped damping term
    shows up as a step far outside the finite-difference error."""
    sc = _small_scene(N=6)
    fr = sc.frame(1)
    p = O.default_params(num_control_points=6, seed=3, lm_iters=1, solver=O.SOLVE_NODE)
    s = O.Stream(p, _intr(O, sc.intr))
    s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    _, _, dbg = s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    ref = O.Stream(p, _intr(O, sc.intr))
    ref.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    ref.frame_begin(fr.depth, fr.feat_xyz, fr.feat_desc)
    ident = np.tile(np.r_[1.0, 0, 0, 0, 0, 0, 0, 0], (6, 1))
    r, _, wa = ref.residuals(ident, jacobian=True)
    assert wa == dbg["w_arap"]
    n = 36
    Jfd = np.zeros((len(r), n))
    h = 1e-6
    for c in range(n):
        e = np.zeros(n)
        e[c] = h
        rp, _ = ref.residuals(ref.apply_increment(ident, e), dq_assoc=ident, w_arap=wa)
        rm, _ = ref.residuals(ref.apply_increment(ident, -e), dq_assoc=ident, w_arap=wa)
        Jfd[:, c] = (rp - rm) / (2 * h)
    lam = dbg["lambda"][0]
    eps = 1e-12 * (Jfd ** 2).sum(0).max()
    want = np.zeros(n)
    for i in range(6):
        Ji = Jfd[:, 6 * i:6 * i + 6]
        damp = np.sqrt(lam * (Ji ** 2).sum(0) + eps)
        aug = np.vstack([Ji, np.diag(damp)])
        want[6 * i:6 * i + 6] = np.linalg.lstsq(aug, np.r_[-r, np.zeros(6)], rcond=None)[0]
    got = dbg["delta0"]
    assert np.linalg.norm(got - want) < 1e-5 * np.linalg.norm(want)
    # the candidate's cost is that of the rebuilt step
    rc, _ = ref.residuals(ref.apply_increment(ident, want), dq_assoc=ident, w_arap=wa)
    assert abs(dbg["cost_new"][0] - (rc ** 2).sum()) < 1e-6 * dbg["cost_new"][0]
    # and the coupled solve takes a different step on the same system
    pd = O.default_params(num_control_points=6, seed=3, lm_iters=1)
    sd = O.Stream(pd, _intr(O, sc.intr))
    sd.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    _, _, dd = sd.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    assert np.linalg.norm(dd["delta0"] - got) > 1e-2 * np.linalg.norm(got)


def test_node_solver_equals_dense_solver_for_one_node(O):
    """With a single control point the only diagonal block is the whole normal matrix, so the
    per-node and the coupled solver take the same steps bit for bit."""
    sc = _small_scene(N=1)
    fr = sc.frame(1)
    out = []
    for solver in (O.SOLVE_DENSE, O.SOLVE_NODE):
        s = O.Stream(O.default_params(num_control_points=1, seed=3, solver=solver), _intr(O, sc.intr))
        s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
        out.append(s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2]["cost_new"], out[1][2]["cost_new"])


def test_node_solver_fixed_point_and_descent(O):
    """Features only with exact o2 = G(o1) for a rigid G. Started at G itself, every residual is
    0 up to FP64 rounding, so the per-node steps vanish and G is returned to 1e-9 mm. Started at
    the identity, each accepted step lowers the cost and the warp moves toward G (each node sees
    only its own block, so after 10 steps it is not yet there, unlike the coupled solve)."""
    pts, feats, R, t = scenes.lattice_scene()
    o2 = feats @ R.T + t
    K = synth.Intrinsics(16, 16, 20.0, 20.0, 8.0, 8.0)
    rng = np.random.default_rng(23)
    desc = rng.integers(0, 256, (25, 32), dtype=np.uint8)
    p = O.default_params(num_control_points=12, lm_iters=10, solver=O.SOLVE_NODE)
    want = pts @ R.T + t
    s = O.Stream(p, _intr(O, K))
    s.set_template(pts.astype(np.float32), feats.astype(np.float32), desc)
    half = 0.5 * math.atan2(40.0, 399.0)
    G = O.dq_from_rt(np.r_[math.cos(half), 0.0, 0.0, math.sin(half)], t)
    s.set_state(np.tile(G, (12, 1)), 0)
    v, _, _ = s.track_frame(np.zeros((16, 16), np.float32), o2.astype(np.float32), desc)
    assert np.abs(v - want).max() < 1e-9
    s.set_state(np.tile(np.r_[1.0, 0, 0, 0, 0, 0, 0, 0], (12, 1)), 0)
    v, dq, dbg = s.track_frame(np.zeros((16, 16), np.float32), o2.astype(np.float32), desc, debug=True)
    acc = dbg["accepted"].astype(bool)
    assert acc.sum() >= 2
    assert np.all(dbg["cost_new"][acc] < dbg["cost_old"][acc])
    assert np.sqrt(((v - want) ** 2).sum(1).mean()) < 0.75 * np.sqrt(((pts - want) ** 2).sum(1).mean())


def test_node_solver_rejected_by_bad_params(O):
    with pytest.raises(O.OracleError):
        O.Stream(O.default_params(num_control_points=4, solver=2), O.intrinsics(16, 16, 20.0, 20.0, 8.0, 8.0))


# ------------------------------------------------------------------------------------------------
# sparse ARAP graph (the alternative to the dense connection of Sec. 2.2)

def _graph(C, k):
    """Brute-force k-nearest-node graph: node a keeps its k nearest others (stable order, so ties
    go to the lower index); a pair is kept if either node keeps the other."""
    N = len(C)
    D2 = ((C[:, None, :] - C[None, :, :]) ** 2).sum(-1)
    adj = np.zeros((N, N), bool)
    for a in range(N):
        d = D2[a].copy()
        d[a] = np.inf
        adj[a, np.argsort(d, kind="stable")[:k]] = True
    return adj | adj.T, D2


def test_sparse_arap_weight_sum_brute_force(O):
    sc = _small_scene(N=10)
    for k in (1, 3):
        s = O.Stream(O.default_params(num_control_points=10, arap_knn=k), _intr(O, sc.intr))
        s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
        info = s.template_info()
        C = sc.pts.astype(np.float64)[info["node_idx"]]
        adj, D2 = _graph(C, k)
        sa = 2.0 * info["sbar"]
        want = np.exp(-D2 / (2 * sa * sa))[adj].sum()
        assert abs(info["s_arap"] - want) <= 1e-12 * want
        assert adj.sum() < 90  # a proper subset of the 90 ordered pairs


def test_sparse_arap_with_every_neighbour_is_dense(O):
    sc = _small_scene(N=6)
    fr = sc.frame(1)
    out = []
    for k in (0, 5):
        s = O.Stream(O.default_params(num_control_points=6, seed=3, arap_knn=k), _intr(O, sc.intr))
        s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
        out.append(s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_sparse_arap_normal_equations(O):
    """With a 2-nearest-node graph: J^T J against a central-difference Jacobian, and every 6x6
    block of a node pair that is off the graph and shares no blend set is exactly zero (in the
    dense connection the same blocks are not)."""
    sc = _small_scene(N=8)
    fr = sc.frame(1)
    rng = np.random.default_rng(33)
    dq = scenes.random_dq(rng, 8, 3.0, 1.0)
    res = {}
    for k in (0, 2):
        s = O.Stream(O.default_params(num_control_points=8, seed=3, arap_knn=k), _intr(O, sc.intr))
        s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
        s.frame_begin(fr.depth, fr.feat_xyz, fr.feat_desc)
        r, J, wa = s.residuals(dq, jacobian=True)
        A, g = s.normal_equations(dq, w_arap=wa)
        res[k] = (s, A, wa)
        if k == 2:
            n = 48
            Jfd = np.zeros_like(J)
            h = 1e-6
            for c in range(n):
                e = np.zeros(n)
                e[c] = h
                rp, _ = s.residuals(s.apply_increment(dq, e), dq_assoc=dq, w_arap=wa)
                rm, _ = s.residuals(s.apply_increment(dq, -e), dq_assoc=dq, w_arap=wa)
                Jfd[:, c] = (rp - rm) / (2 * h)
            assert np.linalg.norm(A - Jfd.T @ Jfd) < 1e-6 * np.linalg.norm(A)
    s2, A2, _ = res[2]
    info = s2.template_info()
    C = sc.pts.astype(np.float64)[info["node_idx"]]
    adj, _ = _graph(C, 2)
    share = np.zeros((8, 8), bool)
    for sets in (info["knn_pts"], info["knn_feat"]):
        for row in sets:
            for a in row:
                share[a, row] = True
    quiet = ~adj & ~share & ~np.eye(8, dtype=bool)
    assert quiet.any()
    A0 = res[0][1]
    for a, b in zip(*np.nonzero(quiet)):
        assert not A2[6 * a:6 * a + 6, 6 * b:6 * b + 6].any()
        assert np.abs(A0[6 * a:6 * a + 6, 6 * b:6 * b + 6]).max() > 0
    for a, b in zip(*np.nonzero(adj & ~share)):
        assert np.abs(A2[6 * a:6 * a + 6, 6 * b:6 * b + 6]).max() > 0


# ------------------------------------------------------------------------------------------------
# z-buffered association (the "rasterization" of Sec. 2 read with visibility)

def test_zbuffer_keeps_only_the_nearest_point_per_pixel(O):
    K, depth, pts, nb, nf = scenes.two_layer_scene()
    rng = np.random.default_rng(34)
    desc = rng.integers(0, 256, (4, 32), dtype=np.uint8)
    fi = np.arange(nb, nb + 4)
    corr = {}
    for zb in (0, 1):
        s = O.Stream(O.default_params(num_control_points=8, lm_iters=1, assoc_zbuffer=zb), _intr(O, K))
        s.set_template(pts, pts[fi], desc)
        _, _, d = s.track_frame(depth, pts[fi], desc, debug=True)
        corr[zb] = d["corr0"]
    pix_front = corr[0][nb:nb + nf]
    assert (pix_front >= 0).all()
    # without the z-buffer the back layer takes the same pixels as the front layer
    assert np.array_equal(corr[0][:nb], pix_front)
    assert corr[0][-1] == pix_front[0]
    # with it the back layer and the later copy are hidden; the front layer keeps its pixels
    assert (corr[1][:nb] == -1).all()
    assert np.array_equal(corr[1][nb:nb + nf], pix_front)
    assert corr[1][-1] == -1


def test_zbuffer_without_collisions_changes_nothing(O):
    """At the identity every config 1 template point has a pixel of its own, so the first
    iteration is the same with and without the z-buffer."""
    sc = synth.make_config1(1)
    fr = sc.frame(1)
    out = []
    for zb in (0, 1):
        s = O.Stream(O.default_params(num_control_points=64, seed=1, lm_iters=1, assoc_zbuffer=zb),
                     _intr(O, sc.intr))
        s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
        out.append(s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][2]["corr0"], out[1][2]["corr0"])
    assert len(np.unique(out[0][2]["corr0"][out[0][2]["corr0"] >= 0])) == (out[0][2]["corr0"] >= 0).sum()


# ------------------------------------------------------------------------------------------------
# closest-point association (the kd-tree search Sec. 2 contrasts with its re-projection)

def test_closest_point_association_is_the_nearest_neighbour_of_a_library_kdtree(O):
    """At the identity the deformed template points are the template points; the association must
    pick, for every one of them, the pixel whose back-projected point is nearest in 3D among the
    pixels with a normal -- as scipy's kd-tree finds it (distances equal; pixels equal wherever the
    nearest point is unique to 1e-9 relative)."""
    from scipy.spatial import cKDTree
    sc = synth.make_config1(1)
    fr = sc.frame(1)
    K = sc.intr
    s = O.Stream(O.default_params(num_control_points=64, seed=1, lm_iters=1, assoc_kdtree=1), _intr(O, K))
    s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    _, _, d = s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    corr = d["corr0"]
    _, val = O.normal_map(fr.depth, _intr(O, K))
    valid = np.flatnonzero(val.reshape(-1))
    u, v = valid % K.width, valid // K.width
    z = fr.depth.reshape(-1)[valid].astype(np.float64)
    q = np.stack([(u - K.cx) / K.fx * z, (v - K.cy) / K.fy * z, z], axis=1)
    dist, idx = cKDTree(q).query(sc.pts.astype(np.float64), k=2)
    assert (corr >= 0).all()
    pos = np.searchsorted(valid, corr)
    assert np.array_equal(valid[pos], corr), "a point was matched to a pixel without a normal"
    dsel = np.linalg.norm(q[pos] - sc.pts.astype(np.float64), axis=1)
    assert np.allclose(dsel, dist[:, 0], rtol=1e-12, atol=1e-12)
    unique = dist[:, 1] > dist[:, 0] * (1 + 1e-9)
    assert unique.mean() > 0.99
    assert np.array_equal(corr[unique], valid[idx[unique, 0]])
    # the residual is the point-to-plane distance at that pixel, as with re-projection
    assert np.isfinite(d["r0"]).all()


def test_closest_point_and_zbuffer_are_exclusive(O):
    with pytest.raises(O.OracleError):
        O.Stream(O.default_params(num_control_points=8, assoc_kdtree=1, assoc_zbuffer=1),
                 O.intrinsics(16, 12, 10, 10, 8, 6))


# ------------------------------------------------------------------------------------------------
# uniform ORB features (Sec. 2.1): FAST corners, neighbour suppression, oriented binary descriptors

_CIRCLE = [(0, -3), (1, -3), (2, -2), (3, -1), (3, 0), (3, 1), (2, 2), (1, 3),
           (0, 3), (-1, 3), (-2, 2), (-3, 1), (-3, 0), (-3, -1), (-2, -2), (-1, -3)]


def _ring_patch(values, centre=100, bg=100):
    """9 x 9 patch with the given 16 circle values around the centre pixel (4, 4)."""
    img = np.full((9, 9), bg, np.uint8)
    img[4, 4] = centre
    for (dx, dy), x in zip(_CIRCLE, values):
        img[4 + dy, 4 + dx] = x
    return img


def test_fast_segment_test_cases(O):
    t = 20
    # all 16 darker: a corner whose response sums the 16 margins
    assert O.fast_response(_ring_patch([50] * 16), 4, 4, t) == 16 * (100 - 50 - t)
    assert O.fast_response(_ring_patch([100] * 16), 4, 4, t) == 0
    # 9 contiguous brighter: corner; 8: not
    nine = [200] * 9 + [100] * 7
    assert O.fast_response(_ring_patch(nine), 4, 4, t) == 9 * (200 - 100 - t)
    assert O.fast_response(_ring_patch([200] * 8 + [100] * 8), 4, 4, t) == 0
    # a run of 9 that wraps past the start of the circle
    wrap = [200] * 5 + [100] * 7 + [200] * 4
    assert O.fast_response(_ring_patch(wrap), 4, 4, t) == 9 * 80
    # exactly at the threshold does not count
    assert O.fast_response(_ring_patch([120] * 16), 4, 4, t) == 0
    assert O.fast_response(_ring_patch([121] * 16), 4, 4, t) == 16
    # 9 brighter split 5 + 4 by a darker pixel is no run of 9; the response is only taken by a corner
    split = [200] * 5 + [50] + [200] * 4 + [100] * 6
    assert O.fast_response(_ring_patch(split), 4, 4, t) == 0
    # 9 pixels exactly at the threshold and 7 above: no run of 9 strictly brighter pixels
    assert O.fast_response(_ring_patch([120] * 9 + [200] * 7), 4, 4, t) == 0
    # both classes present: the larger sum is the response
    mixed = [200] * 9 + [50] * 7
    assert O.fast_response(_ring_patch(mixed), 4, 4, t) == max(9 * 80, 7 * 30)


def _dots(W, H, dots, bg=40):
    img = np.full((H, W), bg, np.uint8)
    for u, v, val in dots:
        img[v, u] = val
    return img


def test_orb_suppression_keeps_the_larger_response_then_the_lower_index(O):
    pat = synth.orb_pattern(0)
    # two isolated dots: both corners, neither suppresses the other (6 px apart)
    r = O.orb_detect(_dots(64, 64, [(30, 30, 200), (36, 30, 200)]), pat)
    assert r["kp"].tolist() == [[30, 30], [36, 30]]
    # adjacent dots: the brighter one (larger response) wins
    r = O.orb_detect(_dots(64, 64, [(30, 30, 200), (31, 30, 250)]), pat)
    assert r["kp"].tolist() == [[31, 30]]
    # adjacent equal dots: the lower pixel index wins; with radius 0 both stay
    r = O.orb_detect(_dots(64, 64, [(30, 30, 200), (31, 31, 200)]), pat)
    assert r["kp"].tolist() == [[30, 30]]
    r = O.orb_detect(_dots(64, 64, [(30, 30, 200), (31, 31, 200)]), pat, nms_radius=0)
    assert r["kp"].tolist() == [[30, 30], [31, 31]]
    # nothing closer than 18 px to the border (64 - 18 = 46 is outside, 45 inside)
    r = O.orb_detect(_dots(64, 64, [(17, 30, 200), (45, 30, 200), (30, 46, 200)]), pat)
    assert r["kp"].tolist() == [[45, 30]]
    # the cap keeps the first corners in raster order and counts them all
    r = O.orb_detect(_dots(64, 64, [(20, 20, 200), (40, 20, 200), (20, 40, 200)]), pat, max_features=2)
    assert r["kp"].tolist() == [[20, 20], [40, 20]] and r["total"] == 3


def test_orb_orientation_bins_of_intensity_ramps(O):
    """A bright dot on a linear intensity ramp rising along angle phi: the intensity centroid
    points along phi, so the orientation bin is phi / 12 deg."""
    pat = synth.orb_pattern(0)
    u = np.arange(64)[None, :] - 32.0
    v = np.arange(64)[:, None] - 32.0
    for b in (0, 4, 9, 17, 26):
        phi = math.radians(12.0 * b)
        img = np.clip(np.floor(100 + 2.5 * (u * math.cos(phi) + v * math.sin(phi)) + 0.5), 0, 255).astype(np.uint8)
        img[32, 32] = 255
        r = O.orb_detect(img, pat, fast_threshold=40)
        k = [i for i, (x, y) in enumerate(r["kp"].tolist()) if (x, y) == (32, 32)]
        assert k, b
        assert r["angle_bin"][k[0]] == b


def test_orb_descriptor_is_invariant_to_a_half_turn(O):
    """Rotating the image by 180 deg maps pixel (u, v) to (W-1-u, H-1-v), negates both moments
    (orientation + 15 bins) and rotates the sampling pattern with it: the keypoints map onto each
    other and the descriptors agree (up to the rare pattern point whose rotated offset rounds the
    other way)."""
    sc = synth.make_small_sequence(seed=12, M=500, N=8, K1=40, width=160, height=120, n_frames=1,
                                   max_step_mm=2.0)
    _, img = sc.image(0)
    pat = synth.orb_pattern(0)
    a = O.orb_detect(img, pat)
    b = O.orb_detect(img[::-1, ::-1].copy(), pat)
    assert len(a["kp"]) > 50
    H, W = img.shape
    mb = {(W - 1 - x, H - 1 - y): i for i, (x, y) in enumerate(b["kp"].tolist())}
    common = 0
    diff_bits = []
    for i, (x, y) in enumerate(a["kp"].tolist()):
        j = mb.get((x, y))
        if j is None:
            continue
        common += 1
        assert (a["angle_bin"][i] + 15) % 30 == b["angle_bin"][j]
        diff_bits.append(int(np.unpackbits(a["desc"][i] ^ b["desc"][j]).sum()))
    assert common >= 0.95 * len(a["kp"])
    assert np.mean(diff_bits) < 2.0 and max(diff_bits) <= 16


def test_orb_matches_follow_the_surface(O):
    """Template features from the textured template image and frame features from frame 1,
    matched by nearest Hamming distance: most matches land within 2 px of where the surface
    point under the template feature moved to (the template point nearest the keypoint, moved
    by the frame's ground-truth warp and projected)."""
    sc = synth.make_small_sequence(seed=12, M=12000, N=8, K1=40, width=160, height=120, n_frames=1,
                                   max_step_mm=2.0)
    d0, i0 = sc.image(0)
    d1, i1 = sc.image(1)
    pat = synth.orb_pattern(0)
    K = _intr(O, sc.intr)
    a = O.orb_detect(i0, pat, d0, K)
    b = O.orb_detect(i1, pat, d1, K)
    idx, dist = O.hamming_match(a["desc"], b["desc"])
    fr = sc.frame(1)
    proj = lambda X: np.stack([sc.intr.fx * X[:, 0] / X[:, 2] + sc.intr.cx,
                               sc.intr.fy * X[:, 1] / X[:, 2] + sc.intr.cy], 1)
    puv = proj(sc.pts.astype(np.float64))
    gt_uv = proj(fr.gt_vertices)
    good = seen = 0
    for i in range(len(a["kp"])):
        j = np.argmin(((puv - a["kp"][i]) ** 2).sum(1))
        if ((puv[j] - a["kp"][i]) ** 2).sum() > 1.0:
            continue
        seen += 1
        moved = gt_uv[j] + (a["kp"][i] - puv[j])
        if idx[i] >= 0 and ((b["kp"][idx[i]] - moved) ** 2).sum() <= 4.0:
            good += 1
    assert seen >= 0.8 * len(a["kp"])
    assert good >= 0.5 * seen, (good, seen)


def test_sparse_arap_graph_ties_go_to_the_lower_index(O):
    """Control points on a square lattice have many equal rest distances; the k nearest are then
    the lowest-indexed of the tied nodes (brute force with a stable sort)."""
    pts, feats, R, t = scenes.lattice_scene()
    rng = np.random.default_rng(35)
    desc = rng.integers(0, 256, (25, 32), dtype=np.uint8)
    for k in (1, 2, 3):
        s = O.Stream(O.default_params(num_control_points=12, arap_knn=k), O.intrinsics(16, 16, 20.0, 20.0, 8.0, 8.0))
        s.set_template(pts.astype(np.float32), feats.astype(np.float32), desc)
        info = s.template_info()
        C = pts.astype(np.float32).astype(np.float64)[info["node_idx"]]
        adj, D2 = _graph(C, k)
        d = D2 + np.diag(np.full(12, np.inf))
        assert any(np.sum(d[a] == np.sort(d[a])[k - 1]) > 1 for a in range(12))  # ties at the k-th
        sa = 2.0 * info["sbar"]
        want = np.exp(-D2 / (2 * sa * sa))[adj].sum()
        assert abs(info["s_arap"] - want) <= 1e-12 * want


def test_orb_descriptor_of_an_unrotated_keypoint_by_brute_force(O):
    """A keypoint whose orientation bin is 0 uses the pattern as drawn: its descriptor is the
    256 comparisons of 5 x 5 box sums at p + (x1, y1) and p + (x2, y2), bit k in byte k // 8 from
    the least significant bit."""
    pat = synth.orb_pattern(0)
    u = np.arange(64)[None, :] - 32.0
    v = np.arange(64)[:, None] - 32.0
    rng = np.random.default_rng(36)
    img = np.clip(np.floor(100 + 2.5 * u + rng.integers(-6, 7, (64, 64)) + 0.5), 0, 255).astype(np.uint8)
    img[32, 32] = 255
    r = O.orb_detect(img, pat, fast_threshold=40)
    k = [i for i, (x, y) in enumerate(r["kp"].tolist()) if (x, y) == (32, 32)]
    assert k and r["angle_bin"][k[0]] == 0
    I = img.astype(np.int64)
    box = lambda x, y: int(I[y - 2:y + 3, x - 2:x + 3].sum())
    want = np.zeros(32, np.uint8)
    for b in range(256):
        x1, y1, x2, y2 = (int(q) for q in pat[b])
        if box(32 + x1, 32 + y1) < box(32 + x2, 32 + y2):
            want[b // 8] |= np.uint8(1 << (b % 8))
    assert np.array_equal(r["desc"][k[0]], want)


def test_orb_descriptor_nearly_invariant_to_a_quarter_turn(O):
    """A quarter turn maps the keypoints onto each other exactly and turns the orientation by -7.5
    bins, so the steered pattern is off by 6 degrees: the descriptors of corresponding keypoints
    still agree in most bits (about 15 of 256 differ), far from the 128 of unrelated ones. A pattern
    steered the wrong way round would not agree."""
    sc = synth.make_small_sequence(seed=12, M=500, N=8, K1=40, width=160, height=120, n_frames=1,
                                   max_step_mm=2.0)
    _, img = sc.image(0)
    pat = synth.orb_pattern(0)
    a = O.orb_detect(img, pat)
    b = O.orb_detect(np.rot90(img).copy(), pat)
    W = img.shape[1]
    mb = {(x, y): i for i, (x, y) in enumerate(b["kp"].tolist())}
    diff = []
    for i, (x, y) in enumerate(a["kp"].tolist()):
        j = mb.get((y, W - 1 - x))
        if j is None:
            continue
        # (x, y) -> (y, W - 1 - x) turns every offset (dx, dy) into (dy, -dx): minus 90 degrees
        assert (b["angle_bin"][j] - a["angle_bin"][i]) % 30 in (22, 23)
        diff.append(int(np.unpackbits(a["desc"][i] ^ b["desc"][j]).sum()))
    assert len(diff) >= 0.9 * len(a["kp"])
    assert np.mean(diff) < 30


def test_orb_points_project_back_onto_their_keypoints(O):
    sc = synth.make_small_sequence(seed=12, M=500, N=8, K1=40, width=160, height=120, n_frames=1,
                                   max_step_mm=2.0)
    depth, img = sc.image(1)
    r = O.orb_detect(img, synth.orb_pattern(0), depth, _intr(O, sc.intr))
    X = r["xyz"].astype(np.float64)
    ok = np.isfinite(X).all(1)
    assert ok.mean() > 0.9
    K = sc.intr
    u = K.fx * X[ok, 0] / X[ok, 2] + K.cx
    v = K.fy * X[ok, 1] / X[ok, 2] + K.cy
    assert np.abs(u - r["kp"][ok, 0]).max() < 1e-3 and np.abs(v - r["kp"][ok, 1]).max() < 1e-3
    assert np.array_equal(X[ok, 2].astype(np.float32), depth[r["kp"][ok, 1], r["kp"][ok, 0]])


# ------------------------------------------------------------------------------------------------
# the LM step rule, the pre-selection thresholds and the per-frame ARAP weight, each on a case
# that takes the branch in question

def _lm_lambdas(lam0, accepted):
    """Damping sequence of Sec. 2's Levenberg-Marquardt rule: /10 after an accepted step, x10
    after a rejected one, kept in [1e-10, 1e10]."""
    lam = [lam0]
    for a in accepted[:-1]:
        lam.append(max(lam[-1] / 10.0, 1e-10) if a else min(lam[-1] * 10.0, 1e10))
    return np.array(lam)


def test_lm_rejects_a_step_that_does_not_lower_the_cost(O):
    """At an exact fixed point (target = template on the dyadic plane) every residual and every
    step is exactly 0, so the candidate's cost equals the iterate's. The iterate is replaced only
    for a strictly lower cost: every step is rejected and the damping grows tenfold each time."""
    K, depth, P = scenes.dyadic_plane()
    pts = P[2:-2, 2:-2].reshape(-1, 3).astype(np.float32)
    rng = np.random.default_rng(22)
    fi = rng.choice(len(pts), 12, replace=False)
    desc = rng.integers(0, 256, (12, 32), dtype=np.uint8)
    s = O.Stream(O.default_params(num_control_points=8, lm_iters=6), _intr(O, K))
    s.set_template(pts, pts[fi], desc)
    _, dq, d = s.track_frame(depth, pts[fi], desc, debug=True)
    assert np.all(d["cost_old"] == 0.0) and np.all(d["cost_new"] == 0.0)
    assert not d["accepted"].any()
    assert np.array_equal(d["lambda"], [1e-4, 1e-3, 1e-2, 1e-1, 1.0, 10.0])
    assert np.array_equal(dq, np.tile(np.r_[1.0, 0, 0, 0, 0, 0, 0, 0], (8, 1)))


def test_lm_rejected_steps_keep_the_iterate_and_raise_the_damping(O):
    """The rigid lattice (features only) converges to rounding level within seven iterations;
    the steps after that do not lower the cost and are rejected in the middle of the frame.
    After a rejected step the damping is multiplied by 10 and the next iteration starts from the
    same warps, so its cost at the iterate is the same number; after an accepted one it is divided
    by 10, down to 1e-10."""
    pts, feats, R, t = scenes.lattice_scene()
    o2 = feats @ R.T + t
    K = synth.Intrinsics(16, 16, 20.0, 20.0, 8.0, 8.0)
    rng = np.random.default_rng(23)
    desc = rng.integers(0, 256, (25, 32), dtype=np.uint8)
    s = O.Stream(O.default_params(num_control_points=12, lm_iters=10), _intr(O, K))
    s.set_template(pts.astype(np.float32), feats.astype(np.float32), desc)
    _, _, d = s.track_frame(np.zeros((16, 16), np.float32), o2.astype(np.float32), desc, debug=True)
    acc, lam, c0, c1 = d["accepted"], d["lambda"], d["cost_old"], d["cost_new"]
    T = len(acc)
    mid_rejects = [i for i in range(T - 1) if not acc[i]]
    assert len(mid_rejects) >= 2, acc
    # the lower clamp is reached: an accepted step whose tenth would fall below 1e-10
    assert any(acc[i] and lam[i] / 10.0 < 1e-10 and lam[i + 1] == 1e-10 for i in range(T - 1)), lam
    assert np.array_equal(lam, _lm_lambdas(1e-4, acc))
    for i in range(T):
        assert bool(acc[i]) == bool(c1[i] < c0[i])
    for i in mid_rejects:
        assert c0[i + 1] == c0[i]
    assert c0[0] > 1e6 and c0[-1] < 1e-20


def test_arap_weight_is_fixed_for_the_whole_frame(O):
    """The dynamic ARAP weight (Sec. 2, after Eq. (1)) is set once per frame from the
    iteration-0 weight sums and used unchanged by every iteration, although the Tukey and feature
    weights move as the surface is re-associated (checked: the iteration-0 and final costs are
    far apart)."""
    sc = synth.make_config1(1)
    fr = sc.frame(1)
    s = O.Stream(O.default_params(num_control_points=64, seed=1, lambda_arap=1.5), _intr(O, sc.intr))
    s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    _, _, d = s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    want = 1.5 * (d["omega0"].sum() + 10.0 * d["orbw0"].sum()) / s.template_info()["s_arap"]
    assert abs(d["w_arap"] - want) < 1e-12 * want
    assert np.all(d["w_arap_iter"] == d["w_arap"])
    assert d["cost_old"][-1] < 0.1 * d["cost_old"][0]
    # a second frame sets its own weight from its own iteration-0 sums
    s2 = O.Stream(O.default_params(num_control_points=64, seed=1, lambda_arap=1.5), _intr(O, sc.intr))
    s2.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
    s2.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc)
    _, _, e = s2.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
    want2 = 1.5 * (e["omega0"].sum() + 10.0 * e["orbw0"].sum()) / s2.template_info()["s_arap"]
    assert abs(e["w_arap"] - want2) < 1e-12 * want2 and e["w_arap"] != d["w_arap"]
    assert np.all(e["w_arap_iter"] == e["w_arap"])


def test_preselect_drops_hypotheses_scoring_below_half_of_the_best(O):
    """Sec. 2.1: a reference whose hypothesis collects a small sum of weights is taken for an
    outlier. Two locally rigid clusters as in the keep test, the second one smaller (12 matches):
    started from unit weights, the alternation leaves its hypotheses with scores on both sides of
    half the best one, several of them between 0.4 and 0.5. Exactly the hypotheses below one half
    are dropped."""
    rng = np.random.default_rng(31)
    H = 3.0
    A = rng.uniform(-10, 10, size=(30, 3))
    B = rng.uniform(-10, 10, size=(12, 3)) + np.array([100.0, 0, 0])
    R = scenes.quat_to_matrix(np.r_[1.0, 0.1, -0.05, 0.0])
    o1 = np.vstack([A, B, rng.uniform(-50, 50, size=(4, 3))])
    o2 = np.vstack([A @ R.T, B @ R.T + np.array([0.0, 40.0, 0.0]),
                    rng.uniform(-50, 50, size=(4, 3)) + 300])
    r = O.preselect(o1, o2, np.ones(46, np.uint8), H, refs=0, iters=10)
    valid = r["hyp_kept"][:46] != 2
    ratio = r["hyp_W"][:46] / r["hyp_W"][:46][valid].max()
    assert valid.all()
    assert np.any((ratio > 0.4) & (ratio < 0.5)), ratio
    assert np.any((ratio >= 0.5) & (ratio < 0.6)), ratio
    assert np.array_equal(r["hyp_kept"][:46], (ratio >= 0.5).astype(np.uint8))
    assert np.all(r["hyp_kept"][:30] == 1) and np.all(r["hyp_kept"][42:46] == 0)


def test_preselect_threshold_is_half(O):
    """Sec. 2.1: a match belongs to the pre-selected set when its weight in some kept hypothesis
    reaches 1/2, i.e. it lies within 2H of that hypothesis's rigid image. Two matches are moved
    off an exact rigid motion by 2.2 H and 1.8 H; with references drawn among the other 20
    (seed 2 of the sampler), their weights (Eq. (4), H / d, d nudged by the weighted rotation fit)
    are about 0.47 and 0.59: the first stays out, the second is in. Neither is within H, so
    neither counts as an inlier of any hypothesis."""
    rng = np.random.default_rng(32)
    H = 3.0
    o1 = rng.uniform(-30, 30, size=(22, 3))
    R = scenes.quat_to_matrix(np.r_[1.0, -0.03, 0.08, 0.02])
    o2 = o1 @ R.T + np.array([4.0, -2.0, 1.0])
    u = _unit(rng, 2)
    o2[20] += 2.2 * H * u[0]
    o2[21] += 1.8 * H * u[1]
    r = O.preselect(o1, o2, np.ones(22, np.uint8), H, refs=12, iters=10, seed=2)
    assert 20 not in r["hyp_k0"][:12] and 21 not in r["hyp_k0"][:12]
    assert np.all(r["hyp_kept"][:12] == 1)
    assert 0.42 < r["wstar"][20] < 0.48, r["wstar"][20]
    assert 0.52 < r["wstar"][21] < 0.62, r["wstar"][21]
    assert not r["preselected"][20] and r["preselected"][21]
    assert r["preselected"][:20].all()
    # each hypothesis counts the matches within H of its rigid image: the 20 exact ones, not the
    # one at 1.8 H
    assert np.all(r["hyp_nin"][:12] == 20), r["hyp_nin"][:12]
