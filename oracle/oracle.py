"""ctypes wrapper of the FP64 oracle library (test infrastructure only).

Loads oracle/libtt_oracle.so (built by oracle/build.py). Arrays are numpy; every call copies in
and out of caller-owned buffers, as the C interface does.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# TT_ORACLE_LIB names another build of the same source (the mutation check loads planted copies)
LIB_PATH = os.environ.get("TT_ORACLE_LIB") or os.path.join(HERE, "libtt_oracle.so")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


class Intrinsics(C.Structure):
    _fields_ = [("width", C.c_int), ("height", C.c_int), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double)]


class Params(C.Structure):
    _fields_ = [("num_control_points", C.c_int), ("knn", C.c_int), ("w_orb", C.c_double),
                ("w_angle", C.c_double), ("w_rotation", C.c_double), ("lambda_arap", C.c_double),
                ("tukey_c", C.c_double), ("H", C.c_double), ("ransac_refs", C.c_int),
                ("ransac_iters", C.c_int), ("lm_iters", C.c_int), ("max_hamming", C.c_int),
                ("lm_lambda0", C.c_double), ("seed", C.c_uint64), ("solver", C.c_int),
                ("arap_knn", C.c_int), ("assoc_zbuffer", C.c_int), ("assoc_kdtree", C.c_int)]


SOLVE_DENSE, SOLVE_NODE = 0, 1


_P = C.c_void_p


class OrbParams(C.Structure):
    _fields_ = [("fast_threshold", C.c_int), ("nms_radius", C.c_int), ("max_features", C.c_int)]


ORB_BORDER = 18


class FrameDebug(C.Structure):
    _fields_ = [(n, _P) for n in (
        "match_idx", "match_dist", "wstar", "preselected", "hyp_k0", "hyp_W", "hyp_nin",
        "hyp_kept", "corr0", "r0", "omega0", "orbw0", "A0", "g0", "w_arap", "cost_old",
        "cost_new", "lambda_", "accepted", "delta0", "w_arap_iter")]


def _declare(L):
    vp = C.c_void_p
    L.tto_default_params.argtypes = [C.POINTER(Params)]
    L.tto_create_stream.argtypes = [C.POINTER(Params), C.POINTER(Intrinsics), C.POINTER(vp)]
    L.tto_destroy.argtypes = [vp]
    L.tto_set_template.argtypes = [vp, vp, C.c_int, vp, vp, C.c_int]
    L.tto_track_frame.argtypes = [vp, vp, vp, vp, C.c_int, vp, vp, C.POINTER(FrameDebug)]
    L.tto_num_nodes.argtypes = [vp]
    L.tto_get_template_info.argtypes = [vp] + [vp] * 7
    L.tto_get_state.argtypes = [vp, vp, vp]
    L.tto_set_state.argtypes = [vp, vp, C.c_int64]
    L.tto_hamming_match.argtypes = [vp, C.c_int, vp, C.c_int, vp, vp]
    L.tto_hamming_match.restype = None
    L.tto_rotation_fit.argtypes = [vp, vp, vp]
    L.tto_preselect.argtypes = [vp, vp, vp, C.c_int, C.c_double, C.c_int, C.c_int, C.c_uint64,
                                C.c_int64, vp, vp, vp, vp, vp, vp]
    L.tto_splitmix64.argtypes = [C.c_uint64, C.c_int, vp]
    L.tto_splitmix64.restype = None
    L.tto_normal_map.argtypes = [vp, C.POINTER(Intrinsics), vp, vp]
    L.tto_normal_map.restype = None
    L.tto_dqb.argtypes = [vp, vp, vp, C.c_int, vp, vp]
    L.tto_dqb.restype = None
    L.tto_dq_transform.argtypes = [vp, vp, vp]
    L.tto_dq_transform.restype = None
    L.tto_dq_from_rt.argtypes = [vp, vp, vp]
    L.tto_dq_from_rt.restype = None
    L.tto_apply_increment.argtypes = [vp, vp, vp, vp]
    L.tto_frame_begin.argtypes = [vp, vp, vp, vp, C.c_int]
    L.tto_num_rows.argtypes = [vp]
    L.tto_residuals.argtypes = [vp, vp, vp, C.c_double, vp, vp, vp]
    L.tto_normal_equations.argtypes = [vp, vp, C.c_double, vp, vp]
    L.tto_cholesky.argtypes = [vp, C.c_int, vp]
    L.tto_cholesky_solve.argtypes = [vp, C.c_int, vp, vp]
    L.tto_cholesky_solve.restype = None
    L.tto_orb_default_params.argtypes = [C.POINTER(OrbParams)]
    L.tto_orb_default_params.restype = None
    L.tto_fast_response.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int]
    L.tto_orb_detect.argtypes = [vp, C.c_int, C.c_int, vp, C.POINTER(Intrinsics), vp, C.POINTER(OrbParams),
                                 vp, vp, vp, vp, vp]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def default_params(**kw):
    p = Params()
    lib().tto_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def intrinsics(width, height, fx, fy, cx, cy):
    return Intrinsics(int(width), int(height), float(fx), float(fy), float(cx), float(cy))


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


class Stream:
    """One tracked surface in the oracle."""

    def __init__(self, params, intr):
        self.params = params
        self.intr = intr
        h = C.c_void_p()
        _check(lib().tto_create_stream(C.byref(params), C.byref(intr), C.byref(h)), "create_stream")
        self.h = h

    def close(self):
        if self.h:
            lib().tto_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- template ---------------------------------------------------------------------------
    def set_template(self, pts, feat_xyz, feat_desc):
        pts = _c(pts, np.float32).reshape(-1, 3)
        feat_xyz = _c(feat_xyz, np.float32).reshape(-1, 3)
        feat_desc = _c(feat_desc, np.uint8).reshape(-1, 32)
        self.M, self.K1 = pts.shape[0], feat_xyz.shape[0]
        rc = lib().tto_set_template(self.h, _ptr(pts), self.M, _ptr(feat_xyz), _ptr(feat_desc), self.K1)
        _check(rc, "set_template")
        self.N = lib().tto_num_nodes(self.h)
        return rc

    def template_info(self):
        kk = self.params.knn
        node_idx = np.zeros(self.N, np.int32)
        knn_pts = np.zeros((self.M, kk), np.int32)
        alpha_pts = np.zeros((self.M, kk))
        knn_feat = np.zeros((max(self.K1, 1), kk), np.int32)
        alpha_feat = np.zeros((max(self.K1, 1), kk))
        sbar = np.zeros(1)
        sarap = np.zeros(1)
        _check(lib().tto_get_template_info(self.h, _ptr(node_idx), _ptr(knn_pts), _ptr(alpha_pts),
                                           _ptr(knn_feat), _ptr(alpha_feat), _ptr(sbar), _ptr(sarap)),
               "get_template_info")
        return dict(node_idx=node_idx, knn_pts=knn_pts, alpha_pts=alpha_pts,
                    knn_feat=knn_feat[:self.K1], alpha_feat=alpha_feat[:self.K1],
                    sbar=float(sbar[0]), s_arap=float(sarap[0]))

    def get_state(self):
        dq = np.zeros((self.N, 8))
        fr = np.zeros(1, np.int64)
        _check(lib().tto_get_state(self.h, _ptr(dq), _ptr(fr)), "get_state")
        return dq, int(fr[0])

    def set_state(self, dq, frame):
        dq = _c(dq, np.float64).reshape(self.N, 8) if dq is not None else None
        _check(lib().tto_set_state(self.h, _ptr(dq), int(frame)), "set_state")

    # -- frame ------------------------------------------------------------------------------
    def _frame_args(self, depth, feat_xyz, feat_desc):
        depth = _c(depth, np.float32)
        feat_xyz = _c(feat_xyz, np.float32).reshape(-1, 3)
        feat_desc = _c(feat_desc, np.uint8).reshape(-1, 32)
        return depth, feat_xyz, feat_desc

    def track_frame(self, depth, feat_xyz, feat_desc, debug=False):
        depth, feat_xyz, feat_desc = self._frame_args(depth, feat_xyz, feat_desc)
        K2 = feat_xyz.shape[0]
        verts = np.zeros((self.M, 3))
        dq = np.zeros((self.N, 8))
        dbg = None
        out = {}
        if debug:
            K1, M, R, T, n = self.K1, self.M, self.params.ransac_refs, self.params.lm_iters, 6 * self.N
            out = dict(match_idx=np.zeros(K1, np.int32), match_dist=np.zeros(K1, np.int32),
                       wstar=np.zeros(K1), preselected=np.zeros(K1, np.uint8),
                       hyp_k0=np.zeros(R, np.int32), hyp_W=np.zeros(R), hyp_nin=np.zeros(R, np.int32),
                       hyp_kept=np.zeros(R, np.uint8), corr0=np.zeros(M, np.int32), r0=np.zeros(M),
                       omega0=np.zeros(M), orbw0=np.zeros(K1), A0=np.zeros((n, n)), g0=np.zeros(n),
                       w_arap=np.zeros(1), cost_old=np.zeros(T), cost_new=np.zeros(T),
                       lambda_=np.zeros(T), accepted=np.zeros(T, np.uint8), delta0=np.full(n, np.nan),
                       w_arap_iter=np.zeros(T))
            dbg = FrameDebug(**{k: _ptr(v) for k, v in out.items()})
        rc = lib().tto_track_frame(self.h, _ptr(depth), _ptr(feat_xyz), _ptr(feat_desc), K2,
                                   _ptr(verts), _ptr(dq), C.byref(dbg) if dbg is not None else None)
        _check(rc, "track_frame")
        if debug:
            out["w_arap"] = float(out["w_arap"][0])
            out["lambda"] = out.pop("lambda_")
        return verts, dq, out

    def frame_begin(self, depth, feat_xyz, feat_desc):
        depth, feat_xyz, feat_desc = self._frame_args(depth, feat_xyz, feat_desc)
        _check(lib().tto_frame_begin(self.h, _ptr(depth), _ptr(feat_xyz), _ptr(feat_desc),
                                     feat_xyz.shape[0]), "frame_begin")

    def num_rows(self):
        return lib().tto_num_rows(self.h)

    def residuals(self, dq_eval, dq_assoc=None, w_arap=-1.0, jacobian=False):
        dq_eval = _c(dq_eval, np.float64)
        dq_assoc = dq_eval if dq_assoc is None else _c(dq_assoc, np.float64)
        rows = self.num_rows()
        r = np.zeros(rows)
        J = np.zeros((rows, 6 * self.N)) if jacobian else None
        wa = np.zeros(1)
        _check(lib().tto_residuals(self.h, _ptr(dq_eval), _ptr(dq_assoc), float(w_arap), _ptr(r),
                                   _ptr(J), _ptr(wa)), "residuals")
        return (r, J, float(wa[0])) if jacobian else (r, float(wa[0]))

    def normal_equations(self, dq, w_arap=-1.0):
        n = 6 * self.N
        A = np.zeros((n, n))
        g = np.zeros(n)
        _check(lib().tto_normal_equations(self.h, _ptr(_c(dq, np.float64)), float(w_arap), _ptr(A), _ptr(g)),
               "normal_equations")
        return A, g

    def apply_increment(self, dq, delta):
        out = np.zeros((self.N, 8))
        _check(lib().tto_apply_increment(self.h, _ptr(_c(dq, np.float64)), _ptr(_c(delta, np.float64)),
                                         _ptr(out)), "apply_increment")
        return out


# -- step-level functions -------------------------------------------------------------------------

def hamming_match(desc1, desc2):
    d1 = _c(desc1, np.uint8).reshape(-1, 32)
    d2 = _c(desc2, np.uint8).reshape(-1, 32)
    idx = np.zeros(d1.shape[0], np.int32)
    dist = np.zeros(d1.shape[0], np.int32)
    lib().tto_hamming_match(_ptr(d1), d1.shape[0], _ptr(d2), d2.shape[0], _ptr(idx), _ptr(dist))
    return idx, dist


def rotation_fit(M):
    M = _c(M, np.float64).reshape(3, 3)
    R = np.zeros((3, 3))
    sig = np.zeros(3)
    deg = lib().tto_rotation_fit(_ptr(M), _ptr(R), _ptr(sig))
    return R, sig, bool(deg)


def preselect(o1, o2, usable, H, refs=30, iters=10, seed=0, frame=0):
    o1 = _c(o1, np.float64).reshape(-1, 3)
    o2 = _c(o2, np.float64).reshape(-1, 3)
    K = o1.shape[0]
    usable = _c(usable, np.uint8)
    nh_alloc = max(refs if refs > 0 else K, 1)
    wstar = np.zeros(K)
    pre = np.zeros(K, np.uint8)
    k0 = np.zeros(nh_alloc, np.int32)
    W = np.zeros(nh_alloc)
    nin = np.zeros(nh_alloc, np.int32)
    kept = np.zeros(nh_alloc, np.uint8)
    nh = lib().tto_preselect(_ptr(o1), _ptr(o2), _ptr(usable), K, float(H), int(refs), int(iters),
                             int(seed) & 0xFFFFFFFFFFFFFFFF, int(frame), _ptr(wstar), _ptr(pre),
                             _ptr(k0), _ptr(W), _ptr(nin), _ptr(kept))
    return dict(n=nh, wstar=wstar, preselected=pre, hyp_k0=k0, hyp_W=W, hyp_nin=nin, hyp_kept=kept)


def splitmix64(state, n):
    out = np.zeros(n, np.uint64)
    lib().tto_splitmix64(int(state) & 0xFFFFFFFFFFFFFFFF, n, _ptr(out))
    return out


def normal_map(depth, intr):
    depth = _c(depth, np.float32)
    H, W = intr.height, intr.width
    nrm = np.zeros((H * W, 3))
    val = np.zeros(H * W, np.uint8)
    lib().tto_normal_map(_ptr(depth), C.byref(intr), _ptr(nrm), _ptr(val))
    return nrm.reshape(H, W, 3), val.reshape(H, W)


def dqb(dq, nodes, alpha, p):
    dq = _c(dq, np.float64)
    nodes = _c(nodes, np.int32)
    alpha = _c(alpha, np.float64)
    p = _c(p, np.float64)
    v = np.zeros(3)
    lib().tto_dqb(_ptr(dq), _ptr(nodes), _ptr(alpha), len(nodes), _ptr(p), _ptr(v))
    return v


def dq_transform(dq, p):
    v = np.zeros(3)
    lib().tto_dq_transform(_ptr(_c(dq, np.float64)), _ptr(_c(p, np.float64)), _ptr(v))
    return v


def dq_from_rt(q, t):
    out = np.zeros(8)
    lib().tto_dq_from_rt(_ptr(_c(q, np.float64)), _ptr(_c(t, np.float64)), _ptr(out))
    return out


def cholesky(A):
    A = _c(A, np.float64)
    n = A.shape[0]
    L = np.zeros_like(A)
    rc = lib().tto_cholesky(_ptr(A), n, _ptr(L))
    return L, rc


def cholesky_solve(L, b):
    L = _c(L, np.float64)
    b = _c(b, np.float64)
    x = np.zeros_like(b)
    lib().tto_cholesky_solve(_ptr(L), L.shape[0], _ptr(b), _ptr(x))
    return x


def orb_params(**kw):
    p = OrbParams()
    lib().tto_orb_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def fast_response(img, u, v, t):
    img = _c(img, np.uint8)
    return lib().tto_fast_response(_ptr(img), img.shape[1], int(u), int(v), int(t))


def orb_detect(img, pattern, depth=None, intr=None, **kw):
    """Uniform ORB keypoints of an 8-bit image: dict(kp [n,2] int32 (u, v), xyz [n,3] float32,
    desc [n,32] uint8, angle_bin [n] int32, total = corners kept before the cap)."""
    img = _c(img, np.uint8)
    H, W = img.shape
    p = orb_params(**kw)
    mx = p.max_features
    kp = np.zeros((max(mx, 1), 2), np.int32)
    xyz = np.zeros((max(mx, 1), 3), np.float32)
    desc = np.zeros((max(mx, 1), 32), np.uint8)
    ang = np.zeros(max(mx, 1), np.int32)
    cnt = np.zeros(2, np.int32)
    d = _c(depth, np.float32) if depth is not None else None
    _check(lib().tto_orb_detect(_ptr(img), W, H, _ptr(d) if d is not None else None,
                                C.byref(intr) if intr is not None else None, _ptr(_c(pattern, np.int8)),
                                C.byref(p), _ptr(kp), _ptr(xyz), _ptr(desc), _ptr(ang), _ptr(cnt)), "orb_detect")
    n = int(cnt[0])
    return dict(kp=kp[:n].copy(), xyz=xyz[:n].copy(), desc=desc[:n].copy(), angle_bin=ang[:n].copy(),
                total=int(cnt[1]))
