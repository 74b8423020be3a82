"""Thin ctypes binding of the HIP library (include/tt.h). Argument marshalling only: every step of
the solve runs in the library's kernels. Raises if the library has not been built.

Names follow the C ABI: default_params, create_stream, Stream.set_template, Stream.track_frame,
Stream.track_frame_device, track_batch_device, Stream.destroy, strerror.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtt.so")

TT_OK, TT_EINVAL, TT_ENOMEM, TT_ESTATE, TT_EDEVICE, TT_EBUSY = 0, -1, -2, -3, -4, -5
TT_FP32, TT_BF16_IR, TT_FP16_IR = 0, 1, 2
TT_SOLVE_DENSE, TT_SOLVE_NODE = 0, 1
STAGES = ("front", "rows", "arap", "data", "solve", "update", "factor")

_lib = None


class TTError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class Intrinsics(C.Structure):
    _fields_ = [("width", C.c_int), ("height", C.c_int), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double)]


class Params(C.Structure):
    _fields_ = [("num_control_points", C.c_int), ("knn", C.c_int), ("w_orb", C.c_double),
                ("w_angle", C.c_double), ("w_rotation", C.c_double), ("lambda_arap", C.c_double),
                ("tukey_c", C.c_double), ("H", C.c_double), ("ransac_refs", C.c_int),
                ("ransac_iters", C.c_int), ("lm_iters", C.c_int), ("max_hamming", C.c_int),
                ("lm_lambda0", C.c_double), ("precision", C.c_int), ("seed", C.c_uint64),
                ("hbm_budget_bytes", C.c_uint64), ("ir_iters", C.c_int),
                ("solver", C.c_int), ("arap_knn", C.c_int),
                ("assoc_zbuffer", C.c_int), ("graph", C.c_int), ("assoc_kdtree", C.c_int)]


_DEBUG_FIELDS = ("match_idx", "match_dist", "wstar", "preselected", "hyp_k0", "hyp_W", "hyp_nin",
                 "hyp_kept", "corr0", "r0", "omega0", "orbw0", "A0", "g0", "w_arap", "cost_old",
                 "cost_new", "lambda_", "accepted", "delta0", "w_arap_iter")


class OrbParams(C.Structure):
    _fields_ = [("fast_threshold", C.c_int), ("nms_radius", C.c_int), ("max_features", C.c_int)]


TT_ORB_BORDER = 18


class FrameDebug(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in _DEBUG_FIELDS]


class FrameDevice(C.Structure):
    _fields_ = [("depth", C.c_void_p), ("feat_xyz", C.c_void_p), ("feat_desc", C.c_void_p), ("K2", C.c_int),
                ("out_vertices", C.c_void_p), ("out_dq", C.c_void_p), ("inputs_ready", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("chol_grid_pct", C.c_int), ("arap_threads", C.c_int), ("fuse_rows_arap", C.c_int),
                ("frame_ms", C.c_double)]


class ServerParams(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_rounds_ahead", C.c_int)]


class ServerStats(C.Structure):
    _fields_ = [("streams_open", C.c_int), ("opens_waiting", C.c_int), ("reserved_bytes", C.c_uint64),
                ("frames_submitted", C.c_int64), ("frames_done", C.c_int64), ("rounds", C.c_int64),
                ("frame_iterations", C.c_int64)]


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2007_08576_amd.build")
        # torch (which owns device memory and streams here) ships its own HIP runtime; loading it
        # first lets the library bind to that same runtime instead of a second copy
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.tt_default_params.argtypes = [C.POINTER(Params)]
        L.tt_default_params.restype = None
        L.tt_create_stream.argtypes = [C.POINTER(Params), C.POINTER(Intrinsics), vp, C.POINTER(vp)]
        L.tt_set_template.argtypes = [vp, vp, C.c_int, vp, vp, C.c_int]
        L.tt_track_frame.argtypes = [vp, vp, vp, vp, C.c_int, vp, vp, C.POINTER(FrameDebug)]
        L.tt_track_frame_device.argtypes = [vp, vp, vp, vp, C.c_int, vp, vp]
        L.tt_track_frame_device_ev.argtypes = [vp, vp, vp, vp, C.c_int, vp, vp, vp]
        L.tt_track_batch_device.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(FrameDevice)]
        L.tt_sync.argtypes = [vp]
        L.tt_get_frame_log.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.tt_hip_stream.argtypes = [vp]
        L.tt_hip_stream.restype = vp
        L.tt_get_template_info.argtypes = [vp] + [vp] * 7
        L.tt_get_state.argtypes = [vp, vp, vp]
        L.tt_set_state.argtypes = [vp, vp, C.c_int64]
        L.tt_device_bytes.argtypes = [vp, C.POINTER(C.c_uint64)]
        L.tt_set_timing.argtypes = [vp, C.c_int]
        L.tt_debug_cholesky_solve.argtypes = [C.c_int, vp, vp, vp, C.POINTER(C.c_int)]
        L.tt_debug_cholesky_solve_ex.argtypes = [C.c_int, vp, vp, vp, C.POINTER(C.c_int), C.c_int, C.c_int]
        L.tt_cholesky_solve_noalloc.argtypes = [C.c_int, vp, vp, vp, vp, vp]
        L.tt_get_timing.argtypes = [vp, vp, vp]
        L.tt_destroy.argtypes = [vp]
        L.tt_strerror.argtypes = [C.c_int]
        L.tt_strerror.restype = C.c_char_p
        L.tt_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.tt_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.tt_autotune.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, C.POINTER(Tuning)]
        L.tt_server_default_params.argtypes = [C.POINTER(ServerParams)]
        L.tt_server_default_params.restype = None
        L.tt_server_create.argtypes = [C.POINTER(ServerParams), vp, C.POINTER(vp)]
        L.tt_server_open.argtypes = [vp, C.POINTER(Params), C.POINTER(Intrinsics), vp, C.c_int, vp, vp, C.c_int,
                                     C.c_int, C.c_double, C.POINTER(vp)]
        L.tt_server_submit.argtypes = [vp, vp, C.POINTER(FrameDevice), C.POINTER(C.c_uint64)]
        L.tt_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.tt_server_wait.argtypes = [vp, C.c_uint64, C.c_double, C.POINTER(C.c_double)]
        L.tt_server_close.argtypes = [vp, vp]
        L.tt_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.tt_server_destroy.argtypes = [vp]
        L.tt_orb_default_params.argtypes = [C.POINTER(OrbParams)]
        L.tt_orb_default_params.restype = None
        L.tt_orb_create.argtypes = [C.POINTER(OrbParams), C.c_int, C.c_int, vp, vp, C.POINTER(vp)]
        L.tt_orb_detect_device.argtypes = [vp, vp, vp, C.POINTER(Intrinsics), vp, vp, vp, vp, vp]
        L.tt_orb_detect.argtypes = [vp, vp, vp, C.POINTER(Intrinsics), vp, vp, vp, vp, vp]
        L.tt_orb_hip_stream.argtypes = [vp]
        L.tt_orb_hip_stream.restype = vp
        L.tt_orb_destroy.argtypes = [vp]
        _lib = L
    return _lib


def strerror(code):
    return lib().tt_strerror(int(code)).decode()


def _check(rc, what):
    if rc != TT_OK:
        raise TTError(rc, what)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def default_params(**kw):
    p = Params()
    lib().tt_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def intrinsics(width, height, fx, fy, cx, cy):
    return Intrinsics(int(width), int(height), float(fx), float(fy), float(cx), float(cy))


def _dev_ptr(t):
    """Device address of a torch tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return C.c_void_p(t)
    return C.c_void_p(t.data_ptr())


class Stream:
    """A tracked surface: library-owned device state behind the C ABI."""

    def __init__(self, params, intr, hip_stream=None):
        self.params = params
        self.intr = intr
        h = C.c_void_p()
        _check(lib().tt_create_stream(C.byref(params), C.byref(intr),
                                      None if hip_stream is None else C.c_void_p(hip_stream), C.byref(h)),
               "tt_create_stream")
        self.h = h
        self.M = self.N = self.K1 = 0

    def destroy(self):
        if self.h:
            lib().tt_destroy(self.h)
            self.h = None

    close = destroy

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def set_template(self, pts, feat_xyz, feat_desc):
        pts = _c(pts, np.float32).reshape(-1, 3)
        feat_xyz = _c(feat_xyz, np.float32).reshape(-1, 3)
        feat_desc = _c(feat_desc, np.uint8).reshape(-1, 32)
        _check(lib().tt_set_template(self.h, _ptr(pts), pts.shape[0], _ptr(feat_xyz), _ptr(feat_desc),
                                     feat_xyz.shape[0]), "tt_set_template")
        self.M, self.K1, self.N = pts.shape[0], feat_xyz.shape[0], self.params.num_control_points

    def track_frame(self, depth, feat_xyz, feat_desc, debug=False):
        """Host-memory frame; returns (vertices [M,3] f64, dq [N,8] f64, debug dict)."""
        depth = _c(depth, np.float32)
        feat_xyz = _c(feat_xyz, np.float32).reshape(-1, 3)
        feat_desc = _c(feat_desc, np.uint8).reshape(-1, 32)
        verts = np.zeros((self.M, 3))
        dq = np.zeros((self.N, 8))
        out = {}
        dbg = None
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
        rc = lib().tt_track_frame(self.h, _ptr(depth), _ptr(feat_xyz), _ptr(feat_desc), feat_xyz.shape[0],
                                  _ptr(verts), _ptr(dq), C.byref(dbg) if dbg is not None else None)
        _check(rc, "tt_track_frame")
        if debug:
            out["w_arap"] = float(out["w_arap"][0])
            out["lambda"] = out.pop("lambda_")
        return verts, dq, out

    def track_frame_device(self, depth, feat_xyz, feat_desc, K2, out_vertices=None, out_dq=None,
                           inputs_ready=None):
        """Device-memory frame (torch tensors or raw addresses); queued, not waited for. inputs_ready:
        a torch.cuda.Event recorded after the inputs were written (tt_track_frame_device_ev), which
        lets the frame's matching and pre-selection overlap the previous frame's solve."""
        if inputs_ready is None:
            _check(lib().tt_track_frame_device(self.h, _dev_ptr(depth), _dev_ptr(feat_xyz), _dev_ptr(feat_desc),
                                               int(K2), _dev_ptr(out_vertices), _dev_ptr(out_dq)),
                   "tt_track_frame_device")
        else:
            _check(lib().tt_track_frame_device_ev(self.h, _dev_ptr(depth), _dev_ptr(feat_xyz), _dev_ptr(feat_desc),
                                                  int(K2), _dev_ptr(out_vertices), _dev_ptr(out_dq),
                                                  _event_ptr(inputs_ready)),
                   "tt_track_frame_device_ev")

    def sync(self):
        _check(lib().tt_sync(self.h), "tt_sync")

    def frame_log(self):
        """LM record of the last frame: cost at the iterate and candidate, damping, accepted,
        ARAP weight and factorisation failure per iteration."""
        T = self.params.lm_iters
        out = dict(cost_old=np.zeros(T), cost_new=np.zeros(T), lambda_=np.zeros(T), accepted=np.zeros(T, np.uint8),
                   w_arap=np.zeros(T), chol_fail=np.zeros(T, np.int32))
        _check(lib().tt_get_frame_log(self.h, *[_ptr(v) for v in out.values()]), "tt_get_frame_log")
        out["lambda"] = out.pop("lambda_")
        return out

    def hip_stream(self):
        return lib().tt_hip_stream(self.h)

    def template_info(self):
        node_idx = np.zeros(self.N, np.int32)
        knn_pts = np.zeros((self.M, 4), np.int32)
        alpha_pts = np.zeros((self.M, 4), np.float32)
        knn_feat = np.zeros((max(self.K1, 1), 4), np.int32)
        alpha_feat = np.zeros((max(self.K1, 1), 4), np.float32)
        sbar = np.zeros(1)
        sarap = np.zeros(1)
        _check(lib().tt_get_template_info(self.h, _ptr(node_idx), _ptr(knn_pts), _ptr(alpha_pts), _ptr(knn_feat),
                                          _ptr(alpha_feat), _ptr(sbar), _ptr(sarap)), "tt_get_template_info")
        return dict(node_idx=node_idx, knn_pts=knn_pts, alpha_pts=alpha_pts, knn_feat=knn_feat[:self.K1],
                    alpha_feat=alpha_feat[:self.K1], sbar=float(sbar[0]), s_arap=float(sarap[0]))

    def get_state(self):
        dq = np.zeros((self.N, 8))
        fr = np.zeros(1, np.int64)
        _check(lib().tt_get_state(self.h, _ptr(dq), _ptr(fr)), "tt_get_state")
        return dq, int(fr[0])

    def set_state(self, dq, frame):
        dq = None if dq is None else _c(dq, np.float64).reshape(self.N, 8)
        _check(lib().tt_set_state(self.h, _ptr(dq), int(frame)), "tt_set_state")

    def set_timing(self, enable=True, stages=None):
        """Stage timers on (every stage, or only the names in `stages`) or off."""
        mask = 0
        if enable:
            names = STAGES if stages is None else stages
            for name in names:
                mask |= 1 << STAGES.index(name)
        _check(lib().tt_set_timing(self.h, mask), "tt_set_timing")

    def get_timing(self):
        """(ms per stage, count per stage) accumulated since the last call; stage order as STAGES."""
        ms = np.zeros(len(STAGES))
        n = np.zeros(len(STAGES), np.int64)
        _check(lib().tt_get_timing(self.h, _ptr(ms), _ptr(n)), "tt_get_timing")
        return ms, n

    def get_tuning(self):
        t = Tuning()
        _check(lib().tt_get_tuning(self.h, C.byref(t)), "tt_get_tuning")
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def set_tuning(self, chol_grid_pct=200, arap_threads=256, fuse_rows_arap=1):
        t = Tuning(int(chol_grid_pct), int(arap_threads), int(fuse_rows_arap), 0.0)
        _check(lib().tt_set_tuning(self.h, C.byref(t)), "tt_set_tuning")

    def autotune(self, depth, feat_xyz, feat_desc, K2, reps=3):
        """tt_autotune on one device-memory frame; returns the chosen tuning (with its frame time)."""
        t = Tuning()
        _check(lib().tt_autotune(self.h, _dev_ptr(depth), _dev_ptr(feat_xyz), _dev_ptr(feat_desc), int(K2), int(reps),
                                 C.byref(t)), "tt_autotune")
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def device_bytes(self):
        b = C.c_uint64()
        _check(lib().tt_device_bytes(self.h, C.byref(b)), "tt_device_bytes")
        return int(b.value)


def debug_cholesky_solve(A, b, precision=TT_FP32, ir_iters=2):
    """Solve A x = b with the library's Cholesky kernels (FP32, or a 16-bit form with refinement);
    returns (x, failed)."""
    A = _c(A, np.float32)
    b = _c(b, np.float32)
    x = np.zeros(b.shape[0], np.float32)
    fail = C.c_int(0)
    _check(lib().tt_debug_cholesky_solve_ex(int(b.shape[0]), _ptr(A), _ptr(b), _ptr(x), C.byref(fail),
                                            int(precision), int(ir_iters)), "tt_debug_cholesky_solve_ex")
    return x, bool(fail.value)


def cholesky_solve_noalloc(n, d_A, d_b, d_x, d_status, hip_stream=None):
    """tt_cholesky_solve_noalloc on device buffers (torch tensors or addresses); queued, not waited
    for."""
    _check(lib().tt_cholesky_solve_noalloc(int(n), _dev_ptr(d_A), _dev_ptr(d_b), _dev_ptr(d_x), _dev_ptr(d_status),
                                           None if hip_stream is None else C.c_void_p(hip_stream)),
           "tt_cholesky_solve_noalloc")


def _event_ptr(ev):
    """hipEvent_t of a torch.cuda.Event (or a raw handle)."""
    if ev is None:
        return None
    h = getattr(ev, "cuda_event", ev)
    return C.c_void_p(int(h))


def track_batch_device(streams, frames):
    """One frame per stream as one batch (tt_track_batch_device). frames: sequence of
    (depth, feat_xyz, feat_desc, K2, out_vertices, out_dq[, inputs_ready]) with torch tensors or
    addresses; inputs_ready as for Stream.track_frame_device."""
    S = len(streams)
    hs = (C.c_void_p * S)(*[s.h.value for s in streams])
    fr = (FrameDevice * S)()
    for q, f in enumerate(frames):
        depth, xyz, desc, K2, ov, oq = f[:6]
        ev = _event_ptr(f[6]) if len(f) > 6 else None
        fr[q] = FrameDevice(_dev_ptr(depth), _dev_ptr(xyz), _dev_ptr(desc), int(K2), _dev_ptr(ov), _dev_ptr(oq),
                            ev.value if ev is not None else None)
    _check(lib().tt_track_batch_device(hs, S, fr), "tt_track_batch_device")


class ServedStream:
    """A stream opened by a Server (the server owns it until Server.close)."""

    def __init__(self, server, h, params, M, K1, K2max):
        self.server, self.h, self.params = server, h, params
        self.M, self.K1, self.N, self.K2max = M, K1, params.num_control_points, K2max


class Server:
    """Many streams on one GPU (tt_server_*): streams admitted against one HBM budget, their frames
    batched at LM-iteration boundaries by the library's scheduler thread."""

    def __init__(self, hbm_budget_bytes=0, max_rounds_ahead=1, hip_stream=None):
        p = ServerParams()
        lib().tt_server_default_params(C.byref(p))
        p.hbm_budget_bytes = int(hbm_budget_bytes)
        p.max_rounds_ahead = int(max_rounds_ahead)
        h = C.c_void_p()
        _check(lib().tt_server_create(C.byref(p), None if hip_stream is None else C.c_void_p(hip_stream),
                                      C.byref(h)), "tt_server_create")
        self.h = h

    def open(self, params, intr, pts, feat_xyz, feat_desc, K2max, wait_s=0.0):
        """tt_server_open: raises TTError (TT_EBUSY) if no room was made within wait_s seconds."""
        pts = _c(pts, np.float32).reshape(-1, 3)
        feat_xyz = _c(feat_xyz, np.float32).reshape(-1, 3)
        feat_desc = _c(feat_desc, np.uint8).reshape(-1, 32)
        h = C.c_void_p()
        _check(lib().tt_server_open(self.h, C.byref(params), C.byref(intr), _ptr(pts), pts.shape[0], _ptr(feat_xyz),
                                    _ptr(feat_desc), feat_xyz.shape[0], int(K2max), float(wait_s), C.byref(h)),
               "tt_server_open")
        return ServedStream(self, h, params, pts.shape[0], feat_xyz.shape[0], int(K2max))

    def submit(self, stream, depth, feat_xyz, feat_desc, K2, out_vertices=None, out_dq=None, inputs_ready=None):
        """Queues one frame (device tensors or addresses, kept unchanged until it is done); returns
        its ticket."""
        ev = _event_ptr(inputs_ready)
        fr = FrameDevice(_dev_ptr(depth), _dev_ptr(feat_xyz), _dev_ptr(feat_desc), int(K2), _dev_ptr(out_vertices),
                         _dev_ptr(out_dq), ev.value if ev is not None else None)
        t = C.c_uint64()
        _check(lib().tt_server_submit(self.h, stream.h, C.byref(fr), C.byref(t)), "tt_server_submit")
        return t.value

    def poll(self, ticket):
        """(done, latency_ms or None); raises TTError if the frame failed."""
        done, lat = C.c_int(), C.c_double()
        _check(lib().tt_server_poll(self.h, int(ticket), C.byref(done), C.byref(lat)), "tt_server_poll")
        return bool(done.value), (lat.value if done.value else None)

    def wait(self, ticket, wait_s=60.0):
        lat = C.c_double()
        _check(lib().tt_server_wait(self.h, int(ticket), float(wait_s), C.byref(lat)), "tt_server_wait")
        return lat.value

    def close(self, stream):
        if stream.h:
            _check(lib().tt_server_close(self.h, stream.h), "tt_server_close")
            stream.h = None

    def stats(self):
        st = ServerStats()
        _check(lib().tt_server_get_stats(self.h, C.byref(st)), "tt_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def destroy(self):
        if self.h:
            _check(lib().tt_server_destroy(self.h), "tt_server_destroy")
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def create_stream(params, intr, hip_stream=None):
    return Stream(params, intr, hip_stream)


def orb_params(**kw):
    p = OrbParams()
    lib().tt_orb_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Orb:
    """Uniform ORB detector for width x height 8-bit images (tt_orb_*)."""

    def __init__(self, params, width, height, pattern, hip_stream=None):
        self.params = params
        self.W, self.H = int(width), int(height)
        self._pattern = _c(pattern, np.int8)
        h = C.c_void_p()
        _check(lib().tt_orb_create(C.byref(params), self.W, self.H, _ptr(self._pattern),
                                   C.c_void_p(hip_stream) if hip_stream else None, C.byref(h)), "tt_orb_create")
        self.h = h

    def detect(self, image, depth=None, intr=None):
        """Host arrays in and out: dict(kp [n,2] int32, xyz [n,3] float32, desc [n,32] uint8,
        angle_bin [n] int32, total)."""
        img = _c(image, np.uint8)
        mx = max(self.params.max_features, 1)
        kp = np.zeros((mx, 2), np.int32)
        xyz = np.zeros((mx, 3), np.float32)
        desc = np.zeros((mx, 32), np.uint8)
        ang = np.zeros(mx, np.int32)
        cnt = np.zeros(2, np.int32)
        d = _c(depth, np.float32) if depth is not None else None
        _check(lib().tt_orb_detect(self.h, _ptr(img), _ptr(d), C.byref(intr) if intr is not None else None,
                                   _ptr(kp), _ptr(xyz), _ptr(desc), _ptr(ang), _ptr(cnt)), "tt_orb_detect")
        n = int(cnt[0])
        return dict(kp=kp[:n].copy(), xyz=xyz[:n].copy(), desc=desc[:n].copy(), angle_bin=ang[:n].copy(),
                    total=int(cnt[1]))

    def detect_device(self, image, depth, intr, kp, xyz, desc, angle, count):
        """Device tensors (or addresses); queued on the detector's HIP stream."""
        _check(lib().tt_orb_detect_device(self.h, _dev_ptr(image), _dev_ptr(depth),
                                          C.byref(intr) if intr is not None else None, _dev_ptr(kp),
                                          _dev_ptr(xyz), _dev_ptr(desc), _dev_ptr(angle), _dev_ptr(count)),
               "tt_orb_detect_device")

    def hip_stream(self):
        return lib().tt_orb_hip_stream(self.h)

    def destroy(self):
        if self.h:
            lib().tt_orb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
