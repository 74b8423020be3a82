"""Seeded synthetic workloads shaped like the paper's experiments (stereo depth + ORB features).

The paper evaluates on stereo laparoscope videos, the Hamlyn phantom and an EM-tracked liver
(Sec. 3); none of that data is available, so these scenes stand in for it:

* config 1 -- 128 x 96 height field z = 80 + 6 sin(u/15) cos(v/20) mm, 3,000 template points,
  64 control points, one target frame warped by three Gaussian bumps plus a 3 deg / 2 mm rigid
  motion, 400 features (25 % outliers), exact feature positions;
* config 2 -- 640 x 480 surface of 20 Gaussian dents over a 100 mm plane, 30,000 template
  points, 400 control points, 2,000 features (30 % outliers), a sequence of frames deformed by
  six oscillating Gaussian bumps whose largest per-frame motion is 15 mm, feature positions
  lifted from the rendered depth;
* config 3 -- config 2 with 1,500 control points and 100,000 template points;
* config 4 -- 16 streams of uneven size (see make_config4);
* config 5 -- 64 stressed streams (see make_config5): in a fifth of the frames 60 % of the matches
  are outliers, 30 % of the depth pixels are occluded by smoke-like blobs, and the camera jumps
  10 deg / 20 mm.

This module holds only the workload recipe (surfaces, warps, a z-buffered mesh rasteriser and
descriptor noise); none of the tracking method's arithmetic. Every draw comes from a
counter-based SplitMix64 stream keyed by (seed, purpose), so any frame can be regenerated alone.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _fnv1a64(s: str) -> int:
    h = 0xCBF29CE484222325
    for ch in s.encode():
        h ^= ch
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


class Rng:
    """Counter-based SplitMix64: output k of a stream is mix(state0 + k * golden)."""

    def __init__(self, seed: int, tag: str):
        with np.errstate(over="ignore"):
            s = np.array([(int(seed) ^ _fnv1a64(tag)) & 0xFFFFFFFFFFFFFFFF], np.uint64)
            self.state0 = _mix(s + GOLDEN)[0]
        self.k = 0

    def u64(self, n: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            ks = np.arange(self.k + 1, self.k + 1 + n, dtype=np.uint64)
            out = _mix(self.state0 + ks * GOLDEN)
        self.k += n
        return out

    def uniform(self, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        u = (self.u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
        return lo + (hi - lo) * u

    def normal(self, n: int) -> np.ndarray:
        u1 = self.uniform(n)
        u2 = self.uniform(n)
        return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)

    def integers(self, n: int, hi: int) -> np.ndarray:
        return np.minimum((self.uniform(n) * hi).astype(np.int64), hi - 1)

    def choice(self, pop: int, k: int) -> np.ndarray:
        """k distinct indices of range(pop), in draw order (random keys, k smallest)."""
        keys = self.u64(pop)
        return np.argsort(keys, kind="stable")[:k]

    def unit_vectors(self, n: int) -> np.ndarray:
        v = np.stack([self.normal(n), self.normal(n), self.normal(n)], 1)
        return v / np.linalg.norm(v, axis=1, keepdims=True)

    def bytes(self, n: int) -> np.ndarray:
        return self.u64((n + 7) // 8).view(np.uint8)[:n].copy()


@dataclasses.dataclass
class Intrinsics:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


def intrinsics_for(width: int, height: int) -> Intrinsics:
    """Pinhole model of the 128 x 96 config (fx = 110, centre (64, 48)) scaled to width."""
    s = width / 128.0
    return Intrinsics(width, height, 110.0 * s, 110.0 * s, width / 2.0, height / 2.0)


def backproject_grid(depth: np.ndarray, K: Intrinsics) -> np.ndarray:
    """(H, W, 3) camera-frame points of every pixel centre (u, v) at the given depth."""
    H, W = depth.shape
    u = np.arange(W, dtype=np.float64)[None, :]
    v = np.arange(H, dtype=np.float64)[:, None]
    z = depth.astype(np.float64)
    return np.stack([(u - K.cx) / K.fx * z, (v - K.cy) / K.fy * z, z], -1)


def render_depth(P: np.ndarray, K: Intrinsics, attr: np.ndarray | None = None):
    """Z-buffered depth of the grid mesh with vertices P (H, W, 3): two triangles per 2 x 2
    quad, perspective-correct depth (1/z interpolated in screen space) at pixel centres.
    Uncovered pixels get depth 0 (invalid). With attr (H, W, C) per vertex, also returns the
    attribute of the visible surface at every pixel centre (perspective-correct, NaN where
    uncovered)."""
    H, W = P.shape[:2]
    X = P.reshape(-1, 3)
    z = X[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        su = K.fx * X[:, 0] / z + K.cx
        sv = K.fy * X[:, 1] / z + K.cy
    idx = np.arange(H * W).reshape(H, W)
    a = idx[:-1, :-1].ravel()
    b = idx[:-1, 1:].ravel()
    c = idx[1:, :-1].ravel()
    d = idx[1:, 1:].ravel()
    tri = np.concatenate([np.stack([a, b, c], 1), np.stack([b, d, c], 1)], 0)
    ok = np.all(z[tri] > 1e-6, axis=1)
    tri = tri[ok]
    tu, tv, tz = su[tri], sv[tri], z[tri]
    u0 = np.ceil(tu.min(1)).astype(np.int64)
    u1 = np.floor(tu.max(1)).astype(np.int64)
    v0 = np.ceil(tv.min(1)).astype(np.int64)
    v1 = np.floor(tv.max(1)).astype(np.int64)
    u0 = np.maximum(u0, 0)
    v0 = np.maximum(v0, 0)
    u1 = np.minimum(u1, W - 1)
    v1 = np.minimum(v1, H - 1)
    bw = np.maximum(u1 - u0 + 1, 0)
    bh = np.maximum(v1 - v0 + 1, 0)
    cnt = bw * bh
    keep = cnt > 0
    tri_i = np.nonzero(keep)[0]
    cnt = cnt[keep]
    total = int(cnt.sum())
    zbuf = np.full(H * W, np.inf)
    if total == 0:
        if attr is not None:
            return np.zeros((H, W), np.float32), np.full((H, W, attr.shape[-1]), np.nan)
        return np.zeros((H, W), np.float32)
    rep = np.repeat(tri_i, cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    off = np.arange(total) - start
    px = u0[rep] + off % bw[rep]
    py = v0[rep] + off // bw[rep]
    x0, x1, x2 = tu[rep, 0], tu[rep, 1], tu[rep, 2]
    y0, y1, y2 = tv[rep, 0], tv[rep, 1], tv[rep, 2]
    area = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)
    with np.errstate(divide="ignore", invalid="ignore"):
        l1 = ((px - x0) * (y2 - y0) - (x2 - x0) * (py - y0)) / area
        l2 = ((x1 - x0) * (py - y0) - (px - x0) * (y1 - y0)) / area
    l0 = 1.0 - l1 - l2
    eps = -1e-9
    inside = (np.abs(area) > 1e-12) & (l0 >= eps) & (l1 >= eps) & (l2 >= eps)
    invz = l0 / tz[rep, 0] + l1 / tz[rep, 1] + l2 / tz[rep, 2]
    inside &= invz > 0
    pix = (py * W + px)[inside]
    zz = 1.0 / invz[inside]
    np.minimum.at(zbuf, pix, zz)
    out = np.where(np.isfinite(zbuf), zbuf, 0.0).astype(np.float32)
    if attr is None:
        return out.reshape(H, W)
    # attribute of the nearest candidate of each pixel
    A = attr.reshape(-1, attr.shape[-1]).astype(np.float64)
    ti = tri[rep][inside]
    w = np.stack([l0[inside] / tz[rep, 0][inside], l1[inside] / tz[rep, 1][inside],
                  l2[inside] / tz[rep, 2][inside]], 1)
    order = np.lexsort((zz, pix))
    first = order[np.r_[True, pix[order][1:] != pix[order][:-1]]]
    vals = (w[first, :, None] * A[ti[first]]).sum(1) * zz[first, None]
    img = np.full((H * W, A.shape[1]), np.nan)
    img[pix[first]] = vals
    return out.reshape(H, W), img.reshape(H, W, -1)


def surface_texture(seed: int, name: str, width: int, height: int):
    """A fixed random texture painted on the template surface, as a function of the template
    image coordinates (u0, v0): value noise (lattice values blended with smoothstep weights) at
    periods of 16, 8 and 4 pixels. Returns f(u0, v0) -> intensity in [0, 255] (float)."""
    rng = Rng(seed, f"{name}/texture")
    octaves = []
    for period, amp in ((16.0, 0.5), (8.0, 0.3), (4.0, 0.2)):
        gw, gh = int(width / period) + 3, int(height / period) + 3
        octaves.append((period, amp, rng.uniform(gw * gh).reshape(gh, gw)))

    def f(u0, v0):
        u0, v0 = np.asarray(u0, np.float64), np.asarray(v0, np.float64)
        bad = ~(np.isfinite(u0) & np.isfinite(v0))
        u0, v0 = np.where(bad, 0.0, u0), np.where(bad, 0.0, v0)
        acc = np.zeros(np.shape(u0))
        for period, amp, g in octaves:
            x = np.clip(u0 / period, 0, g.shape[1] - 2.000001)
            y = np.clip(v0 / period, 0, g.shape[0] - 2.000001)
            ix, iy = np.floor(x).astype(np.int64), np.floor(y).astype(np.int64)
            fx, fy = x - ix, y - iy
            fx, fy = fx * fx * (3 - 2 * fx), fy * fy * (3 - 2 * fy)  # smoothstep: no creases
            val = (g[iy, ix] * (1 - fx) * (1 - fy) + g[iy, ix + 1] * fx * (1 - fy)
                   + g[iy + 1, ix] * (1 - fx) * fy + g[iy + 1, ix + 1] * fx * fy)
            acc = acc + amp * val
        return np.where(bad, np.nan, 255.0 * acc)

    return f


def to_image(intensity: np.ndarray) -> np.ndarray:
    """8-bit grey image from intensities (NaN, i.e. background, is black)."""
    x = np.where(np.isfinite(intensity), intensity, 0.0)
    return np.clip(np.floor(x + 0.5), 0, 255).astype(np.uint8)


def orb_pattern(seed: int = 0) -> np.ndarray:
    """256 point pairs (x1, y1, x2, y2) for binary descriptors: i.i.d. Gaussian offsets with
    sigma = 31 / 5 px (a 31-pixel patch), rounded, redrawn until inside the disc of radius 13.
    Returns (256, 4) int8."""
    rng = Rng(seed, "orb/pattern")
    out = np.zeros((256, 4), np.int8)
    for k in range(256):
        for h in range(2):
            while True:
                x, y = np.floor(rng.normal(2) * (31.0 / 5.0) + 0.5)
                if x * x + y * y <= 169:
                    break
            out[k, 2 * h], out[k, 2 * h + 1] = int(x), int(y)
    return out


def flip_bits(desc: np.ndarray, rng: Rng, nbits: int = 8) -> np.ndarray:
    """Copy of each 32-byte descriptor with exactly nbits distinct bits flipped."""
    out = desc.copy()
    for i in range(desc.shape[0]):
        bits = rng.choice(256, nbits)
        for b in bits:
            out[i, b >> 3] ^= np.uint8(1 << (b & 7))
    return out


def rotation_matrix(axis: np.ndarray, angle: float) -> np.ndarray:
    axis = axis / np.linalg.norm(axis)
    x, y, z = axis
    c, s = math.cos(angle), math.sin(angle)
    C = 1 - c
    return np.array([[c + x * x * C, x * y * C - z * s, x * z * C + y * s],
                     [y * x * C + z * s, c + y * y * C, y * z * C - x * s],
                     [z * x * C - y * s, z * y * C + x * s, c + z * z * C]])


@dataclasses.dataclass
class Frame:
    depth: np.ndarray       # (H, W) float32, mm; 0 = invalid
    feat_xyz: np.ndarray    # (K2, 3) float32; NaN = no depth
    feat_desc: np.ndarray   # (K2, 32) uint8
    gt_vertices: np.ndarray  # (M, 3) float64 ground-truth positions of the template points
    inlier_of: np.ndarray   # (K2,) template feature index of an inlier, -1 for an outlier
    stressed: bool = False   # a stressed frame (config 5)


@dataclasses.dataclass
class Scene:
    name: str
    intr: Intrinsics
    num_control_points: int
    pts: np.ndarray          # (M, 3) float32 template points
    feat_xyz: np.ndarray     # (K1, 3) float32
    feat_desc: np.ndarray    # (K1, 32) uint8
    n_frames: int
    _frame_fn: object = None
    _grid: np.ndarray = None
    _image_fn: object = None

    def frame(self, t: int) -> Frame:
        """Target frame t (1 <= t <= n_frames)."""
        if not 1 <= t <= self.n_frames:
            raise IndexError(t)
        return self._frame_fn(t)

    def image(self, t: int):
        """(depth, 8-bit grey image) of frame t of the textured surface, t = 0 the template's
        own frame (sequence scenes only)."""
        if self._image_fn is None:
            raise ValueError("scene has no texture")
        if not 0 <= t <= self.n_frames:
            raise IndexError(t)
        return self._image_fn(t)


def _features(rng_tag_seed, name, t, tmpl_xyz, tmpl_desc, gt_xyz, target_P, target_valid,
              n_out, exact, K: Intrinsics):
    """Frame features: inliers (template feature warped to the frame, 8 flipped bits) and
    outliers (fresh random descriptors at random valid target pixels), shuffled."""
    rng = Rng(rng_tag_seed, f"{name}/features/{t}")
    K1 = tmpl_xyz.shape[0]
    n_in = K1 - n_out
    which = rng.choice(K1, n_in)
    desc_in = flip_bits(tmpl_desc[which], rng, 8)
    if exact:
        xyz_in = gt_xyz[which]
    else:
        g = gt_xyz[which]
        with np.errstate(divide="ignore", invalid="ignore"):
            u = np.floor(K.fx * g[:, 0] / g[:, 2] + K.cx + 0.5)
            v = np.floor(K.fy * g[:, 1] / g[:, 2] + K.cy + 0.5)
        ok = (g[:, 2] > 0) & (u >= 0) & (u < K.width) & (v >= 0) & (v < K.height)
        ui = np.where(ok, u, 0).astype(np.int64)
        vi = np.where(ok, v, 0).astype(np.int64)
        ok &= target_valid[vi, ui]
        xyz_in = np.where(ok[:, None], target_P[vi, ui], np.nan)
    valid_pix = np.flatnonzero(target_valid.ravel())
    pick = valid_pix[rng.integers(n_out, valid_pix.size)] if n_out else np.zeros(0, np.int64)
    xyz_out = target_P.reshape(-1, 3)[pick]
    desc_out = rng.bytes(32 * n_out).reshape(n_out, 32)
    xyz = np.concatenate([xyz_in, xyz_out], 0)
    desc = np.concatenate([desc_in, desc_out], 0)
    inl = np.concatenate([which, -np.ones(n_out, np.int64)])
    perm = rng.choice(K1, K1)
    return xyz[perm].astype(np.float32), desc[perm].copy(), inl[perm]


def make_config1(seed: int = 1) -> Scene:
    """128 x 96 height field, one target frame (see module docstring)."""
    name = "config1"
    W, H = 128, 96
    K = Intrinsics(W, H, 110.0, 110.0, 64.0, 48.0)
    u = np.arange(W, dtype=np.float64)[None, :]
    v = np.arange(H, dtype=np.float64)[:, None]
    depth0 = (80.0 + 6.0 * np.sin(u / 15.0) * np.cos(v / 20.0)).astype(np.float32)
    P0 = backproject_grid(depth0, K)
    rng = Rng(seed, f"{name}/template")
    tidx = np.sort(rng.choice(W * H, 3000))
    pts = P0.reshape(-1, 3)[tidx]
    fidx = rng.choice(3000, 400)
    feat_xyz = pts[fidx]
    feat_desc = rng.bytes(400 * 32).reshape(400, 32)
    # the warp: three Gaussian bumps along +z (amplitude 4 mm, sigma 15 mm), then 3 deg / 2 mm
    wr = Rng(seed, f"{name}/warp")
    mu = pts[wr.choice(3000, 3)]
    sgn = np.where(wr.uniform(3) < 0.5, -1.0, 1.0)
    Rg = rotation_matrix(wr.unit_vectors(1)[0], math.radians(3.0))
    tg = 2.0 * wr.unit_vectors(1)[0]

    def G(x):
        d2 = ((x[:, None, :] - mu[None, :, :]) ** 2).sum(-1)
        bump = (4.0 * sgn[None, :] * np.exp(-d2 / (2 * 15.0 ** 2))).sum(1)
        y = x.copy()
        y[:, 2] += bump
        return y @ Rg.T + tg

    def frame_fn(t):
        Pt = G(P0.reshape(-1, 3)).reshape(H, W, 3)
        depth = render_depth(Pt, K)
        tP = backproject_grid(depth, K)
        valid = depth > 0
        gt_f = G(feat_xyz.astype(np.float64))
        fx, fd, inl = _features(seed, name, t, feat_xyz, feat_desc, gt_f, tP, valid, 100, True, K)
        return Frame(depth, fx, fd, G(pts.astype(np.float64)), inl)

    return Scene(name, K, 64, pts.astype(np.float32), feat_xyz.astype(np.float32), feat_desc, 1,
                 frame_fn)


@dataclasses.dataclass
class Stress:
    """Stressed frames (config 5): each frame is stressed with probability prob (a draw keyed by the
    frame); a stressed frame has outlier_frac of its matches outliers, exactly invalid_frac of its
    pixels invalid (the largest values of a sum of n_blobs Gaussian blobs with radii U[20, 80] px,
    ties to the lower pixel index), and is seen from the stream's second camera pose: the scene
    rotated by angle_deg about a random axis through the template centroid and moved by shift_mm."""
    prob: float = 0.2
    outlier_frac: float = 0.6
    invalid_frac: float = 0.3
    n_blobs: int = 8
    angle_deg: float = 10.0
    shift_mm: float = 20.0


def stressed_frame(seed: int, name: str, t: int, prob: float) -> bool:
    """Whether frame t of the sequence (seed, name) is stressed (one draw keyed by the frame)."""
    return bool(Rng(seed, f"{name}/stress/{t}").uniform(1)[0] < prob)


def blob_mask(rng: Rng, width: int, height: int, frac: float, n_blobs: int) -> np.ndarray:
    """(H, W) bool: exactly round(frac * W * H) pixels, those with the largest sum of random
    Gaussian blobs (centres uniform in the image, radii U[20, 80] px at 640 wide)."""
    cu = rng.uniform(n_blobs, 0.0, width)
    cv = rng.uniform(n_blobs, 0.0, height)
    rad = rng.uniform(n_blobs, 20.0, 80.0) * (width / 640.0)
    amp = rng.uniform(n_blobs, 0.5, 1.0)
    u = np.arange(width, dtype=np.float64)[None, :, None]
    v = np.arange(height, dtype=np.float64)[:, None, None]
    f = (amp * np.exp(-((u - cu) ** 2 + (v - cv) ** 2) / (2 * rad ** 2))).sum(-1).ravel()
    n = int(round(frac * width * height))
    order = np.lexsort((np.arange(f.size), -f))  # largest first, ties to the lower index
    m = np.zeros(f.size, bool)
    m[order[:n]] = True
    return m.reshape(height, width)


def make_sequence(seed: int = 2, M: int = 30000, N: int = 400, K1: int = 2000,
                  outlier_frac: float = 0.30, width: int = 640, height: int = 480,
                  n_frames: int = 300, max_step_mm: float = 15.0, name: str = "config2",
                  stress: Stress | None = None) -> Scene:
    """Gaussian-dent surface and an oscillating six-bump deformation sequence (config 2/3); with
    stress, some frames are stressed as described by Stress (config 5)."""
    K = intrinsics_for(width, height)
    W, H = width, height
    rng = Rng(seed, f"{name}/surface")
    A = rng.uniform(20, 2.0, 10.0)
    mu = np.stack([rng.uniform(20, 0, W), rng.uniform(20, 0, H)], 1)
    s = rng.uniform(20, 20.0, 80.0) * (W / 640.0)
    u = np.arange(W, dtype=np.float64)[None, :, None]
    v = np.arange(H, dtype=np.float64)[:, None, None]
    d2 = (u - mu[None, None, :, 0]) ** 2 + (v - mu[None, None, :, 1]) ** 2
    depth0 = (100.0 - (A * np.exp(-d2 / (2 * s ** 2))).sum(-1)).astype(np.float32)
    P0 = backproject_grid(depth0, K)
    rt = Rng(seed, f"{name}/template")
    tidx = np.sort(rt.choice(W * H, M))
    pts = P0.reshape(-1, 3)[tidx]
    fidx = rt.choice(M, K1)
    feat_xyz = pts[fidx]
    feat_desc = rt.bytes(K1 * 32).reshape(K1, 32)
    # six oscillating bumps: G_t(x) = x + sum_b A_b (sin(2 pi t / T_b + phi_b) - sin(phi_b)) g_b(x) d_b
    rw = Rng(seed, f"{name}/warp")
    nb = 6
    bmu = pts[rw.choice(M, nb)]
    sig = rw.uniform(nb, 10.0, 25.0)
    T = rw.uniform(nb, 10.0, 40.0)
    phi = rw.uniform(nb, 0.0, 2 * np.pi)
    dirs = np.zeros((nb, 3))
    for b in range(nb):
        while True:
            dvec = rw.unit_vectors(1)[0]
            if abs(dvec[2]) >= 0.5:
                break
        dirs[b] = dvec

    def disp_coeff(x):
        d2 = ((x[:, None, :] - bmu[None, :, :]) ** 2).sum(-1)
        return np.exp(-d2 / (2 * sig[None, :] ** 2))          # (n, nb)

    def osc(t):
        return np.sin(2 * np.pi * t / T + phi) - np.sin(phi)    # (nb,)

    # amplitude scale: largest per-frame displacement change of a template point = max_step_mm
    gtmpl = disp_coeff(pts)
    best = 0.0
    for t in range(1, n_frames + 1):
        dv = (gtmpl * (osc(t) - osc(t - 1))[None, :]) @ dirs
        best = max(best, float(np.sqrt((dv ** 2).sum(1)).max()))
    amp = max_step_mm / best if best > 0 else 0.0

    def G(x, t):
        return x + (disp_coeff(x) * (amp * osc(t))[None, :]) @ dirs

    n_out = int(round(outlier_frac * K1))
    if stress is not None:
        rc = Rng(seed, f"{name}/camera")
        cam_R = rotation_matrix(rc.unit_vectors(1)[0], math.radians(stress.angle_deg))
        cam_t = stress.shift_mm * rc.unit_vectors(1)[0]
        centroid = pts.astype(np.float64).mean(0)

    def frame_fn(t):
        hard = stress is not None and stressed_frame(seed, name, t, stress.prob)

        def Gc(x):  # the deformed scene in this frame's camera coordinates
            y = G(x, t)
            return (y - centroid) @ cam_R.T + centroid + cam_t if hard else y

        Pt = Gc(P0.reshape(-1, 3)).reshape(H, W, 3)
        depth = render_depth(Pt, K)
        if hard:
            occ = blob_mask(Rng(seed, f"{name}/occlusion/{t}"), W, H, stress.invalid_frac, stress.n_blobs)
            depth = np.where(occ, np.float32(0.0), depth).astype(np.float32)
        tP = backproject_grid(depth, K)
        valid = depth > 0
        gt_f = Gc(feat_xyz.astype(np.float64))
        n_o = int(round(stress.outlier_frac * K1)) if hard else n_out
        fx, fd, inl = _features(seed, name, t, feat_xyz, feat_desc, gt_f, tP, valid, n_o, False, K)
        return Frame(depth, fx, fd, Gc(pts.astype(np.float64)), inl, hard)

    tex = surface_texture(seed, name, W, H)
    uv0 = np.stack(np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64)), -1)

    def image_fn(t):
        # the textured surface seen in frame t (t = 0: the template, undeformed)
        if t == 0:
            return depth0, to_image(tex(uv0[..., 0], uv0[..., 1]))
        hard = stress is not None and stressed_frame(seed, name, t, stress.prob)
        y = G(P0.reshape(-1, 3), t)
        if hard:
            y = (y - centroid) @ cam_R.T + centroid + cam_t
        depth, a = render_depth(y.reshape(H, W, 3), K, uv0)
        if hard:
            occ = blob_mask(Rng(seed, f"{name}/occlusion/{t}"), W, H, stress.invalid_frac, stress.n_blobs)
            depth = np.where(occ, np.float32(0.0), depth).astype(np.float32)
        return depth, to_image(tex(a[..., 0], a[..., 1]))

    return Scene(name, K, N, pts.astype(np.float32), feat_xyz.astype(np.float32), feat_desc,
                 n_frames, frame_fn, _image_fn=image_fn)


def make_config2(seed: int = 2, n_frames: int = 300) -> Scene:
    return make_sequence(seed=seed, n_frames=n_frames)


def make_config3(seed: int = 3, n_frames: int = 300) -> Scene:
    return make_sequence(seed=seed, M=100000, N=1500, K1=2000, n_frames=n_frames, name="config3")


def make_config4(seed: int = 4, n_streams: int = 16, n_frames: int = 300):
    """Serving mix (config 4): n_streams independent streams with uneven sizes. Per stream s
    (seeded 1000 * seed + s): control points N ~ U{100..800}, depth map one of 320x240, 480x360,
    640x480 (intrinsics scaled with the width), M = W * H / 10 template points, K ~ U{500..3000}
    features with an outlier fraction ~ U[0.2, 0.4]; each stream is a config-2-style sequence."""
    sizes = ((320, 240), (480, 360), (640, 480))
    scenes = []
    for q in range(n_streams):
        rng = Rng(1000 * seed + q, "config4/stream")
        N = 100 + int(rng.uniform(1, 0.0, 701.0)[0])
        W, H = sizes[int(rng.uniform(1, 0.0, 3.0)[0])]
        K1 = 500 + int(rng.uniform(1, 0.0, 2501.0)[0])
        out = float(rng.uniform(1, 0.2, 0.4)[0])
        scenes.append(make_sequence(seed=1000 * seed + q, M=W * H // 10, N=min(N, 800), K1=min(K1, 3000),
                                    outlier_frac=out, width=W, height=H, n_frames=n_frames,
                                    name=f"config4/{q}"))
    return scenes


def config5_stream(seed: int, q: int, n_frames: int = 300) -> Scene:
    """Stream q of config 5 (seeded 1000 * seed + q): 640 x 480, N ~ U{200..1500} control points,
    M = W * H / 10 template points, 2,000 features with 30 % outliers, stressed frames as Stress()."""
    rng = Rng(1000 * seed + q, "config5/stream")
    N = 200 + int(rng.uniform(1, 0.0, 1301.0)[0])
    return make_sequence(seed=1000 * seed + q, M=640 * 480 // 10, N=min(N, 1500), K1=2000,
                         outlier_frac=0.3, width=640, height=480, n_frames=n_frames,
                         name=f"config5/{q}", stress=Stress())


@dataclasses.dataclass
class StreamSpec:
    """What a stream needs of a Scene, without its frame generator (picklable)."""
    num_control_points: int
    intr: Intrinsics
    pts: np.ndarray
    feat_xyz: np.ndarray
    feat_desc: np.ndarray


def config5_arrays(seed: int, q: int, n_frames: int):
    """Config 5 stream q as plain arrays: (StreamSpec, [(depth, feat_xyz, feat_desc)] for frames
    1 .. n_frames, number of stressed frames among them). For generating streams in worker
    processes."""
    sc = config5_stream(seed, q, n_frames=300)
    frs = [sc.frame(t) for t in range(1, n_frames + 1)]
    spec = StreamSpec(sc.num_control_points, sc.intr, sc.pts, sc.feat_xyz, sc.feat_desc)
    return spec, [(f.depth, f.feat_xyz, f.feat_desc) for f in frs], sum(f.stressed for f in frs)


def config2_arrays(seed: int, n_frames: int, ts):
    """Frames ts of make_config2(seed, n_frames) as plain arrays (depth, feat_xyz, feat_desc,
    gt_vertices). For generating a long sequence in worker processes."""
    sc = make_config2(seed=seed, n_frames=n_frames)
    return [(f.depth, f.feat_xyz, f.feat_desc, f.gt_vertices) for f in (sc.frame(t) for t in ts)]


def make_config5(seed: int = 5, n_streams: int = 64, n_frames: int = 300):
    """Stress serving (config 5): n_streams streams from config5_stream."""
    return [config5_stream(seed, q, n_frames) for q in range(n_streams)]


def make_small_sequence(seed: int = 11, M: int = 2000, N: int = 48, K1: int = 300,
                        width: int = 160, height: int = 120, n_frames: int = 4,
                        max_step_mm: float = 3.0) -> Scene:
    """A reduced sequence (same recipe as config 2) whose oracle frames finish in seconds."""
    return make_sequence(seed=seed, M=M, N=N, K1=K1, width=width, height=height,
                         n_frames=n_frames, max_step_mm=max_step_mm, name="small")
