"""Small hand-built scenes for pinning the oracle against closed forms (CPU only)."""
import math

import numpy as np

from paper_2007_08576_amd import synth


def random_dq(rng: np.random.Generator, n: int, rot_deg: float, trans_mm: float) -> np.ndarray:
    """n unit dual quaternions with random axis-angle rotation up to rot_deg and translation
    up to trans_mm, written out from the textbook definition (qd = t qr / 2)."""
    out = np.zeros((n, 8))
    for i in range(n):
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        th = math.radians(rot_deg) * rng.uniform(0.2, 1.0)
        q = np.array([math.cos(th / 2), *(math.sin(th / 2) * ax)])
        t = rng.normal(size=3)
        t *= trans_mm * rng.uniform(0.2, 1.0) / np.linalg.norm(t)
        out[i, :4] = q
        out[i, 4:] = 0.5 * quat_mul(np.array([0.0, *t]), q)
    return out


def quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def quat_to_matrix(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def dq_rt(dq):
    """Rotation matrix and translation of a unit dual quaternion (textbook)."""
    q = dq[:4]
    t = 2.0 * quat_mul(dq[4:], q * np.array([1, -1, -1, -1]))[1:]
    return quat_to_matrix(q), t


def dyadic_plane(width=32, height=24, fx=128.0):
    """Tilted plane z = 96 + u/4 + v/8 whose depths and back-projections are exact in float32.
    Returns (intrinsics, depth, grid points (H, W, 3) float64)."""
    K = synth.Intrinsics(width, height, fx, fx, float(width // 2), float(height // 2))
    u = np.arange(width, dtype=np.float64)[None, :]
    v = np.arange(height, dtype=np.float64)[:, None]
    depth = (96.0 + u / 4.0 + v / 8.0).astype(np.float32)
    P = synth.backproject_grid(depth, K)
    assert np.array_equal(P.astype(np.float32).astype(np.float64), P)
    return K, depth, P


def lattice_scene(n_side=17, spacing=50.0, z=401.0, f_half=2):
    """Template points on a square grid in the plane z = 401 and (2 f_half + 1)^2 features on
    the lattice 401 (i, j, 1), |i|, |j| <= f_half, with a rotation by atan2(40, 399) about the z axis that maps
    every lattice point to integer coordinates (Pythagorean triple 399^2 + 40^2 = 401^2)."""
    ax = (np.arange(n_side) - n_side // 2) * spacing
    X, Y = np.meshgrid(ax, ax)
    pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], 1)
    ij = np.array([(i, j) for i in range(-f_half, f_half + 1) for j in range(-f_half, f_half + 1)],
                  np.float64)
    feats = np.stack([401.0 * ij[:, 0], 401.0 * ij[:, 1], np.full(len(ij), 401.0)], 1)
    R = np.array([[399.0, -40.0, 0.0], [40.0, 399.0, 0.0], [0.0, 0.0, 401.0]]) / 401.0
    t = np.array([3.0, -2.0, 1.0])
    return pts, feats, R, t


def two_layer_scene():
    """A plane's interior pixel centres (front) and the same points at twice the distance (back,
    on the same camera rays, so on the same pixels), back layer first in index order, plus an
    exact copy of front point 0 at the end (an equal-z tie that the lower index wins).
    Returns (intrinsics, depth, template points float32, back count, front count)."""
    K, depth, P = dyadic_plane()
    front = P[2:-2, 2:-2].reshape(-1, 3)
    back = 2.0 * front
    pts = np.vstack([back, front, front[:1]]).astype(np.float32)
    return K, depth, pts, len(back), len(front)
