"""Seeded synthetic inputs for the near-wall mesh-adaptation path.

This module only *generates* geometry, weights and workload descriptors.  It
holds none of the method's arithmetic (no binning, no separating-axis test, no
refinement, no link fractions), so that the CPU oracle under ``oracle/`` and the
HIP library can both be fed from it without sharing any computational code.

Every generator works in FP64 and rounds to FP32 exactly once at the end.

Workloads (the paper's own test bodies, a circle and a scanned bunny, are
described in the Results section; the bunny mesh is not available, so seeded
star-shaped bodies stand in for an irregular, large triangle count):

* ``C0`` 2D circle, 256 segments, radius 0.25 at (0.5, 0.5); 16x16 root
  quadtrees of 4x4 cells; 3 refinement passes; 32x32 bins; D2Q9.
* ``C1`` icosphere of subdivision 5 (20,480 triangles), radius 0.2 at the
  centre of the unit cube; 16^3 root octrees of 4^3 cells; 3 passes; 64^3 bins;
  D3Q19.
* ``C2`` star body on an icosphere of subdivision 7 (327,680 triangles); 32^3
  roots; 4 passes; 128^3 bins; D3Q27.
* ``C3`` the C1 sphere with every vertex jittered by N(0, 1e-3); loss weights
  U(-1, 1).
* ``C4`` 64 star bodies, subdivisions drawn from {3..7}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Tuple

import numpy as np

# Fixed seeds for every random draw (star coefficients, jitter, weights, batch).
SEED_STAR = 0
SEED_JITTER = 1
SEED_WEIGHTS = 2
SEED_BATCH = 3


# --------------------------------------------------------------------------
# 2D: circle as a closed polyline of equal segments
# --------------------------------------------------------------------------
def circle(n: int = 256, r: float = 0.25, center=(0.5, 0.5)) -> Tuple[np.ndarray, np.ndarray]:
    """Counter-clockwise circle: vertex k at angle 2*pi*k/n, segment (k, k+1 mod n)."""
    k = np.arange(n, dtype=np.float64)
    th = 2.0 * math.pi * k / n
    v = np.stack([center[0] + r * np.cos(th), center[1] + r * np.sin(th)], axis=1)
    f = np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1).astype(np.int32)
    return v.astype(np.float32), f


# --------------------------------------------------------------------------
# 3D: icosphere (icosahedron, 4-way midpoint splits, projected each time)
# --------------------------------------------------------------------------
_PHI = (1.0 + math.sqrt(5.0)) / 2.0
_ICO_V = np.array(
    [[-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
     [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
     [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1]], dtype=np.float64)
_ICO_F = np.array(
    [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
     [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
     [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
     [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)


def _orient_outward(v: np.ndarray, f: np.ndarray) -> np.ndarray:
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, (a + b + c) / 3.0) < 0
    f = f.copy()
    f[flip] = f[flip][:, [0, 2, 1]]
    return f


def icosphere_unit(s: int) -> Tuple[np.ndarray, np.ndarray]:
    """Unit-sphere icosphere of subdivision ``s`` in FP64: 10*4^s+2 vertices, 20*4^s faces,
    outward counter-clockwise triangles."""
    v = _ICO_V / np.linalg.norm(_ICO_V, axis=1, keepdims=True)
    f = _orient_outward(v, _ICO_F)
    for _ in range(s):
        verts = [row for row in v]
        cache: Dict[Tuple[int, int], int] = {}

        def mid(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            idx = cache.get(key)
            if idx is None:
                m = 0.5 * (verts[i] + verts[j])
                m = m / np.linalg.norm(m)
                verts.append(m)
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        nf = np.empty((4 * len(f), 3), dtype=np.int64)
        for t, (a, b, c) in enumerate(f):
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf[4 * t + 0] = (a, ab, ca)
            nf[4 * t + 1] = (b, bc, ab)
            nf[4 * t + 2] = (c, ca, bc)
            nf[4 * t + 3] = (ab, bc, ca)
        v = np.array(verts)
        f = nf
    return v, f.astype(np.int32)


def icosphere(s: int, r: float = 0.2, center=(0.5, 0.5, 0.5)) -> Tuple[np.ndarray, np.ndarray]:
    u, f = icosphere_unit(s)
    v = np.asarray(center, dtype=np.float64) + r * u
    return v.astype(np.float32), f


# --------------------------------------------------------------------------
# 3D: star-shaped body, radius perturbed by real spherical harmonics
# --------------------------------------------------------------------------
def _assoc_legendre(lmax: int, x: np.ndarray) -> Dict[Tuple[int, int], np.ndarray]:
    """P_l^m(x) for 0 <= m <= l <= lmax, without the Condon-Shortley phase."""
    P: Dict[Tuple[int, int], np.ndarray] = {}
    sx = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    pmm = np.ones_like(x)
    for m in range(lmax + 1):
        if m > 0:
            pmm = pmm * (2 * m - 1) * sx
        P[(m, m)] = pmm
        if m + 1 <= lmax:
            P[(m + 1, m)] = x * (2 * m + 1) * pmm
        for l in range(m + 2, lmax + 1):
            P[(l, m)] = ((2 * l - 1) * x * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def real_sph_harm(lmax: int, dirs: np.ndarray) -> Dict[Tuple[int, int], np.ndarray]:
    """Orthonormal real spherical harmonics Y_lm at unit directions (polar angle from +z)."""
    x = np.clip(dirs[:, 2], -1.0, 1.0)
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    P = _assoc_legendre(lmax, x)
    Y: Dict[Tuple[int, int], np.ndarray] = {}
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m == 0:
                Y[(l, m)] = K * P[(l, 0)]
            elif m > 0:
                Y[(l, m)] = math.sqrt(2.0) * K * P[(l, am)] * np.cos(am * phi)
            else:
                Y[(l, m)] = math.sqrt(2.0) * K * P[(l, am)] * np.sin(am * phi)
    return Y


def star_coefficients(seed: int, lmax: int = 8, sigma: float = 0.03) -> List[Tuple[int, int, float]]:
    """a_lm ~ N(0, sigma^2 / l) for l = 1..lmax, m = -l..l, drawn in (l asc, m asc) order."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            out.append((l, m, float(rng.normal(0.0, sigma / math.sqrt(l)))))
    return out


def star_fp64(s: int, seed: int = SEED_STAR, r0: float = 0.2, center=(0.5, 0.5, 0.5),
              lmax: int = 8, sigma: float = 0.03) -> Tuple[np.ndarray, np.ndarray]:
    u, f = icosphere_unit(s)
    Y = real_sph_harm(lmax, u)
    pert = np.zeros(len(u))
    for l, m, a in star_coefficients(seed, lmax, sigma):
        pert += a * Y[(l, m)]
    r = r0 * (1.0 + pert)
    v = np.asarray(center, dtype=np.float64) + r[:, None] * u
    return v, f


def star(s: int, seed: int = SEED_STAR, **kw) -> Tuple[np.ndarray, np.ndarray]:
    v, f = star_fp64(s, seed, **kw)
    return v.astype(np.float32), f


# --------------------------------------------------------------------------
# Perturbations, loss weights, batch draws
# --------------------------------------------------------------------------
def jitter_fp64(v64: np.ndarray, sigma: float = 1e-3, seed: int = SEED_JITTER) -> np.ndarray:
    """Add N(0, sigma^2) per unique vertex and coordinate in FP64 (round later, once)."""
    rng = np.random.default_rng(seed)
    return v64 + rng.normal(0.0, sigma, size=v64.shape)


def weights(n: int, seed: int = SEED_WEIGHTS) -> np.ndarray:
    """One U(-1, 1) draw per (node, direction) slot, in canonical slot order."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=n).astype(np.float32)


# --------------------------------------------------------------------------
# Workload descriptors
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    dim: int
    vertices: np.ndarray          # [Nv, dim] float32
    faces: np.ndarray             # [F, dim] int32
    roots: Tuple[int, int, int]
    levels: int                   # number of refinement passes = finest level
    bins: int                     # bins per axis
    lattice: int                  # 9, 19 or 27
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    extra: dict = field(default_factory=dict)

    def cell_size(self, level: int, axis: int = 0) -> np.float32:
        """Cell edge at ``level`` along ``axis``: (hi-lo)/(4*R*2^level), one FP32 division."""
        span = np.float32(self.hi[axis]) - np.float32(self.lo[axis])
        return np.float32(span / np.float32(4 * self.roots[axis] * (1 << level)))

    def d_spec(self) -> np.ndarray:
        """Near-wall distance per tested level: one cell of that level (d_l = dx_l), or the workload's
        constant distance (extra["d_const"], the paper's setting) on every level."""
        if "d_const" in self.extra:
            return np.full(self.levels, np.float32(self.extra["d_const"]), dtype=np.float32)
        return np.array([self.cell_size(l) for l in range(self.levels)], dtype=np.float32)


def _face_count(s: int) -> int:
    return 20 * 4 ** s


def workload(name: str) -> Workload:
    name = name.upper()
    if name == "C0":
        v, f = circle(256, 0.25, (0.5, 0.5))
        return Workload("C0", 2, v, f, (16, 16, 1), 3, 32, 9)
    if name == "C1":
        v, f = icosphere(5, 0.2)
        return Workload("C1", 3, v, f, (16, 16, 16), 3, 64, 19)
    if name == "C2":
        v, f = star(7, SEED_STAR)
        return Workload("C2", 3, v, f, (32, 32, 32), 4, 128, 27)
    if name == "C3":
        u, f = icosphere_unit(5)
        v64 = np.array([0.5, 0.5, 0.5]) + 0.2 * u
        v = jitter_fp64(v64, 1e-3, SEED_JITTER).astype(np.float32)
        return Workload("C3", 3, v, f, (16, 16, 16), 3, 64, 19,
                        extra={"weights_seed": SEED_WEIGHTS})
    if name == "P0":
        # the paper's 2D study shape: a 12,800-segment circle, 256^2 cells, d = 0.1, two passes
        v, f = circle(12800, 0.25, (0.5, 0.5))
        return Workload("P0", 2, v, f, (64, 64, 1), 2, 8, 9, extra={"d_const": 0.1})
    if name == "P1":
        # the paper's 3D study at the size of its body: a star on an 81,920-face icosphere, 64^3 cells,
        # d = 0.05, two passes
        v, f = star(6, SEED_STAR)
        return Workload("P1", 3, v, f, (16, 16, 16), 2, 8, 19, extra={"d_const": 0.05})
    raise KeyError(name)


def batch_draws(n_bodies: int = 64, seed: int = SEED_BATCH) -> List[dict]:
    """Per-body (subdivision, coefficient seed, roots, passes) for the batched workload.

    Subdivision s ~ U{3..7}; roots 16^3 with 3 passes for s <= 5, 32^3 with 4 passes
    for s >= 6; body b uses star seed 0 + b."""
    rng = np.random.default_rng(seed)
    subs = rng.integers(3, 8, size=n_bodies)
    out = []
    for b, s in enumerate(subs):
        s = int(s)
        R, L = (16, 3) if s <= 5 else (32, 4)
        out.append({"body": b, "s": s, "seed": SEED_STAR + b, "roots": R, "levels": L,
                    "faces": _face_count(s)})
    return out


def batch_body(draw: dict) -> Workload:
    v, f = star(draw["s"], draw["seed"])
    R = draw["roots"]
    return Workload(f"C4.{draw['body']}", 3, v, f, (R, R, R), draw["levels"], 0, 27)


# --------------------------------------------------------------------------
# Tiny shapes for pins
# --------------------------------------------------------------------------
def box_mesh(lo=(0.3, 0.3, 0.3), hi=(0.7, 0.7, 0.7)) -> Tuple[np.ndarray, np.ndarray]:
    """Axis-aligned box surface, 12 outward triangles."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], dtype=np.float64)
    f = np.array([[0, 2, 1], [0, 3, 2], [4, 5, 6], [4, 6, 7],
                  [0, 1, 5], [0, 5, 4], [2, 3, 7], [2, 7, 6],
                  [1, 2, 6], [1, 6, 5], [0, 4, 7], [0, 7, 3]], dtype=np.int64)
    f = _orient_outward(v - v.mean(axis=0), f)
    return v.astype(np.float32), f.astype(np.int32)


def square_loop(lo=(0.3, 0.3), hi=(0.7, 0.7)) -> Tuple[np.ndarray, np.ndarray]:
    """Axis-aligned square as 4 counter-clockwise segments."""
    v = np.array([[lo[0], lo[1]], [hi[0], lo[1]], [hi[0], hi[1]], [lo[0], hi[1]]], dtype=np.float32)
    f = np.array([[0, 1], [1, 2], [2, 3], [3, 0]], dtype=np.int32)
    return v, f


def random_triangles(n: int, seed: int, lo=0.2, hi=0.8, size=0.05) -> Tuple[np.ndarray, np.ndarray]:
    """``n`` independent small triangles (unshared vertices) inside [lo, hi]^3."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(lo, hi, size=(n, 1, 3))
    d = rng.uniform(-size, size, size=(n, 3, 3))
    v = (c + d).reshape(-1, 3)
    f = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    return v.astype(np.float32), f


def random_segments(n: int, seed: int, lo=0.2, hi=0.8, size=0.05) -> Tuple[np.ndarray, np.ndarray]:
    rng = np.random.default_rng(seed)
    c = rng.uniform(lo, hi, size=(n, 1, 2))
    d = rng.uniform(-size, size, size=(n, 2, 2))
    v = (c + d).reshape(-1, 2)
    f = np.arange(2 * n, dtype=np.int32).reshape(n, 2)
    return v.astype(np.float32), f
