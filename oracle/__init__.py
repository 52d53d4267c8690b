"""ctypes wrapper around the plain serial CPU oracle (``agal_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product library.  It shares
no code with the HIP path.

Precision: bins, cell centres and the separating-axis flags are FP32 (the
paper's build is single precision, Results section); link fractions, the
adjoint and finite differences are FP64 on the FP32 inputs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "agal_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# Mutation tests point this at a deliberately broken copy of the oracle.
_OVERRIDE = os.environ.get("AGAL_ORACLE_LIB")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if _OVERRIDE:
        return _OVERRIDE
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build(force=False)
        L = C.CDLL(path)
        P = C.c_void_p
        fp, dp, i32p, i64p, u8p = (C.POINTER(C.c_float), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int64), C.POINTER(C.c_uint8))
        sig = {
            "orc_lattice": (C.c_int, [C.c_int, i32p]),
            "orc_gather": (None, [C.c_int, fp, i32p, C.c_int64, fp]),
            "orc_bin_faces": (P, [C.c_int, fp, C.c_int64, fp, fp, C.c_int]),
            "orc_bin_faces_discrete": (P, [C.c_int, fp, C.c_int64, fp, fp, C.c_int, C.c_float]),
            "orc_bins_free": (None, [P]),
            "orc_bins_nb": (C.c_int64, [P]),
            "orc_bins_P": (C.c_int64, [P]),
            "orc_bins_count": (C.POINTER(C.c_uint32), [P]),
            "orc_bins_off": (C.POINTER(C.c_uint32), [P]),
            "orc_bins_ids": (i32p, [P]),
            "orc_sat": (C.c_int, [C.c_int, fp, fp, C.c_float]),
            "orc_near_face_l2": (C.c_int, [C.c_int, dp, dp, C.c_double]),
            "orc_face_dist2": (C.c_double, [C.c_int, dp, dp]),
            "orc_near_l2_f32": (C.c_int, [C.c_int, fp, fp, C.c_float]),
            "orc_refine": (P, [C.c_int, fp, C.c_int64, P, i32p, C.c_int, fp, fp, fp]),
            "orc_refine_own_bin": (P, [C.c_int, fp, C.c_int64, P, i32p, C.c_int, fp, fp, fp, C.c_int]),
            "orc_forest_free": (None, [P]),
            "orc_forest_n": (C.c_int64, [P, C.c_int]),
            "orc_forest_keys": (C.POINTER(C.c_uint32), [P, C.c_int]),
            "orc_forest_leaf": (u8p, [P, C.c_int]),
            "orc_forest_mark": (u8p, [P, C.c_int]),
            "orc_forest_cell_flag": (u8p, [P, C.c_int]),
            "orc_forest_tests": (C.c_int64, [P, C.c_int]),
            "orc_link_fractions": (P, [C.c_int, fp, C.c_int64, P, P, C.c_int, i64p, C.c_int64]),
            "orc_links_free": (None, [P]),
            "orc_links_n": (C.c_int64, [P]),
            "orc_links_key": (C.POINTER(C.c_uint64), [P]),
            "orc_links_q": (dp, [P]),
            "orc_links_face": (i32p, [P]),
            "orc_links_tests": (C.c_int64, [P]),
            "orc_link_grad": (None, [P, P, fp, i32p, dp, dp]),
            "orc_classify_nodes": (None, [C.c_int, C.c_int, C.c_int64, i32p, fp, u8p]),
            "orc_forest_diff": (None, [C.POINTER(C.c_uint32), u8p, C.c_int64, C.POINTER(C.c_uint32), u8p,
                                       C.c_int64, i32p, u8p, u8p]),
            "orc_link_stable": (None, [P, P, fp, C.c_int64, P, C.c_double, C.c_double, C.c_double,
                                       C.c_double, C.c_double, u8p]),
            "orc_link_t": (C.c_int, [P, C.c_uint64, C.c_int, C.c_int, fp, C.c_int32, dp]),
            "orc_fd_grad": (None, [P, P, fp, C.c_int64, i32p, C.c_int64, P, dp, C.c_double, i64p,
                                   C.c_int64, dp, i64p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _copy(ptr, n, dtype) -> np.ndarray:
    if n == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


# ---------------------------------------------------------------------------
def lattice(Q: int) -> np.ndarray:
    c = np.zeros((27, 3), dtype=np.int32)
    d = lib().orc_lattice(Q, _ptr(c, C.c_int32))
    if d < 0:
        raise ValueError(f"unknown lattice Q={Q}")
    return c[:Q].copy()


def gather(dim: int, verts: np.ndarray, faces: np.ndarray) -> np.ndarray:
    """Index lists -> coordinate list [F, dim(vertex), dim(axis)] (FP32)."""
    verts = np.ascontiguousarray(verts, dtype=np.float32)
    faces = np.ascontiguousarray(faces, dtype=np.int32)
    F = faces.shape[0]
    out = np.zeros((F, dim, dim), dtype=np.float32)
    lib().orc_gather(dim, _ptr(verts, C.c_float), _ptr(faces, C.c_int32), F, _ptr(out, C.c_float))
    return out


def _vec3(x, fill) -> np.ndarray:
    a = np.full(3, fill, dtype=np.float32)
    x = np.asarray(x, dtype=np.float32).ravel()
    a[: len(x)] = x
    return a


class Bins:
    """Bins of the faces: by bounding box (spacing None), or by the paper's sampled points at `spacing`."""

    def __init__(self, dim: int, coords: np.ndarray, lo, hi, B: int, spacing: Optional[float] = None):
        self._coords = np.ascontiguousarray(coords, dtype=np.float32)
        self.dim, self.B = dim, B
        self.lo, self.hi = _vec3(lo, 0.0), _vec3(hi, 1.0)
        F = self._coords.shape[0]
        if spacing is None:
            self.h = lib().orc_bin_faces(dim, _ptr(self._coords, C.c_float), F, _ptr(self.lo, C.c_float),
                                         _ptr(self.hi, C.c_float), B)
        else:
            self.h = lib().orc_bin_faces_discrete(dim, _ptr(self._coords, C.c_float), F, _ptr(self.lo, C.c_float),
                                                  _ptr(self.hi, C.c_float), B, C.c_float(spacing))
        if not self.h:
            raise ValueError(f"bins per axis must be at least 1 (got {B}), dim 2 or 3, spacing positive")
        nb = lib().orc_bins_nb(self.h)
        P = lib().orc_bins_P(self.h)
        self.nb, self.P = nb, P
        self.count = _copy(lib().orc_bins_count(self.h), nb, np.uint32)
        self.offsets = _copy(lib().orc_bins_off(self.h), nb + 1, np.uint32)
        self.ids = _copy(lib().orc_bins_ids(self.h), P, np.int32)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_bins_free(self.h)
            self.h = None


def bin_faces(dim, coords, lo, hi, B) -> Bins:
    return Bins(dim, coords, lo, hi, B)


def bin_faces_discrete(dim, coords, lo, hi, B, spacing) -> Bins:
    """The paper's binning: each face in every bin holding one of its sampled points."""
    return Bins(dim, coords, lo, hi, B, spacing)


def sat(dim: int, face: np.ndarray, m: Sequence[float], h: float) -> bool:
    face = np.ascontiguousarray(face, dtype=np.float32).ravel()
    mm = _vec3(m, 0.0)
    return bool(lib().orc_sat(dim, _ptr(face, C.c_float), _ptr(mm, C.c_float), C.c_float(h)))


def near_face_l2(dim: int, face: np.ndarray, p: Sequence[float], R: float) -> bool:
    """FP64: is p within Euclidean distance R of the closed face?"""
    face = np.ascontiguousarray(face, dtype=np.float64).ravel()
    pp = np.zeros(3, dtype=np.float64)
    pp[:dim] = np.asarray(p, dtype=np.float64)[:dim]
    return bool(lib().orc_near_face_l2(dim, _ptr(face, C.c_double), _ptr(pp, C.c_double), R))


def face_dist2(dim: int, face: np.ndarray, p: Sequence[float]) -> float:
    """FP64 squared Euclidean distance from p to the closed face."""
    face = np.ascontiguousarray(face, dtype=np.float64).ravel()
    pp = np.zeros(3, dtype=np.float64)
    pp[:dim] = np.asarray(p, dtype=np.float64)[:dim]
    return float(lib().orc_face_dist2(dim, _ptr(face, C.c_double), _ptr(pp, C.c_double)))


def near_l2_f32(dim: int, face: np.ndarray, p: Sequence[float], R: float) -> bool:
    """The FP32 decision of the own-bin flag step (fixed rounded sequence)."""
    face = np.ascontiguousarray(face, dtype=np.float32).ravel()
    pp = _vec3(p, 0.0)
    return bool(lib().orc_near_l2_f32(dim, _ptr(face, C.c_float), _ptr(pp, C.c_float), C.c_float(R)))


class Forest:
    """Near-wall refinement.  own_bin=False: separating-axis flags over every bin
    under the query box.  own_bin=True: the paper's own-bin Euclidean flags
    with mark propagation (n_prop < 0: the paper's step count)."""

    def __init__(self, dim, coords, bins: Optional[Bins], roots, L, d_spec, lo, hi, own_bin=False, n_prop=-1):
        self._coords = np.ascontiguousarray(coords, dtype=np.float32)
        self._bins = bins
        self.dim, self.L = dim, L
        r = np.ones(3, dtype=np.int32)
        r[:dim] = np.asarray(roots, dtype=np.int32)[:dim]
        self.roots = r
        d = np.ascontiguousarray(np.asarray(d_spec, dtype=np.float32).reshape(-1))
        if L > 0 and len(d) < L:
            raise ValueError("d_spec needs one entry per pass")
        if len(d) == 0:
            d = np.zeros(1, dtype=np.float32)
        self.lo, self.hi = _vec3(lo, 0.0), _vec3(hi, 1.0)
        if own_bin:
            if bins is None:
                raise ValueError("the own-bin mode needs bins")
            self.h = lib().orc_refine_own_bin(dim, _ptr(self._coords, C.c_float), self._coords.shape[0], bins.h,
                                              _ptr(r, C.c_int32), L, _ptr(d, C.c_float), _ptr(self.lo, C.c_float),
                                              _ptr(self.hi, C.c_float), int(n_prop))
        else:
            self.h = lib().orc_refine(dim, _ptr(self._coords, C.c_float), self._coords.shape[0],
                                      bins.h if bins is not None else None, _ptr(r, C.c_int32), L,
                                      _ptr(d, C.c_float), _ptr(self.lo, C.c_float), _ptr(self.hi, C.c_float))
        if not self.h:
            raise ValueError("oracle refine rejected its arguments")
        cells = 64 if dim == 3 else 16
        self.levels = []
        for l in range(L + 1):
            n = lib().orc_forest_n(self.h, l)
            self.levels.append({
                "keys": _copy(lib().orc_forest_keys(self.h, l), n, np.uint32),
                "leaf": _copy(lib().orc_forest_leaf(self.h, l), n, np.uint8),
                "mark": _copy(lib().orc_forest_mark(self.h, l), n, np.uint8),
                "cell_flag": _copy(lib().orc_forest_cell_flag(self.h, l), n * cells, np.uint8).reshape(n, cells),
            })
        self.tests = [lib().orc_forest_tests(self.h, l) for l in range(L + 1)]

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_forest_free(self.h)
            self.h = None


def refine(dim, coords, bins, roots, L, d_spec, lo, hi, own_bin=False, n_prop=-1) -> Forest:
    return Forest(dim, coords, bins, roots, L, d_spec, lo, hi, own_bin, n_prop)


class Links:
    def __init__(self, dim, coords, bins: Optional[Bins], forest: Forest, Q: int, subset=None):
        self._coords = np.ascontiguousarray(coords, dtype=np.float32)
        self._bins, self._forest = bins, forest
        self.dim, self.Q = dim, Q
        sub = None
        nsub = 0
        if subset is not None:
            sub = np.ascontiguousarray(np.asarray(subset, dtype=np.int64))
            nsub = len(sub)
        self.h = lib().orc_link_fractions(dim, _ptr(self._coords, C.c_float), self._coords.shape[0],
                                          bins.h if bins is not None else None, forest.h, Q,
                                          _ptr(sub, C.c_int64) if sub is not None else None, nsub)
        if not self.h:
            raise ValueError("lattice does not match the dimension")
        n = lib().orc_links_n(self.h)
        self.n = n
        self.key = _copy(lib().orc_links_key(self.h), n, np.uint64)
        self.q = _copy(lib().orc_links_q(self.h), n * Q, np.float64).reshape(n, Q)
        self.face = _copy(lib().orc_links_face(self.h), n * Q, np.int32).reshape(n, Q)
        self.tests = lib().orc_links_tests(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_links_free(self.h)
            self.h = None


def link_fractions(dim, coords, bins, forest, Q, subset=None) -> Links:
    return Links(dim, coords, bins, forest, Q, subset)


def link_grad(forest: Forest, links: Links, coords, fidx, w, n_vertices) -> np.ndarray:
    coords = np.ascontiguousarray(coords, dtype=np.float32)
    fidx = np.ascontiguousarray(fidx, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    if w.size != links.n * links.Q:
        raise ValueError("weights must hold n_nodes * Q entries")
    g = np.zeros((n_vertices, links.dim), dtype=np.float64)
    lib().orc_link_grad(forest.h, links.h, _ptr(coords, C.c_float), _ptr(fidx, C.c_int32),
                        _ptr(w, C.c_double), _ptr(g, C.c_double))
    return g


def classify_nodes(dim: int, Q: int, face: np.ndarray, coords) -> np.ndarray:
    """Per node 1 (fluid), 2 (solid) or 3 (its links disagree), from the orientation of each link's face."""
    face = np.ascontiguousarray(face, dtype=np.int32).reshape(-1, Q)
    coords = np.ascontiguousarray(coords, dtype=np.float32)
    out = np.zeros(face.shape[0], dtype=np.uint8)
    lib().orc_classify_nodes(dim, Q, face.shape[0], _ptr(face, C.c_int32), _ptr(coords, C.c_float),
                             _ptr(out, C.c_uint8))
    return out


def forest_diff(old_levels, new_levels):
    """Per level of two forests over the same root grid: (old_index, state, removed) of orc_forest_diff.
    Levels are dicts with "keys" (sorted uint32) and "leaf" (uint8), as Forest.levels holds them."""
    out = []
    for lo_, ln_ in zip(old_levels, new_levels):
        ok = np.ascontiguousarray(lo_["keys"], dtype=np.uint32)
        ol = np.ascontiguousarray(lo_["leaf"], dtype=np.uint8)
        nk = np.ascontiguousarray(ln_["keys"], dtype=np.uint32)
        nl = np.ascontiguousarray(ln_["leaf"], dtype=np.uint8)
        idx = np.zeros(len(nk), dtype=np.int32)
        st = np.zeros(len(nk), dtype=np.uint8)
        rm = np.zeros(len(ok), dtype=np.uint8)
        lib().orc_forest_diff(_ptr(ok, C.c_uint32), _ptr(ol, C.c_uint8), len(ok), _ptr(nk, C.c_uint32),
                              _ptr(nl, C.c_uint8), len(nk), _ptr(idx, C.c_int32), _ptr(st, C.c_uint8),
                              _ptr(rm, C.c_uint8))
        out.append((idx, st, rm))
    return out


def link_stable(forest, links, coords, bins, h=1e-4, eta_max=0.025, bary_min=0.1, t_lo=0.1, gap=0.1):
    coords = np.ascontiguousarray(coords, dtype=np.float32)
    out = np.zeros((links.n, links.Q), dtype=np.uint8)
    lib().orc_link_stable(forest.h, links.h, _ptr(coords, C.c_float), coords.shape[0],
                          bins.h if bins is not None else None, h, eta_max, bary_min, t_lo, gap,
                          _ptr(out, C.c_uint8))
    return out.astype(bool)


def link_t(forest: Forest, node_key: int, Q: int, i: int, coords, face: int):
    """FP64 fraction at which link (node, direction i) meets `face`, or None."""
    coords = np.ascontiguousarray(coords, dtype=np.float32)
    t = C.c_double()
    hit = lib().orc_link_t(forest.h, int(node_key), Q, i, _ptr(coords, C.c_float), int(face), C.byref(t))
    return t.value if hit else None


def fd_grad(forest, links, verts, fidx, bins, w, h=1e-4, vertex_subset=None):
    verts = np.ascontiguousarray(verts, dtype=np.float32)
    fidx = np.ascontiguousarray(fidx, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    Nv = verts.shape[0]
    if vertex_subset is None:
        vertex_subset = np.arange(Nv)
    vs = np.ascontiguousarray(np.asarray(vertex_subset, dtype=np.int64))
    g = np.zeros((Nv, links.dim), dtype=np.float64)
    nch = np.zeros(1, dtype=np.int64)
    lib().orc_fd_grad(forest.h, links.h, _ptr(verts, C.c_float), Nv, _ptr(fidx, C.c_int32), fidx.shape[0],
                      bins.h if bins is not None else None, _ptr(w, C.c_double), h, _ptr(vs, C.c_int64),
                      len(vs), _ptr(g, C.c_double), _ptr(nch, C.c_int64))
    return g, int(nch[0])


# ---------------------------------------------------------------------------
def run_plain(wl, with_links: bool = True, link_subset=None, brute: bool = False):
    """Bins -> refinement -> link fractions for one workload (see ``geomgen``)."""
    coords = gather(wl.dim, wl.vertices, wl.faces)
    bins = bin_faces(wl.dim, coords, wl.lo[: wl.dim], wl.hi[: wl.dim], wl.bins)
    forest = refine(wl.dim, coords, None if brute else bins, wl.roots[: wl.dim], wl.levels, wl.d_spec(),
                    wl.lo[: wl.dim], wl.hi[: wl.dim])
    out = {"coords": coords, "bins": bins, "forest": forest}
    if with_links:
        out["links"] = link_fractions(wl.dim, coords, None if brute else bins, forest, wl.lattice, link_subset)
    return out
