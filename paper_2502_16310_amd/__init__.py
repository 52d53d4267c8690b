"""Python binding of ``libagal.so`` -- the MI355X near-wall mesh-adaptation path
(bin faces -> refine near the wall -> link fractions -> adjoint).

The module-level ``agal_*`` functions have the names and arguments of the C
ABI in ``include/agal.h`` and only marshal arguments (device pointers are
plain integers, handles are opaque ``ctypes.c_void_p``).  ``Context``,
``Geometry`` ... wrap them for torch tensors, and ``LinkFractions`` is the
``torch.autograd.Function`` around the forward and adjoint.  Every step of
the path runs in the HIP library; there is no fallback: importing this
package without a built library raises ``ImportError``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libagal.so")

AGAL_OK, AGAL_EINVAL, AGAL_ENOMEM, AGAL_EHIP, AGAL_ECAPACITY, AGAL_ESTATE = range(6)
AGAL_D2Q9, AGAL_D3Q19, AGAL_D3Q27 = 9, 19, 27
AGAL_MAX_LEVELS = 8


class AgalError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


class _ForestDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("roots", C.c_int * 3), ("n_levels", C.c_int),
                ("d_spec", C.POINTER(C.c_float)), ("lo", C.c_float * 3), ("hi", C.c_float * 3)]


class _Allocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p),
                ("alloc", C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p))]


class _BodyDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("d_vertices", C.c_void_p), ("n_vertices", C.c_int64), ("d_faces", C.c_void_p),
                ("n_faces", C.c_int64), ("forest", _ForestDesc), ("lattice", C.c_int), ("bins", C.c_int32)]


class _TuneOpts(C.Structure):
    _fields_ = [("tune_bins", C.c_int), ("tune_grid", C.c_int), ("with_adjoint", C.c_int),
                ("capacity_margin", C.c_float), ("cache_path", C.c_char_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                          "or `python paper_2502_16310_amd/build.py`")
    # torch ships its own HIP runtime under the same soname; loading torch first
    # makes this library bind to that copy instead of starting a second runtime
    # in the process (which then finds no device)
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, vp = C.c_void_p, C.c_void_p
    i64, i32 = C.c_int64, C.c_int32
    PP = C.POINTER(C.c_void_p)
    sig = {
        "agal_context_create": [C.POINTER(_Allocator), PP],
        "agal_context_destroy": [P],
        "agal_import_faces": [P, C.c_int, vp, i64, vp, i64, vp, PP],
        "agal_geom_view": [P, C.POINTER(C.c_int), C.POINTER(i64), C.POINTER(i64), PP, PP],
        "agal_bin_faces": [P, C.POINTER(C.c_float), C.POINTER(C.c_float), i32, vp, PP],
        "agal_bins_view": [P, PP, PP, C.POINTER(i64), C.POINTER(i64)],
        "agal_bin_faces_discrete": [P, C.POINTER(C.c_float), C.POINTER(C.c_float), i32, C.c_float, i32, vp, PP],
        "agal_bin_faces_noalloc": [P, C.POINTER(C.c_float), C.POINTER(C.c_float), i32, vp, vp, i64, vp,
                                   C.POINTER(i64)],
        "agal_near_wall_refine": [P, P, C.POINTER(_ForestDesc), vp, PP],
        "agal_near_wall_refine_own_bin": [P, P, C.POINTER(_ForestDesc), C.c_int, vp, PP],
        "agal_forest_level_view": [P, C.c_int, PP, PP, PP, PP, C.POINTER(i64)],
        "agal_forest_info": [P, C.POINTER(C.c_int), C.POINTER(C.c_int)],
        "agal_link_fractions": [P, P, P, C.c_int, vp, PP],
        "agal_links_view": [P, PP, PP, PP, C.POINTER(i64), C.POINTER(C.c_int)],
        "agal_link_fractions_backward": [P, P, vp, vp, vp],
        "agal_classify_nodes": [P, P, vp, vp],
        "agal_forest_diff_create": [P, P, vp, PP],
        "agal_forest_diff_view": [P, C.c_int, PP, PP, PP, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)],
        "agal_destroy_forest_diff": [P],
        "agal_lattice_vectors": [C.c_int, C.POINTER(i32)],
        "agal_profile_enable": [P, C.c_int],
        "agal_context_set_flag_table_limit": [P, C.c_int64],
        "agal_context_set_link_list_limit": [P, C.c_int64],
        "agal_profile_read": [P, C.c_int, C.POINTER(C.c_char_p), C.POINTER(i64), C.POINTER(C.c_double),
                              C.POINTER(C.c_int)],
        "agal_batch_plan_create": [P, C.c_int, C.POINTER(_BodyDesc), C.POINTER(_TuneOpts), vp, PP],
        "agal_batch_run": [P, vp],
        "agal_batch_status": [P, vp],
        "agal_batch_body_view": [P, C.c_int, PP, PP, PP, C.POINTER(i64), C.POINTER(C.c_int), PP, PP,
                                 C.POINTER(i64), C.POINTER(i32)],
        "agal_batch_level_view": [P, C.c_int, C.c_int, PP, PP, PP, PP, C.POINTER(i64)],
        "agal_batch_info": [P, C.POINTER(C.c_int), C.POINTER(C.c_int)],
        "agal_destroy_batch": [P],
        "agal_destroy_geom": [P],
        "agal_destroy_bins": [P],
        "agal_destroy_forest": [P],
        "agal_destroy_links": [P],
        "agal_status_string": [C.c_int],
        "agal_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    for name in ("agal_context_destroy", "agal_destroy_geom", "agal_destroy_bins", "agal_destroy_forest",
                 "agal_destroy_links", "agal_destroy_batch", "agal_destroy_forest_diff"):
        getattr(lib, name).restype = None
    lib.agal_status_string.restype = C.c_char_p
    lib.agal_last_error.restype = C.c_char_p
    return lib


_lib = _load()


def _check(status: int, what: str):
    if status != AGAL_OK:
        msg = _lib.agal_last_error().decode(errors="replace")
        raise AgalError(status, f"{what}: {_lib.agal_status_string(status).decode()}: {msg}")


def _h(x):
    return x.value if isinstance(x, C.c_void_p) else x


# ---------------------------------------------------------------------------
# C ABI, same names (raw device pointers as ints, handles as c_void_p)
# ---------------------------------------------------------------------------
def agal_context_create(allocator: Optional[_Allocator] = None) -> C.c_void_p:
    out = C.c_void_p()
    _check(_lib.agal_context_create(C.byref(allocator) if allocator is not None else None, C.byref(out)),
           "agal_context_create")
    return out


def agal_context_destroy(ctx):
    _lib.agal_context_destroy(_h(ctx))


def agal_import_faces(ctx, dim: int, d_vertices: int, n_vertices: int, d_faces: Optional[int], n_faces: int,
                      stream: int = 0) -> C.c_void_p:
    out = C.c_void_p()
    _check(_lib.agal_import_faces(_h(ctx), dim, d_vertices, n_vertices, d_faces or None, n_faces, stream or None,
                                  C.byref(out)), "agal_import_faces")
    return out


def agal_geom_view(geom):
    dim, F, Nv = C.c_int(), C.c_int64(), C.c_int64()
    co, bb = C.c_void_p(), C.c_void_p()
    _check(_lib.agal_geom_view(_h(geom), C.byref(dim), C.byref(F), C.byref(Nv), C.byref(co), C.byref(bb)),
           "agal_geom_view")
    return dim.value, F.value, Nv.value, co.value, bb.value


def _f3(v, fill):
    a = (C.c_float * 3)(fill, fill, fill)
    for i, x in enumerate(list(v)[:3]):
        a[i] = float(x)
    return a


def agal_bin_faces(geom, lo: Sequence[float], hi: Sequence[float], B: int, stream: int = 0) -> C.c_void_p:
    out = C.c_void_p()
    _check(_lib.agal_bin_faces(_h(geom), _f3(lo, 0.0), _f3(hi, 1.0), int(B), stream or None, C.byref(out)),
           "agal_bin_faces")
    return out


def agal_bin_faces_discrete(geom, lo: Sequence[float], hi: Sequence[float], B: int, spacing: float = 0.0,
                            bin_fraction: int = 0, stream: int = 0) -> C.c_void_p:
    out = C.c_void_p()
    _check(_lib.agal_bin_faces_discrete(_h(geom), _f3(lo, 0.0), _f3(hi, 1.0), int(B), C.c_float(spacing),
                                        int(bin_fraction), stream or None, C.byref(out)), "agal_bin_faces_discrete")
    return out


def agal_bin_faces_noalloc(geom, lo: Sequence[float], hi: Sequence[float], B: int, d_offsets: int,
                           d_face_ids: Optional[int], ids_capacity: int, stream: int = 0) -> int:
    """Bins into caller buffers without device allocation; returns the entry count P."""
    n = C.c_int64()
    _check(_lib.agal_bin_faces_noalloc(_h(geom), _f3(lo, 0.0), _f3(hi, 1.0), int(B), d_offsets, d_face_ids or None,
                                       int(ids_capacity), stream or None, C.byref(n)), "agal_bin_faces_noalloc")
    return n.value


def agal_bins_view(bins):
    off, ids = C.c_void_p(), C.c_void_p()
    nb, P = C.c_int64(), C.c_int64()
    _check(_lib.agal_bins_view(_h(bins), C.byref(off), C.byref(ids), C.byref(nb), C.byref(P)), "agal_bins_view")
    return off.value, ids.value, nb.value, P.value


def forest_desc(dim: int, roots: Sequence[int], n_levels: int, d_spec: Sequence[float], lo: Sequence[float],
                hi: Sequence[float]):
    d = (C.c_float * max(1, n_levels))(*[float(x) for x in list(d_spec)[:n_levels]])
    desc = _ForestDesc()
    desc.dim = dim
    r = list(roots) + [1] * (3 - len(roots))
    desc.roots = (C.c_int * 3)(*[int(x) for x in r[:3]])
    desc.n_levels = n_levels
    desc.d_spec = C.cast(d, C.POINTER(C.c_float))
    desc.lo = _f3(lo, 0.0)
    desc.hi = _f3(hi, 1.0)
    desc._keep = d
    return desc


def agal_near_wall_refine(geom, bins, desc: _ForestDesc, stream: int = 0) -> C.c_void_p:
    out = C.c_void_p()
    _check(_lib.agal_near_wall_refine(_h(geom), _h(bins), C.byref(desc), stream or None, C.byref(out)),
           "agal_near_wall_refine")
    return out


def agal_near_wall_refine_own_bin(geom, bins, desc: _ForestDesc, n_prop: int = -1, stream: int = 0) -> C.c_void_p:
    out = C.c_void_p()
    _check(_lib.agal_near_wall_refine_own_bin(_h(geom), _h(bins), C.byref(desc), int(n_prop), stream or None,
                                              C.byref(out)), "agal_near_wall_refine_own_bin")
    return out


def agal_forest_level_view(forest, level: int):
    k, lf, mk, cf = C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_void_p()
    n = C.c_int64()
    _check(_lib.agal_forest_level_view(_h(forest), level, C.byref(k), C.byref(lf), C.byref(mk), C.byref(cf),
                                       C.byref(n)), "agal_forest_level_view")
    return k.value, lf.value, mk.value, cf.value, n.value


def agal_forest_diff_create(old_forest, new_forest, stream: int = 0):
    out = C.c_void_p()
    _check(_lib.agal_forest_diff_create(_h(old_forest), _h(new_forest), stream or None, C.byref(out)),
           "agal_forest_diff_create")
    return out.value


def agal_forest_diff_view(diff, level: int):
    """(old_index ptr, state ptr, removed ptr, n_new, n_old, [created, refined, coarsened, removed])."""
    oi, st, rm = C.c_void_p(), C.c_void_p(), C.c_void_p()
    nn, no = C.c_int64(), C.c_int64()
    cnt = (C.c_int64 * 4)()
    _check(_lib.agal_forest_diff_view(_h(diff), level, C.byref(oi), C.byref(st), C.byref(rm), C.byref(nn),
                                      C.byref(no), cnt), "agal_forest_diff_view")
    return oi.value, st.value, rm.value, nn.value, no.value, list(cnt)


def agal_destroy_forest_diff(h):
    _lib.agal_destroy_forest_diff(_h(h))


def agal_forest_info(forest):
    dim, L = C.c_int(), C.c_int()
    _check(_lib.agal_forest_info(_h(forest), C.byref(dim), C.byref(L)), "agal_forest_info")
    return dim.value, L.value


def agal_link_fractions(geom, bins, forest, lattice: int, stream: int = 0) -> C.c_void_p:
    out = C.c_void_p()
    _check(_lib.agal_link_fractions(_h(geom), _h(bins), _h(forest), int(lattice), stream or None, C.byref(out)),
           "agal_link_fractions")
    return out


def agal_links_view(links):
    k, q, f = C.c_void_p(), C.c_void_p(), C.c_void_p()
    n, Q = C.c_int64(), C.c_int()
    _check(_lib.agal_links_view(_h(links), C.byref(k), C.byref(q), C.byref(f), C.byref(n), C.byref(Q)),
           "agal_links_view")
    return k.value, q.value, f.value, n.value, Q.value


def agal_link_fractions_backward(geom, links, d_grad_q: int, d_grad_vertices: int, stream: int = 0):
    _check(_lib.agal_link_fractions_backward(_h(geom), _h(links), d_grad_q, d_grad_vertices, stream or None),
           "agal_link_fractions_backward")


def agal_classify_nodes(geom, links, d_class: int, stream: int = 0):
    _check(_lib.agal_classify_nodes(_h(geom), _h(links), d_class, stream or None), "agal_classify_nodes")


def agal_lattice_vectors(lattice: int):
    buf = (C.c_int32 * (3 * lattice))()
    _check(_lib.agal_lattice_vectors(int(lattice), buf), "agal_lattice_vectors")
    return [tuple(buf[3 * i:3 * i + 3]) for i in range(lattice)]


def agal_context_set_flag_table_limit(ctx, max_entries: int):
    _check(_lib.agal_context_set_flag_table_limit(_h(ctx), int(max_entries)), "agal_context_set_flag_table_limit")


def agal_context_set_link_list_limit(ctx, max_blocks_per_face: int):
    _check(_lib.agal_context_set_link_list_limit(_h(ctx), int(max_blocks_per_face)),
           "agal_context_set_link_list_limit")


def agal_profile_enable(ctx, enable: bool = True):
    _check(_lib.agal_profile_enable(_h(ctx), 1 if enable else 0), "agal_profile_enable")


def agal_profile_read(ctx, max_entries: int = 64):
    """{kernel name: (launches, total ms)} recorded since the last read."""
    names = (C.c_char_p * max_entries)()
    launches = (C.c_int64 * max_entries)()
    ms = (C.c_double * max_entries)()
    n = C.c_int()
    _check(_lib.agal_profile_read(_h(ctx), max_entries, names, launches, ms, C.byref(n)), "agal_profile_read")
    return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(n.value)}


def body_desc(dim: int, d_vertices: int, n_vertices: int, d_faces: Optional[int], n_faces: int,
              forest: _ForestDesc, lattice: int, bins: int = 0) -> _BodyDesc:
    b = _BodyDesc()
    b.dim, b.d_vertices, b.n_vertices = dim, d_vertices, n_vertices
    b.d_faces, b.n_faces = d_faces or None, n_faces
    b.forest, b.lattice, b.bins = forest, int(lattice), int(bins)
    b._keep = forest._keep
    return b


def tune_opts(tune_bins: bool = True, tune_grid: bool = True, with_adjoint: bool = False,
              capacity_margin: float = 0.0, cache_path: Optional[str] = None) -> _TuneOpts:
    o = _TuneOpts()
    o.tune_bins, o.tune_grid, o.with_adjoint = int(tune_bins), int(tune_grid), int(with_adjoint)
    o.capacity_margin = float(capacity_margin)
    o.cache_path = cache_path.encode() if cache_path else None
    return o


def agal_batch_plan_create(ctx, bodies: Sequence[_BodyDesc], opts: Optional[_TuneOpts] = None,
                           stream: int = 0) -> C.c_void_p:
    arr = (_BodyDesc * len(bodies))(*bodies)
    out = C.c_void_p()
    _check(_lib.agal_batch_plan_create(_h(ctx), len(bodies), arr, C.byref(opts) if opts is not None else None,
                                       stream or None, C.byref(out)), "agal_batch_plan_create")
    return out


def agal_batch_run(batch, stream: int = 0):
    _check(_lib.agal_batch_run(_h(batch), stream or None), "agal_batch_run")


def agal_batch_status(batch, stream: int = 0):
    _check(_lib.agal_batch_status(_h(batch), stream or None), "agal_batch_status")


def agal_batch_body_view(batch, body: int):
    """(node_key, q, face, n_nodes, Q, grad_q, grad_vertices, node_capacity, bins)"""
    k, q, f, gq, gv = (C.c_void_p() for _ in range(5))
    n, cap = C.c_int64(), C.c_int64()
    Q, B = C.c_int(), C.c_int32()
    _check(_lib.agal_batch_body_view(_h(batch), int(body), C.byref(k), C.byref(q), C.byref(f), C.byref(n),
                                     C.byref(Q), C.byref(gq), C.byref(gv), C.byref(cap), C.byref(B)),
           "agal_batch_body_view")
    return k.value, q.value, f.value, n.value, Q.value, gq.value, gv.value, cap.value, B.value


def agal_batch_level_view(batch, body: int, level: int):
    k, lf, mk, cf = C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_void_p()
    n = C.c_int64()
    _check(_lib.agal_batch_level_view(_h(batch), int(body), int(level), C.byref(k), C.byref(lf), C.byref(mk),
                                      C.byref(cf), C.byref(n)), "agal_batch_level_view")
    return k.value, lf.value, mk.value, cf.value, n.value


def agal_batch_info(batch):
    nb, w = C.c_int(), C.c_int()
    _check(_lib.agal_batch_info(_h(batch), C.byref(nb), C.byref(w)), "agal_batch_info")
    return nb.value, w.value


def agal_destroy_batch(h):
    _lib.agal_destroy_batch(_h(h))


def agal_destroy_geom(h):
    _lib.agal_destroy_geom(_h(h))


def agal_destroy_bins(h):
    _lib.agal_destroy_bins(_h(h))


def agal_destroy_forest(h):
    _lib.agal_destroy_forest(_h(h))


def agal_destroy_links(h):
    _lib.agal_destroy_links(_h(h))


def agal_status_string(s: int) -> str:
    return _lib.agal_status_string(int(s)).decode()


def agal_last_error() -> str:
    return _lib.agal_last_error().decode(errors="replace")


from .torch_api import (Batch, Bins, Context, Forest, ForestDiff, Geometry, LinkFractions, Links,  # noqa: E402
                        NearWallConfig, device_copy, device_write, near_wall)

__all__ = [n for n in dir() if n.startswith("agal_")] + [
    "AgalError", "Batch", "device_write", "Context", "Geometry", "Bins", "Forest", "ForestDiff", "Links", "LinkFractions", "NearWallConfig", "near_wall",
    "forest_desc", "body_desc", "tune_opts", "device_copy", "LIB_PATH"]
