"""torch-facing wrappers over the C ABI: tensors in, tensors out, the current
torch stream as the HIP stream, and the autograd Function for q.

torch only provides device memory and the stream; every step runs in the HIP
library.  Result arrays owned by the library are copied into torch tensors on
the same stream (device-to-device) when asked for.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import torch

from . import (AgalError, agal_bin_faces, agal_bins_view, agal_context_create, agal_context_destroy,
               agal_destroy_bins, agal_destroy_forest, agal_destroy_geom, agal_destroy_links, agal_forest_info,
               agal_forest_level_view, agal_geom_view, agal_import_faces, agal_link_fractions,
               agal_link_fractions_backward, agal_links_view, agal_near_wall_refine, forest_desc)

_hip = None


def _hiprt():
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        _hip.hipMemcpyAsync.restype = C.c_int
    return _hip


def current_stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def device_copy(ptr: int, numel: int, dtype: torch.dtype, device=None) -> torch.Tensor:
    """Copy `numel` elements at device address `ptr` into a new tensor (stream ordered)."""
    t = torch.empty(numel, dtype=dtype, device=device or torch.device("cuda", torch.cuda.current_device()))
    if numel:
        rc = _hiprt().hipMemcpyAsync(t.data_ptr(), ptr, numel * t.element_size(), 3, current_stream() or None)
        if rc != 0:
            raise AgalError(3, f"hipMemcpyAsync failed with code {rc}")
    return t


class Context:
    """One agal_context (HIP stream-ordered pool allocator)."""

    def __init__(self):
        self.h = agal_context_create()

    def __del__(self):
        if getattr(self, "h", None) is not None:
            agal_context_destroy(self.h)
            self.h = None

    def import_faces(self, vertices: torch.Tensor, faces: Optional[torch.Tensor] = None) -> "Geometry":
        return Geometry(self, vertices, faces)


_default_ctx: Optional[Context] = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx


def _require_cuda(t: torch.Tensor, dtype, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    return t.contiguous()


class Geometry:
    def __init__(self, ctx: Context, vertices: torch.Tensor, faces: Optional[torch.Tensor]):
        self.ctx = ctx
        v = _require_cuda(vertices, torch.float32, "vertices")
        dim = v.shape[-1]
        if faces is not None:
            f = _require_cuda(faces, torch.int32, "faces")
            nf = f.shape[0]
            fp = f.data_ptr()
        else:
            f, nf, fp = None, v.shape[0] // dim, None
        self.h = agal_import_faces(ctx.h, dim, v.data_ptr(), v.shape[0], fp, nf, current_stream())
        self.dim, self.n_faces, self.n_vertices, _, _ = agal_geom_view(self.h)

    def __del__(self):
        if getattr(self, "h", None) is not None:
            agal_destroy_geom(self.h)
            self.h = None

    def soa(self) -> Tuple[torch.Tensor, torch.Tensor]:
        _, F, _, co, bb = agal_geom_view(self.h)
        d = self.dim
        return (device_copy(co, d * d * F, torch.float32).view(d * d, F),
                device_copy(bb, 2 * d * F, torch.float32).view(2 * d, F))

    def bin_faces(self, lo, hi, B: int) -> "Bins":
        return Bins(self, lo, hi, B)


class Bins:
    def __init__(self, geom: Geometry, lo, hi, B: int):
        self.geom = geom
        self.h = agal_bin_faces(geom.h, lo, hi, B, current_stream())
        self.B = B
        _, _, self.n_bins, self.n_entries = agal_bins_view(self.h)

    def __del__(self):
        if getattr(self, "h", None) is not None:
            agal_destroy_bins(self.h)
            self.h = None

    def tensors(self) -> Tuple[torch.Tensor, torch.Tensor]:
        off, ids, nb, P = agal_bins_view(self.h)
        return device_copy(off, nb + 1, torch.int32), device_copy(ids, P, torch.int32)


class Forest:
    def __init__(self, geom: Geometry, bins: Bins, dim, roots, n_levels, d_spec, lo, hi):
        self.geom, self.bins = geom, bins
        self.desc = forest_desc(dim, roots, n_levels, d_spec, lo, hi)
        self.h = agal_near_wall_refine(geom.h, bins.h, self.desc, current_stream())
        self.dim, self.n_levels = agal_forest_info(self.h)

    def __del__(self):
        if getattr(self, "h", None) is not None:
            agal_destroy_forest(self.h)
            self.h = None

    def level(self, l: int) -> dict:
        k, lf, mk, cf, n = agal_forest_level_view(self.h, l)
        cells = 4 ** self.dim
        out = {"keys": device_copy(k, n, torch.int32), "leaf": device_copy(lf, n, torch.uint8),
               "mark": device_copy(mk, n, torch.uint8), "n": n}
        out["cell_flag"] = device_copy(cf, n * cells, torch.uint8).view(n, cells) if cf else None
        return out

    def link_fractions(self, lattice: int) -> "Links":
        return Links(self, lattice)


class Links:
    def __init__(self, forest: Forest, lattice: int):
        self.forest = forest
        self.geom = forest.geom
        self.h = agal_link_fractions(forest.geom.h, forest.bins.h, forest.h, lattice, current_stream())
        _, _, _, self.n_nodes, self.Q = agal_links_view(self.h)

    def __del__(self):
        if getattr(self, "h", None) is not None:
            agal_destroy_links(self.h)
            self.h = None

    def tensors(self) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
        k, q, f, n, Q = agal_links_view(self.h)
        return (device_copy(k, n, torch.int64), device_copy(q, n * Q, torch.float32).view(n, Q),
                device_copy(f, n * Q, torch.int32).view(n, Q))

    def backward(self, grad_q: torch.Tensor, grad_vertices: Optional[torch.Tensor] = None) -> torch.Tensor:
        g = _require_cuda(grad_q, torch.float32, "grad_q")
        if g.numel() != self.n_nodes * self.Q:
            raise ValueError("grad_q must hold n_nodes * Q values")
        if grad_vertices is None:
            grad_vertices = torch.zeros((self.geom.n_vertices, self.geom.dim), dtype=torch.float32, device=g.device)
        agal_link_fractions_backward(self.geom.h, self.h, g.data_ptr(), grad_vertices.data_ptr(), current_stream())
        return grad_vertices


@dataclass
class NearWallConfig:
    """Forest, bins and lattice of one near-wall pass.  d_spec=None means one cell of the
    tested level: d_l = (hi - lo) / (4 * roots * 2^l)."""
    dim: int
    roots: Sequence[int]
    n_levels: int
    bins: int
    lattice: int
    lo: Sequence[float] = (0.0, 0.0, 0.0)
    hi: Sequence[float] = (1.0, 1.0, 1.0)
    d_spec: Optional[Sequence[float]] = None

    def distances(self) -> List[float]:
        if self.d_spec is not None:
            return [float(x) for x in self.d_spec]
        import numpy as np
        span = np.float32(self.hi[0]) - np.float32(self.lo[0])
        return [float(np.float32(span / np.float32(4 * self.roots[0] * (1 << l)))) for l in range(self.n_levels)]


def near_wall(vertices: torch.Tensor, faces: Optional[torch.Tensor], cfg: NearWallConfig,
              ctx: Optional[Context] = None, with_links: bool = True):
    """Import -> bins -> refinement -> link fractions on the current stream."""
    ctx = ctx or default_context()
    geom = ctx.import_faces(vertices, faces)
    bins = geom.bin_faces(cfg.lo[:cfg.dim], cfg.hi[:cfg.dim], cfg.bins)
    forest = Forest(geom, bins, cfg.dim, cfg.roots, cfg.n_levels, cfg.distances(), cfg.lo, cfg.hi)
    links = forest.link_fractions(cfg.lattice) if with_links else None
    return geom, bins, forest, links


class LinkFractions(torch.autograd.Function):
    """(vertices, faces, cfg) -> (node_key, q, face); differentiable in the vertices."""

    @staticmethod
    def forward(fctx, vertices, faces, cfg, ctx=None):
        geom, bins, forest, links = near_wall(vertices.detach(), faces, cfg, ctx)
        fctx.keep = (geom, bins, forest, links)
        fctx.vshape = tuple(vertices.shape)
        key, q, face = links.tensors()
        fctx.mark_non_differentiable(key, face)
        return key, q, face

    @staticmethod
    def backward(fctx, g_key, g_q, g_face):
        geom, bins, forest, links = fctx.keep
        grad_v = torch.zeros(fctx.vshape, dtype=torch.float32, device=g_q.device if g_q is not None else "cuda")
        if g_q is not None:
            links.backward(g_q.contiguous(), grad_v)
        return grad_v, None, None, None
