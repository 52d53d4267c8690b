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

from . import (AgalError, agal_batch_body_view, agal_batch_info, agal_batch_level_view, agal_batch_plan_create,
               agal_batch_run, agal_batch_status, agal_bin_faces, agal_bin_faces_discrete, agal_bins_view, agal_context_create,
               agal_context_set_flag_table_limit, agal_context_set_link_list_limit,
               agal_context_destroy, agal_destroy_batch, agal_destroy_bins, agal_destroy_forest, agal_destroy_geom,
               agal_destroy_links, agal_forest_info, agal_forest_level_view, agal_geom_view, agal_import_faces,
               agal_classify_nodes, agal_destroy_forest_diff, agal_forest_diff_create, agal_forest_diff_view,
               agal_link_fractions, agal_link_fractions_backward, agal_links_view, agal_near_wall_refine,
               agal_near_wall_refine_own_bin, body_desc,
               forest_desc, tune_opts)

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


def device_write(ptr: int, src: torch.Tensor):
    """Copy a contiguous device tensor to device address `ptr` (stream ordered)."""
    src = src.contiguous()
    if src.numel():
        rc = _hiprt().hipMemcpyAsync(ptr, src.data_ptr(), src.numel() * src.element_size(), 3,
                                     current_stream() or None)
        if rc != 0:
            raise AgalError(3, f"hipMemcpyAsync failed with code {rc}")


class _TorchAllocator:
    """agal_allocator callbacks over torch's caching allocator: the library's
    device memory comes from (and returns to) torch's pool, on the stream the
    library passes."""

    def __init__(self):
        from . import _Allocator

        def alloc(_ctx, nbytes, stream):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), stream or 0)
            except RuntimeError:
                return None   # out of memory: the library reports AGAL_ENOMEM

        def free(_ctx, ptr, _stream):
            torch.cuda.caching_allocator_delete(ptr)

        ft = _Allocator._fields_
        self._alloc = ft[1][1](alloc)   # the callbacks must outlive every context that uses them
        self._free = ft[2][1](free)
        self.desc = _Allocator(None, self._alloc, self._free)


_torch_allocator: Optional[_TorchAllocator] = None


class _DeviceView:
    """A device array owned by a library handle, exposed to torch without a
    copy (CUDA array interface); holds its owner so the memory outlives every
    tensor made from it."""

    _TYPESTR = {torch.int32: "<i4", torch.int64: "<i8", torch.float32: "<f4", torch.uint8: "|u1"}

    def __init__(self, ptr: int, shape: Tuple[int, ...], dtype: torch.dtype, owner):
        self.owner = owner
        self.__cuda_array_interface__ = {"shape": tuple(int(x) for x in shape), "typestr": self._TYPESTR[dtype],
                                         "data": (int(ptr), False), "version": 2}


def device_view(ptr: int, shape, dtype: torch.dtype, owner) -> torch.Tensor:
    """Tensor aliasing `ptr` (no copy), valid while `owner` lives (the tensor keeps it alive)."""
    shape = tuple(shape)
    numel = 1
    for x in shape:
        numel *= int(x)
    if numel == 0 or not ptr:
        return torch.empty(shape, dtype=dtype, device=torch.device("cuda", torch.cuda.current_device()))
    return torch.as_tensor(_DeviceView(ptr, shape, dtype, owner), device=torch.device("cuda",
                                                                                       torch.cuda.current_device()))


class Context:
    """One agal_context.  By default the library allocates device memory
    through torch's caching allocator; torch_allocator=False selects the
    library's own stream-ordered pool."""

    def __init__(self, torch_allocator: bool = True):
        global _torch_allocator
        if torch_allocator:
            if _torch_allocator is None:
                _torch_allocator = _TorchAllocator()
            self.h = agal_context_create(_torch_allocator.desc)
        else:
            self.h = agal_context_create()

    def __del__(self):
        if getattr(self, "h", None) is not None:
            agal_context_destroy(self.h)
            self.h = None

    def import_faces(self, vertices: torch.Tensor, faces: Optional[torch.Tensor] = None) -> "Geometry":
        return Geometry(self, vertices, faces)

    def set_flag_table_limit(self, max_entries: int):
        """Face-centric flag step for levels whose block grid has at most
        max_entries positions, cell-centric above (0: cell-centric everywhere)."""
        agal_context_set_flag_table_limit(self.h, max_entries)

    def set_link_list_limit(self, max_blocks_per_face: int):
        """Link fractions from per-block candidate lists while the largest face
        has at most this many candidate blocks, from the bins above (0: always
        from the bins)."""
        agal_context_set_link_list_limit(self.h, max_blocks_per_face)


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
        """Views of the coordinate list and bounding boxes (valid while this object lives)."""
        _, F, _, co, bb = agal_geom_view(self.h)
        d = self.dim
        return device_view(co, (d * d, F), torch.float32, self), device_view(bb, (2 * d, F), torch.float32, self)

    def bin_faces(self, lo, hi, B: int) -> "Bins":
        return Bins(self, lo, hi, B)

    def bin_faces_discrete(self, lo, hi, B: int, spacing: float = 0.0, bin_fraction: int = 0) -> "Bins":
        """The paper's binning by sampled points (spacing <= 0: half the smallest bin edge; bin_fraction >= 1:
        the paper's indicator-array form, B^D / bin_fraction bins at a time)."""
        return Bins(self, lo, hi, B, discrete=True, spacing=spacing, bin_fraction=bin_fraction)


class Bins:
    def __init__(self, geom: Geometry, lo, hi, B: int, discrete: bool = False, spacing: float = 0.0,
                 bin_fraction: int = 0):
        self.geom = geom
        if discrete:
            self.h = agal_bin_faces_discrete(geom.h, lo, hi, B, spacing, bin_fraction, current_stream())
        else:
            self.h = agal_bin_faces(geom.h, lo, hi, B, current_stream())
        self.B = B
        _, _, self.n_bins, self.n_entries = agal_bins_view(self.h)

    def __del__(self):
        if getattr(self, "h", None) is not None:
            agal_destroy_bins(self.h)
            self.h = None

    def tensors(self) -> Tuple[torch.Tensor, torch.Tensor]:
        """Views of the CSR offsets (uint32 bits in int32) and face ids."""
        off, ids, nb, P = agal_bins_view(self.h)
        return device_view(off, (nb + 1,), torch.int32, self), device_view(ids, (P,), torch.int32, self)


class Forest:
    """Near-wall refinement.  own_bin=True takes the paper's own form: a cell
    looks at the faces of its own bin with the Euclidean test, and marks
    spread over n_prop rings of blocks (n_prop < 0: the paper's rule)."""

    def __init__(self, geom: Geometry, bins: Bins, dim, roots, n_levels, d_spec, lo, hi, own_bin: bool = False,
                 n_prop: int = -1):
        self.geom, self.bins = geom, bins
        self.desc = forest_desc(dim, roots, n_levels, d_spec, lo, hi)
        if own_bin:
            self.h = agal_near_wall_refine_own_bin(geom.h, bins.h, self.desc, n_prop, current_stream())
        else:
            self.h = agal_near_wall_refine(geom.h, bins.h, self.desc, current_stream())
        self.dim, self.n_levels = agal_forest_info(self.h)

    def __del__(self):
        if getattr(self, "h", None) is not None:
            agal_destroy_forest(self.h)
            self.h = None

    def level(self, l: int) -> dict:
        """Views of one level's arrays (keys are uint32 bits in int32)."""
        k, lf, mk, cf, n = agal_forest_level_view(self.h, l)
        cells = 4 ** self.dim
        out = {"keys": device_view(k, (n,), torch.int32, self), "leaf": device_view(lf, (n,), torch.uint8, self),
               "mark": device_view(mk, (n,), torch.uint8, self), "n": n}
        out["cell_flag"] = device_view(cf, (n, cells), torch.uint8, self) if cf else None
        return out

    def link_fractions(self, lattice: int) -> "Links":
        return Links(self, lattice)

    def diff(self, old: "Forest") -> "ForestDiff":
        """How this forest relates to `old` (the same body's forest before it moved), level by level."""
        return ForestDiff(old, self)


class ForestDiff:
    """Re-adaptation bookkeeping between two forests over the same root grid: per level, for every new block
    its index in the old level (-1: none) and its state (0 kept, 1 created, 2 refined, 3 coarsened), for every
    old block whether it was removed, and the counts [created, refined, coarsened, removed]."""

    def __init__(self, old: Forest, new: Forest):
        self.old, self.new = old, new
        self.h = agal_forest_diff_create(old.h, new.h, current_stream())
        self.n_levels = new.n_levels

    def __del__(self):
        if getattr(self, "h", None) is not None:
            agal_destroy_forest_diff(self.h)
            self.h = None

    def level(self, l: int) -> dict:
        oi, st, rm, nn, no, cnt = agal_forest_diff_view(self.h, l)
        return {"old_index": device_view(oi, (nn,), torch.int32, self), "state": device_view(st, (nn,), torch.uint8, self),
                "removed": device_view(rm, (no,), torch.uint8, self), "counts": cnt}

    def counts(self) -> List[List[int]]:
        return [agal_forest_diff_view(self.h, l)[5] for l in range(self.n_levels + 1)]


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
        """Views of node keys (uint64 bits in int64), q and face ids."""
        k, q, f, n, Q = agal_links_view(self.h)
        return (device_view(k, (n,), torch.int64, self), device_view(q, (n, Q), torch.float32, self),
                device_view(f, (n, Q), torch.int32, self))

    def backward(self, grad_q: torch.Tensor, grad_vertices: Optional[torch.Tensor] = None) -> torch.Tensor:
        g = _require_cuda(grad_q, torch.float32, "grad_q")
        if g.numel() != self.n_nodes * self.Q:
            raise ValueError("grad_q must hold n_nodes * Q values")
        if grad_vertices is None:
            grad_vertices = torch.zeros((self.geom.n_vertices, self.geom.dim), dtype=torch.float32, device=g.device)
        agal_link_fractions_backward(self.geom.h, self.h, g.data_ptr(), grad_vertices.data_ptr(), current_stream())
        return grad_vertices

    def classify(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Side of every boundary node from its links' faces: 1 fluid, 2 solid, 3 mixed (uint8, node order)."""
        if out is None:
            out = torch.empty(self.n_nodes, dtype=torch.uint8, device=torch.device("cuda", torch.cuda.current_device()))
        if not out.is_cuda or out.dtype != torch.uint8 or not out.is_contiguous() or out.numel() != self.n_nodes:
            raise ValueError("out must be a contiguous uint8 device tensor of n_nodes values")
        agal_classify_nodes(self.geom.h, self.h, out.data_ptr(), current_stream())
        return out


@dataclass
class NearWallConfig:
    """Forest, bins and lattice of one near-wall pass.  d_spec=None means one cell of the
    tested level, its largest extent: d_l = max over axes of (hi - lo) / (4 * roots * 2^l)."""
    dim: int
    roots: Sequence[int]
    n_levels: int
    bins: int
    lattice: int
    lo: Sequence[float] = (0.0, 0.0, 0.0)
    hi: Sequence[float] = (1.0, 1.0, 1.0)
    d_spec: Optional[Sequence[float]] = None
    own_bin: bool = False     # the paper's own-bin Euclidean flags with mark propagation
    n_prop: int = -1          # propagation steps of the own-bin form (< 0: the paper's rule)

    def distances(self) -> List[float]:
        if self.d_spec is not None:
            return [float(x) for x in self.d_spec]
        import numpy as np
        out = []
        for l in range(self.n_levels):
            d = [np.float32(np.float32(self.hi[a]) - np.float32(self.lo[a])) / np.float32(4 * self.roots[a] * (1 << l))
                 for a in range(self.dim)]
            out.append(float(max(np.float32(x) for x in d)))
        return out


def near_wall(vertices: torch.Tensor, faces: Optional[torch.Tensor], cfg: NearWallConfig,
              ctx: Optional[Context] = None, with_links: bool = True):
    """Import -> bins -> refinement -> link fractions on the current stream."""
    ctx = ctx or default_context()
    geom = ctx.import_faces(vertices, faces)
    bins = geom.bin_faces(cfg.lo[:cfg.dim], cfg.hi[:cfg.dim], cfg.bins)
    forest = Forest(geom, bins, cfg.dim, cfg.roots, cfg.n_levels, cfg.distances(), cfg.lo, cfg.hi, cfg.own_bin,
                    cfg.n_prop)
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


class Batch:
    """Many bodies, one graph launch per run.

    bodies: sequence of (vertices, faces or None, NearWallConfig); a config with
    bins <= 0 lets the plan's tuner choose the bin density.  The tensors must
    stay alive (and keep their shapes) while the batch lives; their values may
    change between runs."""

    def __init__(self, bodies, tune_bins: bool = True, tune_grid: bool = True, with_adjoint: bool = False,
                 capacity_margin: float = 0.0, cache_path: Optional[str] = None, ctx: Optional[Context] = None):
        self.ctx = ctx or default_context()
        self._inputs = []
        descs = []
        for v, f, cfg in bodies:
            v = v.contiguous()
            f = None if f is None else f.to(torch.int32).contiguous()
            self._inputs.append((v, f))
            fd = forest_desc(cfg.dim, cfg.roots, cfg.n_levels, cfg.distances(), cfg.lo, cfg.hi)
            descs.append(body_desc(cfg.dim, v.data_ptr(), v.shape[0], None if f is None else f.data_ptr(),
                                   f.shape[0] if f is not None else v.shape[0] // cfg.dim, fd, cfg.lattice,
                                   cfg.bins))
        self.cfgs = [b[2] for b in bodies]
        opts = tune_opts(tune_bins, tune_grid, with_adjoint, capacity_margin, cache_path)
        self.h = agal_batch_plan_create(self.ctx.h, descs, opts, current_stream())
        self.n_bodies, self.workgroups_per_cu = agal_batch_info(self.h)

    def __del__(self):
        if getattr(self, "h", None) is not None:
            agal_destroy_batch(self.h)
            self.h = None

    def run(self):
        agal_batch_run(self.h, current_stream())

    def status(self):
        agal_batch_status(self.h, current_stream())

    def bins(self, body: int) -> int:
        return agal_batch_body_view(self.h, body)[8]

    # Results are copies: a run rewrites the plan's buffers in place.
    def links(self, body: int):
        """(node_key int64, q (n, Q) float32, face (n, Q) int32) of the last run (after status())."""
        k, q, f, n, Q, _, _, _, _ = agal_batch_body_view(self.h, body)
        return (device_copy(k, n, torch.int64), device_copy(q, n * Q, torch.float32).view(n, Q),
                device_copy(f, n * Q, torch.int32).view(n, Q))

    def level(self, body: int, level: int):
        k, lf, mk, cf, n = agal_batch_level_view(self.h, body, level)
        cells = 4 ** self.cfgs[body].dim
        return {"keys": device_copy(k, n, torch.int32), "leaf": device_copy(lf, n, torch.uint8),
                "mark": device_copy(mk, n, torch.uint8),
                "cell_flag": None if not cf else device_copy(cf, n * cells, torch.uint8).view(n, cells)}

    def set_grad_q(self, body: int, grad_q: torch.Tensor):
        """Adjoint input of `body` for the next run: (n_nodes, Q) float32, rows in node order."""
        _, _, _, n, Q, gq, _, cap, _ = agal_batch_body_view(self.h, body)
        if grad_q.shape[0] > cap or (grad_q.numel() and grad_q.shape[1] != Q):
            raise AgalError(1, f"grad_q of shape {tuple(grad_q.shape)} does not fit ({cap}, {Q})")
        if not gq:
            raise AgalError(1, "the batch was planned without the adjoint")
        device_write(gq, grad_q.to(torch.float32))

    def grad_vertices(self, body: int) -> torch.Tensor:
        _, _, _, _, _, _, gv, _, _ = agal_batch_body_view(self.h, body)
        v, _ = self._inputs[body]
        return device_copy(gv, v.numel(), torch.float32).view_as(v)
