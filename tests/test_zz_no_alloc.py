"""The allocation-free binning call (agal_bin_faces_noalloc) against agal_bin_faces.

Both are called through the C ABI on the same imported geometry; offsets and
face ids must be identical.  Three calls in a row, each on a smaller input than
the last (the scratch array keeps the previous call's contents), then the
capacity and size errors.  The context's device allocator counts its calls:
the no-allocation entry point must make none."""
import ctypes as C

import numpy as np
import pytest

import geomgen
from _parity import log

pytestmark = pytest.mark.gpu


class _CountingAllocator:
    """agal_allocator callbacks over torch's caching allocator, counting calls."""

    def __init__(self, agal, torch):
        self.allocs = 0
        self.frees = 0
        self.torch = torch

        def alloc(ctx, nbytes, stream):
            self.allocs += 1
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), stream)

        def free(ctx, ptr, stream):
            self.frees += 1
            torch.cuda.caching_allocator_delete(ptr)

        ft = agal._Allocator._fields_
        self._a = ft[1][1](alloc)
        self._f = ft[2][1](free)
        self.desc = agal._Allocator(None, self._a, self._f)


def _bins_plain(agal, torch, g, lo, hi, B, stream):
    b = agal.agal_bin_faces(g, lo, hi, B, stream)
    off_p, ids_p, nb, P = agal.agal_bins_view(b)
    off = agal.device_copy(off_p, nb + 1, torch.int32).cpu().numpy().view(np.uint32)
    ids = agal.device_copy(ids_p, P, torch.int32).cpu().numpy()
    torch.cuda.synchronize()
    agal.agal_destroy_bins(b)
    return off, ids


def test_bin_faces_noalloc_equals_bin_faces():
    import torch
    import paper_2502_16310_amd as agal
    dev = torch.device("cuda", 0)
    cnt = _CountingAllocator(agal, torch)
    ctx = agal.agal_context_create(cnt.desc)
    stream = torch.cuda.current_stream().cuda_stream
    cases = []
    v, f = geomgen.icosphere(5, 0.2)
    cases.append(("sphere 20480 faces, 64^3 bins", 3, v, f, (0, 0, 0), (1, 1, 1), 64))
    v, f = geomgen.circle(256, 0.25)
    cases.append(("circle 256 segments, 32^2 bins", 2, v, f, (0, 0), (1, 1), 32))
    v, f = geomgen.icosphere(2, 0.3)
    cases.append(("sphere 320 faces, 8^3 bins on [0.1, 0.9]^3", 3, v, f, (0.1, 0.1, 0.1), (0.9, 0.9, 0.9), 8))
    for name, dim, v, f, lo, hi, B in cases:
        log(f"case {name}")
        vt = torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(dev)
        ft = torch.from_numpy(np.ascontiguousarray(f, np.int32)).to(dev)
        g = agal.agal_import_faces(ctx, dim, vt.data_ptr(), vt.shape[0], ft.data_ptr(), ft.shape[0], stream)
        off_ref, ids_ref = _bins_plain(agal, torch, g, lo, hi, B, stream)
        nb = B ** dim
        # caller buffers, filled with garbage so that nothing unwritten can pass
        off = torch.full((nb + 1,), -7, dtype=torch.int32, device=dev)
        cap = len(ids_ref) + 100
        ids = torch.full((cap,), -7, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        a0, f0 = cnt.allocs, cnt.frees
        P = agal.agal_bin_faces_noalloc(g, lo, hi, B, off.data_ptr(), ids.data_ptr(), cap, stream)
        torch.cuda.synchronize()
        assert (cnt.allocs, cnt.frees) == (a0, f0), "the no-allocation call used the device allocator"
        assert P == len(ids_ref)
        off_h = off.cpu().numpy().view(np.uint32)
        ids_h = ids.cpu().numpy()
        assert np.array_equal(off_h, off_ref), "offsets differ from agal_bin_faces"
        assert np.array_equal(ids_h[:P], ids_ref), "face ids differ from agal_bin_faces"
        assert (ids_h[P:] == -7).all(), "wrote past the entry count"
        log(f"  P = {P}, {nb} bins: identical to agal_bin_faces")
        agal.agal_destroy_geom(g)
    # errors: too little id capacity (offsets written, no ids), a grid larger than the scratch array
    v, f = geomgen.icosphere(3, 0.2)
    vt = torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(dev)
    ft = torch.from_numpy(np.ascontiguousarray(f, np.int32)).to(dev)
    g = agal.agal_import_faces(ctx, 3, vt.data_ptr(), vt.shape[0], ft.data_ptr(), ft.shape[0], stream)
    off_ref, ids_ref = _bins_plain(agal, torch, g, (0, 0, 0), (1, 1, 1), 16, stream)
    off = torch.zeros(16 ** 3 + 1, dtype=torch.int32, device=dev)
    ids = torch.full((len(ids_ref) - 1,), -7, dtype=torch.int32, device=dev)
    with pytest.raises(agal.AgalError) as e:
        agal.agal_bin_faces_noalloc(g, (0, 0, 0), (1, 1, 1), 16, off.data_ptr(), ids.data_ptr(), ids.numel(), stream)
    assert e.value.status == agal.AGAL_ECAPACITY
    torch.cuda.synchronize()
    assert np.array_equal(off.cpu().numpy().view(np.uint32), off_ref)
    assert (ids.cpu().numpy() == -7).all()
    log(f"  capacity {ids.numel()} < {len(ids_ref)}: {e.value}")
    big = torch.zeros(8, dtype=torch.int32, device=dev)
    with pytest.raises(agal.AgalError) as e:
        agal.agal_bin_faces_noalloc(g, (0, 0, 0), (1, 1, 1), 256, big.data_ptr(), big.data_ptr(), 8, stream)
    assert e.value.status == agal.AGAL_EINVAL
    log(f"  256^3 bins: {e.value}")
    # the plain call still agrees after the no-allocation calls
    off2, ids2 = _bins_plain(agal, torch, g, (0, 0, 0), (1, 1, 1), 16, stream)
    assert np.array_equal(off2, off_ref) and np.array_equal(ids2, ids_ref)
    agal.agal_destroy_geom(g)
    agal.agal_context_destroy(ctx)
    torch.cuda.synchronize()
