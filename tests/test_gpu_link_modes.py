"""Link fractions from per-block candidate lists (node pass + row pass, rows written at their final
place) and from the bins (one pass, staged rows compacted): both must give the same node keys, q and
face ids bit for bit, and match the FP64 oracle.  The cases cover exact ties, det == 0, t in {0, 1},
degenerate faces, faces outside the domain, blocks with more candidates than one staging round, 2D,
and a forest with no refinement (blocks found by their root index instead of the parent table)."""
import numpy as np
import pytest

import geomgen
from _parity import check_face_ties, compare_bins, compare_forest, compare_links, gpu_run, log
from test_gpu_parity import _check_links, _small_sphere

pytestmark = pytest.mark.gpu


def _degenerate():
    v, f = geomgen.random_triangles(240, 12, 0.1, 0.9, 0.08)
    v = v.reshape(-1, 3, 3).copy()
    v[0::4, 1] = v[0::4, 0]
    v[1::4, 1] = v[1::4, 0]
    v[1::4, 2] = v[1::4, 0]
    v[2::4, 2] = v[2::4, 0] + np.float32(2.0) * (v[2::4, 1] - v[2::4, 0])
    return geomgen.Workload("degenerate", 3, v.reshape(-1, 3).astype(np.float32), f, (3, 3, 3), 2, 8, 27)


def _outside():
    v, f = geomgen.random_triangles(300, 9, 0.05, 0.95, 0.08)
    v = v.copy()
    v[:30] += np.float32(0.9)
    return geomgen.Workload("rand-outside", 3, v, f, (3, 3, 3), 2, 10, 27)


def _box():
    v, f = geomgen.box_mesh((81 / 256,) * 3, (175 / 256,) * 3)
    return geomgen.Workload("box", 3, v, f, (4, 4, 4), 3, 16, 27)


def _square():
    v, f = geomgen.square_loop((81 / 256, 81 / 256), (175 / 256, 175 / 256))
    return geomgen.Workload("square", 2, v, f, (4, 4, 1), 3, 16, 9)


def _packed():
    v, f = geomgen.random_triangles(400, 5, 0.47, 0.53, 0.01)
    return geomgen.Workload("packed400", 3, v, f, (4, 4, 4), 2, 4, 19)


def _rseg():
    v, f = geomgen.random_segments(200, 10, 0.05, 0.95, 0.1)
    return geomgen.Workload("rseg", 2, v, f, (5, 3, 1), 3, 9, 9)


def _nd():
    v, f = geomgen.icosphere(3, 0.2)
    return geomgen.Workload("ico3-nd", 3, v, f, (5, 6, 4), 2, 13, 27, lo=(0.05, -0.02, 0.1), hi=(0.97, 1.01, 0.9))


CASES = {
    "C0": lambda: geomgen.workload("C0"),
    "ico3-nd": _nd,
    "box": _box,
    "square": _square,
    "degenerate": _degenerate,
    "rand-outside": _outside,
    "packed400": _packed,
    "rseg": _rseg,
    "zero-levels": lambda: _small_sphere(2, 4, 0, 8, 27),
}


@pytest.mark.parametrize("name", list(CASES))
def test_list_and_walk_modes_agree_and_match_oracle(orc, name):
    import paper_2502_16310_amd as agal
    wl = CASES[name]()
    log(f"case {wl.name}: dim {wl.dim} faces {len(wl.faces)} roots {wl.roots[:wl.dim]} L {wl.levels} "
        f"B {wl.bins} Q {wl.lattice}")
    walk, lists = agal.Context(), agal.Context()
    walk.set_link_list_limit(0)
    lists.set_link_list_limit(1 << 30)
    d_spec = list(wl.d_spec()[:wl.levels])
    gw = gpu_run(wl, ctx=walk, d_spec=d_spec)
    gl = gpu_run(wl, ctx=lists, d_spec=d_spec)
    for k in ("key", "q", "face"):
        assert np.array_equal(gw[k], gl[k]), f"{k} differs between the list and walk modes"
    log(f"  list and walk modes identical: {len(gl['key'])} nodes")
    coords = orc.gather(wl.dim, wl.vertices, wl.faces)
    ob = orc.bin_faces(wl.dim, coords, wl.lo[:wl.dim], wl.hi[:wl.dim], wl.bins)
    compare_bins(gl, ob)
    of = orc.refine(wl.dim, coords, ob, wl.roots[:wl.dim], wl.levels, d_spec, wl.lo[:wl.dim], wl.hi[:wl.dim])
    compare_forest(gl, of, wl.levels)
    lk = orc.link_fractions(wl.dim, coords, ob, of, wl.lattice)
    rep, arrs = compare_links(gl, lk, cells=4 ** wl.dim)
    _check_links(rep)
    nd, bad = check_face_ties(orc, of, coords, wl.lattice, *arrs)
    log(f"  face ids differing at ties: {nd}, not a tie: {bad}")
    assert bad == 0


def test_default_mode_on_the_sphere_is_lists():
    """The sphere workloads take list mode at the default limit (the node pass runs), and a box of
    large faces takes the bin walk."""
    import torch
    import paper_2502_16310_amd as agal
    for wl, want in ((_small_sphere(3, 4, 2, 16, 19), True), (geomgen.workload("C0"), True),
                     (geomgen.Workload("box-big", 3, *geomgen.box_mesh(), (4, 4, 4), 3, 8, 19), False)):
        ctx = agal.Context()
        agal.agal_profile_enable(ctx.h, True)
        gpu_run(wl, ctx=ctx)
        torch.cuda.synchronize()
        names = agal.agal_profile_read(ctx.h)
        agal.agal_profile_enable(ctx.h, False)
        log(f"  {wl.name}: kernels {sorted(names)}")
        assert ("q_nodes" in names) == want
