"""The paper's sampled-point binning on the GPU against the oracle's orc_bin_faces_discrete, bit for bit
(offsets and ids), in both forms (pairs counted and scattered; the paper's bin-fraction form with its
indicator array at several fractions): 2D and 3D, a single bin holding thousands of faces, faces whose bin
range exceeds 64 bins and one LDS chunk, the paper's star body at its bin densities, the default spacing; the
own-bin refinement and list-mode link fractions on these bins against the oracle, and the calls that need
bounding-box bins refusing them."""
import numpy as np
import pytest

import geomgen
from _parity import check_face_ties, compare_forest, compare_links, log
from test_gpu_parity import _check_links

pytestmark = pytest.mark.gpu


def _geom(wl, ctx=None):
    import torch
    import paper_2502_16310_amd as agal
    ctx = ctx or agal.Context()
    v = torch.from_numpy(np.ascontiguousarray(wl.vertices)).cuda()
    f = torch.from_numpy(np.ascontiguousarray(wl.faces)).cuda()
    return ctx, ctx.import_faces(v, f)


def _compare(orc, wl, geom, B, spacing, fractions=(0,)):
    dim = wl.dim
    coords = orc.gather(dim, wl.vertices, wl.faces)
    ob = orc.bin_faces_discrete(dim, coords, wl.lo[:dim], wl.hi[:dim], B, spacing)
    for bf in fractions:
        bins = geom.bin_faces_discrete(wl.lo[:dim], wl.hi[:dim], B, spacing, bf)
        off, ids = bins.tensors()
        off = off.cpu().numpy().view(np.uint32)
        ids = ids.cpu().numpy()
        assert np.array_equal(off, ob.offsets), f"{wl.name} B={B} B_f={bf}: offsets differ"
        assert np.array_equal(ids, ob.ids), f"{wl.name} B={B} B_f={bf}: ids differ"
    box = orc.bin_faces(dim, coords, wl.lo[:dim], wl.hi[:dim], B)
    log(f"  {wl.name} B={B} spacing={spacing:.4g} fractions {list(fractions)}: {ob.P} entries "
        f"(bounding boxes: {box.P}), largest bin {int(np.diff(ob.offsets).max())}")
    return ob


def _sp(wl, B, frac=0.5):
    return float(np.float32(frac) * min(np.float32(np.float32(wl.hi[a]) - np.float32(wl.lo[a])) / np.float32(B)
                                        for a in range(wl.dim)))


@pytest.mark.parametrize("B", [1, 8, 32])
def test_circle(orc, B):
    wl = geomgen.workload("C0")
    _, geom = _geom(wl)
    _compare(orc, wl, geom, B, _sp(wl, B), (0, 1, 3))
    _compare(orc, wl, geom, B, _sp(wl, B, 1 / 16), (0,))


@pytest.mark.parametrize("B", [1, 2, 16])
def test_sphere_one_bin_of_thousands(orc, B):
    v, f = geomgen.icosphere(4, 0.3)
    wl = geomgen.Workload("ico4", 3, v, f, (8, 8, 8), 2, B, 19)
    _, geom = _geom(wl)
    _compare(orc, wl, geom, B, _sp(wl, B), (0, 1, 5))


@pytest.mark.parametrize("B", [16, 128])
def test_large_faces_workgroup_path(orc, B):
    """The box's twelve triangles span whole bin planes: ranges above 64 bins, and at B = 128 above one LDS
    chunk of 32768 bins."""
    v, f = geomgen.box_mesh((0.03, 0.05, 0.02), (0.97, 0.91, 0.95))
    wl = geomgen.Workload("box-big", 3, v, f, (4, 4, 4), 1, B, 19)
    _, geom = _geom(wl)
    _compare(orc, wl, geom, B, _sp(wl, B), (0, 7) if B == 16 else (0, 64))


@pytest.mark.parametrize("B", [1, 2, 8, 16])
def test_paper_star_body(orc, B):
    wl = geomgen.workload("P1")
    _, geom = _geom(wl)
    _compare(orc, wl, geom, B, _sp(wl, B), (0, 1) if B <= 8 else (0, 4))


def test_default_spacing_and_nondyadic_domain(orc):
    v, f = geomgen.icosphere(3, 0.2)
    wl = geomgen.Workload("ico3-nd", 3, v, f, (5, 6, 4), 2, 11, 27, lo=(0.05, -0.02, 0.1), hi=(0.97, 1.01, 0.9))
    _, geom = _geom(wl)
    dim = wl.dim
    coords = orc.gather(dim, wl.vertices, wl.faces)
    ob = orc.bin_faces_discrete(dim, coords, wl.lo[:dim], wl.hi[:dim], 11, _sp(wl, 11))
    off, ids = geom.bin_faces_discrete(wl.lo[:dim], wl.hi[:dim], 11).tensors()
    assert np.array_equal(off.cpu().numpy().view(np.uint32), ob.offsets)
    assert np.array_equal(ids.cpu().numpy(), ob.ids)


def test_own_bin_refinement_and_links_on_sampled_bins(orc):
    """The paper's pipeline: sampled-point bins, own-bin flags and mark propagation, then link fractions (list
    mode; the box-test refinement refuses these bins)."""
    import paper_2502_16310_amd as agal
    wl = geomgen.workload("P1")
    ctx, geom = _geom(wl)
    B = 8
    sp = _sp(wl, B)
    bins = geom.bin_faces_discrete(wl.lo, wl.hi, B, sp)
    d = [float(x) for x in wl.d_spec()]
    fo = agal.Forest(geom, bins, 3, wl.roots, wl.levels, d, wl.lo, wl.hi, own_bin=True)
    coords = orc.gather(3, wl.vertices, wl.faces)
    ob = orc.bin_faces_discrete(3, coords, wl.lo, wl.hi, B, sp)
    of = orc.refine(3, coords, ob, wl.roots, wl.levels, wl.d_spec(), wl.lo, wl.hi, own_bin=True)
    levels = []
    for l in range(wl.levels + 1):
        x = fo.level(l)
        levels.append({"keys": x["keys"].cpu().numpy().view(np.uint32), "leaf": x["leaf"].cpu().numpy(),
                       "mark": x["mark"].cpu().numpy(),
                       "cell_flag": None if x["cell_flag"] is None else x["cell_flag"].cpu().numpy()})
    compare_forest({"levels": levels}, of, wl.levels)
    log(f"  P1 own-bin on sampled bins (B=8): blocks per level {[len(l['keys']) for l in levels]}")
    # list-mode links on the sampled-bin forest, against the oracle's links (candidates from the bounding-box
    # bins, a superset) on 300 sampled finest-level blocks
    k, q, fc = fo.link_fractions(wl.lattice).tensors()
    g = {"key": k.cpu().numpy().view(np.uint64), "q": q.cpu().numpy(), "face": fc.cpu().numpy()}
    ob_box = orc.bin_faces(3, coords, wl.lo, wl.hi, B)
    nL = len(of.levels[wl.levels]["keys"])
    sub = np.sort(np.random.default_rng(2).choice(nL, size=min(nL, 300), replace=False))
    lk = orc.link_fractions(3, coords, ob_box, of, wl.lattice, subset=sub)
    rep, arrs = compare_links(g, lk, restrict_blocks=of.levels[wl.levels]["keys"][sub])
    _check_links(rep)
    nd, bad = check_face_ties(orc, of, coords, wl.lattice, *arrs)
    assert bad == 0
    with pytest.raises(agal.AgalError) as e:
        agal.Forest(geom, bins, 3, wl.roots, wl.levels, d, wl.lo, wl.hi, own_bin=False)
    assert e.value.status == agal.AGAL_EINVAL


def test_bad_arguments():
    import paper_2502_16310_amd as agal
    wl = geomgen.workload("C0")
    _, geom = _geom(wl)
    for B, sp, bf in ((0, 0.1, 0), (8, float("nan"), 0), (8, float("inf"), 0), (8, 0.1, -1)):
        with pytest.raises(agal.AgalError) as e:
            geom.bin_faces_discrete(wl.lo[:2], wl.hi[:2], B, sp, bf)
        assert e.value.status == agal.AGAL_EINVAL
