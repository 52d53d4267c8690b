"""GPU <-> oracle parity through the C ABI: bins and flags bit-exact, q within
1e-5 of the FP64 oracle, gradients against the FP64 adjoint and central
finite differences."""
import numpy as np
import pytest

import geomgen
from _parity import END_TOL, Q_TOL, check_face_ties, compare_bins, compare_forest, compare_links, gpu_run, log

pytestmark = pytest.mark.gpu


def _small_sphere(s=2, R=4, L=3, B=16, Q=19):
    v, f = geomgen.icosphere(s, 0.2)
    return geomgen.Workload(f"ico{s}", 3, v, f, (R, R, R), L, B, Q)


def _check_links(rep, allow_one_sided=0):
    log(f"  links: gpu nodes {rep.nodes_gpu} oracle nodes {rep.nodes_orc} common links {rep.links} "
        f"max|dq| {rep.max_err:.3e} one-sided {rep.one_sided} (not at an end: {rep.one_sided_not_at_end}) "
        f"face-id diffs {rep.face_diff}")
    assert rep.max_err <= Q_TOL
    assert rep.one_sided_not_at_end <= allow_one_sided
    assert rep.links > 0


def _full(orc, wl, B=None, allow_one_sided=0):
    log(f"case {wl.name}: dim {wl.dim} faces {len(wl.faces)} roots {wl.roots[:wl.dim]} L {wl.levels} "
        f"B {B or wl.bins} Q {wl.lattice}")
    g = gpu_run(wl, B=B)
    coords = orc.gather(wl.dim, wl.vertices, wl.faces)
    ob = orc.bin_faces(wl.dim, coords, wl.lo[:wl.dim], wl.hi[:wl.dim], B or wl.bins)
    compare_bins(g, ob)
    of = orc.refine(wl.dim, coords, ob, wl.roots[:wl.dim], wl.levels, wl.d_spec(), wl.lo[:wl.dim], wl.hi[:wl.dim])
    compare_forest(g, of, wl.levels)
    lk = orc.link_fractions(wl.dim, coords, ob, of, wl.lattice)
    rep, arrs = compare_links(g, lk, cells=4 ** wl.dim)
    _check_links(rep, allow_one_sided)
    nd, bad = check_face_ties(orc, of, coords, wl.lattice, *arrs)
    log(f"  face ids differing at ties: {nd}, not a tie: {bad}")
    assert bad == 0
    return g, of, lk


def test_circle_2d_full(orc):
    _full(orc, geomgen.workload("C0"))


def test_small_sphere_full(orc):
    _full(orc, _small_sphere())


def test_small_sphere_d3q27_non_dyadic_domain(orc):
    v, f = geomgen.icosphere(3, 0.2)
    wl = geomgen.Workload("ico3-nd", 3, v, f, (5, 6, 4), 2, 13, 27, lo=(0.05, -0.02, 0.1), hi=(0.97, 1.01, 0.9))
    _full(orc, wl)


@pytest.mark.parametrize("B", [1, 2, 8, 37])
def test_bin_density_invariance(orc, B):
    # B = 1 is the naive all-faces search; tiny B exercises the oversized-bin path
    _full(orc, _small_sphere(3, 4, 2, 16), B=B)


def test_random_triangles_and_outside_faces(orc):
    v, f = geomgen.random_triangles(300, 9, 0.05, 0.95, 0.08)
    v = v.copy()
    v[:30] += np.float32(0.9)  # some faces stick out of the domain
    wl = geomgen.Workload("rand", 3, v, f, (3, 3, 3), 2, 10, 27)
    _full(orc, wl)


def test_random_segments_2d(orc):
    v, f = geomgen.random_segments(200, 10, 0.05, 0.95, 0.1)
    wl = geomgen.Workload("rseg", 2, v, f, (5, 3, 1), 3, 9, 9)
    _full(orc, wl)


def test_no_refinement_when_far(orc):
    # geometry far outside the near-wall distance: nothing is flagged, no links
    v, f = geomgen.icosphere(1, 0.05, (0.5, 0.5, 0.5))
    wl = geomgen.Workload("tiny", 3, v, f, (2, 2, 2), 2, 8, 19)
    g = gpu_run(wl, d_spec=[0.0, 0.0])
    of_levels = [len(l["keys"]) for l in g["levels"]]
    log(f"  levels {of_levels}")
    coords = orc.gather(3, wl.vertices, wl.faces)
    ob = orc.bin_faces(3, coords, (0, 0, 0), (1, 1, 1), 8)
    of = orc.refine(3, coords, ob, (2, 2, 2), 2, [0.0, 0.0], (0, 0, 0), (1, 1, 1))
    compare_forest(g, of, 2)


def test_zero_levels(orc):
    wl = _small_sphere(2, 4, 0, 8)
    g = gpu_run(wl, levels=0, d_spec=[])
    assert len(g["levels"]) == 1 and (g["levels"][0]["leaf"] == 1).all()
    coords = orc.gather(3, wl.vertices, wl.faces)
    ob = orc.bin_faces(3, coords, (0, 0, 0), (1, 1, 1), 8)
    of = orc.refine(3, coords, ob, (4, 4, 4), 0, [], (0, 0, 0), (1, 1, 1))
    lk = orc.link_fractions(3, coords, ob, of, 19)
    rep, _ = compare_links(g, lk)
    _check_links(rep)


def test_sphere_c1_bins_flags_exact_and_sampled_q(orc):
    wl = geomgen.workload("C1")
    log(f"case C1: faces {len(wl.faces)}")
    g = gpu_run(wl)
    coords = orc.gather(3, wl.vertices, wl.faces)
    ob = orc.bin_faces(3, coords, (0, 0, 0), (1, 1, 1), wl.bins)
    compare_bins(g, ob)
    of = orc.refine(3, coords, ob, wl.roots, wl.levels, wl.d_spec(), (0, 0, 0), (1, 1, 1))
    compare_forest(g, of, wl.levels)
    nL = len(of.levels[wl.levels]["keys"])
    rng = np.random.default_rng(7)
    sub = np.sort(rng.choice(nL, size=min(nL, 2500), replace=False))
    lk = orc.link_fractions(3, coords, ob, of, wl.lattice, subset=sub)
    rep, arrs = compare_links(g, lk, restrict_blocks=of.levels[wl.levels]["keys"][sub])
    _check_links(rep)
    nd, bad = check_face_ties(orc, of, coords, wl.lattice, *arrs)
    log(f"  face ids differing at ties: {nd}, not a tie: {bad}")
    assert bad == 0


def test_run_twice_bitwise_equal(orc):
    wl = _small_sphere(3, 4, 2, 16, 27)
    a = gpu_run(wl)
    b = gpu_run(wl)
    for k in ("offsets", "ids", "key", "q", "face"):
        assert np.array_equal(a[k], b[k]), k
    for la, lb in zip(a["levels"], b["levels"]):
        for k in ("keys", "leaf", "mark"):
            assert np.array_equal(la[k], lb[k])
