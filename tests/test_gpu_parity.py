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


def _max_adjoint_queue(face, w, tile=256, waves=4, group=4, lanes=64):
    """Longest per-wave link queue of the adjoint kernel's schedule: a tile of `tile` nodes is one span of
    node * Q slots read in chunks of `lanes`, chunk c by wave c % waves, `group` chunks per step; the live
    slots (direction > 0, face >= 0, weight != 0) are appended and taken `lanes` at a time."""
    n, Q = face.shape
    live = ((face >= 0) & (w != 0)).copy()
    live[:, 0] = False
    worst = 0
    for t0 in range(0, n, tile):
        span = live[t0:t0 + tile].reshape(-1)
        chunks = [span[c:c + lanes].sum() for c in range(0, span.size, lanes)]
        for wv in range(waves):
            mine = chunks[wv::waves]
            q = 0
            for g0 in range(0, len(mine), group):
                q += sum(mine[g0:g0 + group])
                worst = max(worst, q)
                q %= lanes
    return worst


def _adjoint_all_links(orc, wl, g, of, lk, coords):
    """GPU adjoint against the FP64 one with every link weighted (where both sides name the same face)."""
    import torch
    geom, bins_h, forest_h, links_h = g["handles"]
    assert np.array_equal(g["key"], lk.key)
    w = geomgen.weights(lk.n * wl.lattice, 5).astype(np.float64).reshape(lk.n, wl.lattice)
    w[(lk.face < 0) | (g["face"] != lk.face)] = 0.0
    grad = links_h.backward(torch.from_numpy(w.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    ref = orc.link_grad(of, lk, coords, wl.faces, w, len(wl.vertices))
    err = np.abs(grad - ref)
    comp = float((err / np.maximum(np.abs(ref), 1e-2 * np.abs(ref).max())).max())
    norm = float(np.linalg.norm(grad - ref) / np.linalg.norm(ref))
    return comp, norm, w


def test_random_triangles_and_outside_faces(orc):
    v, f = geomgen.random_triangles(300, 9, 0.05, 0.95, 0.08)
    v = v.copy()
    v[:30] += np.float32(0.9)  # some faces stick out of the domain
    wl = geomgen.Workload("rand", 3, v, f, (3, 3, 3), 2, 10, 27)
    _full(orc, wl)


def test_adjoint_dense_link_queues(orc):
    """A soup of large triangles cuts many directions per node, so the adjoint's per-wave link queues hold up
    to 4 x 64 + 63 links between takes (regression: a take moved only 64 of the waiting links, losing some
    and repeating others).  Every link is weighted; the GPU gradient must match the FP64 adjoint."""
    v, f = geomgen.random_triangles(600, 9, 0.05, 0.95, 0.15)
    wl = geomgen.Workload("soup", 3, v, f, (3, 3, 3), 2, 10, 27)
    g, of, lk = _full(orc, wl)
    coords = orc.gather(wl.dim, wl.vertices, wl.faces)
    comp, norm, w = _adjoint_all_links(orc, wl, g, of, lk, coords)
    qmax = _max_adjoint_queue(g["face"], w)
    log(f"  adjoint, all {int((w != 0).sum())} links weighted: max component rel {comp:.2e}, norm rel {norm:.2e}; "
        f"longest link queue {qmax}")
    assert qmax > 128   # the workload does exercise long queues
    assert comp <= 1e-3 and norm <= 1e-4


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


@pytest.mark.parametrize("limit", [0, 4096])
def test_cell_centric_and_mixed_flag_steps(orc, limit):
    """The flag step one wave per block (limit 0: every level) or mixed (levels
    whose block grid exceeds 4096 positions cell-centric, the rest face-centric):
    the same bit-exact forest as the oracle."""
    import paper_2502_16310_amd as agal
    ctx = agal.Context()
    ctx.set_flag_table_limit(limit)
    for wl in (_small_sphere(3, 8, 3, 16, 19), geomgen.workload("C0")):
        log(f"case {wl.name} flag table limit {limit}: roots {wl.roots[:wl.dim]} L {wl.levels}")
        g = gpu_run(wl, with_links=False, ctx=ctx)
        coords = orc.gather(wl.dim, wl.vertices, wl.faces)
        ob = orc.bin_faces(wl.dim, coords, wl.lo[:wl.dim], wl.hi[:wl.dim], wl.bins)
        of = orc.refine(wl.dim, coords, ob, wl.roots[:wl.dim], wl.levels, wl.d_spec(), wl.lo[:wl.dim],
                        wl.hi[:wl.dim])
        compare_forest(g, of, wl.levels)


def test_large_faces_flag_steps(orc):
    """A 12-triangle box much larger than the cells: level 0 takes the face-centric step,
    levels 1 and 2 the cell-centric one (a face would have more than 4096 candidate cells);
    the forest is the oracle's, bit for bit."""
    v, f = geomgen.box_mesh()
    wl = geomgen.Workload("box-L3", 3, v, f, (4, 4, 4), 3, 8, 19)
    log(f"case {wl.name}: faces {len(wl.faces)} roots {wl.roots} L {wl.levels}")
    g = gpu_run(wl, with_links=False)
    coords = orc.gather(3, wl.vertices, wl.faces)
    ob = orc.bin_faces(3, coords, wl.lo, wl.hi, wl.bins)
    of = orc.refine(3, coords, ob, wl.roots, wl.levels, wl.d_spec(), wl.lo, wl.hi)
    compare_forest(g, of, wl.levels)
    assert int(g["levels"][2]["cell_flag"].sum()) > 0


def test_sphere_81920_faces_flags_exact(orc):
    """81,920 faces: the face-centric step runs 8 faces per wave on a 256-CU device (4 on the
    small cases, 16 on the 327,680-face body); the forest is the oracle's, bit for bit."""
    v, f = geomgen.icosphere(6, 0.2)
    wl = geomgen.Workload("ico6", 3, v, f, (8, 8, 8), 2, 32, 19)
    log(f"case {wl.name}: faces {len(wl.faces)} roots {wl.roots} L {wl.levels}")
    g = gpu_run(wl, with_links=False)
    coords = orc.gather(3, wl.vertices, wl.faces)
    ob = orc.bin_faces(3, coords, wl.lo, wl.hi, wl.bins)
    compare_bins(g, ob)
    of = orc.refine(3, coords, ob, wl.roots, wl.levels, wl.d_spec(), wl.lo, wl.hi)
    compare_forest(g, of, wl.levels)


def test_link_staging_round_wider_than_staging_area(orc):
    """400 small triangles packed near one point and 4 bins per axis: one round of 64
    candidates keeps every one of them, more than the 32 faces the link kernel stages at a
    time, so a round is staged in pieces.  Links and q against the oracle."""
    v, f = geomgen.random_triangles(400, 5, 0.47, 0.53, 0.01)
    wl = geomgen.Workload("packed400", 3, v, f, (4, 4, 4), 2, 4, 19)
    _full(orc, wl)


def test_run_twice_bitwise_equal(orc):
    wl = _small_sphere(3, 4, 2, 16, 27)
    a = gpu_run(wl)
    b = gpu_run(wl)
    for k in ("offsets", "ids", "key", "q", "face"):
        assert np.array_equal(a[k], b[k]), k
    for la, lb in zip(a["levels"], b["levels"]):
        for k in ("keys", "leaf", "mark"):
            assert np.array_equal(la[k], lb[k])
