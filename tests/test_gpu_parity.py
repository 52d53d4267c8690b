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
    # B = 1 is the naive all-faces search (one bin of 1,280 ids: still one LDS rank sort)
    _full(orc, _small_sphere(3, 4, 2, 16), B=B)


@pytest.mark.parametrize("s,B", [(4, 1), (4, 2), (5, 2), (5, 3)])
def test_oversized_bins_csr_exact(orc, s, B):
    """Bins and 64-bin groups holding more than the 2,048 ids one LDS rank sort takes: s=4, B=1 puts
    5,120 ids in one bin (the ordered sweep over all faces); s=4, B=2 gives a group of eight bins above
    2,048 ids whose bins fit one by one; s=5 at B=2 and 3 gives several oversized bins at once.  The
    CSR is compared with the oracle's, bit for bit, and the forest as well."""
    v, f = geomgen.icosphere(s, 0.2)
    wl = geomgen.Workload(f"ico{s}-B{B}", 3, v, f, (2, 2, 2), 2, B, 19)
    log(f"case {wl.name}: faces {len(wl.faces)} B {B}")
    g = gpu_run(wl, with_links=False)
    coords = orc.gather(3, wl.vertices, wl.faces)
    ob = orc.bin_faces(3, coords, wl.lo, wl.hi, B)
    counts = np.diff(ob.offsets.astype(np.int64))
    groups = np.add.reduceat(counts, np.arange(0, len(counts), 64))
    log(f"  largest bin {counts.max()} ids, largest 64-bin group {groups.max()} ids")
    assert groups.max() > 2048
    compare_bins(g, ob)
    of = orc.refine(3, coords, ob, wl.roots, wl.levels, wl.d_spec(), wl.lo, wl.hi)
    compare_forest(g, of, wl.levels)


@pytest.mark.parametrize("lo,hi", [(5 / 16, 11 / 16), (81 / 256, 175 / 256)])
def test_box_links_exact_ties_and_grazing(orc, lo, hi):
    """An axis-aligned box of 12 triangles with dyadic corners: links through the shared diagonal edges
    and corners tie exactly between faces, links parallel to a face have det == 0, and with the faces at
    odd multiples of half a finest cell (second case: finest cells of 1/128, centres at odd multiples of
    1/256) cell centres lie on the faces (t = 0) or one cell away (t = 1).  Links, q and face ids
    against the oracle, ties checked."""
    v, f = geomgen.box_mesh((lo,) * 3, (hi,) * 3)
    for Q in (19, 27):
        wl = geomgen.Workload(f"box-Q{Q}", 3, v, f, (4, 4, 4), 3, 16, Q)
        g, of, lk = _full(orc, wl)
        qs = lk.q[lk.face >= 0]
        log(f"  q = 0: {int((qs == 0).sum())}, q = 1: {int((qs == 1).sum())}")


def test_square_links_2d_exact(orc):
    """2D: an axis-aligned square of 4 segments with dyadic corners on finest-level cell centres (exact
    ties at the corners, den == 0 for links along a side, t = 0 and t = 1)."""
    v, f = geomgen.square_loop((81 / 256, 81 / 256), (175 / 256, 175 / 256))
    wl = geomgen.Workload("square", 2, v, f, (4, 4, 1), 3, 16, 9)
    _full(orc, wl)


def test_degenerate_faces(orc):
    """Zero-area triangles mixed into a soup: all three corners equal, two equal, and three distinct
    (nearly) collinear corners.  Bins, flags, links and q against the oracle (a degenerate face meets the
    separating-axis test through its box axes and edge axes only, and links through it have det == 0)."""
    v, f = geomgen.random_triangles(240, 12, 0.1, 0.9, 0.08)
    v = v.reshape(-1, 3, 3).copy()
    v[0::4, 1] = v[0::4, 0]                               # two corners equal
    v[1::4, 1] = v[1::4, 0]
    v[1::4, 2] = v[1::4, 0]                               # all three equal
    v[2::4, 2] = v[2::4, 0] + np.float32(2.0) * (v[2::4, 1] - v[2::4, 0])   # collinear up to FP32 rounding
    wl = geomgen.Workload("degenerate", 3, v.reshape(-1, 3).astype(np.float32), f, (3, 3, 3), 2, 8, 27)
    _full(orc, wl)
    v2, f2 = geomgen.random_segments(120, 13, 0.1, 0.9, 0.08)
    v2 = v2.reshape(-1, 2, 2).copy()
    v2[0::3, 1] = v2[0::3, 0]                             # zero-length segments
    wl2 = geomgen.Workload("degenerate-2d", 2, v2.reshape(-1, 2), f2, (4, 4, 1), 3, 8, 9)
    _full(orc, wl2)


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


def test_sphere_c1_full(orc):
    """The 20,480-face sphere in full: bins and flags bit-exact, every finest-level block's links."""
    wl = geomgen.workload("C1")
    log(f"case C1: faces {len(wl.faces)}")
    g = gpu_run(wl)
    coords = orc.gather(3, wl.vertices, wl.faces)
    ob = orc.bin_faces(3, coords, (0, 0, 0), (1, 1, 1), wl.bins)
    compare_bins(g, ob)
    of = orc.refine(3, coords, ob, wl.roots, wl.levels, wl.d_spec(), (0, 0, 0), (1, 1, 1))
    compare_forest(g, of, wl.levels)
    lk = orc.link_fractions(3, coords, ob, of, wl.lattice)
    rep, arrs = compare_links(g, lk)
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


def _adjoint_2d_case(orc, wl):
    import torch
    g, of, lk = _full(orc, wl)
    coords = orc.gather(2, wl.vertices, wl.faces)
    comp, norm, w = _adjoint_all_links(orc, wl, g, of, lk, coords)
    log(f"  2D adjoint, {int((w != 0).sum())} links weighted: max component rel {comp:.2e}, norm rel {norm:.2e}")
    assert comp <= 1e-3 and norm <= 1e-4
    return g, of, lk, coords


def test_adjoint_2d_against_oracle(orc):
    """D2Q9 backward: every link of the circle and of a segment soup weighted, against the FP64 adjoint
    (pinned by the closed-form segment and 2D finite differences)."""
    _adjoint_2d_case(orc, geomgen.workload("C0"))
    v, f = geomgen.random_segments(200, 10, 0.05, 0.95, 0.1)
    _adjoint_2d_case(orc, geomgen.Workload("rseg", 2, v, f, (5, 3, 1), 3, 9, 9))


def test_adjoint_2d_against_finite_differences(orc):
    """Jittered 96-segment circle: the GPU's D2Q9 gradient on the links stable under the step against
    central differences of the FP64 oracle at h = 1e-5."""
    import torch
    n = 96
    th = 2 * np.pi * np.arange(n) / n
    v64 = geomgen.jitter_fp64(np.stack([0.5 + 0.25 * np.cos(th), 0.5 + 0.25 * np.sin(th)], 1), 1e-3, 1)
    v = v64.astype(np.float32)
    f = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1).astype(np.int32)
    wl = geomgen.Workload("j2", 2, v, f, (4, 4, 1), 3, 16, 9)
    g = gpu_run(wl)
    r = orc.run_plain(wl)
    fo, lk, bins, coords = r["forest"], r["links"], r["bins"], r["coords"]
    assert np.array_equal(g["key"], lk.key)
    stable = orc.link_stable(fo, lk, coords, bins, h=1e-5)
    w = geomgen.weights(lk.n * 9, 2).astype(np.float64).reshape(lk.n, 9)
    w[~stable | (g["face"] != lk.face)] = 0.0
    geom, bins_h, forest_h, links_h = g["handles"]
    grad = links_h.backward(torch.from_numpy(w.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    fd, nch = orc.fd_grad(fo, lk, wl.vertices, wl.faces, bins, w, h=1e-5)
    assert nch == 0
    err = np.abs(grad - fd)
    scale = np.maximum(np.abs(fd), 1e-2 * np.abs(fd).max())
    comp = float((err / scale).max())
    norm = float(np.linalg.norm(grad - fd) / np.linalg.norm(fd))
    log(f"  2D GPU vs FD h=1e-5 on {int((w != 0).sum())} stable links: max component {comp:.2e}, norm {norm:.2e}")
    assert comp <= 1e-3 and norm <= 1e-3


def test_error_conventions():
    """The plain calls reject invalid input with AGAL_EINVAL and leave no handle behind: a NaN or an Inf
    coordinate, a face index out of range, an unknown lattice or one that does not match the dimension,
    B < 1, hi <= lo, a negative distance and a key space overflow."""
    import torch
    import paper_2502_16310_amd as agal
    dev = torch.device("cuda", 0)
    ctx = agal.agal_context_create()
    stream = torch.cuda.current_stream().cuda_stream
    v, f = geomgen.icosphere(1, 0.2)

    def imp(vv, ff, dim=3):
        vt = torch.from_numpy(np.ascontiguousarray(vv)).to(dev)
        ft = torch.from_numpy(np.ascontiguousarray(ff)).to(dev)
        return agal.agal_import_faces(ctx, dim, vt.data_ptr(), vt.shape[0], ft.data_ptr(), ft.shape[0], stream)

    def einval(fn, what):
        with pytest.raises(agal.AgalError) as e:
            fn()
        assert e.value.status == agal.AGAL_EINVAL, (what, e.value)
        log(f"  {what}: {e.value}")

    for bad in (np.nan, np.inf, -np.inf):
        vb = v.copy()
        vb[7, 1] = bad
        einval(lambda: imp(vb, f), f"vertex coordinate {bad}")
    fb = f.copy()
    fb[3, 2] = len(v)
    einval(lambda: imp(v, fb), "index == n_vertices")
    fb[3, 2] = -1
    einval(lambda: imp(v, fb), "negative index")
    einval(lambda: imp(v, f, dim=4), "dim 4")
    g = imp(v, f)   # the context is still usable after the failures
    einval(lambda: agal.agal_bin_faces(g, (0, 0, 0), (1, 1, 1), 0, stream), "B = 0")
    einval(lambda: agal.agal_bin_faces(g, (0, 0, 0), (1, 0, 1), 8, stream), "hi <= lo")
    b = agal.agal_bin_faces(g, (0, 0, 0), (1, 1, 1), 8, stream)
    einval(lambda: agal.agal_near_wall_refine(g, b, agal.forest_desc(3, (4, 4, 4), 2, [0.01, -0.01], (0, 0, 0),
                                                                      (1, 1, 1)), stream), "negative d_spec")
    einval(lambda: agal.agal_near_wall_refine(g, b, agal.forest_desc(2, (4, 4), 2, [0.01, 0.01], (0, 0), (1, 1)),
                                              stream), "forest dim 2 over 3D faces")
    einval(lambda: agal.agal_near_wall_refine(g, b, agal.forest_desc(3, (1024, 1024, 1024), 2, [0.01, 0.01],
                                                                      (0, 0, 0), (1, 1, 1)), stream),
           "key space overflow")
    fo = agal.agal_near_wall_refine(g, b, agal.forest_desc(3, (4, 4, 4), 2, [1 / 16, 1 / 32], (0, 0, 0), (1, 1, 1)),
                                    stream)
    einval(lambda: agal.agal_link_fractions(g, b, fo, agal.AGAL_D2Q9, stream), "D2Q9 on a 3D forest")
    einval(lambda: agal.agal_link_fractions(g, b, fo, 15, stream), "unknown lattice")
    lk = agal.agal_link_fractions(g, b, fo, agal.AGAL_D3Q19, stream)
    assert agal.agal_links_view(lk)[3] > 0
    for h, fn in ((lk, agal.agal_destroy_links), (fo, agal.agal_destroy_forest), (b, agal.agal_destroy_bins),
                  (g, agal.agal_destroy_geom)):
        fn(h)
    agal.agal_context_destroy(ctx)
    torch.cuda.synchronize()


def test_views_alias_library_memory_and_torch_allocator():
    """Result tensors are views of the library's arrays (no copy) that keep their handle alive, and the
    default context takes its device memory from torch's caching allocator."""
    import gc
    import torch
    import paper_2502_16310_amd as agal
    wl = _small_sphere(3, 4, 2, 16, 19)
    v = torch.from_numpy(wl.vertices).cuda()
    f = torch.from_numpy(wl.faces).cuda()
    cfg = agal.NearWallConfig(dim=3, roots=wl.roots, n_levels=wl.levels, bins=wl.bins, lattice=wl.lattice)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    geom, bins, forest, links = agal.near_wall(v, f, cfg, ctx=agal.Context())
    key, q, face = links.tensors()
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - before
    k_p, q_p, f_p, n, Q = agal.agal_links_view(links.h)
    assert (key.data_ptr(), q.data_ptr(), face.data_ptr()) == (k_p, q_p, f_p)
    assert held >= n * (8 + 8 * Q), "library memory is not counted by torch's allocator"
    ref = (key.cpu().clone(), q.cpu().clone(), face.cpu().clone())
    del geom, bins, forest, links
    gc.collect()
    junk = torch.full((1 << 22,), -3.0, device="cuda")   # reuses freed blocks, if any were freed
    torch.cuda.synchronize()
    assert torch.equal(key.cpu(), ref[0]) and torch.equal(q.cpu(), ref[1]) and torch.equal(face.cpu(), ref[2])
    log(f"  {n} nodes viewed in place; torch's allocator holds {held} bytes for the pass")
    del junk
    # the library's own pool: nothing is counted by torch
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    h = agal.near_wall(v, f, cfg, ctx=agal.Context(torch_allocator=False))
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before < n * (8 + 8 * Q)
    del h
