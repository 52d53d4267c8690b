"""Pins for the CPU oracle: each check compares it with something other than
itself -- exact rational geometry, closed forms, brute force, invariants --
chosen so that a dropped term, a wrong sign or index, or a transposed
operand in the oracle fails at least one of them."""
import itertools
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import geomgen
from _exact import (aabb_meets_box, exact_bin, face_meets_box, fr, near_integer, plane_meets_box,
                    segment_segment, segment_triangle)


# ---------------------------------------------------------------------------
# Lattices
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("Q,dim", [(9, 2), (19, 3), (27, 3)])
def test_lattice_sets(orc, Q, dim):
    c = orc.lattice(Q)
    assert c.shape == (Q, 3)
    assert (c[0] == 0).all()
    vecs = {tuple(int(x) for x in v[:dim]) for v in c}
    full = set(itertools.product((-1, 0, 1), repeat=dim))
    if Q == 19:
        full = {v for v in full if sum(x * x for x in v) <= 2}
    assert vecs == full and len(vecs) == Q
    for i in range(1, Q, 2):
        assert (c[i] == -c[i + 1]).all(), "directions come in +/- pairs"
    n2 = (c.astype(int) ** 2).sum(1)
    assert (np.diff(n2) >= 0).all(), "axis, then edge, then corner directions"
    if dim == 2:
        assert (c[:, 2] == 0).all()
    # D3Q19 is the head of D3Q27
    if Q == 19:
        assert (orc.lattice(27)[:19] == c).all()


# ---------------------------------------------------------------------------
# Import and bins
# ---------------------------------------------------------------------------
def test_gather_matches_index_lists(orc):
    v, f = geomgen.icosphere(1)
    coords = orc.gather(3, v, f)
    assert coords.shape == (f.shape[0], 3, 3)
    assert np.array_equal(coords, v[f])


def _csr_members(bins, F):
    seg_bins = np.repeat(np.arange(bins.nb), bins.count.astype(np.int64))
    order = np.lexsort((seg_bins, bins.ids))
    ids_s, bins_s = bins.ids[order], seg_bins[order]
    starts = np.searchsorted(ids_s, np.arange(F + 1))
    return [bins_s[starts[f]:starts[f + 1]] for f in range(F)]


def _check_bins_exact(orc, dim, coords, lo, hi, B, max_ambiguous_frac=0.01):
    lo = np.asarray(lo, dtype=np.float32)
    hi = np.asarray(hi, dtype=np.float32)
    bins = orc.bin_faces(dim, coords, lo, hi, B)
    F = coords.shape[0]
    assert bins.nb == B ** dim
    assert bins.offsets[0] == 0 and bins.offsets[-1] == bins.P
    assert np.array_equal(np.diff(bins.offsets.astype(np.int64)), bins.count.astype(np.int64))
    for b in np.nonzero(bins.count > 1)[0]:
        seg = bins.ids[bins.offsets[b]:bins.offsets[b + 1]]
        assert (np.diff(seg) > 0).all(), "face ids ascend inside a bin"
    members = _csr_members(bins, F)
    ambiguous = 0
    total = 0
    for f in range(F):
        rngs, amb = [], False
        for a in range(dim):
            mn, mx = coords[f, :, a].min(), coords[f, :, a].max()
            amb |= near_integer(mn, lo[a], hi[a], B) or near_integer(mx, lo[a], hi[a], B)
            rngs.append(range(exact_bin(mn, lo[a], hi[a], B), exact_bin(mx, lo[a], hi[a], B) + 1))
        if amb:
            ambiguous += 1
            continue
        if dim == 2:
            exp = sorted(y * B + x for y in rngs[1] for x in rngs[0])
        else:
            exp = sorted((z * B + y) * B + x for z in rngs[2] for y in rngs[1] for x in rngs[0])
        total += len(exp)
        assert list(members[f]) == exp, f"face {f}"
    assert ambiguous <= max_ambiguous_frac * F + 2
    return bins, ambiguous


def test_bins_exact_circle(orc):
    wl = geomgen.workload("C0")
    coords = orc.gather(2, wl.vertices, wl.faces)
    _check_bins_exact(orc, 2, coords, (0.0, 0.0), (1.0, 1.0), 32)


def test_bins_exact_sphere_nondyadic_domain(orc):
    # a non-dyadic domain and bin count make the FP32 index arithmetic round
    v, f = geomgen.icosphere(3)
    coords = orc.gather(3, v, f)
    _check_bins_exact(orc, 3, coords, (0.1, -0.05, 0.03), (0.93, 1.1, 0.97), 37)


def test_bins_clamp_faces_outside_domain(orc):
    # faces partly or wholly outside [lo, hi] land in the edge bins
    v = np.array([[-0.5, 0.2, 0.3], [-0.4, 0.25, 0.3], [-0.45, 0.2, 0.35],
                  [0.9, 0.9, 0.9], [1.7, 0.95, 0.9], [0.95, 0.9, 1.2]], dtype=np.float32)
    f = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    coords = orc.gather(3, v, f)
    bins = orc.bin_faces(3, coords, (0, 0, 0), (1, 1, 1), 4)
    m = _csr_members(bins, 2)
    # face 0: x clamps to bin 0; y = 0.2..0.25 -> bin 0..1, z = 0.3..0.35 -> bin 1
    assert list(m[0]) == [(1 * 4 + 0) * 4 + 0, (1 * 4 + 1) * 4 + 0]
    # face 1: x 0.9..1.7 -> bin 3; y 0.9..0.95 -> 3; z 0.9..1.2 -> 3
    assert list(m[1]) == [(3 * 4 + 3) * 4 + 3]


# ---------------------------------------------------------------------------
# Separating-axis predicate vs exact clipping
# ---------------------------------------------------------------------------
def _sat_cases_3d(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        m = rng.uniform(0.25, 0.75, 3).astype(np.float32)
        h = np.float32(rng.uniform(0.002, 0.05))
        tri = (m + rng.uniform(-3, 3, (3, 3)) * h).astype(np.float32)
        yield tri, m, h


def test_sat_3d_vs_exact_clipping(orc):
    cats = {"aabb": 0, "plane": 0, "edge": 0, "meet": 0}
    skipped = 0
    for tri, m, h in _sat_cases_3d(2500, 11):
        ex = face_meets_box(tri, m, h)
        lo = face_meets_box(tri, m, float(h) * (1 - 1e-4))
        hi = face_meets_box(tri, m, float(h) * (1 + 1e-4))
        if lo != hi:
            skipped += 1
            continue
        got = orc.sat(3, tri, m, float(h))
        assert got == ex, (tri.tolist(), m.tolist(), float(h))
        if ex:
            cats["meet"] += 1
        elif not aabb_meets_box(tri, m, h):
            cats["aabb"] += 1
        elif not plane_meets_box(tri, m, h):
            cats["plane"] += 1
        else:
            cats["edge"] += 1
    # every kind of separating axis must have been exercised
    assert min(cats.values()) >= 20, cats
    assert skipped < 50


def test_sat_2d_vs_exact_clipping(orc):
    rng = np.random.default_rng(12)
    cats = {"aabb": 0, "line": 0, "meet": 0}
    for _ in range(3000):
        m = rng.uniform(0.25, 0.75, 2).astype(np.float32)
        h = np.float32(rng.uniform(0.002, 0.05))
        seg = (m + rng.uniform(-3, 3, (2, 2)) * h).astype(np.float32)
        ex = face_meets_box(seg, m, h)
        if face_meets_box(seg, m, float(h) * (1 - 1e-4)) != face_meets_box(seg, m, float(h) * (1 + 1e-4)):
            continue
        assert orc.sat(2, seg, m, float(h)) == ex, (seg.tolist(), m.tolist(), float(h))
        if ex:
            cats["meet"] += 1
        elif not aabb_meets_box(seg, m, h):
            cats["aabb"] += 1
        else:
            cats["line"] += 1
    assert min(cats.values()) >= 20, cats


def test_sat_closed_sets_touching(orc):
    """Closed sets: a face touching the cube at one point or along an edge meets it; one
    FP32 step further away it does not."""
    m = np.array([0.5, 0.5, 0.5], dtype=np.float32)
    h = 0.125
    x = np.float32(0.625)
    tri = np.array([[x, 0.5, 0.5], [0.8, 0.55, 0.45], [0.8, 0.45, 0.55]], dtype=np.float32)
    assert orc.sat(3, tri, m, h)
    tri2 = tri.copy()
    tri2[0, 0] = np.nextafter(x, np.float32(1))
    assert not orc.sat(3, tri2, m, h)
    # plane through a box corner, tilted: touches only at the corner (0.625, 0.625, 0.625)
    c = np.float32(0.625)
    tri3 = np.array([[c + 0.25, c - 0.125, c - 0.125], [c - 0.125, c + 0.25, c - 0.125],
                     [c - 0.125, c - 0.125, c + 0.25]], dtype=np.float32)  # plane x+y+z = 3c
    assert face_meets_box(tri3, m, h)
    assert orc.sat(3, tri3, m, h)
    tri4 = tri3 + np.float32(1.0 / 1024)
    assert not face_meets_box(tri4, m, h)
    assert not orc.sat(3, tri4, m, h)
    # 2D: segment touching a corner
    seg = np.array([[0.625, 0.75], [0.75, 0.625]], dtype=np.float32)  # line x + y = 1.375
    m2 = np.array([0.5, 0.5], dtype=np.float32)
    assert not orc.sat(2, seg, m2, h)
    seg2 = np.array([[0.5, 0.75], [0.75, 0.5]], dtype=np.float32)  # x + y = 1.25 hits corner
    assert orc.sat(2, seg2, m2, h)


def test_algorithm1_sandwich(orc):
    """L2-near(d) => closed-box predicate(d) => L2-near(sqrt(D) d)."""
    for tri, m, h in _sat_cases_3d(1500, 21):
        s = orc.sat(3, tri, m, float(h))
        near = orc.near_face_l2(3, tri.astype(np.float64), m.astype(np.float64), float(h) * (1 - 1e-5))
        far = orc.near_face_l2(3, tri.astype(np.float64), m.astype(np.float64), float(h) * math.sqrt(3) * (1 + 1e-5))
        if near:
            assert s
        if s:
            assert far


def test_algorithm1_known_distances(orc):
    """Points at a constructed distance from a triangle's interior, an edge and a vertex."""
    rng = np.random.default_rng(5)
    for _ in range(300):
        tri = rng.uniform(0, 1, (3, 3))
        n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
        n /= np.linalg.norm(n)
        lam = rng.dirichlet([1, 1, 1]) * 0.7 + 0.1
        lam /= lam.sum()
        q = lam @ tri
        s = rng.uniform(0.01, 0.2)
        p = q + s * n * rng.choice([-1, 1])
        assert orc.near_face_l2(3, tri, p, s * (1 + 1e-9))
        assert not orc.near_face_l2(3, tri, p, s * (1 - 1e-9))
    # beyond vertex 0 along the outward bisector direction
    tri = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    p = np.array([-0.3, -0.4, 0.0])
    assert orc.near_face_l2(3, tri, p, 0.5 * (1 + 1e-9)) and not orc.near_face_l2(3, tri, p, 0.5 * (1 - 1e-9))
    # beside the hypotenuse edge
    p = np.array([0.5 + 0.3, 0.5 + 0.3, 0.0])
    d = 0.3 * math.sqrt(2)
    assert orc.near_face_l2(3, tri, p, d * (1 + 1e-9)) and not orc.near_face_l2(3, tri, p, d * (1 - 1e-9))
    seg = np.array([[0.0, 0.0], [1.0, 0.0]])
    assert orc.near_face_l2(2, seg, [0.5, 0.2], 0.2 * (1 + 1e-9))
    assert not orc.near_face_l2(2, seg, [0.5, 0.2], 0.2 * (1 - 1e-9))
    assert orc.near_face_l2(2, seg, [1.3, 0.4], 0.5 * (1 + 1e-9))
    assert not orc.near_face_l2(2, seg, [1.3, 0.4], 0.5 * (1 - 1e-9))


# ---------------------------------------------------------------------------
# Refinement
# ---------------------------------------------------------------------------
def _small_sphere(s=2, R=4, L=3, B=16):
    v, f = geomgen.icosphere(s, 0.2)
    return geomgen.Workload("small", 3, v, f, (R, R, R), L, B, 19)


def _forest(orc, wl, B=None, brute=False):
    coords = orc.gather(wl.dim, wl.vertices, wl.faces)
    bins = orc.bin_faces(wl.dim, coords, wl.lo[:wl.dim], wl.hi[:wl.dim], B or wl.bins)
    fo = orc.refine(wl.dim, coords, None if brute else bins, wl.roots[:wl.dim], wl.levels, wl.d_spec(),
                    wl.lo[:wl.dim], wl.hi[:wl.dim])
    return coords, bins, fo


def _forest_equal(a, b):
    for la, lb in zip(a.levels, b.levels):
        for k in ("keys", "leaf", "mark", "cell_flag"):
            assert np.array_equal(la[k], lb[k]), k


def test_binned_equals_brute_force_and_bin_invariance(orc):
    wl = _small_sphere()
    _, _, ref = _forest(orc, wl, brute=True)
    for B in (1, 4, 16, 37):
        _, _, fo = _forest(orc, wl, B=B)
        _forest_equal(ref, fo)
    wl2 = geomgen.workload("C0")
    _, _, ref2 = _forest(orc, wl2, brute=True)
    for B in (1, 8, 32):
        _, _, fo2 = _forest(orc, wl2, B=B)
        _forest_equal(ref2, fo2)


def decode_keys(keys, level, roots, dim):
    """Block coordinates at ``level`` from hierarchical keys."""
    keys = keys.astype(np.int64)
    nch = 1 << dim
    path = np.zeros((len(keys), 3), dtype=np.int64)
    k = keys.copy()
    for j in range(level):
        ci = k % nch
        k //= nch
        for a in range(dim):
            path[:, a] |= ((ci >> a) & 1) << j
    r = np.stack([k % roots[0], (k // roots[0]) % roots[1], k // (roots[0] * roots[1])], 1)
    return (r << level) | path


def _leaf_level_map(fo, roots, dim):
    L = fo.L
    n = [roots[a] << L for a in range(dim)] + [1] * (3 - dim)
    lvl = -np.ones(n[::-1], dtype=np.int64)  # indexed [z, y, x]
    for l, lv in enumerate(fo.levels):
        c = decode_keys(lv["keys"], l, roots, dim)
        s = 1 << (L - l)
        for (x, y, z), leaf in zip(c, lv["leaf"]):
            if leaf:
                zz = slice(z * s, (z + 1) * s) if dim == 3 else slice(0, 1)
                lvl[zz, y * s:(y + 1) * s, x * s:(x + 1) * s] = l
    return lvl


def _check_balance(lvl, dim):
    assert (lvl >= 0).all(), "leaves tile the domain"
    offs = [o for o in itertools.product((-1, 0, 1), repeat=3) if any(o)]
    if dim == 2:
        offs = [o for o in offs if o[0] == 0]
    Z, Y, X = lvl.shape
    for dz, dy, dx in offs:
        a = lvl[max(0, dz):Z + min(0, dz), max(0, dy):Y + min(0, dy), max(0, dx):X + min(0, dx)]
        b = lvl[max(0, -dz):Z + min(0, -dz), max(0, -dy):Y + min(0, -dy), max(0, -dx):X + min(0, -dx)]
        assert np.abs(a - b).max() <= 1, "2:1 balance across faces, edges and corners"


def test_balance_and_structure(orc):
    for wl in (_small_sphere(), geomgen.workload("C0"), _small_sphere(3, 4, 3, 16)):
        _, _, fo = _forest(orc, wl)
        roots = wl.roots
        _check_balance(_leaf_level_map(fo, roots, wl.dim), wl.dim)
        for l, lv in enumerate(fo.levels):
            assert (np.diff(lv["keys"].astype(np.int64)) > 0).all(), "keys sorted, unique"
            flagged = lv["cell_flag"].any(1)
            assert np.array_equal(flagged, lv["mark"] == 1), "mark 1 = OR of cell flags"
            assert np.array_equal(lv["leaf"] == 0, lv["mark"] > 0), "refined iff marked"
            if l < fo.L:
                nxt = fo.levels[l + 1]["keys"].astype(np.int64)
                parents = np.unique(nxt >> (3 if wl.dim == 3 else 2))
                assert np.array_equal(parents, lv["keys"][lv["leaf"] == 0].astype(np.int64))
            else:
                assert (lv["leaf"] == 1).all() and (lv["mark"] == 0).all()


def _closure_forest(fo, roots, dim):
    """Order-independent closure: per pass, refine the flagged blocks, then keep refining any
    leaf that touches a leaf two or more levels finer, until none does."""
    L = fo.L
    leaves = {(0, tuple(c)) for c in decode_keys(fo.levels[0]["keys"], 0, roots, dim)}

    def paint():
        n = [roots[a] << L for a in range(dim)] + [1] * (3 - dim)
        lvl = -np.ones(n[::-1], dtype=np.int64)
        for l, (x, y, z) in leaves:
            s = 1 << (L - l)
            zz = slice(z * s, (z + 1) * s) if dim == 3 else slice(0, 1)
            lvl[zz, y * s:(y + 1) * s, x * s:(x + 1) * s] = l
        return lvl

    def split(l, c):
        leaves.discard((l, c))
        for ci in range(1 << dim):
            cc = tuple(2 * c[a] + ((ci >> a) & 1) if a < dim else 0 for a in range(3))
            leaves.add((l + 1, cc))

    for p in range(L):
        lv = fo.levels[p]
        cs = decode_keys(lv["keys"], p, roots, dim)
        for c, mk in zip(cs, lv["mark"]):
            if mk == 1:
                split(p, tuple(int(x) for x in c))
        while True:
            lvl = paint()
            bad = None
            for l, c in sorted(leaves):
                s = 1 << (L - l)
                lo = [c[a] * s - 1 if a < dim else 0 for a in range(3)]
                hi = [(c[a] + 1) * s + 1 if a < dim else 1 for a in range(3)]
                sub = lvl[max(0, lo[2]):hi[2], max(0, lo[1]):hi[1], max(0, lo[0]):hi[0]]
                if sub.max() >= l + 2:
                    bad = (l, c)
                    break
            if bad is None:
                break
            split(*bad)
    return leaves


def test_balance_is_minimal_closure(orc):
    for wl in (_small_sphere(2, 2, 3, 8), geomgen.workload("C0")):
        _, _, fo = _forest(orc, wl)
        leaves = _closure_forest(fo, wl.roots, wl.dim)
        got = set()
        for l, lv in enumerate(fo.levels):
            for c, leaf in zip(decode_keys(lv["keys"], l, wl.roots, wl.dim), lv["leaf"]):
                if leaf:
                    got.add((l, tuple(int(x) for x in c)))
        assert got == leaves


def _cell_centres(keys, level, roots, dim, dx):
    c = decode_keys(keys, level, roots, dim)
    cells = 64 if dim == 3 else 16
    ci = np.arange(cells)
    off = np.stack([ci & 3, (ci >> 2) & 3, (ci >> 4) & 3], 1)
    g = 4 * c[:, None, :] + off[None]
    return (2 * g + 1) * (dx / 2.0)  # exact for dyadic dx in float64


def test_flags_closed_form_box_body(orc):
    lo_b, hi_b = 5.0 / 16, 11.0 / 16
    v, f = geomgen.box_mesh((lo_b,) * 3, (hi_b,) * 3)
    wl = geomgen.Workload("box", 3, v, f, (4, 4, 4), 3, 16, 27)
    _, _, fo = _forest(orc, wl)
    for l in range(wl.levels):
        lv = fo.levels[l]
        dx = 1.0 / (4 * 4 * 2 ** l)
        h = float(wl.d_spec()[l])
        m = _cell_centres(lv["keys"], l, wl.roots, 3, dx)
        blo, bhi = m - h, m + h
        meets_k = ((bhi >= lo_b) & (blo <= hi_b)).all(-1)
        inside = ((blo > lo_b) & (bhi < hi_b)).all(-1)
        exp = meets_k & ~inside
        tested = np.zeros(len(lv["keys"]), bool)
        # blocks present at the start of pass l are exactly those with no balance-created origin:
        # all level-l blocks whose parent was flagged (mark 1) at level l-1, or all roots.
        if l == 0:
            tested[:] = True
        else:
            par = fo.levels[l - 1]
            pk = par["keys"][par["mark"] == 1].astype(np.int64)
            tested = np.isin(lv["keys"].astype(np.int64) >> 3, pk)
        assert np.array_equal(lv["cell_flag"][tested].astype(bool), exp[tested])
        assert not lv["cell_flag"][~tested].any()


def test_flags_analytic_sphere(orc):
    u, f = geomgen.icosphere_unit(3)
    r, c0 = 0.2, np.array([0.5, 0.5, 0.5])
    v = (c0 + r * u).astype(np.float32)
    wl = geomgen.Workload("sph", 3, v, f, (8, 8, 8), 2, 32, 19)
    _, _, fo = _forest(orc, wl)
    vv = v.astype(np.float64) - c0
    a, b, c = vv[f[:, 0]], vv[f[:, 1]], vv[f[:, 2]]
    n = np.cross(b - a, c - a)
    dplane = np.abs(np.einsum("ij,ij->i", n, a)) / np.linalg.norm(n, axis=1)
    rmax = np.linalg.norm(vv, axis=1).max()
    rmin = dplane.min()
    checked = 0
    for l in range(wl.levels):
        lv = fo.levels[l]
        dx = 1.0 / (4 * 8 * 2 ** l)
        h = float(wl.d_spec()[l])
        m = _cell_centres(lv["keys"], l, wl.roots, 3, dx) - c0
        near = np.clip(np.abs(m) - h, 0, None)
        far = np.abs(m) + h
        dmin, dmax = np.linalg.norm(near, axis=-1), np.linalg.norm(far, axis=-1)
        flag = lv["cell_flag"].astype(bool)
        must_not = (dmax < rmin * (1 - 1e-6)) | (dmin > rmax * (1 + 1e-6))
        must = (dmin < rmin * (1 - 1e-6)) & (dmax > rmax * (1 + 1e-6))
        if l == 0:
            tmask = np.ones(len(flag), bool)
        else:
            par = fo.levels[l - 1]
            tmask = np.isin(lv["keys"].astype(np.int64) >> 3, par["keys"][par["mark"] == 1].astype(np.int64))
        assert not (flag & must_not)[tmask].any()
        assert flag[must & tmask[:, None]].all()
        checked += int((must | must_not)[tmask].sum())
    assert checked > 10000


# ---------------------------------------------------------------------------
# Link fractions
# ---------------------------------------------------------------------------
def _all_level_forest(orc, dim, v, f, roots, L, Q, B=4):
    wl = geomgen.Workload("t", dim, v, f, tuple(roots) + (1,) * (3 - len(roots)), L, B, Q)
    coords = orc.gather(dim, v, f)
    bins = orc.bin_faces(dim, coords, (0,) * dim, (1,) * dim, B)
    big = np.full(max(L, 1), 4.0, dtype=np.float32)   # flag everything: every block refined
    fo = orc.refine(dim, coords, bins, wl.roots[:dim], L, big, (0,) * dim, (1,) * dim)
    return wl, coords, bins, fo


def test_links_exact_random_triangles(orc):
    v, f = geomgen.random_triangles(8, 3, 0.2, 0.8, 0.25)
    wl, coords, bins, fo = _all_level_forest(orc, 3, v, f, (1, 1, 1), 1, 27)
    lk = orc.link_fractions(3, coords, bins, fo, 27)
    lkb = orc.link_fractions(3, coords, None, fo, 27)
    assert np.array_equal(lk.key, lkb.key) and np.array_equal(lk.face, lkb.face)
    assert np.array_equal(lk.q, lkb.q)
    cvec = orc.lattice(27)
    keys = fo.levels[1]["keys"]
    dx = 1.0 / 8
    m = _cell_centres(keys, 1, (1, 1, 1), 3, dx).reshape(-1, 3)
    node_of = {int(k): i for i, k in enumerate(lk.key)}
    nlinks = 0
    for bi, key in enumerate(keys):
        for cell in range(64):
            o = m[bi * 64 + cell]
            nk = int(key) * 64 + cell
            exp_q, exp_f = [-1.0], [-1]
            for i in range(1, 27):
                D = cvec[i] * dx
                best, bf = None, -1
                for fi in range(len(f)):
                    if ((coords[fi].min(0) > o + np.abs(D) + 1e-9).any()
                            or (coords[fi].max(0) < o - np.abs(D) - 1e-9).any()):
                        continue
                    hit = segment_triangle(o, D, coords[fi])
                    if hit is not None and (best is None or hit[0] < best):
                        best, bf = hit[0], fi
                exp_q.append(-1.0 if best is None else float(best))
                exp_f.append(bf)
            if max(exp_f) < 0:
                assert nk not in node_of
                continue
            n = node_of[nk]
            assert list(lk.face[n]) == exp_f
            ok = np.array(exp_f) >= 0
            assert np.allclose(lk.q[n][ok], np.array(exp_q)[ok], rtol=0, atol=1e-12)
            nlinks += ok.sum()
    assert nlinks > 300


def test_links_exact_random_segments(orc):
    v, f = geomgen.random_segments(12, 4, 0.2, 0.8, 0.25)
    wl, coords, bins, fo = _all_level_forest(orc, 2, v, f, (2, 2), 1, 9)
    lk = orc.link_fractions(2, coords, bins, fo, 9)
    cvec = orc.lattice(9)
    keys = fo.levels[1]["keys"]
    dx = 1.0 / 16
    m = _cell_centres(keys, 1, (2, 2, 1), 2, dx).reshape(-1, 3)
    node_of = {int(k): i for i, k in enumerate(lk.key)}
    nl = 0
    for bi, key in enumerate(keys):
        for cell in range(16):
            o = m[bi * 16 + cell][:2]
            exp_f, exp_q = [-1], [-1.0]
            for i in range(1, 9):
                D = cvec[i][:2] * dx
                best, bf = None, -1
                for fi in range(len(f)):
                    hit = segment_segment(o, D, coords[fi])
                    if hit is not None and (best is None or hit[0] < best):
                        best, bf = hit[0], fi
                exp_q.append(-1.0 if best is None else float(best))
                exp_f.append(bf)
            nk = int(key) * 16 + cell
            if max(exp_f) < 0:
                assert nk not in node_of
                continue
            n = node_of[nk]
            assert list(lk.face[n]) == exp_f
            ok = np.array(exp_f) >= 0
            assert np.allclose(lk.q[n][ok], np.array(exp_q)[ok], atol=1e-12, rtol=0)
            nl += ok.sum()
    assert nl > 100


def test_links_closed_form_box(orc):
    """Dyadic axis-aligned cube: q from the six face planes (closed rectangles), exact."""
    lo_b, hi_b = 5.0 / 16, 11.0 / 16
    v, f = geomgen.box_mesh((lo_b,) * 3, (hi_b,) * 3)
    wl = geomgen.Workload("box", 3, v, f, (4, 4, 4), 2, 8, 27)
    coords, bins, fo = _forest(orc, wl)
    lk = orc.link_fractions(3, coords, bins, fo, 27)
    cvec = orc.lattice(27).astype(np.float64)
    L = wl.levels
    dx = 1.0 / (16 * 2 ** L)
    keys = fo.levels[L]["keys"]
    m = _cell_centres(keys, L, wl.roots, 3, dx).reshape(-1, 3)
    nk = (keys.astype(np.int64)[:, None] * 64 + np.arange(64)[None]).reshape(-1)
    exp = np.full((len(m), 27), -1.0)
    for i in range(1, 27):
        D = cvec[i] * dx
        best = np.full(len(m), np.inf)
        for a in range(3):
            if D[a] == 0:
                continue
            for P in (lo_b, hi_b):
                t = (P - m[:, a]) / D[a]
                hit = m + t[:, None] * D[None]
                ok = (t >= 0) & (t <= 1)
                for b in range(3):
                    if b != a:
                        ok &= (hit[:, b] >= lo_b) & (hit[:, b] <= hi_b)
                best = np.where(ok & (t < best), t, best)
        exp[:, i] = np.where(np.isfinite(best), best, -1.0)
    has = (exp >= 0).any(1)
    assert np.array_equal(lk.key.astype(np.int64), nk[has])
    assert np.array_equal(lk.q, exp[has])
    assert ((lk.face >= 0) == (lk.q >= 0)).all()
    # the face reported is the lowest-numbered triangle containing the hit point (dyadic data:
    # the float64 plane/barycentric arithmetic below is exact)
    mh = m[has]
    tri = v.astype(np.float64)[f]
    nodes, dirs = np.nonzero(lk.q >= 0)
    p = mh[nodes] + lk.q[nodes, dirs][:, None] * (cvec[dirs] * dx)
    expf = np.full(len(nodes), -1)
    for j in range(len(f)):
        a, b, c = tri[j]
        ax = int(np.nonzero((a == b) & (b == c))[0][0])
        u_, w_ = [k for k in range(3) if k != ax]
        on = p[:, ax] == a[ax]
        det = (b[u_] - a[u_]) * (c[w_] - a[w_]) - (b[w_] - a[w_]) * (c[u_] - a[u_])
        l1 = ((p[:, u_] - a[u_]) * (c[w_] - a[w_]) - (p[:, w_] - a[w_]) * (c[u_] - a[u_])) / det
        l2 = ((b[u_] - a[u_]) * (p[:, w_] - a[w_]) - (b[w_] - a[w_]) * (p[:, u_] - a[u_])) / det
        inside = on & (l1 >= 0) & (l2 >= 0) & (l1 + l2 <= 1)
        expf = np.where((expf < 0) & inside, j, expf)
    assert (expf >= 0).all()
    assert np.array_equal(lk.face[nodes, dirs], expf)


def test_links_circle_analytic_and_complementary(orc):
    wl = geomgen.workload("C0")
    r = orc.run_plain(wl)
    lk, fo = r["links"], r["forest"]
    L = wl.levels
    dx = float(wl.cell_size(L))
    cvec = orc.lattice(9).astype(np.float64)[:, :2]
    keys = (lk.key // 16).astype(np.int64)
    cells = (lk.key % 16).astype(np.int64)
    bc = decode_keys(keys, L, wl.roots, 2)
    g = 4 * bc[:, :2] + np.stack([cells & 3, cells >> 2], 1)
    o = (2 * g + 1) * (dx / 2) - 0.5
    R = 0.25
    delta = R * (1 - math.cos(math.pi / 256))
    checked = 0
    for i in range(1, 9):
        D = cvec[i] * dx
        has = lk.face[:, i] >= 0
        # smallest root of |o + t D|^2 = R^2
        a = D @ D
        b = 2 * o @ D
        c = (o * o).sum(1) - R * R
        disc = b * b - 4 * a * c
        sq = np.sqrt(np.clip(disc, 0, None))
        t1, t2 = (-b - sq) / (2 * a), (-b + sq) / (2 * a)
        qi = lk.q[:, i]
        tc = np.where(np.abs(qi - t1) <= np.abs(qi - t2), t1, t2)
        p = o + tc[:, None] * D[None]
        cos = np.abs((p @ D) / (np.linalg.norm(p, axis=1) * np.linalg.norm(D)))
        sliver = np.abs(np.linalg.norm(o, axis=1) - R) <= 2 * delta
        good = has & (cos > 0.1) & (disc > 0) & ~sliver
        tol = 2 * delta / (np.linalg.norm(D) * np.maximum(cos, 1e-3)) + 1e-12
        assert (np.abs(lk.q[good, i] - tc[good]) <= tol[good]).all()
        checked += good.sum()
    assert checked > 3000
    # complementary links: q_i(x) + q_opp(x + c_i dx) = 1 on the same face
    idx = {int(k): n for n, k in enumerate(lk.key)}
    node_g = {tuple(gg): n for gg, n in zip(map(tuple, g), range(len(g)))}
    pairs = 0
    for n in range(lk.n):
        for i in range(1, 9):
            fi = lk.face[n, i]
            if fi < 0:
                continue
            j = i + 1 if i % 2 == 1 else i - 1
            gn = (g[n][0] + int(cvec[i][0]), g[n][1] + int(cvec[i][1]))
            m2 = node_g.get(gn)
            if m2 is None or lk.face[m2, j] != fi:
                continue
            assert abs(lk.q[n, i] + lk.q[m2, j] - 1.0) < 1e-9
            pairs += 1
    assert pairs > 1000


def test_links_complementary_sphere(orc):
    wl = _small_sphere(3, 4, 2, 16)
    coords, bins, fo = _forest(orc, wl)
    lk = orc.link_fractions(3, coords, bins, fo, 27)
    L = wl.levels
    cvec = orc.lattice(27)
    bc = decode_keys((lk.key // 64).astype(np.int64), L, wl.roots, 3)
    cells = (lk.key % 64).astype(np.int64)
    g = 4 * bc + np.stack([cells & 3, (cells >> 2) & 3, cells >> 4], 1)
    node_g = {tuple(x): n for n, x in enumerate(map(tuple, g))}
    pairs = 0
    for n in range(lk.n):
        for i in range(1, 27):
            fi = lk.face[n, i]
            if fi < 0:
                continue
            j = i + 1 if i % 2 == 1 else i - 1
            m2 = node_g.get(tuple(g[n] + cvec[i]))
            if m2 is None or lk.face[m2, j] != fi:
                continue
            assert abs(lk.q[n, i] + lk.q[m2, j] - 1.0) < 1e-9
            pairs += 1
    assert pairs > 2000


def test_no_links_possible_on_coarse_leaves(orc):
    """With d_l = dx_l an unflagged cell has no face within one cell along any lattice
    direction: links computed on the coarse leaves of the forest are empty."""
    wl = _small_sphere(3, 4, 2, 16)
    coords, bins, fo = _forest(orc, wl)
    for l in range(wl.levels):
        lv = fo.levels[l]
        leaf_keys = lv["keys"][lv["leaf"] == 1]
        if len(leaf_keys) == 0:
            continue
        # a forest truncated at level l whose finest level is these leaves
        fo_l = orc.refine(3, coords, bins, wl.roots, l, wl.d_spec()[:max(l, 1)], (0, 0, 0), (1, 1, 1))
        keys_l = fo_l.levels[l]["keys"]
        idx = np.nonzero(np.isin(keys_l, leaf_keys))[0]
        lk = orc.link_fractions(3, coords, bins, fo_l, 27, subset=idx)
        assert lk.n == 0, f"links on coarse leaves at level {l}"


# ---------------------------------------------------------------------------
# Adjoint
# ---------------------------------------------------------------------------
def test_adjoint_horizontal_plane_closed_form(orc):
    """Upward link through the plane z = z0 of a horizontal triangle: dq/dv_k = lambda_k / dx
    along z and zero along x, y (golden values in tests/golden/adjoint_plane.txt)."""
    import os
    gold = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "adjoint_plane.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                k, val = line.split("=")
                gold[k.strip()] = [float(x) for x in val.split()]
    v = np.array(gold["triangle"], dtype=np.float32).reshape(3, 3)
    assert (v[:, 2] == gold["z0"][0]).all()
    f = np.array([[0, 1, 2]], dtype=np.int32)
    wl, coords, bins, fo = _all_level_forest(orc, 3, v, f, (1, 1, 1), 1, 27)
    lk = orc.link_fractions(3, coords, bins, fo, 27)
    ox, oy, oz = gold["origin"]
    dx = 1.0 / 8
    g = np.array([ox, oy, oz]) / (dx / 2)
    g = ((g - 1) / 2).astype(int)
    cell = (g[0] % 4) + 4 * (g[1] % 4) + 16 * (g[2] % 4)
    blk = g // 4
    key = int(blk[0] | (blk[1] << 1) | (blk[2] << 2))
    n = int(np.nonzero(lk.key == key * 64 + cell)[0][0])
    up = 5  # (0, 0, 1)
    assert lk.face[n, up] == 0
    assert abs(lk.q[n, up] - gold["q"][0]) < 1e-7
    w = np.zeros((lk.n, 27))
    w[n, up] = 1.0
    grad = orc.link_grad(fo, lk, coords, f, w, 3)
    exp = np.array(gold["grad_z"])
    assert np.allclose(grad[:, 2], exp, rtol=1e-6, atol=0)
    assert np.allclose(grad[:, :2], 0.0, atol=1e-12)


def _golden(name):
    import os
    gold = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                k, val = line.split("=")
                gold[k.strip()] = [float(x) for x in val.split()]
    return gold


def test_adjoint_horizontal_segment_closed_form(orc):
    """2D: an upward and a diagonal link through a horizontal segment, dq/dy_k = lambda_k / dx
    with lambda = (1 - s, s), zero along x (golden values in tests/golden/adjoint_segment.txt)."""
    gold = _golden("adjoint_segment.txt")
    v = np.array(gold["segment"], dtype=np.float32).reshape(2, 2)
    f = np.array([[0, 1]], dtype=np.int32)
    wl, coords, bins, fo = _all_level_forest(orc, 2, v, f, (1, 1), 1, 9)
    lk = orc.link_fractions(2, coords, bins, fo, 9)
    n = int(np.nonzero(lk.key == int(gold["node_key"][0]))[0][0])
    c = orc.lattice(9)
    up = int(np.nonzero((c[:, 0] == 0) & (c[:, 1] == 1))[0][0])
    diag = int(np.nonzero((c[:, 0] == 1) & (c[:, 1] == 1))[0][0])
    for i, qk, gk in ((up, "q_up", "grad_y_up"), (diag, "q_diag", "grad_y_diag")):
        assert lk.face[n, i] == 0
        assert abs(lk.q[n, i] - gold[qk][0]) < 1e-12
        w = np.zeros((lk.n, 9))
        w[n, i] = 1.0
        grad = orc.link_grad(fo, lk, coords, f, w, 2)
        assert np.allclose(grad[:, 1], gold[gk], rtol=1e-12, atol=0), (gk, grad)
        assert np.allclose(grad[:, 0], 0.0, atol=1e-12)


def test_adjoint_2d_matches_finite_differences(orc):
    """2D adjoint against central differences of the oracle's own q on a jittered circle."""
    n = 96
    th = 2 * np.pi * np.arange(n) / n
    v64 = np.stack([0.5 + 0.25 * np.cos(th), 0.5 + 0.25 * np.sin(th)], 1)
    v64 = geomgen.jitter_fp64(v64, 1e-3, 1)
    v = v64.astype(np.float32)
    f = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1).astype(np.int32)
    wl = geomgen.Workload("j2", 2, v, f, (4, 4, 1), 3, 16, 9)
    coords, bins, fo = _forest(orc, wl)
    lk = orc.link_fractions(2, coords, bins, fo, 9)
    stable = orc.link_stable(fo, lk, coords, bins, h=1e-5)
    w = geomgen.weights(lk.n * 9, 2).astype(np.float64).reshape(lk.n, 9)
    w[~stable] = 0.0
    assert stable.sum() > 200
    g = orc.link_grad(fo, lk, coords, f, w, n)
    gfd, nch = orc.fd_grad(fo, lk, v, f, bins, w, h=1e-5)
    assert nch == 0
    err = np.abs(g - gfd)
    scale = np.maximum(np.abs(gfd), 1e-2 * np.abs(gfd).max())
    assert (err <= 1e-3 * scale).all(), float((err / scale).max())
    assert np.linalg.norm(g - gfd) <= 1e-4 * np.linalg.norm(gfd)


def test_adjoint_matches_finite_differences(orc):
    u, f = geomgen.icosphere_unit(2)
    v64 = geomgen.jitter_fp64(np.array([0.5, 0.5, 0.5]) + 0.2 * u, 1e-3, 1)
    v = v64.astype(np.float32)
    wl = geomgen.Workload("j", 3, v, f, (4, 4, 4), 2, 16, 19)
    coords, bins, fo = _forest(orc, wl)
    lk = orc.link_fractions(3, coords, bins, fo, 19)
    # on this coarse mesh (cell 1/64) a 1e-4 step leaves an O(eta^2) truncation error that
    # +/- weights amplify in the sums; 1e-5 keeps truncation ~1e-7 and FP64 round-off ~1e-11
    stable = orc.link_stable(fo, lk, coords, bins, h=1e-5)
    w = geomgen.weights(lk.n * 19, 2).astype(np.float64).reshape(lk.n, 19)
    w[~stable] = 0.0
    assert stable.sum() > 300
    g = orc.link_grad(fo, lk, coords, f, w, len(v))
    gfd, nch = orc.fd_grad(fo, lk, v, f, bins, w, h=1e-5)
    assert nch == 0
    err = np.abs(g - gfd)
    scale = np.maximum(np.abs(gfd), 1e-2 * np.abs(gfd).max())
    assert (err <= 1e-3 * scale).all(), float((err / scale).max())
    assert np.linalg.norm(g - gfd) <= 1e-3 * np.linalg.norm(gfd)
    # translation: summed over all vertices, the gradient is sum_i w_i n/(D.n) -- check the
    # weaker, formula-free identity that moving every vertex by the same small vector moves
    # each stable link by the same amount as a central difference of the whole geometry
    e = np.array([0.3, -0.5, 0.8])
    e /= np.linalg.norm(e)
    hstep = 1e-5
    qs = []
    for sgn in (1, -1):
        vs = (v64.astype(np.float32).astype(np.float64) + sgn * hstep * e)
        cs = vs[f]
        # q with the same link set, recomputed exactly per stable link
        qs.append(cs)
    lin = (g * e[None]).sum()
    num = 0.0
    cvec = orc.lattice(19).astype(np.float64)
    L = wl.levels
    dx = 1.0 / (16 * 2 ** L)
    bc = decode_keys((lk.key // 64).astype(np.int64), L, wl.roots, 3)
    cells = (lk.key % 64).astype(np.int64)
    gg = 4 * bc + np.stack([cells & 3, (cells >> 2) & 3, cells >> 4], 1)
    o = (2 * gg + 1) * (dx / 2)
    for n_, i in zip(*np.nonzero(w)):
        fi = lk.face[n_, i]
        D = cvec[i] * dx
        tp = segment_triangle(o[n_], D, qs[0][fi])
        tm = segment_triangle(o[n_], D, qs[1][fi])
        num += w[n_, i] * float((tp[0] - tm[0]) / (2 * Fr(hstep)))
    assert abs(num - lin) <= 1e-4 * max(1.0, abs(lin))


def test_bins_reject_fewer_than_one_bin(orc):
    """A bin density below one per axis (or a dimension other than 2 and 3) is refused, not binned."""
    coords = np.zeros((1, 3, 3), dtype=np.float32)
    for dim, B in ((3, 0), (3, -2), (4, 8)):
        with pytest.raises(ValueError):
            orc.bin_faces(dim, coords, (0, 0, 0), (1, 1, 1), B)
