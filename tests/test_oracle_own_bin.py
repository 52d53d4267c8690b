"""Pins for the oracle's own-bin refinement mode (paper Sec. II-C-2 with Algorithm 1, and the
propagation paragraph of Sec. II-C-3).

* The Euclidean point-to-face distance against a numerical minimisation over the face (an
  independent method), and the FP32 near decision against that distance away from the boundary
  and on dyadic cases where the FP32 arithmetic is exact (closed sets).
* The own-bin flags and the propagated marks against a re-derivation in Python: each cell's bin
  from its centre, the faces of that bin only, then a breadth-first search of N_prop rings over
  the blocks that exist at the level."""
import itertools
import math

import numpy as np
import pytest
from scipy.optimize import minimize

import geomgen
from test_oracle_pins import _check_balance, _leaf_level_map, decode_keys


# ---------------------------------------------------------------------------
# Distance and the near decision
# ---------------------------------------------------------------------------
def _dist2_numeric(face, p):
    """min over the closed face of |x - p|^2 by constrained minimisation (SLSQP) from several
    starting points; 2D faces are segments, 3D faces triangles."""
    face = np.asarray(face, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    if len(face) == 2:
        a, e = face[0], face[1] - face[0]
        fun = lambda s: float(np.sum((a + s[0] * e - p) ** 2))
        best = min(fun([s0]) for s0 in np.linspace(0, 1, 101))
        for s0 in (0.0, 0.5, 1.0):
            r = minimize(fun, [s0], method="SLSQP", bounds=[(0, 1)], options={"ftol": 1e-16, "maxiter": 500})
            best = min(best, r.fun)
        return best
    a, e1, e2 = face[0], face[1] - face[0], face[2] - face[0]
    fun = lambda x: float(np.sum((a + x[0] * e1 + x[1] * e2 - p) ** 2))
    cons = [{"type": "ineq", "fun": lambda x: 1.0 - x[0] - x[1]}]
    best = math.inf
    for x0 in ((1 / 3, 1 / 3), (0.05, 0.05), (0.9, 0.05), (0.05, 0.9)):
        r = minimize(fun, x0, method="SLSQP", bounds=[(0, 1), (0, 1)], constraints=cons,
                     options={"ftol": 1e-16, "maxiter": 500})
        if r.x[0] >= -1e-12 and r.x[1] >= -1e-12 and r.x[0] + r.x[1] <= 1 + 1e-12:
            best = min(best, r.fun)
    return best


def _random_cases(n, seed, dim):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        face = rng.uniform(0.2, 0.8, (dim, dim))
        # points near vertices, near edges, above the interior and far away
        kind = rng.integers(4)
        if kind == 0:
            p = face[rng.integers(dim)] + rng.normal(0, 0.05, dim)
        elif kind == 1:
            k = rng.integers(dim)
            p = face[k] + rng.uniform(-0.3, 1.3) * (face[(k + 1) % dim] - face[k]) + rng.normal(0, 0.05, dim)
        elif kind == 2:
            lam = rng.dirichlet(np.ones(dim))
            p = lam @ face + rng.normal(0, 0.05, dim)
        else:
            p = rng.uniform(0, 1, dim)
        out.append((face, p))
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_face_distance_vs_numerical_minimisation(orc, dim):
    for face, p in _random_cases(250, 40 + dim, dim):
        d_orc = math.sqrt(orc.face_dist2(dim, face, p))
        d_num = math.sqrt(_dist2_numeric(face, p))
        assert abs(d_orc - d_num) <= 1e-7, (face, p, d_orc, d_num)


@pytest.mark.parametrize("dim", [2, 3])
def test_near_l2_f32_agrees_with_distance_off_the_boundary(orc, dim):
    rng = np.random.default_rng(7 + dim)
    checked = 0
    for face, p in _random_cases(2000, 60 + dim, dim):
        f32 = face.astype(np.float32)
        p32 = p.astype(np.float32)
        d2 = orc.face_dist2(dim, f32.astype(np.float64), p32.astype(np.float64))
        R = np.float32(math.sqrt(d2) * rng.uniform(0.5, 1.5))
        R2 = float(R) ** 2
        if abs(d2 - R2) <= 1e-4 * R2:
            continue
        checked += 1
        assert orc.near_l2_f32(dim, f32, p32, float(R)) == (d2 <= R2), (face, p, R)
    assert checked > 1800


def test_near_l2_f32_closed_boundary_dyadic(orc):
    """Dyadic points at an exact distance: the decision is closed (<=), and false just inside."""
    tri = np.array([[0, 0, 0], [0.5, 0, 0], [0, 0.5, 0]], dtype=np.float32)
    cases3 = [((0.125, 0.125, 0.25), 0.25),        # above the interior: the prism part
              ((0.25, -0.25, 0.0), 0.25),          # beside edge v0-v1: a cylinder
              ((0.5, 0.5, 0.0), math.sqrt(2) / 4),  # beside the hypotenuse (distance irrational)
              ((-0.1875, -0.25, 0.0), 0.3125),     # beyond vertex v0: a sphere
              ((0.5, 0.0, 0.5), 0.5)]              # above vertex v1
    for p, d in cases3:
        R = np.float32(d)
        if float(R) ** 2 == d * d:   # exactly representable distance
            assert orc.near_l2_f32(3, tri, p, float(R)), p
        assert orc.near_l2_f32(3, tri, p, float(np.float32(d * (1 + 1e-5)))), p
        assert not orc.near_l2_f32(3, tri, p, float(np.float32(d * (1 - 1e-5)))), p
        assert orc.near_face_l2(3, tri.astype(np.float64), p, d * (1 + 1e-12))
        assert not orc.near_face_l2(3, tri.astype(np.float64), p, d * (1 - 1e-12))
    seg = np.array([[0, 0], [0.5, 0]], dtype=np.float32)
    for p, d in (((0.25, 0.25), 0.25), ((0.75, 0.0), 0.25), ((-0.1875, 0.25), 0.3125), ((0.5, -0.5), 0.5)):
        assert orc.near_l2_f32(2, seg, p, d)
        assert not orc.near_l2_f32(2, seg, p, float(np.float32(d * (1 - 1e-5))))
    # a degenerate (zero-area) triangle is its longest edge
    deg = np.array([[0, 0, 0], [0.5, 0, 0], [0.25, 0, 0]], dtype=np.float32)
    assert orc.near_l2_f32(3, deg, (0.25, 0.25, 0.0), 0.25)
    assert not orc.near_l2_f32(3, deg, (0.25, 0.25, 0.0), 0.2499)


# ---------------------------------------------------------------------------
# Own-bin flags and propagation
# ---------------------------------------------------------------------------
def _own_bin_forest(orc, wl, B, d):
    coords = orc.gather(wl.dim, wl.vertices, wl.faces)
    bins = orc.bin_faces(wl.dim, coords, wl.lo[:wl.dim], wl.hi[:wl.dim], B)
    dsp = np.full(wl.levels, d, dtype=np.float32)
    fo = orc.refine(wl.dim, coords, bins, wl.roots[:wl.dim], wl.levels, dsp, wl.lo[:wl.dim], wl.hi[:wl.dim],
                    own_bin=True)
    return coords, bins, fo, dsp


def _expected_pass(orc, wl, coords, bins, keys, level, d):
    """Cell flags of the given blocks and the set of propagated block indices, derived in Python."""
    dim, B = wl.dim, bins.B
    cells = 64 if dim == 3 else 16
    dx = np.float32(1.0) / np.float32(4 * wl.roots[0] * 2 ** level)
    c = decode_keys(keys, level, wl.roots, dim)
    ci = np.arange(cells)
    off = np.stack([ci & 3, (ci >> 2) & 3, (ci >> 4) & 3], 1)[:, :dim]
    g = 4 * c[:, None, :dim] + off[None]
    m = (np.float32(0.0) + (2 * g + 1).astype(np.float32) * (np.float32(0.5) * dx)).astype(np.float32)
    s = np.float32(B) / np.float32(1.0)
    ib = np.clip(np.floor((m - np.float32(0.0)) * s), 0, B - 1).astype(np.int64)
    lin = ib[..., 0] + B * ib[..., 1] + (B * B * ib[..., 2] if dim == 3 else 0)
    lo_f = coords.min(1).astype(np.float64)
    hi_f = coords.max(1).astype(np.float64)
    flags = np.zeros((len(keys), cells), np.uint8)
    for bi in range(len(keys)):
        for cc in range(cells):
            b = lin[bi, cc]
            ids = bins.ids[bins.offsets[b]:bins.offsets[b + 1]]
            p = m[bi, cc].astype(np.float64)
            gap = np.clip(np.maximum(lo_f[ids] - p, p - hi_f[ids]), 0, None)
            cand = ids[np.sqrt((gap ** 2).sum(1)) <= 1.001 * d]
            for f in cand:
                if orc.near_l2_f32(dim, coords[f], m[bi, cc], float(d)):
                    flags[bi, cc] = 1
                    break
    marked = flags.any(1)
    nprop = 0 if B == 1 else 1 + int(np.floor(np.float32(d) / (np.float32(4.0) * dx)))
    pos = {tuple(int(x) for x in cc): i for i, cc in enumerate(c)}
    dist = {i: 0 for i in np.nonzero(marked)[0]}
    frontier = list(dist)
    offs = [o for o in itertools.product((-1, 0, 1), repeat=dim) if any(o)]
    for step in range(1, nprop + 1):
        nxt = []
        for i in frontier:
            for o in offs:
                key = tuple(int(c[i][a]) + (o[a] if a < dim else 0) for a in range(3))
                j = pos.get(key)
                if j is not None and j not in dist:
                    dist[j] = step
                    nxt.append(j)
        frontier = nxt
    prop = np.zeros(len(keys), bool)
    prop[[j for j, st in dist.items() if st > 0]] = True
    return flags, marked, prop, nprop


@pytest.mark.parametrize("case", ["sphere-B1", "sphere-B2", "sphere-B8", "circle-B4", "circle-B16"])
def test_own_bin_flags_and_propagation_brute_force(orc, case):
    if case.startswith("sphere"):
        v, f = geomgen.star(2, 0)
        wl = geomgen.Workload("s", 3, v, f, (4, 4, 4), 2, 0, 19)
        d = 0.05
    else:
        v, f = geomgen.circle(200, 0.25)
        wl = geomgen.Workload("c", 2, v, f, (8, 8, 1), 3, 0, 9)
        d = 0.04
    B = int(case.split("-B")[1])
    coords, bins, fo, dsp = _own_bin_forest(orc, wl, B, d)
    _check_balance(_leaf_level_map(fo, wl.roots, wl.dim), wl.dim)
    total_prop = 0
    for l in range(wl.levels):
        lv = fo.levels[l]
        keys = lv["keys"]
        if l == 0:
            tested = np.ones(len(keys), bool)
        else:
            par = fo.levels[l - 1]
            pk = par["keys"][np.isin(par["mark"], (1, 3))].astype(np.int64)
            tested = np.isin(keys.astype(np.int64) >> wl.dim, pk)
        flags, marked, prop, nprop = _expected_pass(orc, wl, coords, bins, keys[tested], l, dsp[l])
        assert np.array_equal(lv["cell_flag"][tested], flags), f"level {l} cell flags"
        assert not lv["cell_flag"][~tested].any()
        mk = lv["mark"][tested]
        assert np.array_equal(mk == 1, marked), f"level {l}: mark 1 = a flagged cell"
        assert np.array_equal(mk == 3, prop), f"level {l}: mark 3 = reached by propagation"
        assert np.array_equal(lv["leaf"] == 0, lv["mark"] > 0), "refined iff marked"
        total_prop += int(prop.sum())
        if B == 1:
            assert nprop == 0 and not prop.any()
    if B > 1:
        assert total_prop > 0, "the case exercises propagation"
