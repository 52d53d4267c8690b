"""Pins of the oracle's node classification (fluid / solid from the orientation of the faces a node's links
first meet) against an independent inside test: the winding number of the closed, outward-oriented surface
around the node's centre (FP64; 3D: the sum of the triangles' signed solid angles over 4 pi, the Van
Oosterom-Strackee formula; 2D: the sum of the segments' signed angles over 2 pi), and against exact
point-in-box tests on a dyadic box.  Nodes whose centre lies on the surface (a link at t = 0) have no side and
are left out, as are winding numbers away from 0 and 1."""
import numpy as np
import pytest

import geomgen


def _centres(wl, keys):
    """Cell centres of the finest level from the node keys (block key * 4^D + cell, the block key built
    root-first with one x-fastest child index per level), by the FP32 rule lo + (2 g + 1) (dx / 2)."""
    dim, level, roots = wl.dim, wl.levels, wl.roots
    keys = np.asarray(keys, dtype=np.uint64)
    cells = 4 ** dim
    k = (keys // np.uint64(cells)).astype(np.int64)
    cell = (keys % np.uint64(cells)).astype(np.int64)
    path = np.zeros((len(k), 3), dtype=np.int64)
    for j in range(level):
        ci = k & ((1 << dim) - 1)
        k = k >> dim
        for a in range(dim):
            path[:, a] |= ((ci >> a) & 1) << j
    r = np.stack([k % roots[0], (k // roots[0]) % roots[1], k // (roots[0] * roots[1])], 1)
    g = 4 * ((r << level) | path) + np.stack([cell & 3, (cell >> 2) & 3, cell >> 4], 1)
    out = np.zeros((len(k), dim), dtype=np.float32)
    for a in range(dim):
        half = np.float32(0.5) * wl.cell_size(level, a)
        out[:, a] = np.float32(wl.lo[a]) + (2 * g[:, a] + 1).astype(np.float32) * half
    return out.astype(np.float64)


def _winding_3d(verts, faces, p):
    a = verts[faces[:, 0]][None] - p[:, None]
    b = verts[faces[:, 1]][None] - p[:, None]
    c = verts[faces[:, 2]][None] - p[:, None]
    la, lb, lc = (np.linalg.norm(x, axis=2) for x in (a, b, c))
    num = np.einsum("pfi,pfi->pf", a, np.cross(b, c))
    den = (la * lb * lc + np.einsum("pfi,pfi->pf", a, b) * lc + np.einsum("pfi,pfi->pf", a, c) * lb
           + np.einsum("pfi,pfi->pf", b, c) * la)
    return (2.0 * np.arctan2(num, den)).sum(axis=1) / (4.0 * np.pi)


def _winding_2d(verts, faces, p):
    a = verts[faces[:, 0]][None] - p[:, None]
    b = verts[faces[:, 1]][None] - p[:, None]
    cr = a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]
    dt = (a * b).sum(axis=2)
    return np.arctan2(cr, dt).sum(axis=1) / (2.0 * np.pi)


def _run(orc, wl):
    res = orc.run_plain(wl)
    lk = res["links"]
    cls = orc.classify_nodes(wl.dim, wl.lattice, lk.face, res["coords"])
    p = _centres(wl, lk.key)
    on_surface = ((lk.q <= 0.0) & (lk.face >= 0)).any(axis=1)
    return cls, p, on_surface


def _check_against_winding(cls, w, on_surface):
    keep = ~on_surface & ((np.abs(w) < 0.1) | (np.abs(w - 1.0) < 0.1))
    expect = np.where(w > 0.5, 2, 1)
    assert keep.sum() > 100
    bad = (cls != expect) & keep
    assert not bad.any(), f"{int(bad.sum())} of {int(keep.sum())} nodes classified against the winding number"
    return int(keep.sum()), int((cls[keep] == 2).sum())


@pytest.mark.parametrize("shape", ["ico3", "star3"])
def test_classify_3d_matches_winding_number(orc, shape):
    v, f = geomgen.icosphere(3, 0.2) if shape == "ico3" else geomgen.star(3)
    wl = geomgen.Workload(shape, 3, v, f, (8, 8, 8), 2, 16, 19)
    cls, p, on_surface = _run(orc, wl)
    w = _winding_3d(v.astype(np.float64), f, p)
    n, solid = _check_against_winding(cls, w, on_surface)
    assert 0 < solid < n


def test_classify_circle_matches_winding_number(orc):
    wl = geomgen.workload("C0")
    cls, p, on_surface = _run(orc, wl)
    w = _winding_2d(wl.vertices.astype(np.float64), wl.faces, p)
    n, solid = _check_against_winding(cls, w, on_surface)
    assert 0 < solid < n


def _box_edge_touch(wl, p, lo, hi, Q, orc):
    """Per node: does one of its links touch an edge or corner of the box [lo, hi]^D (a point of the
    segment with two coordinates on the box's bounds and none outside)?  Such a link meets two faces at
    one point, one it enters and one it leaves when it only grazes the solid.  Dyadic inputs: exact."""
    c = orc.lattice(Q)[:, :wl.dim].astype(np.float64)
    dx = np.array([wl.cell_size(wl.levels, a) for a in range(wl.dim)], dtype=np.float64)
    touch = np.zeros(len(p), dtype=bool)
    for i in range(1, Q):
        step = c[i] * dx
        for a in range(wl.dim):
            if step[a] == 0:
                continue
            for b in (lo, hi):
                t = (b - p[:, a]) / step[a]
                x = p + t[:, None] * step[None]
                x[:, a] = b
                ok = (t >= 0) & (t <= 1) & ((x >= lo) & (x <= hi)).all(axis=1)
                on = ((x == lo) | (x == hi)).sum(axis=1)
                touch |= ok & (on >= 2)
    return touch


@pytest.mark.parametrize("dim", [2, 3])
def test_classify_dyadic_box_exact(orc, dim):
    """Every node off the surface whose links touch no edge or corner of the box takes its exact side; a
    node whose link grazes an edge or corner takes its side or the mixed class 3, and no other node is
    mixed."""
    lo, hi = 81 / 256, 175 / 256
    if dim == 3:
        v, f = geomgen.box_mesh((lo,) * 3, (hi,) * 3)
        wl = geomgen.Workload("box", 3, v, f, (4, 4, 4), 3, 16, 27)
    else:
        v, f = geomgen.square_loop((lo, lo), (hi, hi))
        wl = geomgen.Workload("square", 2, v, f, (4, 4, 1), 3, 16, 9)
    cls, p, on_surface = _run(orc, wl)
    inside = ((p > lo) & (p < hi)).all(axis=1)
    side = np.where(inside, 2, 1)
    touch = _box_edge_touch(wl, p, lo, hi, wl.lattice, orc)
    keep = ~on_surface & ~touch
    assert keep.sum() > 100 and (inside & keep).any() and (~inside & keep).any()
    assert np.array_equal(cls[keep], side[keep])
    graze = ~on_surface & touch
    assert graze.any() and np.all((cls[graze] == side[graze]) | (cls[graze] == 3))
    assert (cls[graze] == 3).any()
