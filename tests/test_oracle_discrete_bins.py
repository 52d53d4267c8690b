"""Pins of the oracle's sampled-point binning (orc_bin_faces_discrete, the paper's own binning) on dyadic faces,
where every sample point is an exact rational: every bin a face is assigned to meets the face (exact clipping),
the bins of its vertices are always among them, a spacing no smaller than the face samples exactly its
vertices, a 2D segment is in every bin its chord crosses over more than the spacing (exact clipping), and the
assignment is a subset of the bounding-box binning."""
import itertools
from fractions import Fraction as Fr

import numpy as np
import pytest

from _exact import clip_halfspace, exact_bin, face_meets_box


def _dyadic_faces(rng, F, dim, size, bits=8):
    """F faces with coordinates k / 2^bits in [0, 1], extent up to `size`."""
    q = 1 << bits
    c = rng.integers(0, q, size=(F, 1, dim))
    d = rng.integers(-int(size * q), int(size * q) + 1, size=(F, dim, dim))
    pts = np.clip(c + d, 0, q - 1)
    return (pts / q).astype(np.float32)


def _pairs(bins, B, dim):
    out = set()
    for b in range(bins.nb):
        for f in bins.ids[bins.offsets[b]:bins.offsets[b + 1]]:
            out.add((int(f), b))
    return out


def _bin_of(p, B, dim):
    ix = [exact_bin(p[a], 0.0, 1.0, B) for a in range(dim)] + [0] * (3 - dim)
    return (ix[2] * B + ix[1]) * B + ix[0]


def _bin_box(b, B, dim):
    ix = (b % B, (b // B) % B, b // (B * B))
    return [(ix[a] + 0.5) / B for a in range(dim)], 0.5 / B


@pytest.mark.parametrize("dim,spacing", [(3, 1 / 16), (3, 1 / 64), (2, 1 / 32), (2, 1 / 128)])
def test_assigned_bins_meet_the_face_and_hold_its_vertices(orc, dim, spacing):
    rng = np.random.default_rng(7 + dim)
    B = 8
    coords = _dyadic_faces(rng, 150, dim, 0.3)
    bn = orc.bin_faces_discrete(dim, coords, (0,) * dim, (1,) * dim, B, spacing)
    pairs = _pairs(bn, B, dim)
    box = _pairs(orc.bin_faces(dim, coords, (0,) * dim, (1,) * dim, B), B, dim)
    assert pairs <= box, "a sampled bin outside the face's bounding-box bins"
    for f, b in pairs:
        m, h = _bin_box(b, B, dim)
        assert face_meets_box(coords[f], m, h), f"face {f} assigned to bin {b} it does not meet"
    for f in range(len(coords)):
        for v in coords[f]:
            assert (f, _bin_of(v, B, dim)) in pairs, f"face {f} misses the bin of its vertex {v}"
    assert len(pairs) < len(box), "the sampled binning is not just the bounding-box binning"


@pytest.mark.parametrize("dim", [2, 3])
def test_spacing_above_the_face_samples_its_vertices_only(orc, dim):
    rng = np.random.default_rng(3)
    B = 16
    coords = _dyadic_faces(rng, 200, dim, 0.15)
    bn = orc.bin_faces_discrete(dim, coords, (0,) * dim, (1,) * dim, B, 0.5)
    want = {(f, _bin_of(v, B, dim)) for f in range(len(coords)) for v in coords[f]}
    assert _pairs(bn, B, dim) == want


def _chord_linf(seg, m, h):
    poly = [tuple(Fr(float(x)) for x in p) for p in seg]
    for a in range(2):
        poly = clip_halfspace(poly, a, Fr(m[a]) - Fr(h), True)
        if not poly:
            return Fr(-1)
        poly = clip_halfspace(poly, a, Fr(m[a]) + Fr(h), False)
        if not poly:
            return Fr(-1)
    return max(max(abs(p[a] - q[a]) for a in range(2)) for p, q in itertools.combinations(poly, 2)) if len(poly) > 1 else Fr(0)


@pytest.mark.parametrize("spacing", [1 / 32, 1 / 64])
def test_segments_cover_every_bin_they_cross_by_more_than_the_spacing(orc, spacing):
    rng = np.random.default_rng(11)
    B = 16
    coords = _dyadic_faces(rng, 120, 2, 0.4)
    pairs = _pairs(orc.bin_faces_discrete(2, coords, (0, 0), (1, 1), B, spacing), B, 2)
    checked = 0
    for f in range(len(coords)):
        for b in range(B * B):
            m, h = _bin_box(b, B, 2)
            if _chord_linf(coords[f], m, h) > Fr(spacing):
                checked += 1
                assert (f, b) in pairs, f"segment {f} crosses bin {b} over more than the spacing but is not in it"
    assert checked > 200


def test_discrete_bins_refuse_bad_arguments(orc):
    coords = np.zeros((1, 3, 3), dtype=np.float32)
    for B, sp in ((0, 0.1), (8, 0.0), (8, -1.0), (8, float("nan"))):
        with pytest.raises(ValueError):
            orc.bin_faces_discrete(3, coords, (0, 0, 0), (1, 1, 1), B, sp)
