"""Node classification on the GPU (side of every boundary node from the orientation of the faces its
links meet) against the oracle's orc_classify_nodes, bit for bit, on the GPU's own link rows (so that
face ids chosen at ties are the same on both sides), and against the classes of the oracle's links where
the two link sets name the same faces.  Closed bodies in 2D and 3D, the three lattices, a box with links
grazing its edges and corners (class 3), an open surface, and a node set of one row."""
import numpy as np
import pytest

import geomgen
from _parity import gpu_run, log
from test_gpu_link_modes import _box, _nd, _outside, _square

pytestmark = pytest.mark.gpu


def _sphere(Q):
    v, f = geomgen.icosphere(3, 0.2)
    return geomgen.Workload(f"ico3-q{Q}", 3, v, f, (8, 8, 8), 2, 16, Q)


def _star():
    v, f = geomgen.star(3)
    return geomgen.Workload("star3", 3, v, f, (8, 8, 8), 2, 8, 19)


CASES = {
    "C0": lambda: geomgen.workload("C0"),
    "ico3-q19": lambda: _sphere(19),
    "ico3-q27": lambda: _sphere(27),
    "star3": _star,
    "ico3-nd": _nd,
    "box": _box,
    "square": _square,
    "rand-outside": _outside,
}


def _classify(orc, wl, g):
    geom, bins, forest, links = g["handles"]
    cls = links.classify().cpu().numpy()
    coords = orc.gather(wl.dim, wl.vertices, wl.faces)
    exp = orc.classify_nodes(wl.dim, wl.lattice, g["face"], coords)
    assert cls.shape == exp.shape
    bad = np.flatnonzero(cls != exp)
    assert len(bad) == 0, f"{len(bad)} nodes differ, first {bad[:5]}: gpu {cls[bad[:5]]} oracle {exp[bad[:5]]}"
    return cls, coords


@pytest.mark.parametrize("name", list(CASES))
def test_classify_matches_oracle(orc, name):
    wl = CASES[name]()
    g = gpu_run(wl)
    cls, coords = _classify(orc, wl, g)
    counts = np.bincount(cls, minlength=4)[1:].tolist()
    log(f"  {wl.name}: {len(cls)} nodes, fluid / solid / mixed {counts}")
    # the oracle's own links: where both sides name the same faces the classes agree
    r = orc.run_plain(wl)
    lk = r["links"]
    assert np.array_equal(lk.key, g["key"])
    same = (lk.face == g["face"]).all(axis=1)
    ocls = orc.classify_nodes(wl.dim, wl.lattice, lk.face, coords)
    assert np.array_equal(ocls[same], cls[same])
    if name != "rand-outside":
        assert counts[0] > 0 and counts[1] > 0, "a closed body has boundary nodes on both sides"
    if name in ("box", "square"):
        assert counts[2] > 0, "links grazing the box's edges and corners give mixed nodes"


def test_classify_output_checks():
    import torch
    wl = _sphere(19)
    g = gpu_run(wl)
    links = g["handles"][3]
    n = links.n_nodes
    out = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
    assert links.classify(out) is out
    torch.cuda.synchronize()
    assert int(out.max()) <= 3 and int(out.min()) >= 1
    with pytest.raises(ValueError):
        links.classify(torch.empty(n + 1, dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError):
        links.classify(torch.empty(n, dtype=torch.int32, device="cuda"))
