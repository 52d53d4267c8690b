"""The paper's own form of near-wall refinement on the GPU (Euclidean point-face test against the faces of
the cell centre's own bin, then mark propagation over rings of blocks) against the oracle's
orc_refine_own_bin: keys, leaf bits, marks (1 flagged, 2 balance, 3 propagation) and cell flags bit for
bit, over bin densities from the naive single bin to fine bins, the propagation rule and overrides, 2D
and 3D, the paper's constant distance, a non-dyadic domain; and link fractions on such a forest."""
import numpy as np
import pytest

import geomgen
from _parity import compare_forest, compare_links, gpu_run, log
from test_gpu_parity import _check_links

pytestmark = pytest.mark.gpu


def _check(orc, wl, B, d_spec, n_prop=-1, with_links=False):
    g = gpu_run(wl, B=B, d_spec=d_spec, own_bin=True, n_prop=n_prop, with_links=with_links)
    coords = orc.gather(wl.dim, wl.vertices, wl.faces)
    ob = orc.bin_faces(wl.dim, coords, wl.lo[:wl.dim], wl.hi[:wl.dim], B)
    of = orc.refine(wl.dim, coords, ob, wl.roots[:wl.dim], wl.levels, d_spec, wl.lo[:wl.dim], wl.hi[:wl.dim],
                    own_bin=True, n_prop=n_prop)
    compare_forest(g, of, wl.levels)
    marks = [np.bincount(l["mark"], minlength=4)[1:4].tolist() for l in g["levels"][:wl.levels]]
    log(f"  {wl.name} B={B} n_prop={n_prop}: blocks per level {[len(l['keys']) for l in g['levels']]}, "
        f"marks (flag, balance, propagation) per level {marks}")
    return g, of, coords, ob


@pytest.mark.parametrize("B", [1, 2, 8, 32])
def test_own_bin_circle(orc, B):
    wl = geomgen.workload("C0")
    _check(orc, wl, B, list(wl.d_spec()))


@pytest.mark.parametrize("B,n_prop", [(1, -1), (4, -1), (16, -1), (16, 0), (16, 2)])
def test_own_bin_sphere(orc, B, n_prop):
    v, f = geomgen.icosphere(3, 0.2)
    wl = geomgen.Workload("ico3", 3, v, f, (8, 8, 8), 3, B, 19)
    _check(orc, wl, B, list(wl.d_spec()), n_prop)


@pytest.mark.parametrize("B", [2, 8])
def test_own_bin_star_constant_distance(orc, B):
    """The paper's setting at a small scale: a star body, constant d = 0.05 over two passes (several
    block lengths, so several propagation steps)."""
    v, f = geomgen.star(4)
    wl = geomgen.Workload("star4", 3, v, f, (8, 8, 8), 2, B, 19)
    _check(orc, wl, B, [0.05, 0.05])


def test_own_bin_non_dyadic_domain_and_links(orc):
    v, f = geomgen.icosphere(3, 0.2)
    wl = geomgen.Workload("ico3-nd", 3, v, f, (5, 6, 4), 2, 7, 27, lo=(0.05, -0.02, 0.1), hi=(0.97, 1.01, 0.9))
    g, of, coords, ob = _check(orc, wl, 7, list(wl.d_spec()), with_links=True)
    lk = orc.link_fractions(3, coords, ob, of, 27)
    rep, _ = compare_links(g, lk, cells=64)
    _check_links(rep)


def test_own_bin_segments_2d(orc):
    v, f = geomgen.random_segments(200, 10, 0.05, 0.95, 0.1)
    wl = geomgen.Workload("rseg", 2, v, f, (5, 3, 1), 3, 9, 9)
    _check(orc, wl, 9, [0.02, 0.01, 0.005])
