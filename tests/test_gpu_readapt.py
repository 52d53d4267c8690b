"""Re-adaptation of a moving body on the GPU: the forest of the moved geometry (refined from the roots) against
the oracle's refinement, and its relation to the previous forest (old index, kept / created / refined /
coarsened per new block, removed per old block, counts per level) against the oracle's orc_forest_diff on the
same two forests, bit for bit; a sequence of steps of a moving sphere, a moving circle, the 327,680-face star
moved by a fraction of a cell, and forests over different grids refused."""
import numpy as np
import pytest

import geomgen
from _parity import compare_forest, gpu_run, log

pytestmark = pytest.mark.gpu


def _moved(wl, shift, name=None):
    v = (wl.vertices + np.asarray(shift[:wl.dim], dtype=np.float32)).astype(np.float32)
    return geomgen.Workload(name or wl.name + "-moved", wl.dim, v, wl.faces, wl.roots, wl.levels, wl.bins,
                            wl.lattice, wl.lo, wl.hi, dict(wl.extra))


def _check_diff(orc, ga, gb, L):
    fa, fb = ga["handles"][2], gb["handles"][2]
    d = fb.diff(fa)
    ref = orc.forest_diff(ga["levels"], gb["levels"])
    counts = d.counts()
    for l in range(L + 1):
        lv = d.level(l)
        oi, st, rm = lv["old_index"].cpu().numpy(), lv["state"].cpu().numpy(), lv["removed"].cpu().numpy()
        ri, rs, rr = ref[l]
        assert np.array_equal(oi, ri), f"level {l}: old index"
        assert np.array_equal(st, rs), f"level {l}: state"
        assert np.array_equal(rm, rr), f"level {l}: removed"
        want = [int((rs == 1).sum()), int((rs == 2).sum()), int((rs == 3).sum()), int(rr.sum())]
        assert counts[l] == want, f"level {l}: counts {counts[l]} != {want}"
    return counts


def _sphere():
    v, f = geomgen.icosphere(3, 0.2)
    return geomgen.Workload("ico3", 3, v, f, (8, 8, 8), 3, 16, 19)


@pytest.mark.parametrize("name", ["ico3", "C0"])
def test_moving_body_steps(orc, name):
    wl = _sphere() if name == "ico3" else geomgen.workload("C0")
    step = np.array([0.0131, -0.0077, 0.0049])
    prev = gpu_run(wl, with_links=False)
    for k in range(1, 4):
        cur_wl = _moved(wl, step * k, f"{wl.name}-step{k}")
        cur = gpu_run(cur_wl, with_links=False)
        coords = orc.gather(wl.dim, cur_wl.vertices, cur_wl.faces)
        ob = orc.bin_faces(wl.dim, coords, wl.lo[:wl.dim], wl.hi[:wl.dim], wl.bins)
        of = orc.refine(wl.dim, coords, ob, wl.roots[:wl.dim], wl.levels, wl.d_spec(), wl.lo[:wl.dim],
                        wl.hi[:wl.dim])
        compare_forest(cur, of, wl.levels)
        counts = _check_diff(orc, prev, cur, wl.levels)
        log(f"  {cur_wl.name}: [created, refined, coarsened, removed] per level {counts}")
        assert sum(c[0] + c[3] for c in counts) > 0, "a moved body changes its forest"
        prev = cur


def test_same_forest_is_all_kept(orc):
    wl = _sphere()
    a, b = gpu_run(wl, with_links=False), gpu_run(wl, with_links=False)
    counts = _check_diff(orc, a, b, wl.levels)
    assert all(c == [0, 0, 0, 0] for c in counts)


def test_star_c2_moved_by_a_fraction_of_a_cell(orc):
    wl = geomgen.workload("C2")
    a = gpu_run(wl, with_links=False)
    dx = float(wl.cell_size(wl.levels))
    b = gpu_run(_moved(wl, (0.37 * dx, 0.21 * dx, -0.13 * dx)), with_links=False)
    counts = _check_diff(orc, a, b, wl.levels)
    log(f"  C2 moved by (0.37, 0.21, -0.13) cells: [created, refined, coarsened, removed] per level {counts}")


def test_forests_over_different_grids_are_refused():
    import paper_2502_16310_amd as agal
    wl = _sphere()
    a = gpu_run(wl, with_links=False)
    other = geomgen.Workload("ico3-r4", 3, wl.vertices, wl.faces, (4, 4, 4), 3, 16, 19)
    b = gpu_run(other, with_links=False)
    with pytest.raises(agal.AgalError) as e:
        b["handles"][2].diff(a["handles"][2])
    assert e.value.status == agal.AGAL_EINVAL
