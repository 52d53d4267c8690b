"""Pins of the oracle's re-adaptation bookkeeping (orc_forest_diff): the relation between the forest of a
body and the forest of the same body moved, level by level.  Checked against a brute-force computation with
Python sets and dictionaries, against the structure of complete 2^D families (a refined block's children all
appear, a coarsened block's children all disappear, nothing appears or disappears without its parent), and
against the symmetries of the definition (a forest against itself; swapping old and new)."""
import numpy as np
import pytest

import geomgen


def _forest(orc, wl):
    coords = orc.gather(wl.dim, wl.vertices, wl.faces)
    bins = orc.bin_faces(wl.dim, coords, wl.lo[:wl.dim], wl.hi[:wl.dim], wl.bins)
    return orc.refine(wl.dim, coords, bins, wl.roots[:wl.dim], wl.levels, wl.d_spec(), wl.lo[:wl.dim],
                      wl.hi[:wl.dim])


def _moved(wl, shift):
    v = (wl.vertices + np.asarray(shift[:wl.dim], dtype=np.float32)).astype(np.float32)
    return geomgen.Workload(wl.name + "-moved", wl.dim, v, wl.faces, wl.roots, wl.levels, wl.bins, wl.lattice,
                            wl.lo, wl.hi)


def _bodies():
    v, f = geomgen.icosphere(3, 0.2)
    s3 = geomgen.Workload("ico3", 3, v, f, (8, 8, 8), 3, 16, 19)
    c2 = geomgen.workload("C0")
    return [(s3, (0.037, -0.021, 0.013)), (c2, (0.011, 0.043, 0.0))]


def _brute(old, new):
    out = []
    for lo_, ln_ in zip(old.levels, new.levels):
        pos = {int(k): j for j, k in enumerate(lo_["keys"])}
        newset = set(int(k) for k in ln_["keys"])
        idx, st = [], []
        for i, k in enumerate(ln_["keys"]):
            j = pos.get(int(k), -1)
            idx.append(j)
            if j < 0:
                st.append(1)
            elif lo_["leaf"][j] and not ln_["leaf"][i]:
                st.append(2)
            elif not lo_["leaf"][j] and ln_["leaf"][i]:
                st.append(3)
            else:
                st.append(0)
        rm = [0 if int(k) in newset else 1 for k in lo_["keys"]]
        out.append((np.array(idx, dtype=np.int32), np.array(st, dtype=np.uint8), np.array(rm, dtype=np.uint8)))
    return out


@pytest.mark.parametrize("case", [0, 1])
def test_diff_matches_brute_force(orc, case):
    wl, shift = _bodies()[case]
    old, new = _forest(orc, wl), _forest(orc, _moved(wl, shift))
    got = orc.forest_diff(old.levels, new.levels)
    ref = _brute(old, new)
    changed = 0
    for l, ((gi, gs, gr), (ri, rs, rr)) in enumerate(zip(got, ref)):
        assert np.array_equal(gi, ri), f"level {l} old_index"
        assert np.array_equal(gs, rs), f"level {l} state"
        assert np.array_equal(gr, rr), f"level {l} removed"
        changed += int((gs != 0).sum() + gr.sum())
    assert changed > 0


@pytest.mark.parametrize("case", [0, 1])
def test_diff_family_structure(orc, case):
    wl, shift = _bodies()[case]
    D = wl.dim
    old, new = _forest(orc, wl), _forest(orc, _moved(wl, shift))
    d = orc.forest_diff(old.levels, new.levels)
    for l in range(wl.levels):
        idx, st, rm = d[l]
        nk, nl = new.levels[l]["keys"].astype(np.int64), new.levels[l]["leaf"]
        ok, ol = old.levels[l]["keys"].astype(np.int64), old.levels[l]["leaf"]
        _, st1, rm1 = d[l + 1]
        nk1, ok1 = new.levels[l + 1]["keys"].astype(np.int64), old.levels[l + 1]["keys"].astype(np.int64)
        # children that appear: exactly those of new non-leaf blocks that were leaves or absent before
        grow = nk[(nl == 0) & ((st == 1) | (st == 2))]
        expect_created = np.sort((grow[:, None] * (1 << D) + np.arange(1 << D)[None]).reshape(-1))
        assert np.array_equal(np.sort(nk1[st1 == 1]), expect_created), f"level {l + 1} created children"
        # children that disappear: exactly those of old non-leaf blocks that are gone or now leaves
        gone = set(ok[rm == 1].tolist())
        coarsened = set(nk[st == 3].tolist())
        shrink = np.array([k for k, leaf in zip(ok.tolist(), ol.tolist()) if not leaf and (k in gone or k in coarsened)],
                          dtype=np.int64)
        expect_removed = np.sort((shrink[:, None] * (1 << D) + np.arange(1 << D)[None]).reshape(-1))
        assert np.array_equal(np.sort(ok1[rm1 == 1]), expect_removed), f"level {l + 1} removed children"
        # kept blocks keep their index mapping consistent
        kept = idx >= 0
        assert np.array_equal(ok[idx[kept]], nk[kept])


def test_diff_identity_and_swap(orc):
    wl, shift = _bodies()[0]
    a, b = _forest(orc, wl), _forest(orc, _moved(wl, shift))
    for idx, st, rm in orc.forest_diff(a.levels, a.levels):
        assert np.array_equal(idx, np.arange(len(idx))) and not st.any() and not rm.any()
    ab, ba = orc.forest_diff(a.levels, b.levels), orc.forest_diff(b.levels, a.levels)
    for l in range(wl.levels + 1):
        ka, kb = a.levels[l]["keys"], b.levels[l]["keys"]
        assert np.array_equal(np.sort(kb[ab[l][1] == 1]), np.sort(kb[ba[l][2] == 1])), "created vs removed"
        assert np.array_equal(np.sort(kb[ab[l][1] == 2]), np.sort(ka[ba[l][1] == 3])), "refined vs coarsened"
