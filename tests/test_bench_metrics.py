"""The benchmark's workload count (cell-face tests) is computed on the host from
the bins and the forest; it must equal the oracle's own count of the pairs it
visits."""
import numpy as np

import geomgen
from bench import cell_face_tests


def _small_sphere():
    v, f = geomgen.icosphere(3, 0.2)
    return geomgen.Workload("s", 3, v, f, (4, 4, 4), 3, 16, 19)


def test_counts_match_oracle(orc):
    for wl in (geomgen.workload("C0"), _small_sphere()):
        r = orc.run_plain(wl)
        fo, lk, bins = r["forest"], r["links"], r["bins"]
        t_flag, t_q = cell_face_tests(bins.offsets, wl.bins, wl.dim, fo.levels, wl.roots, wl.levels,
                                      wl.d_spec(), wl.lo, wl.hi)
        assert t_flag == fo.tests[:wl.levels]
        assert t_q == lk.tests
