"""Helpers for the GPU <-> oracle parity tests: run the HIP path through the
binding, bring results to the host, and compare with the oracle's arrays."""
from __future__ import annotations

import sys
from dataclasses import dataclass

import numpy as np

Q_TOL = 1e-5          # |q_gpu (FP32) - q_oracle (FP64)|
END_TOL = 1e-5        # a link may exist on one side only when its t is this close to 0 or 1


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_run(wl, B=None, with_links=True, lattice=None, d_spec=None, levels=None, ctx=None, own_bin=False, n_prop=-1):
    import torch
    import paper_2502_16310_amd as agal
    dev = torch.device("cuda", 0)
    v = torch.from_numpy(np.ascontiguousarray(wl.vertices)).to(dev)
    f = torch.from_numpy(np.ascontiguousarray(wl.faces)).to(dev)
    L = wl.levels if levels is None else levels
    cfg = agal.NearWallConfig(dim=wl.dim, roots=wl.roots[:wl.dim], n_levels=L, bins=B or wl.bins,
                              lattice=lattice or wl.lattice, lo=wl.lo[:wl.dim], hi=wl.hi[:wl.dim],
                              d_spec=list(wl.d_spec()[:L]) if d_spec is None else list(d_spec), own_bin=own_bin,
                              n_prop=n_prop)
    geom, bins, forest, links = agal.near_wall(v, f, cfg, ctx=ctx, with_links=with_links)
    off, ids = bins.tensors()
    out = {"handles": (geom, bins, forest, links), "cfg": cfg,
           "offsets": off.cpu().numpy().view(np.uint32), "ids": ids.cpu().numpy()}
    levs = []
    for l in range(L + 1):
        d = forest.level(l)
        levs.append({"keys": d["keys"].cpu().numpy().view(np.uint32), "leaf": d["leaf"].cpu().numpy(),
                     "mark": d["mark"].cpu().numpy(),
                     "cell_flag": None if d["cell_flag"] is None else d["cell_flag"].cpu().numpy()})
    out["levels"] = levs
    if with_links:
        k, q, fc = links.tensors()
        out["key"] = k.cpu().numpy().view(np.uint64)
        out["q"] = q.cpu().numpy()
        out["face"] = fc.cpu().numpy()
    torch.cuda.synchronize()
    return out


def compare_bins(g, ob):
    assert np.array_equal(g["offsets"], ob.offsets), "bin offsets differ"
    assert np.array_equal(g["ids"], ob.ids), "binned face ids differ"


def compare_forest(g, of, L):
    for l in range(L + 1):
        gl, ol = g["levels"][l], of.levels[l]
        assert np.array_equal(gl["keys"], ol["keys"]), f"level {l} keys differ"
        assert np.array_equal(gl["leaf"], ol["leaf"]), f"level {l} leaf flags differ"
        assert np.array_equal(gl["mark"], ol["mark"]), f"level {l} marks differ"
        if l < L:
            assert np.array_equal(gl["cell_flag"], ol["cell_flag"]), f"level {l} cell flags differ"
        else:
            assert gl["cell_flag"] is None


@dataclass
class LinkReport:
    nodes_gpu: int
    nodes_orc: int
    links: int
    max_err: float
    one_sided: int
    one_sided_not_at_end: int
    face_diff: int


def check_face_ties(orc, forest, coords, Q, GQ, GF, OQ, OF, allk, tol=2.4e-7):
    """Where both sides link but name different faces, the GPU's face must also be hit
    (FP64) at the oracle's fraction to within two FP32 steps: ties between faces sharing an edge
    or vertex are broken on the FP32-rounded fraction, then by the lower face id."""
    bad = 0
    rows, cols = np.nonzero((GF >= 0) & (OF >= 0) & (GF != OF))
    for r, c in zip(rows, cols):
        t = orc.link_t(forest, int(allk[r]), Q, int(c), coords, int(GF[r, c]))
        if t is None or abs(t - OQ[r, c]) > tol:
            bad += 1
    return len(rows), bad


def compare_links(g, lk, restrict_blocks=None, cells=64):
    """Join GPU and oracle nodes by key; q within Q_TOL where both sides have a link;
    a link on one side only must sit within END_TOL of a segment end (else counted)."""
    gk, gq, gf = g["key"], g["q"].astype(np.float64), g["face"]
    if restrict_blocks is not None:
        sel = np.isin(gk // np.uint64(cells), restrict_blocks.astype(np.uint64))
        gk, gq, gf = gk[sel], gq[sel], gf[sel]
    ok_, oq, of_ = lk.key, lk.q, lk.face
    allk = np.union1d(gk, ok_)
    Q = gq.shape[1] if len(gq) else oq.shape[1]
    GQ = np.full((len(allk), Q), -1.0)
    GF = np.full((len(allk), Q), -1, dtype=np.int64)
    OQ = np.full((len(allk), Q), -1.0)
    OF = np.full((len(allk), Q), -1, dtype=np.int64)
    gi = np.searchsorted(allk, gk)
    oi = np.searchsorted(allk, ok_)
    GQ[gi], GF[gi] = gq, gf
    OQ[oi], OF[oi] = oq, of_
    both = (GF >= 0) & (OF >= 0)
    err = np.abs(GQ - OQ)[both]
    max_err = float(err.max()) if err.size else 0.0
    one = (GF >= 0) != (OF >= 0)
    qq = np.where(GF >= 0, GQ, OQ)[one]
    at_end = (qq <= END_TOL) | (qq >= 1 - END_TOL)
    return LinkReport(len(gk), len(ok_), int(both.sum()), max_err, int(one.sum()), int((~at_end).sum()),
                      int((GF != OF)[both].sum())), (GQ, GF, OQ, OF, allk)
