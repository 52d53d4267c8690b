"""Full-size parity: the 327,680-triangle star body (bins and flags bit-exact, q on
sampled finest-level blocks, the side of every boundary node) and the differentiated jittered sphere (GPU adjoint
against the FP64 analytic adjoint and against central finite differences)."""
import numpy as np
import pytest

import geomgen
from _parity import check_face_ties, compare_bins, compare_forest, compare_links, gpu_run, log

pytestmark = pytest.mark.gpu


def test_star_c2_bins_flags_exact_and_sampled_q(orc):
    wl = geomgen.workload("C2")
    log(f"case C2: faces {len(wl.faces)} roots {wl.roots} L {wl.levels} B {wl.bins} Q {wl.lattice}")
    g = gpu_run(wl)
    coords = orc.gather(3, wl.vertices, wl.faces)
    ob = orc.bin_faces(3, coords, (0, 0, 0), (1, 1, 1), wl.bins)
    compare_bins(g, ob)
    of = orc.refine(3, coords, ob, wl.roots, wl.levels, wl.d_spec(), (0, 0, 0), (1, 1, 1))
    compare_forest(g, of, wl.levels)
    log(f"  blocks per level {[len(l['keys']) for l in of.levels]}")
    nL = len(of.levels[wl.levels]["keys"])
    rng = np.random.default_rng(11)
    sub = np.sort(rng.choice(nL, size=min(nL, 2000), replace=False))
    lk = orc.link_fractions(3, coords, ob, of, wl.lattice, subset=sub)
    rep, arrs = compare_links(g, lk, restrict_blocks=of.levels[wl.levels]["keys"][sub])
    log(f"  links: gpu nodes {rep.nodes_gpu} oracle nodes {rep.nodes_orc} common {rep.links} "
        f"max|dq| {rep.max_err:.3e} one-sided {rep.one_sided}")
    assert rep.max_err <= 1e-5 and rep.one_sided_not_at_end == 0 and rep.links > 10000
    nd, bad = check_face_ties(orc, of, coords, wl.lattice, *arrs)
    log(f"  face ids differing at ties: {nd}, not a tie: {bad}")
    assert bad == 0
    # node classification over every boundary node, against the oracle on the GPU's own link rows
    cls = g["handles"][3].classify().cpu().numpy()
    exp = orc.classify_nodes(3, wl.lattice, g["face"], coords)
    assert np.array_equal(cls, exp), f"{int((cls != exp).sum())} node classes differ"
    log(f"  classes fluid / solid / mixed {np.bincount(cls, minlength=4)[1:].tolist()}")


def _rel_checks(g, ref, comp_tol, norm_tol):
    err = np.abs(g - ref)
    scale = np.maximum(np.abs(ref), 1e-2 * np.abs(ref).max())
    comp = float((err / scale).max())
    norm = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
    return comp, norm, comp <= comp_tol and norm <= norm_tol


def test_c3_adjoint_against_fp64_adjoint_and_finite_differences(orc):
    import torch
    wl = geomgen.workload("C3")
    log(f"case C3: jittered sphere, faces {len(wl.faces)} vertices {len(wl.vertices)}")
    g = gpu_run(wl)
    r = orc.run_plain(wl)
    fo, lk, bins, coords = r["forest"], r["links"], r["bins"], r["coords"]
    assert np.array_equal(g["key"], lk.key), "node sets differ"
    assert np.array_equal(g["face"] >= 0, lk.face >= 0), "link sets differ"
    # weights U(-1, 1) per slot in canonical order, kept on the links stable under a 1e-4 step
    stable = orc.link_stable(fo, lk, coords, bins, h=1e-4)
    w = geomgen.weights(lk.n * wl.lattice, 2).astype(np.float64).reshape(lk.n, wl.lattice)
    w[~stable] = 0.0
    # ... and on which both sides name the same face (ties make the gradient one-sided)
    w[g["face"] != lk.face] = 0.0
    log(f"  stable links weighted: {int((w != 0).sum())} of {int((lk.face >= 0).sum())}")
    geom, bins_h, forest_h, links_h = g["handles"]
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    grad = links_h.backward(wt).cpu().numpy().astype(np.float64)
    g_ref = orc.link_grad(fo, lk, coords, wl.faces, w, len(wl.vertices))
    comp, norm, ok = _rel_checks(grad, g_ref, 1e-3, 1e-4)
    log(f"  GPU vs FP64 adjoint: max component rel {comp:.2e}, norm rel {norm:.2e}")
    assert ok
    # every link weighted (dense link queues in the adjoint's waves: up to 4 x 64 + 63 entries wait between
    # takes; a take that moved only 64 of them lost some links and repeated others)
    w_all = geomgen.weights(lk.n * wl.lattice, 3).astype(np.float64).reshape(lk.n, wl.lattice)
    w_all[(lk.face < 0) | (g["face"] != lk.face)] = 0.0
    grad_all = links_h.backward(torch.from_numpy(w_all.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    g_all = orc.link_grad(fo, lk, coords, wl.faces, w_all, len(wl.vertices))
    comp, norm, ok = _rel_checks(grad_all, g_all, 1e-3, 1e-4)
    log(f"  all {int((w_all != 0).sum())} links weighted: GPU vs FP64 adjoint max component rel {comp:.2e}, "
        f"norm rel {norm:.2e}")
    assert ok
    sub = np.sort(np.random.default_rng(4).choice(len(wl.vertices), 1024, replace=False))
    fd4, ch4 = orc.fd_grad(fo, lk, wl.vertices, wl.faces, bins, w, h=1e-4, vertex_subset=sub)
    fd5, ch5 = orc.fd_grad(fo, lk, wl.vertices, wl.faces, bins, w, h=1e-5, vertex_subset=sub)
    assert ch4 == 0 and ch5 == 0, "an arg-min face changed under the finite-difference step"
    c4, n4, _ = _rel_checks(grad[sub], fd4[sub], 1, 1)
    c5, n5, ok5 = _rel_checks(grad[sub], fd5[sub], 1e-3, 1e-3)
    log(f"  GPU vs FD h=1e-4: norm rel {n4:.2e} (max component {c4:.2e}); h=1e-5: max component {c5:.2e}, "
        f"norm rel {n5:.2e}")
    assert n4 <= 1e-3
    assert ok5
