"""Benchmark of the near-wall mesh-adaptation hot path on one MI355X.

One step = import the faces (device-resident inputs), bin them, refine the
forest level by level near the wall, compute the link fractions q and run
the adjoint for a weighted sum of q -- every row of the hot path, on
synthetic seeded geometry (see geomgen).  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--config C2|C1|C4|P0|P1|M0] [--no-cpu-baseline]

The default workload is C2 (327,680-face star body, 32^3 roots, 4 passes,
D3Q27), the largest single-body configuration.

--config C4 times the batched form (64 bodies, one graph launch, forward and
adjoint) against the same bodies through the single-body calls.  --config P0 /
P1 runs the paper's bin-density study on its own refinement form (own-bin
Euclidean flags with mark propagation) for B = 1, 2, 8, 16.  --config M0 moves
the C2 body by a fraction of a cell per step and times the whole re-adaptation
step (import, bins, refinement, forest relation to the previous step, q, node
classes).  The C2 line also reports node classification (`classify`) and the
adjoint on the jittered 20,480-face sphere (`grad_C3`).

Beside the GPU line: the FP64 oracle on one host core (`cpu_baseline`) and the same sample with its q phase
split over 16 oracle processes (`cpu_baseline_all_cores`; `--cpu-workers`).

`value` is cell-face tests per second: the number of (cell, face) pairs the
bins put in front of the cells (tested cells of every pass against the faces
of the bins under their query box, plus finest-level cells against the faces
under their link box; a fixed property of the workload) divided by the step
time.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0              # MI355X HBM3E
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # non-packed FP32 lane ops/s: 39.3 T
EPS = 2.0 ** -20
METRIC = "cell-face tests/s and near-wall pass ms (bin+flag+q) at 1 GPU; % HBM peak; grad ms"


# ---------------------------------------------------------------------------
# workload size: cell-face tests (host-side count from the bins and the forest)
# ---------------------------------------------------------------------------
def _bin_index_f32(x, lo, s, B):
    t = (x.astype(np.float32) - np.float32(lo)) * np.float32(s)
    f = np.floor(t)
    return np.clip(f, 0, B - 1).astype(np.int64)


def _bin_index_f64(x, lo, s, B):
    f = np.floor((x - lo) * s)
    return np.clip(f, 0, B - 1).astype(np.int64)


def _decode(keys, level, roots, dim):
    k = keys.astype(np.int64)
    path = np.zeros((len(k), 3), dtype=np.int64)
    for j in range(level):
        ci = k & ((1 << dim) - 1)
        k = k >> dim
        for a in range(dim):
            path[:, a] |= ((ci >> a) & 1) << j
    r = np.stack([k % roots[0], (k // roots[0]) % roots[1], k // (roots[0] * roots[1])], 1)
    return (r << level) | path


def cell_face_tests(offsets, B, dim, levels, roots, L, d_spec, lo, hi):
    """(T_flag per pass, T_q): sum over cells of the face counts of the bins under each
    cell's query box [m - h - eps, m + h + eps] (FP32 bin index) for the cells tested in
    each pass, and [x - dx - eps, x + dx + eps] (FP64) for every finest-level cell."""
    counts = np.diff(offsets.astype(np.int64))
    shape = (B,) * dim
    S = np.zeros(tuple(n + 1 for n in shape), dtype=np.int64)
    if dim == 3:
        S[1:, 1:, 1:] = counts.reshape(shape).cumsum(0).cumsum(1).cumsum(2)
    else:
        S[1:, 1:] = counts.reshape(shape).cumsum(0).cumsum(1)
    lo32 = np.asarray(lo, np.float32)[:dim]
    hi32 = np.asarray(hi, np.float32)[:dim]
    s32 = np.float32(B) / (hi32 - lo32)
    cells = 4 ** dim
    ci = np.arange(cells)
    off = np.stack([ci & 3, (ci >> 2) & 3, (ci >> 4) & 3], 1)[:, :dim]

    def box_sum(il, ih):
        if dim == 3:
            z0, y0, x0 = il[:, 2], il[:, 1], il[:, 0]
            z1, y1, x1 = ih[:, 2] + 1, ih[:, 1] + 1, ih[:, 0] + 1
            return (S[z1, y1, x1] - S[z0, y1, x1] - S[z1, y0, x1] - S[z1, y1, x0]
                    + S[z0, y0, x1] + S[z0, y1, x0] + S[z1, y0, x0] - S[z0, y0, x0])
        y0, x0 = il[:, 1], il[:, 0]
        y1, x1 = ih[:, 1] + 1, ih[:, 0] + 1
        return S[y1, x1] - S[y0, x1] - S[y1, x0] + S[y0, x0]

    def centres(keys, level, f64):
        c = _decode(keys, level, roots, dim)[:, :dim]
        g = (4 * c[:, None, :] + off[None]).reshape(-1, dim)
        dx = np.array([np.float32((hi32[a] - lo32[a]) / np.float32(4 * roots[a] * (1 << level))) for a in range(dim)])
        m = lo32 + (2 * g + 1).astype(np.float32) * (np.float32(0.5) * dx)
        return m.astype(np.float32), dx

    t_flag = []
    for l in range(L):
        lv = levels[l]
        if l == 0:
            tested = np.ones(len(lv["keys"]), bool)
        else:
            par = levels[l - 1]
            pk = par["keys"][par["mark"] == 1].astype(np.int64)
            tested = np.isin(lv["keys"].astype(np.int64) >> dim, pk)
        keys = lv["keys"][tested]
        if len(keys) == 0:
            t_flag.append(0)
            continue
        m, _ = centres(keys, l, False)
        h = np.float32(d_spec[l])
        ql = (m - h) - np.float32(EPS)
        qh = (m + h) + np.float32(EPS)
        il = np.stack([_bin_index_f32(ql[:, a], lo32[a], s32[a], B) for a in range(dim)], 1)
        ih = np.stack([_bin_index_f32(qh[:, a], lo32[a], s32[a], B) for a in range(dim)], 1)
        t_flag.append(int(box_sum(il, ih).sum()))
    keys = levels[L]["keys"]
    if len(keys) == 0:
        return t_flag, 0
    m, dx = centres(keys, L, True)
    m64, dx64 = m.astype(np.float64), dx.astype(np.float64)
    s64 = B / (hi32.astype(np.float64) - lo32.astype(np.float64))
    il = np.stack([_bin_index_f64(m64[:, a] - dx64[a] - EPS, float(lo32[a]), s64[a], B) for a in range(dim)], 1)
    ih = np.stack([_bin_index_f64(m64[:, a] + dx64[a] + EPS, float(lo32[a]), s64[a], B) for a in range(dim)], 1)
    return t_flag, int(box_sum(il, ih).sum())


# ---------------------------------------------------------------------------
def host_info():
    model, cores = platform.processor() or "unknown", os.cpu_count()
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return model, cores


Q_SAMPLE_BLOCKS = 4000   # finest-level blocks whose q the CPU baseline computes when a full pass is too long
Q_SAMPLE_SEED = 5


def cpu_baseline(wl, w_slots, T_total):
    """The CPU oracle as it stands, serial, on the same workload: bins and every refinement pass in full, then
    FP64 q and the FP64 adjoint for every finest-level block, or, when the finest level has more than
    Q_SAMPLE_BLOCKS blocks (a full q pass of the 327,680-face body is about 20 minutes on one core), for a seeded
    uniform sample of Q_SAMPLE_BLOCKS of them.  The rate is the cell-face tests the oracle performed divided by
    its time."""
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    r = oracle.run_plain(wl, with_links=False)
    t1 = time.perf_counter()
    fo = r["forest"]
    n_fin = len(fo.levels[wl.levels]["keys"])
    sub = None
    if n_fin > Q_SAMPLE_BLOCKS:
        rng = np.random.default_rng(Q_SAMPLE_SEED)
        sub = np.sort(rng.choice(n_fin, Q_SAMPLE_BLOCKS, replace=False))
    lk = oracle.link_fractions(wl.dim, r["coords"], r["bins"], fo, wl.lattice, sub)
    w = np.zeros((lk.n, wl.lattice))
    n = min(lk.n * wl.lattice, len(w_slots))
    w.reshape(-1)[:n] = w_slots[:n]
    w[lk.face < 0] = 0.0
    oracle.link_grad(fo, lk, r["coords"], wl.faces, w, len(wl.vertices))
    t2 = time.perf_counter()
    dt = t2 - t0
    T_orc = sum(fo.tests) + lk.tests
    model, _ = host_info()
    what = ("every finest-level cell" if sub is None else
            f"the cells of {len(sub)} of the {n_fin} finest-level blocks (seeded uniform sample, seed {Q_SAMPLE_SEED})")
    return {"value": T_orc / dt, "unit": "cell-face tests/s", "cores": 1, "kind": "oracle",
            "sample": f"{wl.name} on one host core ({model}): bins and {wl.levels} refinement passes in full "
                      f"(FP32 flags, {t1 - t0:.1f} s), then FP64 q and the FP64 adjoint for {what} "
                      f"({t2 - t1:.1f} s); rate = cell-face tests performed / time",
            "seconds": dt, "tests": int(T_orc), "refine_seconds": t1 - t0, "q_seconds": t2 - t1,
            "refine_tests": int(sum(fo.tests)), "q_tests": int(lk.tests),
            "q_blocks": n_fin if sub is None else len(sub), "finest_blocks": n_fin}


CPU_WORKERS = 16   # host cores that go with one GPU on the GPU machine


def _oracle_q_chunk(job):
    """One worker of the all-cores baseline: the oracle's bins and refinement of the workload, then FP64 q and the
    FP64 adjoint for one chunk of the sampled finest-level blocks; returns (q tests, q + adjoint seconds)."""
    name, sub = job
    import geomgen
    import oracle
    oracle.build(force=False)
    wl = geomgen.workload(name)
    r = oracle.run_plain(wl, with_links=False)
    t0 = time.perf_counter()
    lk = oracle.link_fractions(wl.dim, r["coords"], r["bins"], r["forest"], wl.lattice, sub)
    w = np.zeros((lk.n, wl.lattice))
    w_slots = geomgen.weights(max(1, lk.n * wl.lattice), 2)
    w.reshape(-1)[:] = w_slots[: lk.n * wl.lattice]
    w[lk.face < 0] = 0.0
    oracle.link_grad(r["forest"], lk, r["coords"], wl.faces, w, len(wl.vertices))
    return int(lk.tests), time.perf_counter() - t0


def cpu_all_cores(wl, serial, workers=CPU_WORKERS):
    """The serial baseline's sample with its q + adjoint phase split over `workers` processes, each running the
    oracle as it stands on one core (bins and refinement are one serial call in the oracle: their measured serial
    time is kept).  Rate = (refinement tests + q tests) / (serial refinement time + the slowest worker's q time)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    n_fin = serial["finest_blocks"]
    if n_fin > Q_SAMPLE_BLOCKS:
        sub = np.sort(np.random.default_rng(Q_SAMPLE_SEED).choice(n_fin, Q_SAMPLE_BLOCKS, replace=False))
    else:
        sub = np.arange(n_fin)
    chunks = [c for c in np.array_split(sub, min(workers, len(sub))) if len(c)]
    # fresh interpreters (spawn): the parent holds the GPU; a worker that dies ends the pool with an error
    # instead of being restarted, and the whole leg is bounded in time
    try:
        with cf.ProcessPoolExecutor(max_workers=len(chunks), mp_context=mp.get_context("spawn")) as ex:
            res = list(ex.map(_oracle_q_chunk, [(wl.name, c) for c in chunks], timeout=600))
    except Exception as e:   # noqa: BLE001 -- the baseline is reported as missing, with the reason
        print(f"bench: all-cores CPU baseline failed: {e!r}", file=sys.stderr, flush=True)
        return None
    q_tests = sum(t for t, _ in res)
    q_wall = max(dt for _, dt in res)
    T = serial["refine_tests"] + q_tests
    dt = serial["refine_seconds"] + q_wall
    model, _ = host_info()
    return {"value": T / dt, "unit": "cell-face tests/s", "cores": len(chunks), "kind": "oracle",
            "sample": f"{wl.name} on {len(chunks)} host cores ({model}): the serial sample's bins and refinement "
                      f"({serial['refine_seconds']:.1f} s, one core: the oracle refines in one call), then FP64 q "
                      f"and the FP64 adjoint of its {len(sub)} blocks split over {len(chunks)} processes "
                      f"(slowest {q_wall:.2f} s); rate = cell-face tests performed / time",
            "q_rate": q_tests / q_wall, "q_rate_one_core": serial["q_tests"] / serial["q_seconds"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=CPU_WORKERS,
                    help="host processes for the all-cores CPU baseline (1: the one-core baseline only)")
    ap.add_argument("--no-graph", action="store_true", help="skip the one-body graph timing")
    ap.add_argument("--no-grad-leg", action="store_true",
                    help="skip the gradient leg on the jittered 20,480-face sphere (profiling runs of one workload)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times) and exit: the reference kernel that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters into bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import torch
    import geomgen
    import paper_2502_16310_amd as agal

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 3}), flush=True)
        return
    if args.config.upper() == "C4":
        return bench_batch(args)
    if args.config.upper() in ("P0", "P1"):
        return bench_bin_density(args)
    if args.config.upper() == "M0":
        return bench_moving(args)
    wl = geomgen.workload(args.config)
    dim, Q = wl.dim, wl.lattice
    print(f"bench: {wl.name} faces={len(wl.faces)} roots={wl.roots[:dim]} levels={wl.levels} bins={wl.bins} "
          f"Q={Q}", file=sys.stderr, flush=True)
    v = torch.from_numpy(wl.vertices).to(dev)
    f = torch.from_numpy(wl.faces).to(dev)
    d_spec = [float(x) for x in wl.d_spec()]
    ctx = agal.agal_context_create()
    stream = torch.cuda.current_stream().cuda_stream
    desc = agal.forest_desc(dim, wl.roots[:dim], wl.levels, d_spec, wl.lo[:dim], wl.hi[:dim])
    grad = torch.zeros((len(wl.vertices), dim), dtype=torch.float32, device=dev)
    w_host = geomgen.weights(4 ** dim * 4 * 10 ** 6, 2)  # enough slots; first n*Q used
    w_dev = None

    def step(keep=False, ev=None):
        nonlocal w_dev
        g = agal.agal_import_faces(ctx, dim, v.data_ptr(), v.shape[0], f.data_ptr(), f.shape[0], stream)
        if ev:
            ev[0].record()
        b = agal.agal_bin_faces(g, wl.lo[:dim], wl.hi[:dim], wl.bins, stream)
        fo = agal.agal_near_wall_refine(g, b, desc, stream)
        lk = agal.agal_link_fractions(g, b, fo, Q, stream)
        if ev:
            ev[1].record()
        n_nodes = agal.agal_links_view(lk)[3]
        if w_dev is None or w_dev.numel() < n_nodes * Q:
            w_dev = torch.from_numpy(w_host[: max(1, n_nodes * Q)].copy()).to(dev)
        grad.zero_()
        agal.agal_link_fractions_backward(g, lk, w_dev.data_ptr(), grad.data_ptr(), stream)
        if ev:
            ev[2].record()
        if keep:
            return g, b, fo, lk
        for h, fn in ((lk, agal.agal_destroy_links), (fo, agal.agal_destroy_forest), (b, agal.agal_destroy_bins),
                      (g, agal.agal_destroy_geom)):
            fn(h)
        return None

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # workload size, from this GPU run's own bins and forest (outside the timed region)
    g, b, fo, lk = step(keep=True)
    torch.cuda.synchronize()
    off_p, _, nb, P = agal.agal_bins_view(b)
    off = agal.device_copy(off_p, nb + 1, torch.int32).cpu().numpy().view(np.uint32)
    levels = []
    for l in range(wl.levels + 1):
        kp, _, mp, _, n = agal.agal_forest_level_view(fo, l)
        levels.append({"keys": agal.device_copy(kp, n, torch.int32).cpu().numpy().view(np.uint32),
                       "mark": agal.device_copy(mp, n, torch.uint8).cpu().numpy()})
    n_nodes = agal.agal_links_view(lk)[3]
    t_flag, t_q = cell_face_tests(off, wl.bins, dim, levels, wl.roots, wl.levels, d_spec, wl.lo, wl.hi)
    T = sum(t_flag) + t_q
    n_links = int((agal.device_copy(agal.agal_links_view(lk)[2], n_nodes * Q, torch.int32) >= 0).sum().item())
    n_blocks = [len(l["keys"]) for l in levels]
    classify = classify_leg(args, agal, torch, g, lk, n_nodes, Q, dim, len(wl.faces), stream)
    for h, fn in ((lk, agal.agal_destroy_links), (fo, agal.agal_destroy_forest), (b, agal.agal_destroy_bins),
                  (g, agal.agal_destroy_geom)):
        fn(h)

    # timed region: K whole steps (the value).  HIP events on the launch
    # stream (torch's current stream) bracket the near-wall pass (bins ->
    # refinement -> q, in-pass host synchronisations included) and the adjoint
    # of every step.
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(ev=evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    pass_ev = sorted(e[0].elapsed_time(e[1]) for e in evs)
    grad_ev = sorted(e[1].elapsed_time(e[2]) for e in evs)
    # second timed region: the same K steps with the library recording events
    # around each of its kernels (per-kernel averages and the roofline; the
    # extra event records would otherwise inflate the step time above)
    agal.agal_profile_read(ctx)
    agal.agal_profile_enable(ctx, True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    agal.agal_profile_enable(ctx, False)
    prof = agal.agal_profile_read(ctx)
    ms_profiled = (tp1 - tp0) * 1e3 / args.steps
    graph = None if args.no_graph else graph_step(args, agal, torch, wl, v, f, w_host, n_nodes, T)
    pass_ms_median = pass_ev[len(pass_ev) // 2]
    grad_step_median = grad_ev[len(grad_ev) // 2]
    copy_gbs = copy_bandwidth(torch, dev)
    kern = {k: {"launches_per_step": n / args.steps, "ms_per_step": t / args.steps, "avg_us": 1e3 * t / n}
            for k, (n, t) in prof.items()}
    pass_kernels = ("bin_count", "bin_scatter", "bin_canon", "bin_canon_big", "scan_exclusive", "flag_sat",
                    "balance_ripple", "child_gen") + Q_STEP
    pass_kernel_ms = sum(kern[k]["ms_per_step"] for k in pass_kernels if k in kern)
    grad_ms = kern.get("q_adjoint", {}).get("ms_per_step", 0.0)
    # the link step as one unit (candidate lists, node pass, row pass; or the bin walk and compaction): its
    # algorithmic work is one figure for the whole step
    q_ms = sum(kern[k]["ms_per_step"] for k in Q_STEP if k in kern)
    groups = {k: v for k, v in kern.items() if k not in Q_STEP}
    groups["q_step"] = {"launches_per_step": 1.0, "ms_per_step": q_ms, "avg_us": 1e3 * q_ms,
                        "kernels": [k for k in Q_STEP if k in kern]}
    dominant = max(groups, key=lambda k: groups[k]["ms_per_step"])
    hbm_pass = pass_hbm_bytes(dim, Q, len(wl.faces), nb, P, n_blocks, n_nodes, wl.levels)

    # roofline of the dominant kernel
    F = len(wl.faces)
    roof = roofline(dominant, groups[dominant], dim=dim, Q=Q, F=F, nb=nb, P=P, n_blocks=n_blocks, n_nodes=n_nodes,
                    t_flag=t_flag, t_q=t_q, L=wl.levels, workload=wl.name)

    out = {
        "metric": METRIC, "value": T / (ms * 1e-3), "unit": "cell-face tests/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{wl.name}: " + describe(wl), "faces": F, "roots": list(wl.roots[:dim]),
                   "levels": wl.levels, "bins": wl.bins, "lattice": f"D{dim}Q{Q}", "global_batch": 1,
                   "seq_len": 0, "parallelism": "none"},
        "ms_per_step_with_kernel_events": ms_profiled, "graph": graph,
        "near_wall_pass_ms": pass_ms_median, "near_wall_pass_kernel_ms": pass_kernel_ms,
        "grad_ms": grad_ms, "grad_step_ms": grad_step_median,
        "near_wall_pass_hbm": {"algorithmic_bytes": hbm_pass,
                               "GBps": hbm_pass / (pass_ms_median * 1e-3) / 1e9,
                               "frac_of_peak": hbm_pass / (pass_ms_median * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               "frac_of_copy": hbm_pass / (pass_ms_median * 1e-3) / 1e9 / copy_gbs,
                               "copy_GBps": copy_gbs},
        "cell_face_tests": {"flag_per_pass": t_flag, "q": t_q, "total": T,
                            "per_s_pass": T / (pass_ms_median * 1e-3),
                            "flag_per_s": sum(t_flag) / (kern["flag_sat"]["ms_per_step"] * 1e-3)
                            if "flag_sat" in kern else None,
                            "q_per_s": t_q / (q_ms * 1e-3) if q_ms > 0 else None},
        "forest_blocks_per_level": n_blocks, "boundary_nodes": n_nodes, "links": n_links,
        "kernels": kern, "roofline": roof, "classify": classify,
    }
    if wl.name != "C3" and not args.no_grad_leg:
        out["grad_C3"] = grad_c3(args, agal, torch, dev)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on the same workload", file=sys.stderr, flush=True)
        cb = cpu_baseline(wl, w_host.astype(np.float64), T)
        out["cpu_baseline"] = cb
        if args.cpu_workers > 1:
            print(f"bench: the same sample on {args.cpu_workers} host cores", file=sys.stderr, flush=True)
            out["cpu_baseline_all_cores"] = cpu_all_cores(wl, cb, args.cpu_workers)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def classify_leg(args, agal, torch, g, lk, n_nodes, Q, dim, F, stream):
    """The step after q: the side of every boundary node (agal_classify_nodes), timed on its own with HIP
    events on the launch stream over 20 launches on this step's links.  Algorithmic HBM bytes: the face-id
    rows (n_nodes x Q x 4 B) read once, one class byte per node written, every face record (16 FP32 in 3D,
    8 in 2D) read once for the per-face sign words, which are written and read back once (8 B each way)."""
    if n_nodes == 0:
        return None
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.empty(n_nodes, dtype=torch.uint8, device=dev)
    agal.agal_classify_nodes(g, lk, out.data_ptr(), stream)
    torch.cuda.synchronize()
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        agal.agal_classify_nodes(g, lk, out.data_ptr(), stream)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = n_nodes * Q * 4 + n_nodes + F * ((64 if dim == 3 else 32) + 16)
    counts = torch.bincount(out.long(), minlength=4)[1:].tolist()
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"ms": ms, "algorithmic_bytes": nbytes, "GBps": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
            "nodes_fluid_solid_mixed": counts}


def grad_c3(args, agal, torch, dev):
    """The differentiated form on its own workload: the jittered 20,480-face sphere (C3, D3Q19) with weights
    U(-1, 1) (seed 2) on every link slot.  HIP events on the launch stream time the adjoint launch alone and the
    whole forward (import, bins, refinement, q) plus backward; medians over K runs."""
    import geomgen
    wl = geomgen.workload("C3")
    dim, Q = wl.dim, wl.lattice
    print(f"bench: gradient leg on {wl.name} ({len(wl.faces)} faces, D{dim}Q{Q})", file=sys.stderr, flush=True)
    ctx = agal.agal_context_create()
    stream = torch.cuda.current_stream().cuda_stream
    v = torch.from_numpy(wl.vertices).to(dev)
    f = torch.from_numpy(wl.faces).to(dev)
    desc = agal.forest_desc(dim, wl.roots[:dim], wl.levels, [float(x) for x in wl.d_spec()], wl.lo[:dim],
                            wl.hi[:dim])
    grad = torch.zeros((len(wl.vertices), dim), dtype=torch.float32, device=dev)
    w_host = None
    w_dev = None
    adj, tot = [], []
    n_links = 0
    for k in range(args.warmup + args.steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        g = agal.agal_import_faces(ctx, dim, v.data_ptr(), v.shape[0], f.data_ptr(), f.shape[0], stream)
        b = agal.agal_bin_faces(g, wl.lo[:dim], wl.hi[:dim], wl.bins, stream)
        fo = agal.agal_near_wall_refine(g, b, desc, stream)
        lk = agal.agal_link_fractions(g, b, fo, Q, stream)
        n = agal.agal_links_view(lk)[3]
        if w_dev is None:
            face = agal.device_copy(agal.agal_links_view(lk)[2], n * Q, torch.int32)
            w_host = geomgen.weights(n * Q, wl.extra["weights_seed"])
            w_dev = torch.from_numpy(w_host).to(dev) * (face >= 0)
            n_links = int((face >= 0).sum().item())
        grad.zero_()
        e[1].record()
        agal.agal_link_fractions_backward(g, lk, w_dev.data_ptr(), grad.data_ptr(), stream)
        e[2].record()
        for h, fn in ((lk, agal.agal_destroy_links), (fo, agal.agal_destroy_forest), (b, agal.agal_destroy_bins),
                      (g, agal.agal_destroy_geom)):
            fn(h)
        torch.cuda.synchronize()
        if k >= args.warmup:
            adj.append(e[1].elapsed_time(e[2]))
            tot.append(e[0].elapsed_time(e[2]))
    agal.agal_context_destroy(ctx)
    adj.sort()
    tot.sort()
    return {"workload": "C3: icosphere subdivision 5 (20480 triangles) r=0.2, vertices jittered N(0,1e-3) seed 1, "
                        "weights U(-1,1) seed 2, D3Q19",
            "adjoint_ms": adj[len(adj) // 2], "forward_backward_ms": tot[len(tot) // 2], "live_links": n_links}


def graph_step(args, agal, torch, wl, v, f, w_host, n_nodes, T):
    """The same step as the batched form with one body: planned once (untimed, the plan runs the single-body
    calls to size every array), then K replays of one captured graph (import, bins, refinement, q, adjoint;
    no host synchronisation inside).  Results are identical to the single-body calls (tests/test_gpu_batch.py)."""
    dim, Q = wl.dim, wl.lattice
    cfg = agal.NearWallConfig(dim=dim, roots=wl.roots[:dim], n_levels=wl.levels, bins=wl.bins, lattice=Q,
                              lo=wl.lo[:dim], hi=wl.hi[:dim], d_spec=list(wl.d_spec()[:wl.levels]))
    t0 = time.perf_counter()
    bt = agal.Batch([(v, f, cfg)], tune_bins=False, tune_grid=True, with_adjoint=True)
    plan_s = time.perf_counter() - t0
    bt.run()
    bt.status()
    n = bt.links(0)[0].numel()
    assert n == n_nodes, (n, n_nodes)
    bt.set_grad_q(0, torch.from_numpy(w_host[: max(1, n * Q)][: n * Q].reshape(n, Q)).to(v.device))
    for _ in range(args.warmup):
        bt.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bt.run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    bt.status()
    return {"ms_per_step": ms, "value": T / (ms * 1e-3), "plan_s": plan_s, "workgroups_per_cu": bt.workgroups_per_cu}


def bench_batch(args):
    """64 star bodies (subdivision 3..7, D3Q27) as one graph launch (forward q + adjoint), against the
    same bodies run one after another through the single-body calls at the plan's bin densities."""
    import torch
    import geomgen
    import paper_2502_16310_amd as agal

    dev = torch.device("cuda", 0)
    draws = geomgen.batch_draws(64)
    wls = [geomgen.batch_body(d) for d in draws]
    ts = [(torch.from_numpy(w.vertices).to(dev), torch.from_numpy(w.faces).to(dev)) for w in wls]
    F_total = sum(len(w.faces) for w in wls)
    print(f"bench: C4 batch of {len(wls)} star bodies, {F_total} faces", file=sys.stderr, flush=True)
    cfgs = [agal.NearWallConfig(dim=3, roots=w.roots, n_levels=w.levels, bins=0, lattice=w.lattice,
                                d_spec=list(w.d_spec()[:w.levels])) for w in wls]
    t0 = time.perf_counter()
    bt = agal.Batch([(v, f, c) for (v, f), c in zip(ts, cfgs)], tune_bins=True, tune_grid=True, with_adjoint=True)
    plan_s = time.perf_counter() - t0
    bins = [bt.bins(i) for i in range(len(wls))]
    print(f"bench: plan {plan_s:.1f} s, grid {bt.workgroups_per_cu} workgroups/CU, bins {sorted(set(bins))}",
          file=sys.stderr, flush=True)
    bt.run()
    bt.status()
    weights = []
    for i, w in enumerate(wls):
        n = bt.links(i)[0].numel()
        wt = torch.from_numpy(geomgen.weights(max(1, n * w.lattice), 2 + i)[: n * w.lattice].reshape(n, w.lattice))
        weights.append(wt.to(dev))
        bt.set_grad_q(i, weights[-1])

    # single-body path, body after body, same bins and adjoint weights
    ctx = agal.agal_context_create()
    stream = torch.cuda.current_stream().cuda_stream
    grads = [torch.zeros_like(v) for v, _ in ts]
    descs = [agal.forest_desc(3, w.roots, w.levels, [float(x) for x in w.d_spec()], w.lo, w.hi) for w in wls]

    def plain_all(keep=False):
        kept = []
        for i, w in enumerate(wls):
            v, f = ts[i]
            g = agal.agal_import_faces(ctx, 3, v.data_ptr(), v.shape[0], f.data_ptr(), f.shape[0], stream)
            b = agal.agal_bin_faces(g, w.lo, w.hi, bins[i], stream)
            fo = agal.agal_near_wall_refine(g, b, descs[i], stream)
            lk = agal.agal_link_fractions(g, b, fo, w.lattice, stream)
            grads[i].zero_()
            agal.agal_link_fractions_backward(g, lk, weights[i].data_ptr(), grads[i].data_ptr(), stream)
            hs = ((lk, agal.agal_destroy_links), (fo, agal.agal_destroy_forest), (b, agal.agal_destroy_bins),
                  (g, agal.agal_destroy_geom))
            if keep:
                kept.append((g, b, fo, lk))
            else:
                for h, fn in hs:
                    fn(h)
        return kept

    for _ in range(args.warmup):
        plain_all()
        bt.run()
    torch.cuda.synchronize()
    # workload size per body from the single-body results (identical to the batch's)
    T = 0
    T_flag = T_q = 0
    kept = plain_all(keep=True)
    torch.cuda.synchronize()
    n_nodes = 0
    for i, (w, (g, b, fo, lk)) in enumerate(zip(wls, kept)):
        off_p, _, nb, P = agal.agal_bins_view(b)
        off = agal.device_copy(off_p, nb + 1, torch.int32).cpu().numpy().view(np.uint32)
        levels = []
        for l in range(w.levels + 1):
            kp, _, mp, _, n = agal.agal_forest_level_view(fo, l)
            levels.append({"keys": agal.device_copy(kp, n, torch.int32).cpu().numpy().view(np.uint32),
                           "mark": agal.device_copy(mp, n, torch.uint8).cpu().numpy()})
        tf, tq = cell_face_tests(off, bins[i], 3, levels, w.roots, w.levels, [float(x) for x in w.d_spec()],
                                 w.lo, w.hi)
        T += sum(tf) + tq
        T_flag += sum(tf)
        T_q += tq
        n_nodes += agal.agal_links_view(lk)[3]
        for h, fn in ((lk, agal.agal_destroy_links), (fo, agal.agal_destroy_forest), (b, agal.agal_destroy_bins),
                      (g, agal.agal_destroy_geom)):
            fn(h)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_all()
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3 / args.steps

    agal.agal_profile_read(bt.ctx.h)
    agal.agal_profile_enable(bt.ctx.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bt.run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    agal.agal_profile_enable(bt.ctx.h, False)
    prof = agal.agal_profile_read(bt.ctx.h)
    bt.status()
    graph_us = 1e3 * prof["batch_graph"][1] / prof["batch_graph"][0] if "batch_graph" in prof else None

    out = {
        "metric": METRIC, "value": T / (ms * 1e-3), "unit": "cell-face tests/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "C4: 64 star bodies, icosphere subdivisions 3-7, roots 16^3 (3 levels) or 32^3 "
                               "(4 levels), D3Q27, forward q + adjoint, one graph launch",
                   "faces": F_total, "bodies": len(wls), "global_batch": len(wls), "seq_len": 0,
                   "parallelism": "none"},
        "batch_graph_ms": ms, "batch_graph_event_us": graph_us, "plain_sum_ms": plain_ms,
        "speedup_vs_plain": plain_ms / ms, "plan_s": plan_s, "workgroups_per_cu": bt.workgroups_per_cu,
        "bins_per_body": bins, "cell_face_tests": T, "boundary_nodes": n_nodes,
        "roofline": batch_roofline(T_flag, T_q, graph_us if graph_us else 1e3 * ms),
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        # the oracle on one subdivision-4 body of the batch (its rate in the batch's unit)
        i = next(i for i, d in enumerate(draws) if d["s"] == 4)
        print(f"bench: timing the CPU oracle on body {i} of the batch", file=sys.stderr, flush=True)
        import dataclasses
        wl_i = dataclasses.replace(wls[i], bins=bins[i])   # the bin density the plan chose for it
        cb = cpu_baseline(wl_i, geomgen.weights(4 ** 3 * 4 * 10 ** 6, 2 + i).astype(np.float64), None)
        cb["sample"] = f"body {i} of the batch ({len(wls[i].faces)} faces): " + cb["sample"]
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def batch_roofline(t_flag, t_q, graph_us):
    """Roofline of the whole batched graph as one unit: its arithmetic work is the flag tests (24 ops per
    (cell, candidate face) pair) plus the link step (8 ops per pair), against the non-packed FP32 VALU peak;
    the graph's other kernels (bins, scans, balance, adjoint) count as time but not as work."""
    ops = OPS_PER_PAIR["flag_sat"] * t_flag + OPS_PER_PAIR["q_step"] * t_q
    tops = ops / (graph_us * 1e-6) / 1e12
    return {"bound": "alu", "achieved": tops, "peak": VALU_PEAK_TOPS, "unit": "TFLOP/s",
            "frac": tops / VALU_PEAK_TOPS, "traffic": None, "kernel": "batch_graph (whole graph)",
            "ops_per_launch": ops, "flag_pairs": t_flag, "q_pairs": t_q, "avg_launch_us": graph_us}


def bench_moving(args):
    """A moving body: the 327,680-face star translated by (0.37, 0.21, -0.13) finest cells per step.  Each step
    re-adapts from the moved faces: import, bins, refinement from the roots, the relation to the previous
    step's forest (kept / created / refined / coarsened / removed blocks), link fractions and node classes.
    The vertex positions of every step are prepared on the device before the timed region; HIP events on the
    launch stream bracket each step; per-kernel times come from a second, profiled pass."""
    import torch
    import geomgen
    import paper_2502_16310_amd as agal

    dev = torch.device("cuda", 0)
    wl = geomgen.workload("C2")
    dim, Q = wl.dim, wl.lattice
    dx = float(wl.cell_size(wl.levels))
    step = np.array([0.37, 0.21, -0.13]) * dx
    K, W = args.steps, args.warmup
    print(f"bench: M0 moving star, {len(wl.faces)} faces, {K} steps of {step.tolist()}", file=sys.stderr, flush=True)
    f = torch.from_numpy(wl.faces).to(dev)
    vs = [torch.from_numpy((wl.vertices + (step * k).astype(np.float32)).astype(np.float32)).to(dev)
          for k in range(W + 2 * K + 1)]
    d_spec = [float(x) for x in wl.d_spec()]
    ctx = agal.agal_context_create()
    stream = torch.cuda.current_stream().cuda_stream
    desc = agal.forest_desc(dim, wl.roots[:dim], wl.levels, d_spec, wl.lo[:dim], wl.hi[:dim])
    cls = torch.empty(8 << 20, dtype=torch.uint8, device=dev)

    def build(k):
        v = vs[k]
        g = agal.agal_import_faces(ctx, dim, v.data_ptr(), v.shape[0], f.data_ptr(), f.shape[0], stream)
        b = agal.agal_bin_faces(g, wl.lo[:dim], wl.hi[:dim], wl.bins, stream)
        fo = agal.agal_near_wall_refine(g, b, desc, stream)
        return g, b, fo

    def step_once(prev, k, ev=None):
        nonlocal cls
        if ev:
            ev[0].record()
        g, b, fo = build(k)
        d = agal.agal_forest_diff_create(prev[2], fo, stream)
        lk = agal.agal_link_fractions(g, b, fo, Q, stream)
        n = agal.agal_links_view(lk)[3]
        if n > cls.numel():
            cls = torch.empty(2 * n, dtype=torch.uint8, device=dev)
        agal.agal_classify_nodes(g, lk, cls.data_ptr(), stream)
        if ev:
            ev[1].record()
        counts = [agal.agal_forest_diff_view(d, l)[5] for l in range(wl.levels + 1)]
        agal.agal_destroy_forest_diff(d)
        agal.agal_destroy_links(lk)
        for h, fn in ((prev[2], agal.agal_destroy_forest), (prev[1], agal.agal_destroy_bins),
                      (prev[0], agal.agal_destroy_geom)):
            fn(h)
        return (g, b, fo), counts, n

    cur = build(0)
    k = 1
    for _ in range(W):
        cur, _, _ = step_once(cur, k)
        k += 1
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(K)]
    all_counts, nodes = [], []
    t0 = time.perf_counter()
    for i in range(K):
        cur, c, n = step_once(cur, k, evs[i])
        all_counts.append(c)
        nodes.append(n)
        k += 1
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / K
    ev_ms = sorted(e[0].elapsed_time(e[1]) for e in evs)
    agal.agal_profile_read(ctx)
    agal.agal_profile_enable(ctx, True)
    for _ in range(K):
        cur, _, _ = step_once(cur, k)
        k += 1
    torch.cuda.synchronize()
    agal.agal_profile_enable(ctx, False)
    prof = agal.agal_profile_read(ctx)
    for h, fn in ((cur[2], agal.agal_destroy_forest), (cur[1], agal.agal_destroy_bins), (cur[0], agal.agal_destroy_geom)):
        fn(h)
    kern = {name: {"ms_per_step": t / K, "launches_per_step": n / K} for name, (n, t) in prof.items()}
    tot = np.array(all_counts).sum(axis=0)   # levels x 4
    out = {
        "metric": "moving-body re-adaptation steps/s", "value": 1e3 / ms, "unit": "steps/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "M0: C2 star body translated by (0.37, 0.21, -0.13) finest cells per step; per step "
                               "import, bins, refinement, forest relation, D3Q27 link fractions, node classes",
                   "faces": len(wl.faces), "roots": list(wl.roots[:dim]), "levels": wl.levels, "bins": wl.bins},
        "step_event_ms_median": ev_ms[len(ev_ms) // 2], "boundary_nodes_mean": float(np.mean(nodes)),
        "blocks_per_step_created_refined_coarsened_removed": (tot / K).tolist(),
        "kernels": kern,
    }
    print(json.dumps(out), flush=True)


def bench_bin_density(args):
    """The paper's bin-density study on its own refinement form: the Euclidean near test against the
    faces of each cell centre's own bin, then mark propagation (P0: 12,800-segment circle, 256^2 cells,
    d = 0.1; P1: 81,920-face star, 64^3 cells, d = 0.05; two passes), for B in 1, 2, 8, 16: bin setup and
    refinement times (HIP events, medians of K runs) and the blocks the refinement inserts, beside the
    bin-independent closed-box refinement of the same body."""
    import torch
    import geomgen
    import paper_2502_16310_amd as agal

    dev = torch.device("cuda", 0)
    wl = geomgen.workload(args.config)
    dim = wl.dim
    print(f"bench: {wl.name} own-bin refinement, faces={len(wl.faces)} roots={wl.roots[:dim]} "
          f"levels={wl.levels} d={float(wl.d_spec()[0])}", file=sys.stderr, flush=True)
    v = torch.from_numpy(wl.vertices).to(dev)
    f = torch.from_numpy(wl.faces).to(dev)
    ctx = agal.agal_context_create()
    stream = torch.cuda.current_stream().cuda_stream
    desc = agal.forest_desc(dim, wl.roots[:dim], wl.levels, [float(x) for x in wl.d_spec()], wl.lo[:dim],
                            wl.hi[:dim])
    g = agal.agal_import_faces(ctx, dim, v.data_ptr(), v.shape[0], f.data_ptr(), f.shape[0], stream)

    def run(B, own_bin, binning="box", bf=0):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        if binning == "box":
            b = agal.agal_bin_faces(g, wl.lo[:dim], wl.hi[:dim], B, stream)
        else:
            b = agal.agal_bin_faces_discrete(g, wl.lo[:dim], wl.hi[:dim], B, 0.0, bf, stream)
        e[1].record()
        fo = (agal.agal_near_wall_refine_own_bin(g, b, desc, -1, stream) if own_bin
              else agal.agal_near_wall_refine(g, b, desc, stream))
        e[2].record()
        torch.cuda.synchronize()
        levels = []
        for l in range(wl.levels + 1):
            _, _, mp, _, n = agal.agal_forest_level_view(fo, l)
            marks = agal.device_copy(mp, n, torch.uint8).cpu().numpy() if n else np.zeros(0, np.uint8)
            levels.append((n, np.bincount(marks, minlength=4)[:4].tolist()))
        agal.agal_destroy_forest(fo)
        agal.agal_destroy_bins(b)
        return e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), levels

    curve = []
    # own-bin refinement on bounding-box bins and on the paper's sampled-point bins (the pairs form) over the
    # paper's bin densities; the closed-box refinement; then the paper's bin-fraction form at one density
    paper_Bs = (1, 2, 4, 6, 7, 8, 9, 10, 12, 14, 16)
    plan = [(True, B, "box", 0) for B in (1, 2, 8, 16)] + [(True, B, "sampled", 0) for B in paper_Bs] + \
           [(False, 8, "box", 0)] + [(True, 16, "sampled", bf) for bf in (1, 2, 4, 8, 16)]
    for own_bin, B, binning, bf in plan:
        for _ in range(args.warmup):
            run(B, own_bin, binning, bf)
        t_bin, t_ref = [], []
        for _ in range(args.steps):
            tb, tr, levels = run(B, own_bin, binning, bf)
            t_bin.append(tb)
            t_ref.append(tr)
        t_bin.sort()
        t_ref.sort()
        blocks = [n for n, _ in levels]
        form = "own-bin Euclidean + propagation" if own_bin else "closed box (all bins under it)"
        bins_kind = ("bounding-box bins" if binning == "box" else
                     "sampled-point bins" + (f", bin fraction {bf}" if bf else ", pairs form"))
        curve.append({"form": form, "bins": bins_kind, "B": B, "bin_fraction": bf,
                      "bin_ms": t_bin[len(t_bin) // 2], "refine_ms": t_ref[len(t_ref) // 2],
                      "blocks_per_level": blocks, "inserted_blocks": int(sum(blocks[1:])),
                      "marks_flag_balance_propagation": [m[1:4] for _, m in levels[:-1]]})
        print(f"bench: {form}, {bins_kind}, B={B}: bins {curve[-1]['bin_ms']:.3f} ms, refinement "
              f"{curve[-1]['refine_ms']:.3f} ms, blocks {blocks}", file=sys.stderr, flush=True)
    agal.agal_destroy_geom(g)
    agal.agal_context_destroy(ctx)
    best = min((c for c in curve if c["form"].startswith("own") and c["bins"] == "bounding-box bins"),
               key=lambda c: c["bin_ms"] + c["refine_ms"])
    out = {"metric": "near-wall refinement ms (bins + passes) vs bin density, own-bin form", "value":
           best["bin_ms"] + best["refine_ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": best["bin_ms"] + best["refine_ms"], "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{wl.name}: " + describe(wl), "faces": len(wl.faces), "roots": list(wl.roots[:dim]),
                      "levels": wl.levels, "d": float(wl.d_spec()[0]), "global_batch": 1, "seq_len": 0,
                      "parallelism": "none"},
           "best_B": best["B"], "curve": curve, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def copy_bandwidth(torch, dev, mib=1024, reps=5):
    """Device-to-device copy rate (read + write bytes / s): the measured second denominator for % HBM."""
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    return gbs


def describe(wl):
    if wl.name == "C0":
        return "2D circle r=0.25, 256 segments"
    if wl.name == "C1":
        return "icosphere subdivision 5 (20480 triangles) r=0.2"
    if wl.name == "C2":
        return "star body on icosphere subdivision 7 (327680 triangles), seed 0"
    if wl.name == "C3":
        return "C1 sphere jittered N(0,1e-3), seed 1"
    if wl.name == "P0":
        return "circle r=0.25, 12800 segments, 256^2 cells, d=0.1, 2 passes"
    if wl.name == "P1":
        return "star body on icosphere subdivision 6 (81920 triangles), 64^3 cells, d=0.05, 2 passes"
    return wl.name


# FP32 operations charged per (cell, candidate face) pair: the least work a candidate costs.  Link kernel: one
# face-box cull against the link box, 8 ops; flag kernel: the rejection of one separating-axis test by the box
# axes, 24 ops.
OPS_PER_PAIR = {"q_step": 8, "flag_sat": 24}

# Library timing names of the link step's kernels: list mode (candidate lists, node pass, node map + row pass)
# and walk mode (the bin walk, then the compaction).
Q_STEP = ("q_lists", "q_nodes", "q_links", "q_compact")

# Library timing names -> the kernel symbols (as profilers list them) launched under that name, and the source
# each is built from.
KERNEL_SYMBOL = {"flag_sat": (("k_flag_faces",), "refine.hip"), "q_links": (("k_node_map", "k_links_rows"), "links.hip"),
                 "q_nodes": (("k_links_nodes",), "links.hip"), "q_lists": (("k_link_blocks", "k_link_faces"), "links.hip"),
                 "q_adjoint": (("k_adjoint",), "links.hip"), "q_compact": (("k_compact_nodes",), "links.hip"),
                 "bin_canon": (("k_bin_canon_small", "k_bin_canon_medium"), "bins.hip"),
                 "classify": (("k_classify_nodes",), "links.hip")}


def kernel_source_hash(name):
    """sha256 of the sources a kernel is compiled from (its .hip file and the shared device headers)."""
    import hashlib
    if name not in KERNEL_SYMBOL:
        return None
    csrc = os.path.join(ROOT, "paper_2502_16310_amd", "csrc")
    h = hashlib.sha256()
    for fn in (KERNEL_SYMBOL[name][1], "kernels.hpp", "device.hpp"):
        with open(os.path.join(csrc, fn), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name, workload):
    """HBM bytes per launch of timing name `name` (all the kernels launched under it) on `workload` from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (profiles/traffic.json, counters scaled by a plain copy of
    known size); None when there is none or the kernels' sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        table = json.load(fh)
    e = table.get(workload, {}).get(name)
    if not e or e.get("source_sha256") != kernel_source_hash(name):
        return None
    return e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]


def roofline(name, k, dim, Q, F, nb, P, n_blocks, n_nodes, t_flag, t_q, L, workload=None):
    """Roofline entry of kernel `name` from its average launch time.

    flag_sat / q_links are arithmetic kernels: algorithmic work = the (cell,
    candidate face) pairs the bins present (t_flag per pass / t_q) times the
    OPS_PER_PAIR every candidate costs at least, against the FP32 VALU peak
    without packed math or FMA (256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T
    op/s).
    Streaming kernels are charged their compulsory HBM bytes."""
    us = k["avg_us"]
    launches = k["launches_per_step"]
    cells = 4 ** dim
    face_bytes = F * (4 * dim * dim + 8 * dim)           # SoA coordinates + bounding boxes
    csr_bytes = 4 * (nb + 1) + 4 * P
    if name in ("flag_sat", "q_step"):
        pairs = (sum(t_flag) / max(1, launches)) if name == "flag_sat" else t_q
        ops = OPS_PER_PAIR[name] * pairs
        tops = ops / (us * 1e-6) / 1e12
        if name == "q_step":
            parts = [measured_traffic(kn, workload) for kn in k["kernels"]]
            traffic = sum(parts) if parts and all(x is not None for x in parts) else None
        else:
            traffic = measured_traffic(name, workload)
        out = {"bound": "alu", "achieved": tops, "peak": VALU_PEAK_TOPS, "unit": "TFLOP/s",
               "frac": tops / VALU_PEAK_TOPS, "traffic": traffic, "kernel": name,
               "ops_per_pair": OPS_PER_PAIR[name], "ops_per_launch": ops,
               "cell_face_pairs_per_launch": pairs, "avg_launch_us": us}
        if name == "q_step":
            out["step_kernels"] = k["kernels"]
        return out
    if name == "q_adjoint":
        byts = n_nodes * (8 + 8 * Q) + face_bytes + 4 * F * dim + 4 * dim * 4 * F
    elif name == "q_compact":
        byts = 2 * n_nodes * (8 + 8 * Q)
    elif name == "bin_canon":
        byts = 2 * 4 * P + 4 * (nb + 1)
    else:
        byts = None
    if byts is None:
        return {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                "traffic": None, "kernel": name}
    gbs = byts / (us * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": measured_traffic(name, workload), "kernel": name, "bytes_per_launch": byts,
            "avg_launch_us": us}


def pass_hbm_bytes(dim, Q, F, nb, P, n_blocks, n_nodes, L):
    """Compulsory HBM bytes of one near-wall pass (bins + all levels + q write-back)."""
    cells = 4 ** dim
    face_bytes = F * (4 * dim * dim + 8 * dim)
    bins = face_bytes + 8 * (nb + 1) + 8 * P
    flags = sum(n_blocks[:L]) * (4 + cells + 1) + L * (face_bytes + 4 * (nb + 1) + 4 * P)
    refine = sum(n_blocks) * 8
    q = 4 * n_blocks[L] + face_bytes + 4 * (nb + 1) + 4 * P + n_nodes * (8 + 8 * Q)
    return bins + flags + refine + q


if __name__ == "__main__":
    main()
