"""Benchmark: iHS core loci per second on one MI355X.

Workload (synthetic, seeded): 204 haplotypes x 22,147 biallelic SNPs over
35 Mb, copying model with 40 founders and switch probability 0.003, one
planted sweep carried by 70% of the haplotypes (the chromosome-22-shaped
configuration; the paper's CEU chr22 data are not available).

A step is one pass of the whole hot path on device-resident inputs: bit
packing of the uint8 allele matrix, site counts and MAF filter, the EHH walks
with trapezoid iHH, the log-ratios and the frequency-bin standardization
(ss_pack + ss_ihs).  The XPEHH scan of the same sites against 210 haplotypes
is timed the same way and reported beside it.

Two more workloads are reported in the same line:
  * "batched": 5,000 haplotypes x 10^6 SNPs over 250 Mb (200 founders,
    switch probability 0.001, 20 planted sweeps), every qualifying core locus
    in one persistent launch captured in a HIP graph with an autotuned
    configuration, against the plain per-locus class-id kernel on the same
    GPU;
  * "served": 4,096 region-scan requests (Poisson arrivals at 200/s, iHS with
    probability 0.6 else XPEHH, 100-5,000 haplotypes per population and
    1,000-200,000 SNPs, both log-uniform) through the continuous-batching
    server, against the same requests scanned back to back one at a time;
    p50 / p99 latency and throughput for both.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12   # 256 CUs x 64 int32 lanes/clk x 2.4 GHz
PROXY_OPS_PER_CELL = 51.0 / 256.0           # int32 lane-ops per haplotype-cell of the refinement
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_traffic.json")
# the walk kernel's sources: the mask walk and the class-id walk it falls back on
WALK_SRC = [os.path.join(ROOT, "paper_1403_6854_amd", "csrc", f)
            for f in ("ss_walk_mask.hip", "ss_walk_ids.hpp", "ss_internal.hpp")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def walk_src_sha() -> str:
    h = hashlib.sha256()
    for f in WALK_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per walk launch from committed rocprofv3 counter runs, if they
    were taken on the current walk kernel source."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    e = t.get(workload)
    if not e or e.get("walk_src_sha") != walk_src_sha():
        return None
    return e.get("hbm_bytes_per_launch")


def cells(steps: np.ndarray, n_c: np.ndarray) -> int:
    """Algorithmic work: markers walked by each core times its haplotypes."""
    return int((steps.astype(np.int64) * n_c.astype(np.int64)).sum())


def time_scan(fn, warmup: int, steps: int, ss, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ss.timing_read(reset=True)
    ss.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ss.timing_enable(False)
    walk_ms, launches = ss.timing_read(reset=True)
    return (t1 - t0), walk_ms / max(1, launches), launches


def bench_batched(ss, torch, dev, autotune: bool = True, reps: int = 3):
    """5,000 x 10^6 iHS: one persistent launch in a graph vs the plain kernel."""
    import hapgen
    log("batched: generating 5000 x 1e6 on the device")
    alleles, pos, gpos, sweeps = hapgen.large_batch_input(None, device=dev)
    h = ss.hapmat(alleles, torch.from_numpy(pos).to(dev), torch.from_numpy(gpos).to(dev))
    n, M = int(alleles.shape[1]), int(alleles.shape[0])
    del alleles
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    stream = torch.cuda.Stream()
    req = ss.ScanRequest(h)
    ss.alloc_outputs(req, steps=True)
    ss.set_batch_config(ss.BatchConfig())
    tune_s = tune_ms = 0.0
    ws = None
    if autotune:
        log("batched: autotuning the persistent walk")
        t0 = time.perf_counter()
        cfg, tune_ms, ws = ss.autotune_batch([req], stream=stream, sample_items=400_000)
        tune_s = time.perf_counter() - t0
    cfg = ss.get_batch_config()
    # walk kernel alone (eager, timed with events on the stream)
    ws = ss.scan_batch([req], stream=stream, ws=ws, validate=False)
    stream.synchronize()
    ss.timing_read(reset=True)
    ss.timing_enable(True)
    ss.scan_batch([req], stream=stream, ws=ws, validate=False)
    stream.synchronize()
    ss.timing_enable(False)
    walk_ms, _ = ss.timing_read(reset=True)
    # whole scan as a graph replay
    ss.set_graph(True)
    ss.scan_batch([req], stream=stream, ws=ws, validate=False)    # capture + first replay
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ss.scan_batch([req], stream=stream, ws=ws, validate=False)
    stream.synchronize()
    graph_s = (time.perf_counter() - t0) / reps
    ss.set_graph(False)
    ss.graph_clear()
    status = req.out["status"]
    loci = int((status != 1).sum().item())
    # algorithmic work: markers walked by each core times its haplotypes
    n1 = torch.round(req.out["freq"] * n).to(torch.int64)
    n_c = torch.stack([n - n1, n1], dim=1)[:, None, :]
    cells_w = int((req.out["steps"].to(torch.int64) * n_c).sum().item())
    # the plain per-locus kernel (one workgroup per site and direction)
    log("batched: plain per-locus kernel on the same input")
    ss.set_walk_kernel(1)
    plain = ss.ihs(h, validate=False)
    torch.cuda.synchronize()
    ss.timing_read(reset=True)
    ss.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        plain = ss.ihs(h, validate=False)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / reps
    ss.timing_enable(False)
    plain_walk_ms, launches = ss.timing_read(reset=True)
    ss.set_walk_kernel(0)
    same = bool(torch.equal(plain["status"], status)) and bool(
        torch.equal(plain["unstd"].nan_to_num(-7.0), req.out["unstd"].nan_to_num(-7.0)))
    res = {"workload": "ihs_batched_5000x1e6", "n_haps": n, "n_sites": M, "core_loci": loci,
           "sweeps": len(sweeps), "value": round(loci / graph_s, 1), "unit": "core loci/s",
           "scan_ms": round(graph_s * 1e3, 3), "walk_kernel_ms": round(walk_ms, 3),
           "graph": True, "config": dataclasses.asdict(cfg), "autotune_s": round(tune_s, 2),
           "autotune_sample_ms": round(tune_ms, 3),
           "plain_kernel": {"value": round(loci / plain_s, 1), "scan_ms": round(plain_s * 1e3, 3),
                            "walk_kernel_ms": round(plain_walk_ms / max(1, launches), 3)},
           "speedup_vs_plain": round(plain_s / graph_s, 3), "identical_results": same,
           "work_cells": cells_w,
           "achieved_TOPs": round(cells_w / (walk_ms * 1e-3) / 1e12, 4),
           "roofline_frac": round(cells_w / (walk_ms * 1e-3) / 1e12 / PEAK_INT32_TOPS, 5)}
    del req, plain, h, ws
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


# The paper's runtime data sets (Sec. 2.1, Table 1; Sec. 2.2, Table 2): haplotypes
# and SNPs over a 4 Mbp region.  Stand-ins from the copying model: 40 founders,
# the per-bp switch rate of the chromosome-22 workload (0.003 per SNP at 1.58 kb
# per SNP), so that a walk's length in markers grows with the SNP density.
SCALING_IHS = [("IHS250", 250, 9625), ("IHS500", 500, 10646), ("IHS1000", 1000, 11655),
               ("IHS2000", 2000, 12724)]
SCALING_XP = [("XP250", 125, 12920), ("XP500", 250, 14989), ("XP1000", 500, 17142),
              ("XP2000", 1000, 19567)]
SCALING_DENSITY = [2500, 5000, 10000, 20000, 40000]   # SNPs over 4 Mbp at 500 haplotypes
SCALING_BP = 4_000_000
SWITCH_PER_BP = 0.003 / 1580.0


def bench_scaling(ss, torch, dev, reps: int = 10):
    """GPU time of whole scans against haplotypes N and SNP density D at the
    paper's runtime shapes, with the least-squares exponents of
    time ~ N^b D^c (the paper states O(N D^2), Sec. 3)."""
    import hapgen

    def region(n, m, seed, nb=0):
        s = min(0.5, SWITCH_PER_BP * SCALING_BP / m)
        a = hapgen.copying_model(n, m, SCALING_BP, 40, s, seed)
        b = None
        if nb:
            rng = np.random.default_rng(seed + 1)
            b = hapgen.copy_haplotypes(rng, hapgen.derive_founders(rng, a.founders, 0.8), nb, s, 0.001)
        return a, b

    def run(name, n, m, seed, nb=0):
        a, b = region(n, m, seed, nb)
        pos = torch.from_numpy(a.pos_bp).to(dev)
        gpos = torch.from_numpy(a.gpos_cm).to(dev)
        ha = ss.hapmat(torch.from_numpy(a.alleles).to(dev), pos, gpos)
        hb = ss.hapmat(torch.from_numpy(b).to(dev), pos, gpos) if nb else None
        op = ss.OP_XPEHH if nb else ss.OP_IHS
        ws = torch.empty(ss.workspace_bytes(op, ha, hb) + 256, dtype=torch.uint8, device=dev)
        scan = (lambda out: ss.xpehh(ha, hb, steps=True, ws=ws, out=out, validate=False)) if nb else \
               (lambda out: ss.ihs(ha, steps=True, ws=ws, out=out, validate=False))
        out = scan(None)
        el, walk_ms, _ = time_scan(lambda: scan(out), 2, reps, ss, torch)
        st = out["status"].cpu().numpy()
        stp = out["steps"].cpu().numpy().astype(np.int64)
        if nb:
            loci = int(st.size)
            w = int(stp.sum()) * (n + nb)
        else:
            loci = int((st != 1).sum())
            n1 = a.alleles.sum(axis=1).astype(np.int64)
            nc = np.stack([n - n1, n1], axis=1)[:, None, :]
            w = int((stp * nc).sum())
        ms = el / reps * 1e3
        return {"shape": name, "n_haps": n + nb, "n_sites": m, "snps_per_kb": round(m / 4000.0, 3),
                "scan_ms": round(ms, 4), "walk_ms": round(walk_ms, 4), "core_loci": loci,
                "core_loci_per_s": round(loci / (ms * 1e-3), 1), "work_cells": w,
                "mean_markers_per_walk": round(float(stp.sum()) / max(1, (stp > 0).sum()), 1)}

    log("scaling: paper shapes and a density sweep")
    ihs = [run(nm, n, m, 3000 + i) for i, (nm, n, m) in enumerate(SCALING_IHS)]
    xp = [run(nm, n, m, 3100 + i, nb=n) for i, (nm, n, m) in enumerate(SCALING_XP)]
    dens = [run("D%d" % m, 500, m, 3200 + i) for i, m in enumerate(SCALING_DENSITY)]
    pts = ihs + dens
    X = np.stack([np.ones(len(pts)), np.log([p["n_haps"] for p in pts]),
                  np.log([p["snps_per_kb"] for p in pts])], axis=1)
    fit = {}
    for key in ("scan_ms", "walk_ms"):
        coef, *_ = np.linalg.lstsq(X, np.log([p[key] for p in pts]), rcond=None)
        fit[key] = {"exponent_N": round(float(coef[1]), 3), "exponent_D": round(float(coef[2]), 3)}
    cw, *_ = np.linalg.lstsq(X, np.log([p["work_cells"] for p in pts]), rcond=None)
    fit["work_cells"] = {"exponent_N": round(float(cw[1]), 3), "exponent_D": round(float(cw[2]), 3)}
    return {"region_bp": SCALING_BP, "founders": 40, "switch_per_bp": SWITCH_PER_BP,
            "ihs": ihs, "xpehh": xp, "density_n500": dens,
            "fit_ihs": fit, "paper_claim": "O(N D^2) (Sec. 3)"}


def bench_served(ss, torch, dev, args):
    """The served request stream: continuous batching vs back to back."""
    import hapgen
    from paper_1403_6854_amd import serve
    specs = hapgen.request_stream(args.serve_requests)

    def make(spec):
        def f():
            a, b, pos, gpos = hapgen.device_region(spec, dev)
            ha = ss.hapmat(a, pos, gpos)
            hb = ss.hapmat(b, pos, gpos) if b is not None else None
            return ha, hb
        return f

    def reqs_of(sp):
        return [serve.ServeRequest(s.rid, s.arrival_s, s.kind,
                                   serve.request_bytes(s.kind, s.n_a, s.n_b, s.n_sites),
                                   make(s), s.n_sites,
                                   serve.request_work(s.kind, s.n_a, s.n_b, s.n_sites))
                for s in sp]

    def loci_of(done, sp):
        kinds = {s.rid: s for s in sp}
        tot = 0
        for c in done:
            if c.out is None:    # a request that failed every attempt
                continue
            st = c.out["status"]
            tot += int((st != 1).sum().item()) if kinds[c.rid].kind == "ihs" else int(st.numel())
        return tot

    budget = int(args.serve_budget_gb * (1 << 30))
    # warm-up (library, generator and allocator first-use costs stay out of
    # the measured runs) and autotuning of the persistent walk on a batch of
    # the mix (requests drawn like the stream's, with other seeds)
    ss.set_batch_config(ss.BatchConfig())
    tune_specs = [dataclasses.replace(s, rid=100000 + i, seed=s.seed + (1 << 24), arrival_s=0.0)
                  for i, s in enumerate(hapgen.request_stream(48))]
    tune = []
    for r in reqs_of(tune_specs):
        a, b = r.make()
        q = ss.ScanRequest(a, b)
        ss.alloc_outputs(q)
        tune.append(q)
    if args.no_autotune:
        cfg = ss.get_batch_config()
    else:
        cfg, _, _ = ss.autotune_batch(tune, sample_items=0)
    del tune
    warm = [dataclasses.replace(s, arrival_s=0.0) for s in specs[:12]]
    serve.Server(serve.TorchBackend(args.serve_streams), budget).run(reqs_of(warm))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    stream = torch.cuda.Stream()

    def run_one(r):
        with torch.cuda.stream(stream):
            ha, hb = r.make()
            out = ss.ihs(ha, validate=False) if hb is None else ss.xpehh(ha, hb, validate=False)
        stream.synchronize()
        return {"status": out["status"]}

    def both(sp, label):
        log("served: %d requests at %g/s, continuous batching" % (len(sp), label))
        srv = serve.Server(serve.TorchBackend(args.serve_streams), budget, max_batch=64,
                           work_ratio=args.serve_work_ratio)
        done = srv.run(reqs_of(sp))
        torch.cuda.synchronize()
        s1 = serve.summarize(done)
        s1["core_loci_per_s"] = round(loci_of(done, sp) / s1["makespan_s"], 1)
        s1.update({"batches": srv.batches, "mean_batch": round(float(np.mean(srv.batch_sizes)), 2),
                   "peak_admitted_GB": round(srv.peak_bytes / 2**30, 2), "failed_batches": srv.failures,
                   "errors": sum(1 for c in done if c.error)})
        del done
        torch.cuda.empty_cache()
        log("served: %d requests at %g/s, back to back (plain scans)" % (len(sp), label))
        ss.set_walk_kernel(2)    # bitmask kernel when it applies, else the plain class-id kernel
        seq = serve.run_back_to_back(reqs_of(sp), run_one)
        ss.set_walk_kernel(0)
        s2 = serve.summarize(seq)
        s2["core_loci_per_s"] = round(loci_of(seq, sp) / s2["makespan_s"], 1)
        del seq
        torch.cuda.empty_cache()
        return s1, s2

    s1, s2 = both(specs, hapgen.SERVE["rate_per_s"])
    s1.update({"streams": args.serve_streams, "budget_GB": args.serve_budget_gb,
               "work_ratio": args.serve_work_ratio, "config": dataclasses.asdict(cfg),
               "group_tuning": ss.group_tuning()})
    res = {"workload": "served_mixed_4096", "requests": len(specs),
           "arrivals_per_s": hapgen.SERVE["rate_per_s"],
           "continuous_batching": s1, "back_to_back": s2,
           "throughput_ratio": round(s1["requests_per_s"] / s2["requests_per_s"], 3),
           "p99_ratio": round(s2["p99_ms"] / s1["p99_ms"], 3)}
    if args.serve_low_rate > 0:
        low = hapgen.request_stream(args.serve_low_requests, args.serve_low_rate)
        l1, l2 = both(low, args.serve_low_rate)
        res["below_saturation"] = {"requests": len(low), "arrivals_per_s": args.serve_low_rate,
                                   "continuous_batching": l1, "back_to_back": l2,
                                   "p50_ratio": round(l2["p50_ms"] / l1["p50_ms"], 3),
                                   "p99_ratio": round(l2["p99_ms"] / l1["p99_ms"], 3)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=10,
                    help="full oracle scans on all host threads (about 1 s of wall time each 10)")
    ap.add_argument("--cpu-reps-one", type=int, default=4,
                    help="full oracle scans on one thread (about 1.4 s each)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-scaling", action="store_true")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--serve-budget-gb", type=float, default=48.0)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-low-rate", type=float, default=150.0,
                    help="also serve a stream arriving at this rate (below saturation); 0: skip")
    ap.add_argument("--serve-low-requests", type=int, default=2048)
    ap.add_argument("--serve-work-ratio", type=float, default=4.0,
                    help="close a served batch at a request whose estimated work differs "
                         "from the batch's first by more than this factor (0: off)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default persistent-walk configuration (profiling runs)")
    ap.add_argument("--micro-only", action="store_true",
                    help="only run the measurement kernels (achievable peaks) and print them")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy_mb:
        import torch
        x = torch.arange(args.calibrate_copy_mb * (1 << 20) // 8, dtype=torch.int64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1, out=y)       # reads and writes calibrate_copy_mb MiB each
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8}))
        return
    if args.micro_only:
        import torch
        import hapgen
        import paper_1403_6854_amd as ss
        d = hapgen.config_input(1)
        print(json.dumps(ss.micro(ss.pack(torch.from_numpy(d.alleles).cuda()))))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import hapgen
    import paper_1403_6854_amd as ss

    dev = torch.device("cuda:0")
    log("generating inputs")
    a, b = hapgen.config_input(2)          # a = the 204 x 22,147 iHS workload
    M, n = a.alleles.shape
    A = torch.from_numpy(a.alleles).to(dev)
    B = torch.from_numpy(b.alleles).to(dev)
    pos = torch.from_numpy(a.pos_bp).to(dev)
    gpos = torch.from_numpy(a.gpos_cm).to(dev)
    params = ss.Params()

    # --- iHS ---------------------------------------------------------------
    h = ss.hapmat(A, pos, gpos)
    h.validate()
    ws = torch.empty(ss.workspace_bytes(ss.OP_IHS, h, None, params) + 256, dtype=torch.uint8,
                     device=dev)
    out = ss.ihs(h, params, steps=True, ws=ws)
    torch.cuda.synchronize()
    status = out["status"].cpu().numpy()
    stp = out["steps"].cpu().numpy()
    n1 = a.alleles.sum(axis=1).astype(np.int64)
    n_c = np.stack([n - n1, n1], axis=1)             # [M, 2] cores 0 and 1
    W = cells(stp, n_c[:, None, :].repeat(2, axis=1))
    core_loci = int((status != 1).sum())

    def ihs_step():
        hb = ss.HapMat(ss.pack(A), n, pos, gpos)
        ss.ihs(hb, params, steps=False, ws=ws, out=out, validate=False)

    log("timing iHS")
    el, walk_ms, launches = time_scan(ihs_step, args.warmup, args.steps, ss, torch)
    ms_step = el / args.steps * 1e3
    value = core_loci / (el / args.steps)

    # --- XPEHH -------------------------------------------------------------
    hA = ss.hapmat(A, pos, gpos)
    hB = ss.hapmat(B, pos, gpos)
    wsx = torch.empty(ss.workspace_bytes(ss.OP_XPEHH, hA, hB, params) + 256, dtype=torch.uint8,
                      device=dev)
    outx = ss.xpehh(hA, hB, params, steps=True, ws=wsx)
    torch.cuda.synchronize()
    stx = outx["steps"].cpu().numpy()
    Wx = int(stx.astype(np.int64).sum()) * (n + b.alleles.shape[1])

    def xp_step():
        ha = ss.HapMat(ss.pack(A), n, pos, gpos)
        hb2 = ss.HapMat(ss.pack(B), b.alleles.shape[1], pos, gpos)
        ss.xpehh(ha, hb2, params, steps=False, ws=wsx, out=outx, validate=False)

    log("timing XPEHH")
    elx, walk_ms_x, _ = time_scan(xp_step, args.warmup, args.steps, ss, torch)
    value_x = M / (elx / args.steps)

    # --- roofline of the dominant kernel (the iHS walk) ----------------------
    # Algorithmic work is W haplotype-cells (markers walked x core haplotypes);
    # the operations a cell needs are those of the cell-update proxy, whose
    # compiled loop refines 256 cells per lane and row with 51 int32 VALU
    # instructions (gfx950; the profile of the measurement kernels checks it).
    micro = None
    if not args.no_micro:
        log("measurement kernels")
        micro = ss.micro(ss.pack(A))
    ops_per_cell = PROXY_OPS_PER_CELL
    achieved = W * ops_per_cell / (walk_ms * 1e-3) / 1e12
    traffic = measured_traffic("ihs_chr22_204x22147")
    cells_s = W / (walk_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": round(achieved, 5), "peak": round(PEAK_INT32_TOPS, 3),
                "unit": "TOP/s", "frac": round(achieved / PEAK_INT32_TOPS, 6),
                "traffic": traffic,
                "kernel": "mask_walk_kernel<CORE,4,1,1>",
                "kernel_ms": round(walk_ms, 5),
                "work_cells": W, "ops_per_cell": round(ops_per_cell, 5),
                "ops_per_cell_source": "cell-update proxy: 51 VALU lane-ops per 256 cells",
                "achieved_Gcells": round(cells_s / 1e9, 2),
                "algorithmic_bytes": W // 8,
                "algorithmic_GBps": round(W / 8 / (walk_ms * 1e-3) / 1e9, 3)}
    if micro:
        roofline.update({
            "measured": micro,
            "frac_of_measured_valu": round(achieved / micro["valu_int32_TOPs"], 6),
            "frac_of_cell_proxy": round(cells_s / 1e9 / micro["cell_proxy_Gcells"], 6),
            "frac_of_measured_hbm": round(W / 8 / (walk_ms * 1e-3) / 1e9 / micro["hbm_copy_GBps"], 6)})

    # --- CPU baseline: the oracle on this host's cores ------------------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.default_threads()
        log("timing the CPU oracle on %d threads" % threads)
        t0 = time.perf_counter()
        for _ in range(args.cpu_reps):
            ref = oracle.ihs(a.alleles, a.pos_bp, a.gpos_cm, threads=threads)
        t_cpu = (time.perf_counter() - t0) / args.cpu_reps
        assert np.array_equal(ref["status"], status)
        # one thread, for the paper's single-thread column (Table 1)
        log("timing the CPU oracle on 1 thread")
        t0 = time.perf_counter()
        for _ in range(args.cpu_reps_one):
            ref1 = oracle.ihs(a.alleles, a.pos_bp, a.gpos_cm, threads=1)
        t_one = (time.perf_counter() - t0) / args.cpu_reps_one
        assert np.array_equal(ref1["status"], status)
        cpu = {"value": round(core_loci / t_cpu, 1), "unit": "core loci/s", "cores": threads,
               "kind": "oracle",
               "sample": "%d full iHS scans of the 204 x 22,147 workload (%d core loci each), "
                         "%.2f s per scan" % (args.cpu_reps, core_loci, t_cpu),
               "one_thread": {"value": round(core_loci / t_one, 1), "unit": "core loci/s", "cores": 1,
                              "sample": "%d full iHS scans of the same workload, %.2f s per scan"
                                        % (args.cpu_reps_one, t_one)}}

    scaling = None if args.no_scaling else bench_scaling(ss, torch, dev)
    batched = None if args.no_batched else bench_batched(ss, torch, dev, not args.no_autotune)
    served = None if args.no_served else bench_served(ss, torch, dev, args)

    line = {
        "metric": "iHS core loci/sec on 1 MI355X (XPEHH beside it)",
        "value": round(value, 1),
        "unit": "core loci/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ihs_chr22_204x22147", "n_haps": n, "n_sites": M,
                   "core_loci": core_loci, "step": "ss_pack + ss_ihs (device-resident uint8 alleles)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "xpehh": {"workload": "xpehh_chr22_204+210x22147", "value": round(value_x, 1),
                  "unit": "core loci/s", "ms_per_step": round(elx / args.steps * 1e3, 5),
                  "walk_kernel_ms": round(walk_ms_x, 5), "work_cells": Wx,
                  "achieved_TOPs": round(Wx / (walk_ms_x * 1e-3) / 1e12, 4)},
        "scaling_sweep": scaling,
        "batched": batched,
        "served": served,
        "context": {"paper_cpu_loci_per_s": {"ihs_ceu22_1thread": 62.7, "ihs_ceu22_16threads": 671,
                                             "xpehh_ceuyri22_1thread": 38.3,
                                             "xpehh_ceuyri22_16threads": 426},
                    "note": "paper: real CEU/YRI chr22 on a 2x6-core Xeon; here synthetic inputs"},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
