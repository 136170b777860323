#!/usr/bin/env python3
"""Throughput of the exhaustive three-way K2 scan on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one pass of the whole path over one synthetic input that is
already resident in device memory: encode (bit-planes + pairwise tables),
count + FP32 K2 of every triplet, exact top-k (FP32 screen, FP64 re-score,
ordering), copy of the hits to the host.  Prints one JSON line.

Metric: sample-triplets per second = C(M,3) * N / seconds (the paper counts
processed elements as combinations times samples, Experimental Results
section), in units of 1e12.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tera sample-triplets/s; batched-permutation vs plain speedup at exact top-k"
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12      # INT32 lane-ops/s: CUs x lanes x clock
VALU_OPS_PER_ST = 16.0 / 32.0                  # 8 AND + 8 v_bcnt per triplet per 32 samples

MFMA_I8_PEAK_TOPS = 5000.0                     # dense int8 matrix-core ops/s (MI355X)
MFMA_FP4_PEAK_TFLOPS = 10100.0                 # dense FP4 matrix-core flop/s (MI355X)
MFMA_OPS_PER_ST = 16.0                         # plain: 8 corner cells x (multiply + add) per sample-triplet
MFMA_OPS_PER_STQ = 16.0 * 65.0 / 64.0          # batch: the same per phenotype plus the all-sample
                                               # (totals) column shared by 64 phenotypes
PAIR_OPS_PER_SP = 8.0 / 32.0                   # 4 AND + 4 v_bcnt per pair per 32 samples (pairwise tables)
QUAD_MFMA_OPS_PER_SQ = 32.0                    # 16 quad corner cells x (multiply + add) per sample-quad

WORKLOADS = {
    "plain1": dict(cfg=1, kind="plain", desc="plain scan, 64 SNPs x 1024 samples (512 cases), top-10"),
    "plain2": dict(cfg=2, kind="plain", desc="plain scan, 512 SNPs x 4096 samples (50% cases), top-100"),
    "plain3": dict(cfg=3, kind="plain", desc="plain scan, 2048 SNPs x 16384 samples (50% cases), top-1000"),
    "plain6": dict(cfg=6, kind="plain", desc="plain scan, 8192 SNPs x 16384 samples (50% cases), top-1000, "
                   "selected by bound (no score plane)"),
    "perm4": dict(cfg=4, kind="perm", desc="batched permutations: 1024 SNPs x 8192 samples (3277 cases), "
                  "64 phenotype permutations in one launch, top-10 each"),
    "pairs3": dict(cfg=3, kind="pairs", desc="second-order (pair) scan, 2048 SNPs x 16384 samples "
                   "(50% cases), top-1000"),
    "quads2": dict(cfg=2, kind="quads", snps=256, desc="fourth-order (quad) scan, first 256 SNPs of the "
                   "512 x 4096 data set (50% cases), top-100"),
    "uneven5": dict(cfg=5, kind="uneven", desc="batched uneven data sets: 32 data sets, SNPs ~ U[128,1024], "
                    "samples ~ U[1024,16384], one launch, top-10 each"),
}
DEFAULT_WORKLOAD = "perm4"


def recorded_traffic(key: str):
    """HBM bytes per launch of the dominant kernel of "workload|variant" from the
    committed counter summary (profiles/traffic.json), or None when the kernel's
    sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(key)
    if not rec:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return rec["traffic_bytes"] if h.hexdigest() == rec["source_sha256"] else None


def cpu_cores() -> int:
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(d, k: int, budget_s: float = 20.0) -> dict:
    """The oracle (plain CPU loops) timed on a bounded sample of the workload:
    the first M' SNPs of the same data set, M' chosen so the run takes about
    `budget_s` seconds at the oracle's measured rate."""
    import oracle
    from math import comb
    cores = cpu_cores()
    N = d.n_samples
    # calibrate on a small prefix, then size the sample
    m0 = min(d.n_snps, 48)
    t0 = time.perf_counter()
    oracle.scan_topk(d.geno[:m0], d.pheno, k, nthreads=cores, counts=False)
    rate = comb(m0, 3) * N / max(time.perf_counter() - t0, 1e-6)
    m = m0
    while m < d.n_snps and comb(m + 1, 3) * N / rate < budget_s:
        m += 1
    t0 = time.perf_counter()
    oracle.scan_topk(d.geno[:m], d.pheno, k, nthreads=cores, counts=False)
    dt = time.perf_counter() - t0
    work = comb(m, 3) * N
    return {"value": work / dt / 1e12, "unit": "T sample-triplets/s", "cores": cores,
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": f"first {m} of {d.n_snps} SNPs x all {N} samples, top-{k} "
                      f"({work:.3e} sample-triplets)"}


def cpu_host_scan(d, k: int, budget_s: float = 5.0) -> dict:
    """The host-CPU scan (vector popcount, OpenMP; a separate library the GPU
    path never calls) timed on a bounded sample of the workload, like the
    oracle baseline: the first M' SNPs, M' sized to about `budget_s` seconds.
    An auxiliary figure: if its library is not built, the line says so."""
    from math import comb
    try:
        from paper_2201_10956_amd import host
    except (ImportError, OSError) as e:
        return {"value": None, "error": f"host scan library unavailable: {e}"}
    cores = cpu_cores()
    N = d.n_samples
    m0 = min(d.n_snps, 192)
    t0 = time.perf_counter()
    host.scan_topk(d.geno[:m0], d.pheno, k, threads=cores)
    rate = comb(m0, 3) * N / max(time.perf_counter() - t0, 1e-6)
    m = m0
    while m < d.n_snps and comb(m + 1, 3) * N / rate < budget_s:
        m += 1
    t0 = time.perf_counter()
    host.scan_topk(d.geno[:m], d.pheno, k, threads=cores)
    dt = time.perf_counter() - t0
    work = comb(m, 3) * N
    return {"value": work / dt / 1e12, "unit": "T sample-triplets/s", "cores": cores,
            "kind": "host scan (vector AND + popcount, OpenMP)",
            "isa": host.ISA_NAMES[host.best_isa()], "seconds": round(dt, 3),
            "sample": f"first {m} of {d.n_snps} SNPs x all {N} samples, top-{k} "
                      f"({work:.3e} sample-triplets), encoding included"}


def run_plain(args, wl):
    import torch
    from paper_2201_10956_amd import epi3
    from synth import CONFIGS, make_config

    c = CONFIGS[wl["cfg"]]
    d = make_config(wl["cfg"])
    M, N, k = d.n_snps, d.n_samples, c["k"]
    geno = torch.from_numpy(d.geno).to("cuda")          # resident before timing
    ds = epi3.encode(geno, d.pheno)
    variant = epi3.tile_for(ds, "auto") if args.variant == "auto" else args.variant
    if args.tile:  # the forced tile replaces the tuned table's rules for this variant
        epi3.tile_rules_clear()
        epi3.tile_rule(variant, 0, 0, args.tile)
    tile = epi3.tile_for(ds, variant)
    sc = epi3.Scanner(ds, k, variant)

    def step():
        epi3.encode(geno, d.pheno, into=ds)
        return sc.run()

    dt, hits = _timed_steps(step, args.steps, args.warmup)
    cnt_ms, cnt_n, sel_ms, fin_ms = _kernel_times(step)
    T = epi3.n_triplets(M)
    work = T * N
    ms_step = dt * 1e3
    value = work / dt / 1e12
    out = _base(args, wl, value, ms_step, {"valu": "u32", "mfma": "i8", "mfma_fp4": "fp4"}[variant], {
        "workload": wl["desc"], "snps": M, "samples": N, "cases": int(d.pheno.sum()),
        "top_k": k, "triplets": T, "variant": variant, "tile": tile})
    if variant == "valu":
        achieved = work * VALU_OPS_PER_ST / (cnt_ms / 1e3) / 1e12
        out["roofline"] = {
            "bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 3),
            "unit": "T int32-lane-ops/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": recorded_traffic(f"{args.workload}|valu"),
            "traffic_unit": "bytes per launch (FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated)",
            "kernel": "count_valu_kernel", "kernel_ms": round(cnt_ms / max(cnt_n, 1), 4),
            "ops_per_launch": work * VALU_OPS_PER_ST / max(cnt_n, 1)}
    else:
        peak = MFMA_FP4_PEAK_TFLOPS if variant == "mfma_fp4" else MFMA_I8_PEAK_TOPS
        achieved = MFMA_OPS_PER_ST * work / (cnt_ms / 1e3) / 1e12
        out["roofline"] = {
            "bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
            "unit": "TFLOP/s (fp4)" if variant == "mfma_fp4" else "TOP/s (int8)",
            "frac": round(achieved / peak, 4),
            "traffic": recorded_traffic(f"{args.workload}|{variant}"),
            "traffic_unit": "bytes per launch (FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated)",
            "kernel": "count_mfma_plain_kernel", "kernel_ms": round(cnt_ms / max(cnt_n, 1), 4),
            "launches_per_step": cnt_n,
            "ops_per_launch": MFMA_OPS_PER_ST * work / max(cnt_n, 1)}
    out["breakdown_ms"] = {"count_kernels": round(cnt_ms, 4), "finish_kernels": round(fin_ms, 4),
                           "selection": round(sel_ms, 4)}
    out["best"] = {"ijk": [int(hits["i"][0]), int(hits["j"][0]), int(hits["k"][0])],
                   "k2": float(hits["k2"][0])}
    if epi3.n_triplets(M) * 4 <= (16 << 30):  # a score plane exists (AUTO keeps it up to 16 GiB)
        sc.run()
        out["k2_fp32_error"] = plane_k2_error(epi3, ds, sc.score_plane())
    out["k2_fp32_error_hits"] = k2_error(hits["k2_f32"], hits["k2"], epi3.k2_error_bound(N),
                                         f"the {len(hits)} hits")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(d, k, args.cpu_budget)
        out["cpu_fast"] = cpu_host_scan(d, k)
    return out


def cpu_baseline_pairs(d, k: int, budget_s: float = 20.0) -> dict:
    """The oracle's pair scan timed on the first M' SNPs (all of them when the
    whole scan fits the budget)."""
    import oracle
    from math import comb
    cores = cpu_cores()
    N = d.n_samples
    m0 = min(d.n_snps, 256)
    t0 = time.perf_counter()
    oracle.scan_pairs_topk(d.geno[:m0], d.pheno, k, nthreads=cores, counts=False)
    rate = comb(m0, 2) * N / max(time.perf_counter() - t0, 1e-6)
    m = m0
    while m < d.n_snps and comb(m + 1, 2) * N / rate < budget_s:
        m += 1
    t0 = time.perf_counter()
    oracle.scan_pairs_topk(d.geno[:m], d.pheno, k, nthreads=cores, counts=False)
    dt = time.perf_counter() - t0
    work = comb(m, 2) * N
    return {"value": work / dt / 1e12, "unit": "T sample-pairs/s", "cores": cores,
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": f"first {m} of {d.n_snps} SNPs x all {N} samples, top-{k} "
                      f"({work:.3e} sample-pairs)"}


def run_pairs(args, wl):
    import torch
    from paper_2201_10956_amd import epi3
    from synth import CONFIGS, make_config

    c = CONFIGS[wl["cfg"]]
    d = make_config(wl["cfg"])
    M, N, k = d.n_snps, d.n_samples, c["k"]
    geno = torch.from_numpy(d.geno).to("cuda")
    ds = epi3.encode(geno, d.pheno, values=False)
    sc = epi3.PairScanner(ds, k)

    def step():  # encode (planes + pairwise tables) + pair scores + exact top-k
        epi3.encode(geno, d.pheno, into=ds, values=False)
        return sc.run()

    dt, hits = _timed_steps(step, args.steps, args.warmup)
    torch.cuda.synchronize()
    epi3.timing_reset()
    epi3.timing_enable(True)
    reps = 2
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    epi3.timing_enable(False)
    pt_ms, pt_n = epi3.timing_query(4)
    sc_ms, _ = epi3.timing_query(0)
    se_ms, _ = epi3.timing_query(1)
    P = epi3.n_pairs(M)
    work = P * N
    out = _base(args, wl, work / dt / 1e12, dt * 1e3, "u32", {
        "workload": wl["desc"], "snps": M, "samples": N, "cases": int(d.pheno.sum()),
        "top_k": k, "pairs": P})
    out["metric"] = "tera sample-pairs/s at exact top-k (second-order scan)"
    out["unit"] = "T sample-pairs/s"
    ops = work * PAIR_OPS_PER_SP
    kern_ms = pt_ms / max(pt_n, 1)
    achieved = ops / (kern_ms / 1e3) / 1e12
    out["roofline"] = {
        "bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 3),
        "unit": "T int32-lane-ops/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
        "traffic": recorded_traffic(f"{args.workload}|valu"),
        "traffic_unit": "bytes per launch (FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated)",
        "kernel": "pairs_kernel", "kernel_ms": round(kern_ms, 4), "ops_per_launch": ops}
    out["breakdown_ms"] = {"pairwise_tables": round(pt_ms / reps, 4),
                           "pair_scores": round(sc_ms / reps, 4), "selection": round(se_ms / reps, 4)}
    out["best"] = {"ij": [int(hits["i"][0]), int(hits["j"][0])], "k2": float(hits["k2"][0])}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_pairs(d, k, args.cpu_budget)
    return out


def cpu_baseline_quads(geno, pheno, k: int, budget_s: float = 20.0) -> dict:
    """The oracle's quad scan timed on the first M' SNPs."""
    import oracle
    from math import comb
    cores = cpu_cores()
    N = pheno.size
    m0 = min(geno.shape[0], 24)
    t0 = time.perf_counter()
    oracle.scan_quads_topk(geno[:m0], pheno, k, nthreads=cores, counts=False)
    rate = comb(m0, 4) * N / max(time.perf_counter() - t0, 1e-6)
    m = m0
    while m < geno.shape[0] and comb(m + 1, 4) * N / rate < budget_s:
        m += 1
    t0 = time.perf_counter()
    oracle.scan_quads_topk(geno[:m], pheno, k, nthreads=cores, counts=False)
    dt = time.perf_counter() - t0
    work = comb(m, 4) * N
    return {"value": work / dt / 1e12, "unit": "T sample-quads/s", "cores": cores,
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": f"first {m} of {geno.shape[0]} SNPs x all {N} samples, top-{k} "
                      f"({work:.3e} sample-quads)"}


def run_quads(args, wl):
    import torch
    from paper_2201_10956_amd import epi3
    from synth import CONFIGS, make_config

    c = CONFIGS[wl["cfg"]]
    d = make_config(wl["cfg"])
    M, N, k = wl["snps"], d.n_samples, c["k"]
    g_host = np.ascontiguousarray(d.geno[:M])
    geno = torch.from_numpy(g_host).to("cuda")
    ds = epi3.encode(geno, d.pheno)   # value planes: the quad counts run on the matrix cores
    sc = epi3.QuadScanner(ds, k)

    def step():  # encode + triplet corners + quad counts (matrix cores) + scores + exact top-k
        epi3.encode(geno, d.pheno, into=ds)
        return sc.run()

    dt, hits = _timed_steps(step, args.steps, args.warmup)
    cnt_ms, cnt_n, sel_ms, fin_ms = _kernel_times(step)
    Qn = epi3.n_quads(M)
    work = Qn * N
    out = _base(args, wl, work / dt / 1e12, dt * 1e3, "fp4", {
        "workload": wl["desc"], "snps": M, "samples": N, "cases": int(d.pheno.sum()),
        "top_k": k, "quads": Qn, "variant": "mfma_fp4"})
    out["metric"] = "tera sample-quads/s at exact top-k (fourth-order scan)"
    out["unit"] = "T sample-quads/s"
    ops = work * QUAD_MFMA_OPS_PER_SQ
    kern_ms = cnt_ms / max(cnt_n, 1)
    achieved = ops / (cnt_ms / 1e3) / 1e12
    out["roofline"] = {
        "bound": "mfma", "achieved": round(achieved, 2), "peak": MFMA_FP4_PEAK_TFLOPS,
        "unit": "TFLOP/s (fp4)", "frac": round(achieved / MFMA_FP4_PEAK_TFLOPS, 4),
        "traffic": recorded_traffic(f"{args.workload}|mfma_fp4"),
        "traffic_unit": "bytes per launch (FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated)",
        "kernel": "count_mfma_quad_kernel", "kernel_ms": round(kern_ms, 4),
        "launches_per_step": cnt_n, "ops_per_launch": ops / max(cnt_n, 1)}
    out["breakdown_ms"] = {"quad_count_kernels": round(cnt_ms, 4), "finish_kernels": round(fin_ms, 4),
                           "selection": round(sel_ms, 4)}
    out["best"] = {"ijkl": [int(hits[f][0]) for f in ("i", "j", "k", "l")], "k2": float(hits["k2"][0])}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_quads(g_host, d.pheno, k, args.cpu_budget)
    return out


def k2_error(k2_32, k2_64, bound: float, where: str) -> dict:
    """Largest |K2_fp32 - K2_fp64| (absolute and relative) over matched
    scores, next to the error bound e(N) the selection screens with."""
    a = np.asarray(k2_32, dtype=np.float64)
    b = np.asarray(k2_64, dtype=np.float64)
    d = np.abs(a - b)
    return {"max_abs": float(d.max()), "max_rel": float((d / np.abs(b)).max()),
            "bound": bound, "n": int(d.size), "over": where}


def plane_k2_error(epi3, ds, plane, n: int = 10000, seed: int = 5) -> dict:
    """The error report on n sampled ranks of a score plane: FP32 from the
    plane, FP64 from the library's re-score of the same triplets."""
    import torch
    from math import comb
    from synth import SplitMix64
    M = ds.M
    T = comb(M, 3)
    ranks = np.unique((SplitMix64(seed, 0).uniform(0, n) * T).astype(np.int64))
    ijk = _unrank3(M, ranks)
    _, _, k64 = epi3.score_triplets(ds, ijk)
    got = plane[torch.as_tensor(ranks, device=plane.device)].cpu().numpy()
    return k2_error(got, k64.cpu().numpy(), epi3.k2_error_bound(ds.N),
                    f"{ranks.size} sampled triplets of the score plane")


def _unrank3(M: int, ranks) -> np.ndarray:
    """(i, j, k) of lexicographic ranks among the triplets of M SNPs: the
    first index is the last whose block of triplets starts at or before the
    rank (binary search), then likewise for the second."""
    from math import comb
    C = comb(M, 3)
    out = np.empty((len(ranks), 3), dtype=np.uint32)
    for x, r in enumerate(ranks):
        r = int(r)
        lo, hi = 0, M - 3
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if C - comb(M - mid, 3) <= r:
                lo = mid
            else:
                hi = mid - 1
        i, r1 = lo, r - (C - comb(M - lo, 3))
        lo, hi = i + 1, M - 2
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if comb(M - 1 - i, 2) - comb(M - mid, 2) <= r1:
                lo = mid
            else:
                hi = mid - 1
        j = lo
        out[x] = (i, j, r1 - (comb(M - 1 - i, 2) - comb(M - j, 2)) + j + 1)
    return out


def hits_equal(a, b) -> bool:
    """Same triplets, FP64 K2 and counts (the FP32 screen value may differ in
    its last bits between count kernels that sum a table in another order)."""
    return (len(a) == len(b) and all(np.array_equal(a[f], b[f]) for f in ("i", "j", "k", "k2", "counts")))


def _timed_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def _kernel_times(fn, reps=2):
    """Per-step ms of the count stage (all its launches), the selection and the
    table-completion kernel, from the library's HIP events on the launch stream
    (measurement mode), plus count launches per step."""
    import torch
    from paper_2201_10956_amd import epi3
    torch.cuda.synchronize()
    epi3.timing_reset()
    epi3.timing_enable(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    epi3.timing_enable(False)
    c_ms, c_n = epi3.timing_query(0)
    s_ms, s_n = epi3.timing_query(1)
    f_ms, f_n = epi3.timing_query(3)
    return c_ms / reps, c_n / reps, s_ms / reps, f_ms / reps


def _base(args, wl, value, ms_step, dtype, config):
    return {"metric": METRIC, "value": round(value, 4), "unit": "T sample-triplets/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype,
            "data": "synthetic (seeded HWE genotypes, planted triplet)", "config": config}


def run_perm(args, wl):
    import torch
    from paper_2201_10956_amd import epi3
    from synth import CONFIGS, make_config
    from math import comb

    c = CONFIGS[wl["cfg"]]
    d, perms = make_config(wl["cfg"])
    M, N, k, Q = d.n_snps, d.n_samples, c["k"], c["n_perm"]
    geno = torch.from_numpy(d.geno).to("cuda")
    masks = torch.from_numpy(epi3.pack_masks(perms).view(np.int32)).to("cuda")
    ds = epi3.encode(geno, d.pheno, layout="masked")
    variant = "mfma" if args.variant == "mfma" else "mfma_fp4"
    bs = epi3.BatchScanner(ds, k, masks=masks, variant=variant)

    def step():  # encode (planes, bytes, pairwise tables) + one batched launch
        epi3.encode(geno, d.pheno, layout="masked", into=ds)
        return bs.run()

    dt, res = _timed_steps(step, args.steps, args.warmup)
    T = comb(M, 3)
    work = T * N * Q
    value = work / dt / 1e12
    k_ms, k_n, sel_ms, fin_ms = _kernel_times(bs.run)
    t_kernel = k_ms / 1e3  # all count launches of one step
    achieved = MFMA_OPS_PER_STQ * T * N * Q / t_kernel / 1e12

    # plain references: one encode + scan + top-k per phenotype, with the
    # vector-ALU count (the paper's method) and with the tuned plain path
    pds = epi3.encode(geno, perms[0])
    best_variant = epi3.tile_for(pds, "auto")

    def plain_all(variant):
        sc = epi3.Scanner(pds, k, variant)

        def run():
            out = []
            for q in range(Q):
                sc.ds = epi3.encode(geno, perms[q], into=pds)
                out.append(sc.run())
            return out
        return run

    p_dt, plain_res = _timed_steps(plain_all("valu"), 1, 1)
    same = all(a.tobytes() == b.tobytes() for a, b in zip(res, plain_res))
    plain_value = work / p_dt / 1e12
    b_dt, best_res = _timed_steps(plain_all(best_variant), 1, 1)
    same_best = all(hits_equal(a, b) for a, b in zip(res, best_res))
    best_value = work / b_dt / 1e12
    out = _base(args, wl, value, dt * 1e3, "fp4" if variant == "mfma_fp4" else "i8", {
        "workload": wl["desc"], "snps": M, "samples": N, "phenotypes": Q, "top_k": k,
        "triplets": T, "variant": variant, "counted": "sample-triplets per phenotype, summed"})
    out["speedup_vs_plain"] = round(value / plain_value, 3)
    out["plain"] = {"value": round(plain_value, 4), "unit": "T sample-triplets/s",
                    "ms_for_all_phenotypes": round(p_dt * 1e3, 3),
                    "how": "64 x (encode split planes + VALU count + top-k), same data",
                    "hits_identical_to_batched": bool(same)}
    out["speedup_vs_plain_best"] = round(value / best_value, 3)
    out["plain_best"] = {"value": round(best_value, 4), "unit": "T sample-triplets/s",
                         "ms_for_all_phenotypes": round(b_dt * 1e3, 3),
                         "how": f"64 x (encode + {best_variant} plain scan + top-k), same data",
                         "hits_equal_to_batched": bool(same_best)}
    peak = MFMA_FP4_PEAK_TFLOPS if variant == "mfma_fp4" else MFMA_I8_PEAK_TOPS
    # no finish launches: the library counted and scored in one kernel
    fused = fin_ms == 0.0
    out["roofline"] = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                       "unit": "TFLOP/s (fp4)" if variant == "mfma_fp4" else "TOP/s (int8)",
                       "frac": round(achieved / peak, 4),
                       "traffic": recorded_traffic(f"{args.workload}|{variant}" + ("|fused" if fused else "")),
                       "traffic_unit": "bytes per launch (FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated)",
                       "kernel": "count_score_perm_kernel" if fused else "count_mfma_perm_kernel",
                       "kernel_ms": round(k_ms / max(k_n, 1), 4),
                       "launches_per_step": k_n,
                       "ops_per_launch": MFMA_OPS_PER_STQ * T * N * Q / max(k_n, 1)}
    out["breakdown_ms"] = {"count_kernels": round(k_ms, 3), "finish_kernels": round(fin_ms, 3),
                           "selection": round(sel_ms, 3)}
    out["min_k2_per_phenotype"] = [round(float(h["k2"][0]), 6) for h in res[:4]] + ["..."]
    out["k2_fp32_error"] = k2_error(np.concatenate([h["k2_f32"] for h in res]),
                                    np.concatenate([h["k2"] for h in res]),
                                    epi3.k2_error_bound(N), f"the {sum(len(h) for h in res)} hits "
                                    f"of all {Q} phenotypes")
    # permutation significance of the observed phenotype's best triplet: its
    # lowest K2 from a plain scan of the unpermuted phenotype (untimed), the
    # permutations' lowest from hit 0 of each job of the timed batch
    obs = epi3.scan_topk(epi3.encode(geno, d.pheno), 1, best_variant)
    obs_k2 = float(obs["k2"][0])
    out["significance"] = {
        "observed_best": {"ijk": [int(obs["i"][0]), int(obs["j"][0]), int(obs["k"][0])],
                          "k2": obs_k2, "planted": [int(x) for x in d.planted]},
        "p_value": epi3.perm_pvalue(obs_k2, [float(h["k2"][0]) for h in res]),
        "permutations": Q, "how": "(1 + #{q: min K2_q <= observed}) / (Q + 1)"}
    if not args.no_cpu_baseline:
        d0 = type(d)(d.geno, perms[0], d.planted, d.maf, d.seed)
        out["cpu_baseline"] = cpu_baseline(d0, k, args.cpu_budget)
        out["cpu_baseline"]["sample"] += ", phenotype permutation 0"
        out["cpu_fast"] = cpu_host_scan(d0, k)
        out["cpu_fast"]["sample"] += ", phenotype permutation 0"
    return out


def run_uneven(args, wl):
    import torch
    from paper_2201_10956_amd import epi3
    from synth import CONFIGS, make_config
    from math import comb

    c = CONFIGS[wl["cfg"]]
    dsets = make_config(wl["cfg"])
    k = c["k"]
    genos = [torch.from_numpy(d.geno).to("cuda") for d in dsets]
    enc = [epi3.encode(g, d.pheno) for g, d in zip(genos, dsets)]
    variant = args.variant if args.variant in ("auto", "valu", "mfma", "mfma_fp4") else "auto"
    bs = epi3.BatchScanner(enc, k, variant=variant)

    def step():
        for x, (g, d) in enumerate(zip(genos, dsets)):
            epi3.encode(g, d.pheno, into=enc[x])
        return bs.run()

    dt, res = _timed_steps(step, args.steps, args.warmup)
    work = sum(comb(d.n_snps, 3) * d.n_samples for d in dsets)
    value = work / dt / 1e12
    k_ms, k_n, sel_ms, fin_ms = _kernel_times(bs.run)
    # roofline of the count kernel family that does most of the work, timed on
    # its own subset of the data sets (one batched call each)
    kinds = [epi3.tile_for(e, "auto") if variant == "auto" else variant for e in enc]
    on_mfma = [x for x in range(len(enc)) if kinds[x] != "valu"]
    on_valu = [x for x in range(len(enc)) if kinds[x] == "valu"]
    w_mfma = sum(comb(dsets[x].n_snps, 3) * dsets[x].n_samples for x in on_mfma)
    w_valu = work - w_mfma
    if w_mfma >= w_valu:
        sub = epi3.BatchScanner([enc[x] for x in on_mfma], k, variant=variant)
        m_ms, m_n, _, m_fin = _kernel_times(sub.run)
        fp4 = all(kinds[x] == "mfma_fp4" for x in on_mfma)
        peak = MFMA_FP4_PEAK_TFLOPS if fp4 else MFMA_I8_PEAK_TOPS
        achieved = MFMA_OPS_PER_ST * w_mfma / (m_ms / 1e3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                "unit": "TFLOP/s (fp4)" if fp4 else "TOP/s (int8)", "frac": round(achieved / peak, 4),
                "traffic": recorded_traffic(f"{args.workload}|{'mfma_fp4' if fp4 else 'mfma'}"),
                "traffic_unit": "bytes per launch of the matrix-core subset's count kernel "
                                "(FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated)",
                "kernel": "count_mfma_plain_kernel",
                "kernel_ms": round(m_ms / max(m_n, 1), 4), "launches": m_n,
                "datasets_timed": len(on_mfma), "ops": MFMA_OPS_PER_ST * w_mfma}
    else:
        sub = epi3.BatchScanner([enc[x] for x in on_valu], k, variant=variant) if on_mfma else bs
        v_ms, v_n, _, _ = _kernel_times(sub.run)
        achieved = w_valu * VALU_OPS_PER_ST / (v_ms / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 3),
                "unit": "T int32-lane-ops/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": recorded_traffic(f"{args.workload}|valu"),
                "kernel": "count_valu_kernel", "kernel_ms": round(v_ms, 4),
                "datasets_timed": len(on_valu), "ops": w_valu * VALU_OPS_PER_ST}

    def seq():
        return [epi3.scan_topk(e, k, variant) for e in enc]

    s_dt, seq_res = _timed_steps(seq, 1, 1)
    same = all(a.tobytes() == b.tobytes() for a, b in zip(res, seq_res))
    dtype = "u32" if variant == "valu" else ("i8" if variant == "mfma" else "fp4+u32")
    out = _base(args, wl, value, dt * 1e3, dtype, {
        "workload": wl["desc"], "datasets": len(dsets), "top_k": k,
        "snps": [d.n_snps for d in dsets], "samples": [d.n_samples for d in dsets],
        "sample_triplets": work, "variant": variant,
        "count_kernels_per_dataset": [epi3.tile_for(e, "auto") if variant == "auto" else variant
                                      for e in enc]})
    out["sequential"] = {"value": round(work / s_dt / 1e12, 4), "ms": round(s_dt * 1e3, 3),
                         "how": "one plain scan per data set", "hits_identical": bool(same)}
    out["roofline"] = roof
    out["breakdown_ms"] = {"count_kernels": round(k_ms, 4), "finish_kernels": round(fin_ms, 4),
                           "selection": round(sel_ms, 4)}
    out["work_split"] = {"matrix_core_datasets": len(on_mfma), "vector_alu_datasets": len(on_valu),
                         "matrix_core_sample_triplets": w_mfma, "vector_alu_sample_triplets": w_valu}
    if not args.no_cpu_baseline:
        big = max(dsets, key=lambda d: d.n_samples)
        out["cpu_baseline"] = cpu_baseline(big, k, args.cpu_budget)
        out["cpu_fast"] = cpu_host_scan(big, k)
    return out


def copy_calibration(nbytes: int = 1 << 30, reps: int = 3) -> None:
    """A plain device-to-device copy of known size, for scaling the HBM byte
    counters (FETCH_SIZE / WRITE_SIZE) read by the profiler."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes,
                      "reps": reps}), flush=True)


def peak_microbench(reps: int = 5) -> dict:
    """Sustained rates of register-only chains on this GPU (paper_2201_10956_amd/peak):
    FP4 32x32x64 and int8 32x32x32 matrix-core products, AND + v_bcnt on the
    vector ALU; 2048 workgroups of 256 threads (8 waves per SIMD)."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2201_10956_amd", "peak", "libepi3_peak.so"))
    lib.epi3_peak_run.restype = ctypes.c_int
    lib.epi3_peak_run.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
    blocks = torch.cuda.get_device_properties(0).multi_processor_count * 8
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    res = {}
    for kind, name, iters, unit, pub in ((0, "mfma_fp4_32x32x64", 200, "TFLOP/s", MFMA_FP4_PEAK_TFLOPS),
                                         (1, "mfma_i8_32x32x32", 200, "TOP/s", MFMA_I8_PEAK_TOPS),
                                         (2, "valu_and_bcnt", 200000, "T int32-lane-ops/s",
                                          VALU_PEAK_TOPS)):
        ms, ops = ctypes.c_double(0), ctypes.c_double(0)
        rc = lib.epi3_peak_run(kind, iters, blocks, reps, ctypes.c_void_p(out.data_ptr()),
                               ctypes.byref(ms), ctypes.byref(ops))
        if rc != 0:
            raise RuntimeError(f"epi3_peak_run({name}) returned {rc}")
        rate = ops.value / (ms.value / 1e3) / 1e12
        res[name] = {"rate": round(rate, 2), "unit": unit, "ms_per_launch": round(ms.value, 4),
                     "published_peak": round(pub, 2), "frac_of_published": round(rate / pub, 4)}
    return {"peak_microbench": res, "blocks": blocks, "threads_per_block": 256}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--variant", default="auto", choices=["auto", "valu", "mfma", "mfma_fp4"])
    ap.add_argument("--tile", type=int, default=0,
                    help="force the count kernel's tile (plain workloads; 0: tuned table)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--peak", action="store_true",
                    help="print the peak-rate microbenchmarks instead of a workload")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.peak:
        print(json.dumps(peak_microbench()), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this benchmark measures one GPU only; run with --gpus 1"}))
        sys.exit(2)
    wl = WORKLOADS[args.workload]
    run = {"plain": run_plain, "perm": run_perm, "uneven": run_uneven, "pairs": run_pairs,
           "quads": run_quads}[wl["kind"]]
    out = run(args, wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
