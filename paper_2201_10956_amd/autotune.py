"""Autotuner for the count kernels' tile shapes and for the variant that AUTO
selects in plain scans.

For each (M, N) shape of a grid it encodes a seeded random data set on the
GPU, times a whole plain scan (count + selection, HIP events on the scan's
stream, median of `reps` runs after one warm-up) for every variant and tile
candidate, and keeps the fastest.  The winners become tile rules keyed by
the shape (a rule applies to data sets at least that large, see
epi3_tile_rule) and are written as JSON; the binding registers the rules of
`paper_2201_10956_amd/tiles.json` when it is imported.

    python -m paper_2201_10956_amd.autotune --out tiles.json
"""
from __future__ import annotations

import argparse
import json
import time

from . import epi3

CANDIDATES = {"valu": (4, 8), "mfma": (2, 4, 8), "mfma_fp4": (2, 4, 8)}
GRID_M = (64, 256, 1024, 2048)
GRID_N = (1024, 4096, 16384)


def _dataset(M, N, seed, device):
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    geno = torch.randint(0, 3, (M, N), generator=g, dtype=torch.uint8).to(device)
    pheno = (torch.rand(N, generator=g) < 0.5).to(torch.uint8).numpy()
    return epi3.encode(geno, pheno)


def _time_scan(ds, variant, k, reps):
    import torch
    sc = epi3.Scanner(ds, k, variant)
    sc.scan()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        sc.scan()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    sc.topk()
    times.sort()
    return times[len(times) // 2]


def tune(grid_m=GRID_M, grid_n=GRID_N, candidates=CANDIDATES, k=10, reps=3, device="cuda",
         log=print):
    """Returns the tile table {"rules": [...], "measurements": [...]}."""
    import torch
    epi3.tile_rules_clear()
    rules, meas = [], []
    for M in grid_m:
        for N in grid_n:
            ds = _dataset(M, N, seed=M * 100003 + N, device=device)
            best = {}
            for variant, tiles in candidates.items():
                for t in tiles:
                    epi3.tile_rules_clear()
                    epi3.tile_rule(variant, 0, 0, t)
                    try:
                        ms = _time_scan(ds, variant, k, reps)
                    except epi3.Epi3Error as e:  # variant not available for this shape
                        log(f"M={M} N={N} {variant} tile={t}: {e}")
                        continue
                    meas.append({"M": M, "N": N, "variant": variant, "tile": t, "ms": ms})
                    log(f"M={M} N={N} {variant} tile={t}: {ms:.3f} ms")
                    if variant not in best or ms < best[variant][1]:
                        best[variant] = (t, ms)
            for variant, (t, _) in best.items():
                rules.append({"variant": variant, "min_snps": M, "min_samples": N, "tile": t})
            if best:
                fastest = min(best, key=lambda v: best[v][1])
                rules.append({"variant": "auto", "min_snps": M, "min_samples": N,
                              "tile": fastest})
            del ds
            torch.cuda.empty_cache()
    epi3.tile_rules_clear()
    return {"device": torch.cuda.get_device_name(0), "created": time.strftime("%Y-%m-%d"),
            "k": k, "reps": reps, "rules": rules, "measurements": meas}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=epi3.TILES_PATH)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--m", type=int, nargs="*", default=list(GRID_M))
    ap.add_argument("--n", type=int, nargs="*", default=list(GRID_N))
    a = ap.parse_args(argv)
    table = tune(a.m, a.n, reps=a.reps, log=lambda s: print(s, flush=True))
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
    epi3.load_tiles(a.out)
    print(f"wrote {len(table['rules'])} rules to {a.out}", flush=True)


if __name__ == "__main__":
    main()
