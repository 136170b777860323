"""Writes the stored oracle results for the full-size workloads.

Every value written here comes from the CPU oracle (package `oracle`) run on
inputs drawn by `synth`; nothing comes from the GPU library.  Each fixture
records the SHA-256 of its inputs so a test can tell whether the generator
still reproduces them.

    python tests/golden/make_fixtures.py 3          # plain 2048 x 16384, top-1000
    python tests/golden/make_fixtures.py 4 --perm 0:64
    python tests/golden/make_fixtures.py 5
    python tests/golden/make_fixtures.py 4 --observed   # the unpermuted phenotype, top-10
    python tests/golden/make_fixtures.py 2 --quads 256  # quads of the first 256 SNPs, top-100
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import CONFIGS, make_config, manifest_sha256  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _save(name: str, **arrays) -> str:
    path = os.path.join(HERE, name)
    np.savez_compressed(path, **arrays)
    return path


def plain(cfg: int, threads: int) -> None:
    c = CONFIGS[cfg]
    d = make_config(cfg)
    t0 = time.time()
    ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, c["k"], nthreads=threads)
    dt = time.time() - t0
    p = _save(f"oracle_cfg{cfg}_top{c['k']}.npz", ijk=ijk, k2=k2, counts=cc,
              sha256=np.array(manifest_sha256([d.geno, d.pheno])),
              seconds=np.array(dt), threads=np.array(threads))
    print(f"cfg{cfg}: {dt:.1f}s on {threads} threads -> {p}", flush=True)


def perm(cfg: int, threads: int, lo: int, hi: int) -> None:
    c = CONFIGS[cfg]
    d, perms = make_config(cfg)
    for p in range(lo, hi):
        name = f"oracle_cfg{cfg}_perm{p:02d}_top{c['k']}.npz"
        if os.path.exists(os.path.join(HERE, name)):
            continue
        t0 = time.time()
        ijk, k2, cc = oracle.scan_topk(d.geno, perms[p], c["k"], nthreads=threads)
        dt = time.time() - t0
        _save(name, ijk=ijk, k2=k2, counts=cc,
              sha256=np.array(manifest_sha256([d.geno, perms[p]])),
              seconds=np.array(dt), threads=np.array(threads))
        print(f"cfg{cfg} perm {p}: {dt:.1f}s", flush=True)


def observed(cfg: int, threads: int) -> None:
    """The permutation workload's own (unpermuted) phenotype."""
    c = CONFIGS[cfg]
    d, _ = make_config(cfg)
    t0 = time.time()
    ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, c["k"], nthreads=threads)
    dt = time.time() - t0
    p = _save(f"oracle_cfg{cfg}_observed_top{c['k']}.npz", ijk=ijk, k2=k2, counts=cc,
              sha256=np.array(manifest_sha256([d.geno, d.pheno])),
              seconds=np.array(dt), threads=np.array(threads))
    print(f"cfg{cfg} observed: {dt:.1f}s -> {p}", flush=True)


def quads(cfg: int, snps: int, threads: int, k: int = 100) -> None:
    """Fourth-order scan of the first `snps` SNPs of a plain workload."""
    d = make_config(cfg)
    g = np.ascontiguousarray(d.geno[:snps])
    t0 = time.time()
    q, k2, cc = oracle.scan_quads_topk(g, d.pheno, k, nthreads=threads)
    dt = time.time() - t0
    p = _save(f"oracle_cfg{cfg}_quads{snps}_top{k}.npz", ijkl=q, k2=k2, counts=cc,
              sha256=np.array(manifest_sha256([g, d.pheno])),
              seconds=np.array(dt), threads=np.array(threads))
    print(f"cfg{cfg} quads of {snps} SNPs: {dt:.1f}s -> {p}", flush=True)


def uneven(cfg: int, threads: int) -> None:
    c = CONFIGS[cfg]
    ds = make_config(cfg)
    out = {}
    t0 = time.time()
    for x, d in enumerate(ds):
        ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, c["k"], nthreads=threads)
        out[f"ijk{x}"] = ijk
        out[f"k2{x}"] = k2
        out[f"counts{x}"] = cc
        out[f"sha{x}"] = np.array(manifest_sha256([d.geno, d.pheno]))
        print(f"cfg{cfg} dataset {x} ({d.n_snps}x{d.n_samples}) done at {time.time() - t0:.0f}s",
              flush=True)
    out["seconds"] = np.array(time.time() - t0)
    out["threads"] = np.array(threads)
    print(_save(f"oracle_cfg{cfg}_top{c['k']}.npz", **out))


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("cfg", type=int)
    ap.add_argument("--threads", type=int, default=oracle.nthreads_default())
    ap.add_argument("--perm", default="0:64")
    ap.add_argument("--observed", action="store_true")
    ap.add_argument("--quads", type=int, default=0)
    a = ap.parse_args()
    kind = CONFIGS[a.cfg]["kind"]
    if a.quads:
        quads(a.cfg, a.quads, a.threads)
    elif a.observed:
        observed(a.cfg, a.threads)
    elif kind == "plain":
        plain(a.cfg, a.threads)
    elif kind == "perm":
        lo, hi = (int(x) for x in a.perm.split(":"))
        perm(a.cfg, a.threads, lo, hi)
    else:
        uneven(a.cfg, a.threads)
