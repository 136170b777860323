"""Seeded generator for synthetic case-control genotype data.

Data model (paper, Problem Formulation section): a data set holds M SNPs and
N samples; each genotype is 0 (homozygous major), 1 (heterozygous) or 2
(homozygous minor) and each sample carries a phenotype 0 (control) or
1 (case).  The paper measures on synthetic data of 2048-8192 SNPs by 16384
samples (Experimental Results section); the workloads below are synthetic
stand-ins with the same structure.

Random numbers come from counter-based SplitMix64 streams (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): the
n-th output of a stream with start state x0 is mix64(x0 + (n + 1) * GAMMA),
so every array below depends only on (seed, stream id, index), not on numpy's
distribution code.  Nothing here computes a contingency table or a score.
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_SEED_MUL = np.uint64(0xD1B54A32D192ED03)
_STREAM_MUL = np.uint64(0x8CB92BA72F3D8DD7)


def _mix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


class SplitMix64:
    """Counter-based SplitMix64 stream keyed by (seed, stream)."""

    def __init__(self, seed: int, stream: int):
        with np.errstate(over="ignore"):
            s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
            t = np.uint64(stream & 0xFFFFFFFFFFFFFFFF)
            x = (s + np.uint64(1)) * _SEED_MUL ^ (t + np.uint64(1)) * _STREAM_MUL
            self.x0 = _mix64(np.asarray([x], dtype=np.uint64))[0]

    def u64(self, start: int, count: int) -> np.ndarray:
        n = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        with np.errstate(over="ignore"):
            return _mix64(self.x0 + n * _GAMMA)

    def uniform(self, start: int, count: int) -> np.ndarray:
        """Doubles in [0, 1) with 53 random bits."""
        return (self.u64(start, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclasses.dataclass
class Dataset:
    geno: np.ndarray            # uint8 [M][N], SNP-major, values {0,1,2}
    pheno: np.ndarray           # uint8 [N], 1 = case
    planted: Tuple[int, int, int]
    maf: np.ndarray             # float64 [M]
    seed: int

    @property
    def n_snps(self) -> int:
        return int(self.geno.shape[0])

    @property
    def n_samples(self) -> int:
        return int(self.geno.shape[1])

    @property
    def n_cases(self) -> int:
        return int(self.pheno.sum())


def _genotypes(M: int, N: int, maf_lo: float, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Hardy-Weinberg genotypes: P(0) = (1-q)^2, P(1) = 2q(1-q), P(2) = q^2."""
    q = maf_lo + (0.5 - maf_lo) * SplitMix64(seed, 0).uniform(0, M)
    geno = np.empty((M, N), dtype=np.uint8)
    g_stream = SplitMix64(seed, 1)
    rows = max(1, (1 << 22) // max(N, 1))
    for m0 in range(0, M, rows):
        m1 = min(M, m0 + rows)
        u = g_stream.uniform(m0 * N, (m1 - m0) * N).reshape(m1 - m0, N)
        qq = q[m0:m1, None]
        p0 = (1.0 - qq) ** 2
        p01 = 1.0 - qq * qq
        geno[m0:m1] = np.where(u < p0, 0, np.where(u < p01, 1, 2)).astype(np.uint8)
    return geno, q


def _choose_distinct(M: int, count: int, stream: SplitMix64) -> Tuple[int, ...]:
    """Partial Fisher-Yates draw of `count` distinct indices from range(M)."""
    pool = list(range(M))
    u = stream.uniform(0, count)
    for t in range(count):
        r = t + int(u[t] * (M - t))
        pool[t], pool[r] = pool[r], pool[t]
    return tuple(sorted(pool[:count]))


def make_dataset(M: int, N: int, case_frac: float, maf_lo: float, seed: int,
                 planted_mode: str = "any_minor", risk: float = 2.0) -> Dataset:
    """One case-control data set with one planted triplet.

    Exactly round(case_frac * N) samples are cases.  They are drawn without
    replacement with weights w_s (Efraimidis-Spirakis: the samples with the
    smallest -ln(u_s) / w_s), where w_s = `risk` for samples whose genotypes
    at the planted SNPs fall in the raised-risk cells and 1 otherwise.
    planted_mode "any_minor": all three planted genotypes are >= 1;
    "all_minor": all three are 2; "none": no planted signal.
    """
    geno, q = _genotypes(M, N, maf_lo, seed)
    n_cases = int(round(case_frac * N))
    planted: Tuple[int, int, int] = (-1, -1, -1)
    w = np.ones(N, dtype=np.float64)
    if planted_mode != "none" and M >= 3:
        planted = _choose_distinct(M, 3, SplitMix64(seed, 2))  # type: ignore[assignment]
        ga, gb, gc = (geno[s] for s in planted)
        if planted_mode == "any_minor":
            hit = (ga >= 1) & (gb >= 1) & (gc >= 1)
        elif planted_mode == "all_minor":
            hit = (ga == 2) & (gb == 2) & (gc == 2)
        else:
            raise ValueError(planted_mode)
        w[hit] = risk
    u = 1.0 - SplitMix64(seed, 3).uniform(0, N)          # (0, 1]
    key = -np.log(u) / w
    order = np.argsort(key, kind="stable")
    pheno = np.zeros(N, dtype=np.uint8)
    pheno[order[:n_cases]] = 1
    return Dataset(geno=geno, pheno=pheno, planted=planted, maf=q, seed=seed)


def make_parity_fixture(seed: int, M: int = 32, N: int = 512, flip: float = 0.10) -> Dataset:
    """Strong planted signal: case iff the planted genotypes sum to an odd
    number, with a fraction `flip` of labels flipped."""
    geno, q = _genotypes(M, N, 0.05, seed)
    planted = _choose_distinct(M, 3, SplitMix64(seed, 2))
    s = geno[planted[0]].astype(np.int32) + geno[planted[1]] + geno[planted[2]]
    pheno = (s % 2).astype(np.uint8)
    flips = SplitMix64(seed, 4).uniform(0, N) < flip
    pheno[flips] ^= 1
    return Dataset(geno=geno, pheno=pheno, planted=planted, maf=q, seed=seed)  # type: ignore[arg-type]


def make_permutations(pheno: np.ndarray, n_perm: int, seed: int) -> np.ndarray:
    """n_perm seed-fixed permutations of a phenotype vector, uint8 [P][N].

    Permutation p orders the samples by the uniforms of stream (seed, 100 + p),
    which is a uniformly random permutation."""
    N = pheno.shape[0]
    out = np.empty((n_perm, N), dtype=np.uint8)
    for p in range(n_perm):
        perm = np.argsort(SplitMix64(seed, 100 + p).uniform(0, N), kind="stable")
        out[p] = pheno[perm]
    return out


def make_uneven(n_datasets: int, seed: int, m_range=(128, 1024), n_range=(1024, 16384),
                frac_range=(0.3, 0.7), maf_lo: float = 0.05,
                scale: float = 1.0) -> List[Dataset]:
    """Independent data sets of uneven shape, each with one planted triplet.
    `scale` shrinks both size ranges (for small test batches)."""
    st = SplitMix64(seed, 7)
    u = st.uniform(0, 3 * n_datasets).reshape(n_datasets, 3)
    m_lo, m_hi = (max(3, int(x * scale)) for x in m_range)
    n_lo, n_hi = (max(8, int(x * scale)) for x in n_range)
    out = []
    for d in range(n_datasets):
        M = m_lo + int(u[d, 0] * (m_hi - m_lo + 1))
        N = n_lo + int(u[d, 1] * (n_hi - n_lo + 1))
        frac = frac_range[0] + (frac_range[1] - frac_range[0]) * u[d, 2]
        out.append(make_dataset(M, N, frac, maf_lo, seed * 1000 + d))
    return out


# Workloads: the synthetic scan configurations the library is measured on.
CONFIGS: Dict[int, dict] = {
    1: dict(kind="plain", M=64, N=1024, case_frac=0.5, maf_lo=0.05, seed=1001, k=10),
    2: dict(kind="plain", M=512, N=4096, case_frac=0.5, maf_lo=0.05, seed=1002, k=100),
    3: dict(kind="plain", M=2048, N=16384, case_frac=0.5, maf_lo=0.01, seed=1003, k=1000),
    4: dict(kind="perm", M=1024, N=8192, case_frac=0.4, maf_lo=0.05, seed=1004, k=10,
            n_perm=64, perm_seed=2000),
    5: dict(kind="uneven", n_datasets=32, seed=3000, k=10),
    # the largest synthetic shape of the paper's GPU study (8192 SNPs x 16384
    # samples): its FP32 score plane would take 366 GB, so the scan selects by bound
    6: dict(kind="plain", M=8192, N=16384, case_frac=0.5, maf_lo=0.01, seed=1006, k=1000),
}


def make_config(cfg: int, **override):
    """Inputs of one workload: a Dataset (plain), (Dataset, perms) or a list."""
    c = dict(CONFIGS[cfg])
    c.update(override)
    if c["kind"] == "plain":
        return make_dataset(c["M"], c["N"], c["case_frac"], c["maf_lo"], c["seed"])
    if c["kind"] == "perm":
        d = make_dataset(c["M"], c["N"], c["case_frac"], c["maf_lo"], c["seed"])
        return d, make_permutations(d.pheno, c["n_perm"], c["perm_seed"])
    if c["kind"] == "uneven":
        return make_uneven(c["n_datasets"], c["seed"], scale=c.get("scale", 1.0))
    raise ValueError(c["kind"])


def manifest_sha256(arrays: Sequence[np.ndarray]) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()
