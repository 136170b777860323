"""Candidate sets above 16384 entries are ordered by a bitonic sort of
(FP64 key, index) instead of counting, for each candidate, the candidates
before it.  Hits must still equal the oracle's top-k bit for bit, including
runs of exactly equal K2 (identical SNP rows), for triplets (plain and
phenotype batches), pairs and quads."""
import numpy as np
import pytest

import oracle
from synth import SplitMix64, make_dataset, make_permutations
from tests.gpu_util import assert_hits_equal_oracle, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _with_ties(M, N, seed, dup):
    """M SNPs of which every dup-th repeats the row before it (equal tables,
    equal K2: ties broken by index)."""
    u = SplitMix64(seed, 31).uniform(0, M * N + N)
    geno = np.minimum((u[: M * N] * 3).astype(np.uint8), 2).reshape(M, N)
    for r in range(dup, M, dup):
        geno[r] = geno[r - 1]
    pheno = (u[M * N:] < 0.45).astype(np.uint8)
    return np.ascontiguousarray(geno), pheno


@pytest.mark.parametrize("variant", ["valu", "mfma_fp4"])
@pytest.mark.parametrize("k", [3000, 20000])
def test_triplets_sorted_candidates(env, variant, k):
    torch, epi3 = env
    print(f"[case] triplets large k={k} variant={variant}", flush=True)
    geno, pheno = _with_ties(60, 500, 9001, 7)       # 34220 triplets
    ds = epi3.encode(to_dev(geno), pheno)
    h = epi3.Scanner(ds, k, variant, cand_cap=30000).run()
    ijk, k2, cc = oracle.scan_topk(geno, pheno, k)
    assert_hits_equal_oracle(h, ijk, k2, cc)


def test_pairs_sorted_candidates(env):
    torch, epi3 = env
    geno, pheno = _with_ties(400, 300, 9002, 11)     # 79800 pairs
    ds = epi3.encode(to_dev(geno), pheno, values=False)
    h = epi3.PairScanner(ds, 5000, cand_cap=40000).run()
    ij, k2, cc = oracle.scan_pairs_topk(geno, pheno, 5000)
    got = np.stack([h["i"], h["j"]], axis=1).astype(np.int32)
    np.testing.assert_array_equal(got, ij)
    np.testing.assert_array_equal(h["k2"], k2)
    np.testing.assert_array_equal(h["counts"].astype(np.int64), cc.astype(np.int64))


@pytest.mark.parametrize("values", [True, False])
def test_quads_sorted_candidates(env, values):
    torch, epi3 = env
    geno, pheno = _with_ties(32, 300, 9003, 5)       # 35960 quads
    ds = epi3.encode(to_dev(geno), pheno, values=values)
    h = epi3.QuadScanner(ds, 2000, cand_cap=30000).run()
    q, k2, cc = oracle.scan_quads_topk(geno, pheno, 2000)
    got = np.stack([h["i"], h["j"], h["k"], h["l"]], axis=1).astype(np.int32)
    np.testing.assert_array_equal(got, q)
    np.testing.assert_array_equal(h["k2"], k2)
    np.testing.assert_array_equal(h["counts"].astype(np.int64), cc.astype(np.int64))


def test_phenotype_batch_sorted_candidates(env):
    torch, epi3 = env
    d = make_dataset(60, 700, 0.4, 0.05, seed=9004)  # 34220 triplets per phenotype
    perms = make_permutations(d.pheno, 3, seed=9005)
    ds = epi3.encode(to_dev(d.geno), d.pheno, layout="masked")
    masks = torch.from_numpy(epi3.pack_masks(perms).view(np.int32)).to("cuda")
    res = epi3.BatchScanner(ds, 1500, masks=masks, variant="mfma_fp4", cand_cap=20000).run()
    for q in range(3):
        ijk, k2, cc = oracle.scan_topk(d.geno, perms[q], 1500)
        assert_hits_equal_oracle(res[q], ijk, k2, cc)
