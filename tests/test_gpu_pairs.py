"""GPU parity of the second-order (pair) scan against the oracle's pair scan:
every pair's FP32 score within the pair error bound, and hits (pair, FP64 K2
bit for bit, both 9-row tables) equal to the oracle's top-k."""
import numpy as np
import pytest

import oracle
from synth import CONFIGS, SplitMix64, make_config, make_dataset
from tests.gpu_util import require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _tiny(seed, M, N, p_case):
    u = SplitMix64(seed, 23).uniform(0, M * N + N)
    geno = np.minimum((u[: M * N] * 3).astype(np.uint8), 2).reshape(M, N)
    pheno = (u[M * N:] < p_case).astype(np.uint8)
    return geno, pheno


def assert_pair_hits_equal_oracle(h, ij, k2, counts):
    assert len(h) == len(ij), (len(h), len(ij))
    np.testing.assert_array_equal(np.stack([h["i"], h["j"]], axis=1).astype(np.int32), ij)
    np.testing.assert_array_equal(h["k2"], k2)
    np.testing.assert_array_equal(h["counts"].astype(np.int64), counts.astype(np.int64))


def assert_pair_k2_close(got32, ref64, N, epi3):
    diff = np.abs(np.asarray(got32, dtype=np.float64) - ref64)
    e = epi3.k2_error_bound_pairs(N)
    assert np.all(diff <= e), (diff.max(), e)
    assert np.all(diff / np.maximum(np.abs(ref64), 1e-30) <= 1e-4)


@pytest.mark.parametrize("M,N,p", [(2, 1, 0.5), (2, 64, 0.0), (3, 33, 1.0), (5, 31, 0.3),
                                   (64, 95, 0.5), (257, 129, 0.45), (300, 1000, 0.2),
                                   (130, 4097, 0.5)])
def test_every_pair_score_and_topk(env, M, N, p):
    torch, epi3 = env
    print(f"[case] pairs M={M} N={N} p={p}", flush=True)
    geno, pheno = _tiny(100 * M + N, M, N, p)
    ds = epi3.encode(to_dev(geno), pheno)
    k = min(40, M * (M - 1) // 2)
    sc = epi3.PairScanner(ds, k)
    h = sc.run()
    ref_k2, _ = oracle.scan_pairs_all(geno, pheno, counts=False)
    assert_pair_k2_close(sc.score_plane().cpu().numpy(), ref_k2, N, epi3)
    ij, rk2, rcc = oracle.scan_pairs_topk(geno, pheno, k)
    assert_pair_hits_equal_oracle(h, ij, rk2, rcc)


@pytest.mark.parametrize("cfg", [2, 3])
def test_pairs_at_full_size(env, cfg):
    """512 x 4096 (top-100) and 2048 x 16384 (top-1000): hits equal the
    oracle's; sampled FP32 scores within the bound."""
    torch, epi3 = env
    c = CONFIGS[cfg]
    print(f"[case] pairs cfg shape {c['M']}x{c['N']} top-{c['k']}", flush=True)
    d = make_config(cfg)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    sc = epi3.PairScanner(ds, c["k"])
    h = sc.run()
    ij, rk2, rcc = oracle.scan_pairs_topk(d.geno, d.pheno, c["k"])
    assert_pair_hits_equal_oracle(h, ij, rk2, rcc)
    P = epi3.n_pairs(d.n_snps)
    ranks = np.unique((SplitMix64(77, 0).uniform(0, 2000) * P).astype(np.int64))
    lex = oracle.lex_pairs(d.n_snps)[ranks]
    ref = np.array([oracle.k2_rows(oracle.pair_table(d.geno, d.pheno, int(a), int(b)),
                                   oracle.log_factorial(d.n_samples + 1)) for a, b in lex[:200]])
    got = sc.score_plane()[torch.as_tensor(ranks[:200], device="cuda")].cpu().numpy()
    assert_pair_k2_close(got, ref, d.n_samples, epi3)


def test_pairs_edge_cases(env):
    torch, epi3 = env
    # one class only, ties between identical SNP rows (broken by (i, j)), k > C(M,2)
    base, _ = _tiny(3, 1, 200, 0.5)
    geno = np.repeat(base, 6, axis=0)
    for ph in (np.zeros(200, np.uint8), np.ones(200, np.uint8)):
        ds = epi3.encode(to_dev(geno), ph)
        h = epi3.scan_pairs(ds, 50)
        ij, rk2, rcc = oracle.scan_pairs_topk(geno, ph, 50)
        assert len(h) == 15
        assert_pair_hits_equal_oracle(h, ij, rk2, rcc)
    # fewer than two SNPs: no pairs
    ds = epi3.encode(to_dev(geno[:1]), np.zeros(200, np.uint8))
    assert len(epi3.scan_pairs(ds, 5)) == 0


def test_pairs_candidate_capacity_retry(env):
    """A tiny candidate capacity overflows (EPI3_E_CAPACITY with the needed
    size); the scanner retries with it and returns the oracle's hits."""
    torch, epi3 = env
    d = make_dataset(200, 3000, 0.5, 0.05, seed=41)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    sc = epi3.PairScanner(ds, 30, cand_cap=10)
    sc.scan()
    rc, need = sc.topk()
    assert rc == epi3.E_CAPACITY and need >= 30
    h = epi3.PairScanner(ds, 30, cand_cap=need).run()
    ij, rk2, rcc = oracle.scan_pairs_topk(d.geno, d.pheno, 30)
    assert_pair_hits_equal_oracle(h, ij, rk2, rcc)


def test_pairs_refuse_masked_layout(env):
    torch, epi3 = env
    geno, pheno = _tiny(9, 10, 100, 0.5)
    ds = epi3.encode(to_dev(geno), pheno, layout="masked")
    with pytest.raises(epi3.Epi3Error) as e:
        epi3.scan_pairs(ds, 3)
    assert e.value.code == epi3.E_UNSUPPORTED
