"""Plain scans selecting by bound (no FP32 score plane): a sample pass over
every stride-th tile bounds the k-th score, the full pass lists only the
scores under the bound.  Hits must equal the oracle's top-k bit for bit (the
stored full-size result at 2048 x 16384 included), for both matrix-core
operand types, at shapes where the sample is every tile and where it is a
small fraction of them; the vector-ALU variant and the score-plane hook
refuse the mode; a list too short for the scores under the bound is
reported as a capacity error and holds them on the retry."""
import os

import numpy as np
import pytest

import oracle
from synth import CONFIGS, SplitMix64, make_config, make_dataset, manifest_sha256
from tests.gpu_util import assert_hits_equal_oracle, hits_ijk, require_gpu, to_dev

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def env():
    torch, epi3 = require_gpu()
    epi3.set_scan_select("bounded")
    yield torch, epi3
    epi3.set_scan_select("auto")
    epi3.set_compact_cap(0)


def _tiny(seed, M, N, p_case):
    u = SplitMix64(seed, 41).uniform(0, M * N + N)
    geno = np.minimum((u[: M * N] * 3).astype(np.uint8), 2).reshape(M, N)
    pheno = (u[M * N:] < p_case).astype(np.uint8)
    return geno, pheno


@pytest.mark.parametrize("variant", ["mfma", "mfma_fp4"])
@pytest.mark.parametrize("M,N,p,k", [(5, 31, 0.3, 3), (40, 300, 0.5, 25), (97, 300, 0.2, 100),
                                     (130, 700, 0.5, 10), (300, 1000, 0.5, 50)])
def test_bounded_equals_oracle(env, variant, M, N, p, k):
    torch, epi3 = env
    print(f"[case] bounded {variant} M={M} N={N} k={k}", flush=True)
    geno, pheno = _tiny(7 * M + N, M, N, p)
    ds = epi3.encode(to_dev(geno), pheno)
    h = epi3.Scanner(ds, k, variant).run()
    ijk, rk2, rcc = oracle.scan_topk(geno, pheno, k)
    assert_hits_equal_oracle(h, ijk, rk2, rcc)


@pytest.mark.parametrize("variant", ["mfma", "mfma_fp4"])
@pytest.mark.parametrize("M,N,p,k", [(2, 30, 0.5, 5), (3, 40, 0.5, 1), (4, 50, 0.4, 10),
                                     (5, 31, 0.3, 10), (12, 3, 0.5, 7), (30, 64, 0.0, 5),
                                     (30, 64, 1.0, 5)])
def test_bounded_edges(env, variant, M, N, p, k):
    """No triplet, one triplet, k at and above C(M,3), three samples, and a
    class with no samples (all controls, all cases)."""
    torch, epi3 = env
    print(f"[case] bounded edge {variant} M={M} N={N} p={p} k={k}", flush=True)
    geno, pheno = _tiny(7 * M + N, M, N, p)
    ds = epi3.encode(to_dev(geno), pheno)
    h = epi3.Scanner(ds, k, variant).run()
    ijk, rk2, rcc = oracle.scan_topk(geno, pheno, k)
    assert_hits_equal_oracle(h, ijk, rk2, rcc)


def test_bounded_ties(env):
    """Runs of identical SNP rows give exactly equal K2: ties broken by index."""
    torch, epi3 = env
    geno, pheno = _tiny(77, 120, 400, 0.45)
    for r in range(5, 120, 5):
        geno[r] = geno[r - 1]
    geno = np.ascontiguousarray(geno)
    ds = epi3.encode(to_dev(geno), pheno)
    h = epi3.Scanner(ds, 200, "mfma_fp4").run()
    ijk, rk2, rcc = oracle.scan_topk(geno, pheno, 200)
    assert_hits_equal_oracle(h, ijk, rk2, rcc)


def test_bounded_cfg2(env):
    """512 SNPs x 4096 samples, top-100: the sample is about 1 tile in 6."""
    torch, epi3 = env
    c = CONFIGS[2]
    d = make_config(2)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    h = epi3.Scanner(ds, c["k"], "mfma_fp4").run()
    ijk, rk2, rcc = oracle.scan_topk(d.geno, d.pheno, c["k"])
    assert_hits_equal_oracle(h, ijk, rk2, rcc)


def test_bounded_full_size(env):
    """2048 SNPs x 16384 samples, top-1000, without the 5.7 GB score plane:
    the stored oracle result."""
    torch, epi3 = env
    c = CONFIGS[3]
    d = make_config(3)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    h = epi3.Scanner(ds, c["k"], "mfma_fp4").run()
    fx = os.path.join(GOLDEN, f"oracle_cfg3_top{c['k']}.npz")
    if os.path.exists(fx):
        z = np.load(fx)
        assert str(z["sha256"]) == manifest_sha256([d.geno, d.pheno])
        assert_hits_equal_oracle(h, z["ijk"], z["k2"], z["counts"])
    else:
        rc, rk = oracle.score_list(d.geno, d.pheno, hits_ijk(h))
        np.testing.assert_array_equal(h["k2"], rk)


def test_bounded_refusals(env):
    torch, epi3 = env
    geno, pheno = _tiny(3, 30, 200, 0.5)
    ds = epi3.encode(to_dev(geno), pheno)
    with pytest.raises(epi3.Epi3Error) as e:
        epi3.Scanner(ds, 5, "valu").run()
    assert e.value.code == epi3.E_UNSUPPORTED
    sc = epi3.Scanner(ds, 5, "mfma_fp4")
    sc.scan()
    with pytest.raises(epi3.Epi3Error) as e:
        sc.score_plane()
    assert e.value.code == epi3.E_UNSUPPORTED


def test_bounded_list_overflow(env):
    """A list of 16 entries cannot hold the scores under the bound of a top-50
    of 4 million triplets: capacity error; with the default list the same
    scan equals the oracle."""
    torch, epi3 = env
    d = make_dataset(290, 2000, 0.5, 0.05, seed=4242)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    epi3.set_compact_cap(16)
    try:
        sc = epi3.Scanner(ds, 50, "mfma_fp4")
        with pytest.raises(epi3.Epi3Error) as e:
            sc.run(retry=False)
        assert e.value.code == epi3.E_CAPACITY
    finally:
        epi3.set_compact_cap(0)
    h = epi3.Scanner(ds, 50, "mfma_fp4").run()
    ijk, rk2, rcc = oracle.scan_topk(d.geno, d.pheno, 50)
    assert_hits_equal_oracle(h, ijk, rk2, rcc)


def test_8192_snps_properties(env):
    """8192 SNPs x 16384 samples, top-1000 (the paper's largest synthetic GPU
    shape; the plane would take 366 GB, so AUTO selects by bound too).  The
    oracle cannot rank 9.2e10 triplets here, so: hits in strict (K2, i, j, k)
    order with FP64 K2 and all 54 counts equal to the oracle's for the same
    triplets, and none of 20000 sampled triplets outside the hits ranks before
    the last hit."""
    torch, epi3 = env
    from math import comb
    c = CONFIGS[6]
    d = make_config(6)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    epi3.set_scan_select("auto")
    try:
        h = epi3.Scanner(ds, c["k"], "mfma_fp4").run()
    finally:
        epi3.set_scan_select("bounded")
    assert len(h) == c["k"]
    ijk = hits_ijk(h)
    keys = list(zip(h["k2"].tolist(), ijk[:, 0].tolist(), ijk[:, 1].tolist(), ijk[:, 2].tolist()))
    assert all(a < b for a, b in zip(keys, keys[1:]))
    rc, rk = oracle.score_list(d.geno, d.pheno, ijk)
    np.testing.assert_array_equal(h["k2"], rk)
    np.testing.assert_array_equal(h["counts"].astype(np.int64), rc.astype(np.int64))
    T = comb(c["M"], 3)
    ranks = np.unique((SplitMix64(606, 0).uniform(0, 20000) * T).astype(np.int64))
    from tests.gpu_util import lex_unrank
    smp = lex_unrank(c["M"], ranks)
    _, sk = oracle.score_list(d.geno, d.pheno, smp)
    hit_set = set(map(tuple, ijk.tolist()))
    last = keys[-1]
    for (i, j, k), v in zip(smp.tolist(), sk.tolist()):
        if (i, j, k) not in hit_set:
            assert (v, i, j, k) > last, ((i, j, k), v, last)
