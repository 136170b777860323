"""GPU parity of the plain scan (encode -> count + K2 -> top-k) against the oracle."""
import itertools
import os

import numpy as np
import pytest

import oracle
from synth import CONFIGS, SplitMix64, make_config, make_dataset, manifest_sha256
from tests.gpu_util import (assert_hits_equal_oracle, assert_k2_close, hits_ijk, lex_rank,
                            lex_unrank, require_gpu, to_dev)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _tiny(seed, M, N, p_case):
    u = SplitMix64(seed, 21).uniform(0, M * N + N)
    geno = np.minimum((u[: M * N] * 3).astype(np.uint8), 2).reshape(M, N)
    pheno = (u[M * N:] < p_case).astype(np.uint8)
    return geno, pheno


def test_cfg1_every_table_and_score(env):
    torch, epi3 = env
    d = make_config(1)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    cc, k2 = epi3.scan_tables(ds, "valu")
    ref_k2, ref_cc = oracle.scan_all(d.geno, d.pheno)
    np.testing.assert_array_equal(cc.cpu().numpy(), ref_cc)
    assert_k2_close(k2.cpu().numpy(), ref_k2, d.n_samples, epi3)


def test_cfg1_topk(env):
    torch, epi3 = env
    c = CONFIGS[1]
    d = make_config(1)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    h = epi3.scan_topk(ds, c["k"], "valu")
    ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, c["k"])
    assert_hits_equal_oracle(h, ijk, k2, cc)


@pytest.mark.parametrize("M,N,p", [(3, 1, 0.5), (3, 64, 0.0), (4, 33, 1.0), (5, 31, 0.3),
                                   (9, 95, 0.5), (17, 257, 0.7), (66, 130, 0.45), (130, 70, 0.5)])
def test_ragged_shapes_every_table(env, M, N, p):
    torch, epi3 = env
    geno, pheno = _tiny(1000 * M + N, M, N, p)
    ds = epi3.encode(to_dev(geno), pheno)
    cc, k2 = epi3.scan_tables(ds, "valu")
    ref_k2, ref_cc = oracle.scan_all(geno, pheno)
    np.testing.assert_array_equal(cc.cpu().numpy(), ref_cc)
    assert_k2_close(k2.cpu().numpy(), ref_k2, N, epi3)
    k = min(25, len(ref_k2))
    h = epi3.scan_topk(ds, k, "valu")
    ijk, rk2, rcc = oracle.scan_topk(geno, pheno, k)
    assert_hits_equal_oracle(h, ijk, rk2, rcc)


def test_strided_rows_and_identical_snps(env):
    torch, epi3 = env
    base, pheno = _tiny(5, 1, 77, 0.5)
    geno = np.repeat(base, 7, axis=0)
    big = np.zeros((7, 200), dtype=np.uint8)
    big[:, :77] = geno
    g = to_dev(big)[:, :77]          # row stride 200
    ds = epi3.encode(g, pheno)
    h = epi3.scan_topk(ds, 35, "valu")
    assert [tuple(x) for x in hits_ijk(h)] == list(itertools.combinations(range(7), 3))
    assert np.all(h["k2"] == h["k2"][0])


def test_k_larger_than_triplets_and_too_few_snps(env):
    torch, epi3 = env
    geno, pheno = _tiny(8, 6, 40, 0.5)
    ds = epi3.encode(to_dev(geno), pheno)
    h = epi3.scan_topk(ds, 100, "valu")
    ijk, k2, cc = oracle.scan_topk(geno, pheno, 100)
    assert len(h) == 20
    assert_hits_equal_oracle(h, ijk, k2, cc)
    ds2 = epi3.encode(to_dev(geno[:2]), pheno)
    assert len(epi3.scan_topk(ds2, 5, "valu")) == 0


@pytest.mark.parametrize("variant", ["valu", "mfma_fp4"])
def test_many_exact_ties_rank_over_several_chunks(env, variant):
    """30 SNPs drawn from 4 distinct rows: thousands of triplets share their
    K2 exactly, and k = all 4060 triplets puts every one through the rank
    kernel (several 1024-candidate chunks, ties broken by (i, j, k))."""
    torch, epi3 = env
    print(f"[case] exact ties, 30 SNPs x 200 samples, k=4060, {variant}", flush=True)
    base, pheno = _tiny(77, 4, 200, 0.4)
    pick = SplitMix64(78, 1).uniform(0, 30)
    geno = np.ascontiguousarray(base[np.minimum((pick * 4).astype(np.int64), 3)])
    ds = epi3.encode(to_dev(geno), pheno)
    h = epi3.scan_topk(ds, 4060, variant)
    ijk, k2, cc = oracle.scan_topk(geno, pheno, 4060)
    assert len(h) == 4060 and len(np.unique(k2)) < 400
    assert_hits_equal_oracle(h, ijk, k2, cc)


def test_bits_only_encoding(env):
    """A data set encoded without value planes scans with the popcount kernel
    (AUTO falls back to it) to the oracle's hits, and the matrix-core kernels
    refuse it; pair and quad scans on it equal those on a full encoding."""
    torch, epi3 = env
    print("[case] bits-only encoding, 24 SNPs x 900 samples", flush=True)
    d = make_dataset(24, 900, 0.4, 0.05, seed=91)
    g = to_dev(d.geno)
    ds = epi3.encode(g, d.pheno, values=False)
    assert not ds.c.bytes and not ds.c.nibbles
    ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, 15)
    for variant in ("auto", "valu"):
        assert_hits_equal_oracle(epi3.scan_topk(ds, 15, variant), ijk, k2, cc)
    for variant in ("mfma", "mfma_fp4"):
        with pytest.raises(epi3.Epi3Error) as e:
            epi3.scan_topk(ds, 15, variant)
        assert e.value.code == epi3.E_UNSUPPORTED
    full = epi3.encode(g, d.pheno)
    assert epi3.scan_pairs(ds, 20).tobytes() == epi3.scan_pairs(full, 20).tobytes()
    assert epi3.scan_quads(ds, 20).tobytes() == epi3.scan_quads(full, 20).tobytes()
    # re-encoding into the same buffer keeps the flag's effect
    again = epi3.encode(g, d.pheno, into=ds, values=False)
    assert not again.c.bytes
    assert_hits_equal_oracle(epi3.scan_topk(again, 15, "valu"), ijk, k2, cc)


def test_bad_genotype_and_phenotype(env):
    torch, epi3 = env
    geno, pheno = _tiny(9, 5, 40, 0.5)
    geno[3, 17] = 3
    ds = epi3.encode(to_dev(geno), pheno)
    with pytest.raises(epi3.Epi3Error) as e:
        epi3.scan_topk(ds, 3, "valu")
    assert e.value.code == epi3.E_GENOTYPE
    geno[3, 17] = 1
    bad = pheno.copy()
    bad[4] = 2
    with pytest.raises(epi3.Epi3Error) as e:
        epi3.encode(to_dev(geno), bad)
    assert e.value.code == epi3.E_PHENOTYPE


def test_capacity_overflow_then_retry(env):
    torch, epi3 = env
    d = make_config(1)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    sc = epi3.Scanner(ds, 10, "valu", cand_cap=3)
    sc.scan()
    with pytest.raises(epi3.Epi3Error) as e:
        sc.topk()
    assert e.value.code == epi3.E_CAPACITY
    h = sc.run()               # retries with the reported capacity
    ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, 10)
    assert_hits_equal_oracle(h, ijk, k2, cc)


def test_cfg2_score_plane_and_topk(env):
    torch, epi3 = env
    c = CONFIGS[2]
    d = make_config(2)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    sc = epi3.Scanner(ds, c["k"], "valu")
    h = sc.run()
    ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, c["k"])
    assert_hits_equal_oracle(h, ijk, k2, cc)
    plane = sc.score_plane().cpu().numpy()
    ref_k2, _ = oracle.scan_all(d.geno, d.pheno, counts=False)
    assert_k2_close(plane, ref_k2, d.n_samples, epi3)
    # the FP32 value carried by each hit is the plane's value
    ranks = [lex_rank(d.n_snps, *x) for x in ijk]
    np.testing.assert_array_equal(h["k2_f32"], plane[ranks])


def test_score_triplets_sampled(env):
    torch, epi3 = env
    d = make_config(2)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    u = SplitMix64(77, 0).uniform(0, 3 * 3000).reshape(-1, 3)
    ijk = np.sort((u * d.n_snps).astype(np.int64), axis=1)
    keep = (ijk[:, 0] < ijk[:, 1]) & (ijk[:, 1] < ijk[:, 2])
    ijk = ijk[keep].astype(np.int32)
    cc, kf, kd = epi3.score_triplets(ds, ijk)
    rc, rk = oracle.score_list(d.geno, d.pheno, ijk)
    np.testing.assert_array_equal(cc.cpu().numpy(), rc)
    np.testing.assert_array_equal(kd.cpu().numpy(), rk)
    assert_k2_close(kf.cpu().numpy(), rk, d.n_samples, epi3)


def test_repeat_runs_bit_identical(env):
    torch, epi3 = env
    d = make_config(1)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    sc = epi3.Scanner(ds, 50, "valu")
    a = sc.run()
    p1 = sc.score_plane().clone()
    b = sc.run()
    p2 = sc.score_plane().clone()
    assert a.tobytes() == b.tobytes()
    assert torch.equal(p1, p2)


def test_cfg3_full_size(env):
    """2048 SNPs x 16384 samples, top-1000: hits equal the stored oracle result;
    sampled scores of the whole plane and sampled tables equal the oracle's."""
    torch, epi3 = env
    c = CONFIGS[3]
    d = make_config(3)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    sc = epi3.Scanner(ds, c["k"], "valu")
    h = sc.run()
    fx = os.path.join(GOLDEN, f"oracle_cfg3_top{c['k']}.npz")
    if os.path.exists(fx):
        z = np.load(fx)
        assert str(z["sha256"]) == manifest_sha256([d.geno, d.pheno])
        assert_hits_equal_oracle(h, z["ijk"], z["k2"], z["counts"])
    else:  # no stored result: check the hits one by one against the oracle
        rc, rk = oracle.score_list(d.geno, d.pheno, hits_ijk(h))
        np.testing.assert_array_equal(h["k2"], rk)
        np.testing.assert_array_equal(h["counts"].astype(np.int64), rc)
    plane = sc.score_plane()
    T = epi3.n_triplets(d.n_snps)
    u = SplitMix64(33, 0).uniform(0, 4000)
    ranks = np.unique((u * T).astype(np.int64))
    M = d.n_snps
    lex = lex_unrank(M, ranks)
    rc, rk = oracle.score_list(d.geno, d.pheno, lex)
    got = plane[torch.as_tensor(ranks, device=plane.device)].cpu().numpy()
    assert_k2_close(got, rk, d.n_samples, epi3)
    # every sampled triplet that beats the returned k-th best is among the hits
    hit_set = set(map(tuple, hits_ijk(h).tolist()))
    for x in np.nonzero(rk < h["k2"][-1])[0]:
        assert tuple(lex[x].tolist()) in hit_set
    cc, kf, kd = epi3.score_triplets(ds, lex)
    np.testing.assert_array_equal(cc.cpu().numpy(), rc)
    np.testing.assert_array_equal(kf.cpu().numpy(), got)


@pytest.mark.parametrize("ccap", [1, 3, 40])
def test_compaction_overflow_falls_back_to_plane(env, ccap):
    """A compaction capacity too small for the low end of the plane: the later
    selection passes read the whole plane again and the hits stay exact."""
    torch, epi3 = env
    d = make_config(1)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    try:
        epi3.set_compact_cap(ccap)
        h = epi3.scan_topk(ds, 10, "valu")
    finally:
        epi3.set_compact_cap(0)
    ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, 10)
    assert_hits_equal_oracle(h, ijk, k2, cc)


@pytest.mark.parametrize("variant", ["valu", "mfma_fp4"])
def test_sampled_bound_with_compaction_overflow(env, variant):
    """512 SNPs x 4096 samples (22 M triplets): the first bound comes from the
    sampled select; with a compaction capacity of 16 the list overflows and the
    later passes read the plane.  Hits stay exact either way."""
    torch, epi3 = env
    print(f"[case] sampled bound, {variant}", flush=True)
    d = make_config(2)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, 100)
    h = epi3.scan_topk(ds, 100, variant)
    assert_hits_equal_oracle(h, ijk, k2, cc)
    try:
        epi3.set_compact_cap(16)
        h = epi3.scan_topk(ds, 100, variant)
    finally:
        epi3.set_compact_cap(0)
    assert_hits_equal_oracle(h, ijk, k2, cc)
