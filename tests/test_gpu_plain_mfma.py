"""GPU parity of the plain scan with the matrix-core count kernels (int8 bytes
and FP4 nibbles) against the oracle, and against the vector-ALU kernel's
tables and score plane (already pinned to the oracle)."""
import os

import numpy as np
import pytest

import oracle
from synth import CONFIGS, SplitMix64, make_config, make_dataset, manifest_sha256
from tests.gpu_util import (assert_hits_equal_oracle, assert_k2_close, hits_ijk, lex_unrank,
                            require_gpu, to_dev)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
VARIANTS = ["mfma", "mfma_fp4"]


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _tiny(seed, M, N, p_case):
    u = SplitMix64(seed, 21).uniform(0, M * N + N)
    geno = np.minimum((u[: M * N] * 3).astype(np.uint8), 2).reshape(M, N)
    pheno = (u[M * N:] < p_case).astype(np.uint8)
    return geno, pheno


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("M,N,p", [(3, 1, 0.5), (3, 64, 0.0), (4, 33, 1.0), (5, 31, 0.3),
                                   (9, 95, 0.5), (34, 129, 0.5), (66, 257, 0.45),
                                   (130, 70, 0.5), (97, 300, 0.2)])
def test_ragged_shapes_every_table(env, M, N, p, variant):
    torch, epi3 = env
    print(f"[case] {variant} M={M} N={N} p={p}", flush=True)
    geno, pheno = _tiny(1000 * M + N, M, N, p)
    ds = epi3.encode(to_dev(geno), pheno)
    cc, k2 = epi3.scan_tables(ds, variant)
    ref_k2, ref_cc = oracle.scan_all(geno, pheno)
    np.testing.assert_array_equal(cc.cpu().numpy(), ref_cc)
    assert_k2_close(k2.cpu().numpy(), ref_k2, N, epi3)
    k = min(25, len(ref_k2))
    h = epi3.scan_topk(ds, k, variant)
    ijk, rk2, rcc = oracle.scan_topk(geno, pheno, k)
    assert_hits_equal_oracle(h, ijk, rk2, rcc)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("M,N,p", [(300, 1000, 0.5), (257, 700, 0.1), (40, 20000, 0.5)])
def test_tables_equal_vector_alu(env, M, N, p, variant):
    """Several workgroup tiles in both directions and long sample loops: every
    table and FP32 score equals the vector-ALU kernel's bit for bit."""
    torch, epi3 = env
    print(f"[case] {variant} M={M} N={N} p={p}", flush=True)
    d = make_dataset(M, N, p, 0.05, seed=M + N)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    cv, kv = epi3.scan_tables(ds, "valu")
    cm, km = epi3.scan_tables(ds, variant)
    assert torch.equal(cv, cm)
    assert torch.equal(kv, km)


@pytest.mark.parametrize("variant", VARIANTS)
def test_cfg1_cfg2_topk(env, variant):
    torch, epi3 = env
    for cfg in (1, 2):
        c = CONFIGS[cfg]
        d = make_config(cfg)
        ds = epi3.encode(to_dev(d.geno), d.pheno)
        sc = epi3.Scanner(ds, c["k"], variant)
        h = sc.run()
        ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, c["k"])
        assert_hits_equal_oracle(h, ijk, k2, cc)
        plane = sc.score_plane().clone()
        ref = epi3.Scanner(ds, c["k"], "valu")
        ref.run()
        assert torch.equal(plane, ref.score_plane())


@pytest.mark.parametrize("variant", VARIANTS)
def test_all_controls_or_all_cases(env, variant):
    torch, epi3 = env
    for p in (0.0, 1.0):
        geno, pheno = _tiny(44, 20, 300, p)
        ds = epi3.encode(to_dev(geno), pheno)
        h = epi3.scan_topk(ds, 9, variant)
        ijk, k2, cc = oracle.scan_topk(geno, pheno, 9)
        assert_hits_equal_oracle(h, ijk, k2, cc)


def test_cfg3_full_size_fp4(env):
    """2048 SNPs x 16384 samples, top-1000 through the FP4 matrix-core kernel
    (many passes through both scratch buffers): hits equal the stored oracle
    result; sampled scores of the plane equal the oracle's within the bound."""
    torch, epi3 = env
    c = CONFIGS[3]
    d = make_config(3)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    sc = epi3.Scanner(ds, c["k"], "mfma_fp4")
    h = sc.run()
    fx = os.path.join(GOLDEN, f"oracle_cfg3_top{c['k']}.npz")
    if os.path.exists(fx):
        z = np.load(fx)
        assert str(z["sha256"]) == manifest_sha256([d.geno, d.pheno])
        assert_hits_equal_oracle(h, z["ijk"], z["k2"], z["counts"])
    else:
        rc, rk = oracle.score_list(d.geno, d.pheno, hits_ijk(h))
        np.testing.assert_array_equal(h["k2"], rk)
        np.testing.assert_array_equal(h["counts"].astype(np.int64), rc)
    plane = sc.score_plane()
    T = epi3.n_triplets(d.n_snps)
    ranks = np.unique((SplitMix64(34, 0).uniform(0, 3000) * T).astype(np.int64))
    lex = lex_unrank(d.n_snps, ranks)
    rc, rk = oracle.score_list(d.geno, d.pheno, lex)
    got = plane[torch.as_tensor(ranks, device=plane.device)].cpu().numpy()
    assert_k2_close(got, rk, d.n_samples, epi3)


def test_class_too_large_for_matrix_cores(env):
    """Class sizes above 65535 are refused by the matrix-core variants."""
    torch, epi3 = env
    geno, pheno = _tiny(5, 3, 66000, 0.0)
    ds = epi3.encode(to_dev(geno), pheno)
    with pytest.raises(epi3.Epi3Error) as e:
        epi3.scan_topk(ds, 1, "mfma")
    assert e.value.code == epi3.E_UNSUPPORTED
    h = epi3.scan_topk(ds, 1, "valu")
    assert len(h) == 1


@pytest.mark.parametrize("variant", ["valu"] + VARIANTS)
def test_large_sample_count(env, variant):
    """50000 samples: the log-factorial table no longer fits in LDS and the
    kernels read it from global memory; tables and hits still match."""
    torch, epi3 = env
    geno, pheno = _tiny(61, 12, 50000, 0.45)
    ds = epi3.encode(to_dev(geno), pheno)
    cc, k2 = epi3.scan_tables(ds, variant)
    ref_k2, ref_cc = oracle.scan_all(geno, pheno)
    np.testing.assert_array_equal(cc.cpu().numpy(), ref_cc)
    assert_k2_close(k2.cpu().numpy(), ref_k2, 50000, epi3)
    h = epi3.scan_topk(ds, 7, variant)
    ijk, rk2, rcc = oracle.scan_topk(geno, pheno, 7)
    assert_hits_equal_oracle(h, ijk, rk2, rcc)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("jb", [2, 4, 8])
def test_tile_shapes_and_small_passes(env, variant, jb):
    """Every tile shape (16 i x JB j x 256/JB k), and scratch passes of 3
    tiles (many passes, both buffers, a ragged last pass): tables and scores
    equal the vector-ALU kernel's; hits equal the oracle's."""
    torch, epi3 = env
    print(f"[case] {variant} JB={jb}", flush=True)
    d = make_dataset(150, 900, 0.4, 0.05, seed=jb)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    cv, kv = epi3.scan_tables(ds, "valu")
    try:
        epi3.tile_rule(variant, 0, 0, jb)
        assert epi3.tile_for(ds, variant) == jb
        cm, km = epi3.scan_tables(ds, variant)
        assert torch.equal(cv, cm) and torch.equal(kv, km)
        epi3.set_pass_bytes(3 * 2 * 16 * 256 * 16)
        cm, km = epi3.scan_tables(ds, variant)
        assert torch.equal(cv, cm) and torch.equal(kv, km)
        h = epi3.scan_topk(ds, 20, variant)
    finally:
        epi3.set_pass_bytes(0)
        epi3.tile_rules_clear()
        epi3.load_tiles()
    ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, 20)
    assert_hits_equal_oracle(h, ijk, k2, cc)
