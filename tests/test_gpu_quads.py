"""GPU parity of the fourth-order (quad) scan against the oracle's quad scan:
every quad's FP32 score within the 81-row error bound, and hits (quad, FP64
K2 bit for bit, both 81-row tables) equal to the oracle's top-k.  Each case
runs on a data set with FP4 value planes (counts on the matrix cores) and on
one encoded without them (counts by popcount)."""
import numpy as np
import pytest

import oracle
from synth import SplitMix64, make_dataset
from tests.gpu_util import require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _tiny(seed, M, N, p_case):
    u = SplitMix64(seed, 29).uniform(0, M * N + N)
    geno = np.minimum((u[: M * N] * 3).astype(np.uint8), 2).reshape(M, N)
    pheno = (u[M * N:] < p_case).astype(np.uint8)
    return geno, pheno


def _quad_unrank(M, r):
    """The quad of lexicographic rank r among all i < j < k < l < M: walk the
    first index up while whole blocks of quads fit below r, then the next."""
    from math import comb
    out, lo = [], 0
    for left in (4, 3, 2, 1):
        x = lo
        while comb(M - 1 - x, left - 1) <= r:
            r -= comb(M - 1 - x, left - 1)
            x += 1
        out.append(x)
        lo = x + 1
    return tuple(out)


def assert_quad_hits_equal_oracle(h, q, k2, counts):
    assert len(h) == len(q), (len(h), len(q))
    got = np.stack([h["i"], h["j"], h["k"], h["l"]], axis=1).astype(np.int32)
    np.testing.assert_array_equal(got, q)
    np.testing.assert_array_equal(h["k2"], k2)
    np.testing.assert_array_equal(h["counts"].astype(np.int64), counts.astype(np.int64))


def assert_quad_k2_close(got32, ref64, N, epi3):
    diff = np.abs(np.asarray(got32, dtype=np.float64) - ref64)
    e = epi3.k2_error_bound_quads(N)
    assert np.all(diff <= e), (diff.max(), e)
    assert np.all(diff / np.maximum(np.abs(ref64), 1e-30) <= 1e-4)


VALUES = [pytest.param(True, id="mfma"), pytest.param(False, id="popcount")]


@pytest.mark.parametrize("values", VALUES)
@pytest.mark.parametrize("M,N,p", [(4, 1, 0.5), (4, 64, 0.0), (5, 33, 1.0), (7, 31, 0.3),
                                   (12, 95, 0.5), (20, 129, 0.45), (40, 300, 0.2),
                                   (33, 2000, 0.5), (70, 333, 0.4)])
def test_every_quad_score_and_topk(env, M, N, p, values):
    torch, epi3 = env
    print(f"[case] quads M={M} N={N} p={p} values={values}", flush=True)
    geno, pheno = _tiny(100 * M + N, M, N, p)
    ds = epi3.encode(to_dev(geno), pheno, values=values)
    k = min(30, M * (M - 1) * (M - 2) * (M - 3) // 24)
    sc = epi3.QuadScanner(ds, k)
    h = sc.run()
    ref_k2, _ = oracle.scan_quads_all(geno, pheno, counts=False)
    assert_quad_k2_close(sc.score_plane().cpu().numpy(), ref_k2, N, epi3)
    q, rk2, rcc = oracle.scan_quads_topk(geno, pheno, k)
    assert_quad_hits_equal_oracle(h, q, rk2, rcc)


@pytest.mark.parametrize("values", VALUES)
def test_quads_128_snps(env, values):
    """128 SNPs x 4096 samples (10.7 M quads), top-100 equal to the oracle's;
    sampled FP32 scores within the bound."""
    torch, epi3 = env
    print(f"[case] quads 128 x 4096 values={values}", flush=True)
    d = make_dataset(128, 4096, 0.5, 0.05, seed=44)
    ds = epi3.encode(to_dev(d.geno), d.pheno, values=values)
    sc = epi3.QuadScanner(ds, 100)
    h = sc.run()
    q, rk2, rcc = oracle.scan_quads_topk(d.geno, d.pheno, 100)
    assert_quad_hits_equal_oracle(h, q, rk2, rcc)
    Q = epi3.n_quads(128)
    ranks = np.unique((SplitMix64(78, 0).uniform(0, 300) * Q).astype(np.int64))
    lex = oracle.lex_quads(128)[ranks]
    L = oracle.log_factorial(d.n_samples + 1)
    ref = np.array([oracle.k2_rows(oracle.quad_table(d.geno, d.pheno, *map(int, x)), L) for x in lex])
    got = sc.score_plane()[torch.as_tensor(ranks, device="cuda")].cpu().numpy()
    assert_quad_k2_close(got, ref, d.n_samples, epi3)


@pytest.mark.parametrize("values", VALUES)
def test_quads_large_sample_count(env, values):
    """50000 samples: the log-factorial table is read from global memory."""
    torch, epi3 = env
    geno, pheno = _tiny(71, 9, 50000, 0.45)
    ds = epi3.encode(to_dev(geno), pheno, values=values)
    sc = epi3.QuadScanner(ds, 12)
    h = sc.run()
    ref_k2, _ = oracle.scan_quads_all(geno, pheno, counts=False)
    assert_quad_k2_close(sc.score_plane().cpu().numpy(), ref_k2, 50000, epi3)
    q, rk2, rcc = oracle.scan_quads_topk(geno, pheno, 12)
    assert_quad_hits_equal_oracle(h, q, rk2, rcc)


@pytest.mark.parametrize("values", VALUES)
def test_quads_edge_cases(env, values):
    torch, epi3 = env
    base, _ = _tiny(3, 1, 150, 0.5)
    geno = np.repeat(base, 6, axis=0)           # identical rows: ties broken by index
    for ph in (np.zeros(150, np.uint8), np.ones(150, np.uint8)):  # one class empty
        ds = epi3.encode(to_dev(geno), ph, values=values)
        h = epi3.scan_quads(ds, 40)
        q, rk2, rcc = oracle.scan_quads_topk(geno, ph, 40)
        assert len(h) == 15
        assert_quad_hits_equal_oracle(h, q, rk2, rcc)
    ds = epi3.encode(to_dev(geno[:3]), np.zeros(150, np.uint8))
    assert len(epi3.scan_quads(ds, 5)) == 0
    ds = epi3.encode(to_dev(geno), np.zeros(150, np.uint8), layout="masked")
    with pytest.raises(epi3.Epi3Error) as e:
        epi3.scan_quads(ds, 3)
    assert e.value.code == epi3.E_UNSUPPORTED


@pytest.mark.parametrize("values", VALUES)
def test_quads_candidate_capacity_retry(env, values):
    torch, epi3 = env
    d = make_dataset(30, 2000, 0.5, 0.05, seed=45)
    ds = epi3.encode(to_dev(d.geno), d.pheno, values=values)
    sc = epi3.QuadScanner(ds, 20, cand_cap=5)
    sc.scan()
    rc, need = sc.topk()
    assert rc == epi3.E_CAPACITY and need >= 20
    h = epi3.QuadScanner(ds, 20, cand_cap=need).run()
    q, rk2, rcc = oracle.scan_quads_topk(d.geno, d.pheno, 20)
    assert_quad_hits_equal_oracle(h, q, rk2, rcc)


@pytest.mark.parametrize("values", VALUES)
def test_quads_256_snps_bench_workload(env, values):
    """The benchmark's fourth-order workload, the first 256 SNPs of the
    512 x 4096 data set (174 M quads): top-100 equal to the stored oracle
    result, 2000 sampled FP32 scores within the bound."""
    import os
    from synth import CONFIGS, make_config, manifest_sha256
    torch, epi3 = env
    print(f"[case] quads 256 x 4096 values={values}", flush=True)
    d = make_config(2)
    g = np.ascontiguousarray(d.geno[:256])
    ds = epi3.encode(to_dev(g), d.pheno, values=values)
    sc = epi3.QuadScanner(ds, 100)
    h = sc.run()
    z = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                             "oracle_cfg2_quads256_top100.npz"))
    assert str(z["sha256"]) == manifest_sha256([g, d.pheno])
    assert_quad_hits_equal_oracle(h, z["ijkl"], z["k2"], z["counts"])
    Q = epi3.n_quads(256)
    ranks = np.unique((SplitMix64(79, 0).uniform(0, 2000) * Q).astype(np.int64))
    lex = [_quad_unrank(256, int(r)) for r in ranks]
    L = oracle.log_factorial(d.n_samples + 1)
    ref = np.array([oracle.k2_rows(oracle.quad_table(g, d.pheno, *map(int, x)), L) for x in lex])
    got = sc.score_plane()[torch.as_tensor(ranks, device="cuda")].cpu().numpy()
    assert_quad_k2_close(got, ref, d.n_samples, epi3)


@pytest.mark.parametrize("M,N,p,pass_tiles", [(70, 700, 0.45, 3), (97, 513, 0.3, 0), (131, 260, 0.6, 7)])
def test_matrix_core_quads_equal_popcount_quads(env, M, N, p, pass_tiles):
    """Every FP32 score of the matrix-core quad scan equals the popcount quad
    scan's bit for bit (same cells, same expression and row order), over M
    not a multiple of the 16 x 32 tile blocks, ragged class sizes and many
    scratch passes; hits equal the oracle's."""
    torch, epi3 = env
    print(f"[case] quads mfma vs popcount M={M} N={N} pass_tiles={pass_tiles}", flush=True)
    geno, pheno = _tiny(7 * M + N, M, N, p)
    dv = epi3.encode(to_dev(geno), pheno, values=True)
    db = epi3.encode(to_dev(geno), pheno, values=False)
    try:
        if pass_tiles:
            epi3.set_pass_bytes(pass_tiles * 128 * 1024)
        sv = epi3.QuadScanner(dv, 25)
        hv = sv.run()
    finally:
        epi3.set_pass_bytes(0)
    sb = epi3.QuadScanner(db, 25)
    hb = sb.run()
    assert torch.equal(sv.score_plane(), sb.score_plane())
    q, rk2, rcc = oracle.scan_quads_topk(geno, pheno, 25)
    assert_quad_hits_equal_oracle(hv, q, rk2, rcc)
    assert_quad_hits_equal_oracle(hb, q, rk2, rcc)
