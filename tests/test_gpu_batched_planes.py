"""Element-wise parity of the phenotype-batch count and table-completion
kernels: every FP32 score they write equals the vector-ALU plain scan's score
of the same phenotype bit for bit (the same row order and bracketing of
Eq. 1 from the same FP32 table) and the oracle's FP64 K2 within the error
bound e(N) and 1e-4 relative; plus full-size int8 runs and concurrent calls
on two streams."""
import os
import threading

import numpy as np
import pytest

import oracle
from synth import CONFIGS, SplitMix64, make_config, make_dataset, make_permutations
from tests.gpu_util import (assert_hits_equal_oracle, assert_k2_close, hits_ijk, lex_unrank,
                            require_gpu, to_dev)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TILE_SCRATCH = 64 * 64 * 16 + 64 * 16  # bytes of one phenotype-batch tile in a pass buffer


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _masks(epi3, perms):
    import torch
    return torch.from_numpy(epi3.pack_masks(perms).view(np.int32)).to("cuda")


def _valu_plane(epi3, g, pheno):
    sc = epi3.Scanner(epi3.encode(g, pheno), 1, "valu")
    sc.scan()
    return sc.score_plane().clone()


@pytest.mark.parametrize("variant", ["mfma", "mfma_fp4"])
@pytest.mark.parametrize("M,N,Q,pass_tiles", [
    (130, 3000, 64, 7),    # many passes, both scratch buffers, pivots cut by pass ends
    (67, 1500, 20, 0),     # M one past a multiple of 16 and of 64; Q < 64
    (45, 700, 70, 0),      # two groups of phenotypes (64 + 6)
    (19, 257, 1, 0),       # one phenotype, one ragged sample chunk
])
def test_perm_score_block_every_score(env, M, N, Q, pass_tiles, variant):
    torch, epi3 = env
    print(f"[case] score block {variant} M={M} N={N} Q={Q} pass_tiles={pass_tiles}", flush=True)
    d = make_dataset(M, N, 0.4, 0.05, seed=700 + M)
    perms = make_permutations(d.pheno, Q, seed=800 + N)
    g = to_dev(d.geno)
    ds = epi3.encode(g, d.pheno, layout="masked")
    try:
        epi3.set_pass_bytes(pass_tiles * TILE_SCRATCH)
        epi3.set_batch_select("plane")
        bs = epi3.BatchScanner(ds, 5, masks=_masks(epi3, perms), variant=variant)
        res = bs.run()
        planes = [bs.score_plane(q).clone() for q in range(Q)]
    finally:
        epi3.set_pass_bytes(0)
        epi3.set_batch_select("auto")
    worst = 0.0
    for q in range(Q):
        ref = _valu_plane(epi3, g, perms[q])
        assert torch.equal(planes[q], ref), q
        k2_64, _ = oracle.scan_all(d.geno, perms[q], counts=False)
        diff, _ = assert_k2_close(planes[q].cpu().numpy(), k2_64, N, epi3)
        worst = max(worst, diff)
        ijk, k2, cc = oracle.scan_topk(d.geno, perms[q], 5)
        assert_hits_equal_oracle(res[q], ijk, k2, cc)
    print(f"[fp32] max |K2_32 - K2_64| = {worst:.3e}, bound {epi3.k2_error_bound(N):.3e}")


@pytest.mark.parametrize("variant", ["mfma_fp4", "mfma"])
def test_cfg4_score_block_full_size(env, variant):
    """1024 SNPs x 8192 samples x 64 phenotypes with the score plane kept
    (the default for this size selects by bound and keeps none):
    every phenotype's whole FP32 plane equals its vector-ALU plain scan's bit
    for bit, 10^4 sampled ranks per phenotype equal the oracle's FP64 K2
    within e(N), and each top-10 equals the stored oracle result."""
    torch, epi3 = env
    print(f"[case] cfg4 score block {variant}", flush=True)
    c = CONFIGS[4]
    d, perms = make_config(4)
    g = to_dev(d.geno)
    ds = epi3.encode(g, d.pheno, layout="masked")
    try:
        epi3.set_batch_select("plane")  # kept while the planes are read
        bs = epi3.BatchScanner(ds, c["k"], masks=_masks(epi3, perms), variant=variant)
        res = bs.run()
        planes = [bs.score_plane(q) for q in range(c["n_perm"])]
    finally:
        epi3.set_batch_select("auto")
    T = epi3.n_triplets(d.n_snps)
    worst_abs = worst_rel = 0.0
    for q in range(c["n_perm"]):
        plane = planes[q]
        assert torch.equal(plane, _valu_plane(epi3, g, perms[q])), q
        ranks = np.unique((SplitMix64(4000 + q, 0).uniform(0, 10000) * T).astype(np.int64))
        _, rk = oracle.score_list(d.geno, perms[q], lex_unrank(d.n_snps, ranks))
        got = plane[torch.as_tensor(ranks, device=plane.device)].cpu().numpy()
        a, r = assert_k2_close(got, rk, d.n_samples, epi3)
        worst_abs, worst_rel = max(worst_abs, a), max(worst_rel, r)
        fx = os.path.join(GOLDEN, f"oracle_cfg4_perm{q:02d}_top{c['k']}.npz")
        z = np.load(fx)
        assert_hits_equal_oracle(res[q], z["ijk"], z["k2"], z["counts"])
    print(f"[fp32] cfg4 sampled max abs {worst_abs:.3e} rel {worst_rel:.3e}, "
          f"bound {epi3.k2_error_bound(d.n_samples):.3e}")


def test_cfg3_full_size_int8(env):
    """2048 SNPs x 16384 samples, top-1000 through the int8 matrix-core kernel:
    hits equal the stored oracle result and the plane equals the FP4 kernel's."""
    torch, epi3 = env
    print("[case] cfg3 int8", flush=True)
    c = CONFIGS[3]
    d = make_config(3)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    sc = epi3.Scanner(ds, c["k"], "mfma")
    h = sc.run()
    z = np.load(os.path.join(GOLDEN, f"oracle_cfg3_top{c['k']}.npz"))
    assert_hits_equal_oracle(h, z["ijk"], z["k2"], z["counts"])
    plane = sc.score_plane().clone()
    sf = epi3.Scanner(ds, c["k"], "mfma_fp4")
    sf.scan()
    assert torch.equal(plane, sf.score_plane())


def test_concurrent_calls_two_streams(env):
    """A matrix-core plain scan and a phenotype batch issued from two host
    threads on two streams at once, many passes each (small pass buffers),
    repeated: every result equals the oracle's."""
    torch, epi3 = env
    print("[case] concurrent plain + batch", flush=True)
    d1 = make_dataset(150, 2000, 0.5, 0.05, seed=71)
    d2 = make_dataset(90, 1500, 0.4, 0.05, seed=72)
    perms = make_permutations(d2.pheno, 16, seed=73)
    want1 = oracle.scan_topk(d1.geno, d1.pheno, 12)
    want2 = [oracle.scan_topk(d2.geno, perms[q], 6) for q in range(16)]
    ds1 = epi3.encode(to_dev(d1.geno), d1.pheno)
    ds2 = epi3.encode(to_dev(d2.geno), d2.pheno, layout="masked")
    masks = _masks(epi3, perms)
    try:
        epi3.set_pass_bytes(5 * TILE_SCRATCH)  # many passes on both paths
        sc = epi3.Scanner(ds1, 12, "mfma_fp4")
        bs = epi3.BatchScanner(ds2, 6, masks=masks, variant="mfma_fp4")
        torch.cuda.synchronize()
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        out1, out2, errs = [], [], []

        def plain():
            try:
                for _ in range(4):
                    out1.append(sc.run(stream=s1))
            except Exception as e:  # surfaced below
                errs.append(e)

        def batch():
            try:
                for _ in range(4):
                    out2.append(bs.run(stream=s2))
            except Exception as e:
                errs.append(e)

        ta, tb = threading.Thread(target=plain), threading.Thread(target=batch)
        ta.start()
        tb.start()
        ta.join()
        tb.join()
        torch.cuda.synchronize()
    finally:
        epi3.set_pass_bytes(0)
    assert not errs, errs
    assert len(out1) == 4 and len(out2) == 4
    for h in out1:
        assert_hits_equal_oracle(h, *want1)
    for res in out2:
        for q in range(16):
            assert_hits_equal_oracle(res[q], *want2[q])
