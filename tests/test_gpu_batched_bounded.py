"""Phenotype batches selected by bound (no score plane): a sample pass over
every stride-th tile bounds each job's k-th FP32 score, the full pass lists
only the scores under that bound.  The list must hold exactly the scores of
the plane at or below its bound, the bound must cover the k-th smallest
score plus 2 e(N), and the hits must equal both the plane-selected batch's
and the oracle's."""
import contextlib

import numpy as np
import pytest

import oracle
from synth import CONFIGS, make_config, make_dataset, make_permutations
from tests.gpu_util import assert_hits_equal_oracle, require_gpu, to_dev

pytestmark = pytest.mark.gpu
TILE_SCRATCH = 64 * 64 * 16 + 64 * 16


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _masks(epi3, perms):
    import torch
    return torch.from_numpy(epi3.pack_masks(perms).view(np.int32)).to("cuda")


@contextlib.contextmanager
def _settings(epi3, mode, pass_tiles=0):
    """Process-wide settings for a batch and every later look into its
    workspace (the hooks lay the workspace out under the current settings)."""
    try:
        epi3.set_batch_select(mode)
        epi3.set_pass_bytes(pass_tiles * TILE_SCRATCH)
        yield
    finally:
        epi3.set_batch_select("auto")
        epi3.set_pass_bytes(0)


def _run(epi3, ds, k, masks, variant, mode, pass_tiles=0):
    with _settings(epi3, mode, pass_tiles):
        bs = epi3.BatchScanner(ds, k, masks=masks, variant=variant)
        return bs, bs.run()


@pytest.mark.parametrize("variant", ["mfma", "mfma_fp4"])
@pytest.mark.parametrize("M,N,Q,k,pass_tiles", [
    (130, 3000, 70, 5, 5),    # two groups, sample and full passes cut into many passes
    (300, 1200, 16, 25, 0),   # a sample of one tile in five
    (40, 500, 3, 1, 0),
])
def test_bounded_list_equals_plane(env, M, N, Q, k, pass_tiles, variant):
    torch, epi3 = env
    print(f"[case] bounded {variant} M={M} N={N} Q={Q} k={k}", flush=True)
    d = make_dataset(M, N, 0.4, 0.05, seed=900 + M)
    perms = make_permutations(d.pheno, Q, seed=901 + N)
    ds = epi3.encode(to_dev(d.geno), d.pheno, layout="masked")
    m = _masks(epi3, perms)
    with _settings(epi3, "plane", pass_tiles):
        bp = epi3.BatchScanner(ds, k, masks=m, variant=variant)
        res_p = bp.run()
        planes = [bp.score_plane(q).cpu().numpy() for q in range(Q)]
        with pytest.raises(epi3.Epi3Error) as e:
            bp.bound_list(0)  # a plane batch keeps no list
        assert e.value.code == epi3.E_UNSUPPORTED
    with _settings(epi3, "bounded", pass_tiles):
        bb = epi3.BatchScanner(ds, k, masks=m, variant=variant)
        res_b = bb.run()
        lists = [bb.bound_list(q) for q in range(Q)]
        with pytest.raises(epi3.Epi3Error) as e:
            bb.score_plane(0)
        assert e.value.code == epi3.E_UNSUPPORTED
    e2 = 2 * epi3.k2_error_bound(N)
    for q in range(Q):
        assert res_b[q].tobytes() == res_p[q].tobytes(), q
        ijk, k2, cc = oracle.scan_topk(d.geno, perms[q], k)
        assert_hits_equal_oracle(res_b[q], ijk, k2, cc)
        scores, ranks, bound = lists[q]
        want = np.flatnonzero(planes[q] <= bound)
        assert np.array_equal(np.sort(ranks), want), q
        np.testing.assert_array_equal(scores, planes[q][ranks])
        kth = np.partition(planes[q], k - 1)[k - 1]
        assert float(bound) >= float(kth) + e2


def test_bounded_list_overflow_is_a_capacity_error(env):
    torch, epi3 = env
    d = make_dataset(60, 700, 0.5, 0.05, seed=95)
    perms = make_permutations(d.pheno, 4, seed=96)
    ds = epi3.encode(to_dev(d.geno), d.pheno, layout="masked")
    m = _masks(epi3, perms)
    try:
        epi3.set_compact_cap(2)            # lists of 2 entries cannot hold 3 hits
        with pytest.raises(epi3.Epi3Error) as e:
            _run(epi3, ds, 3, m, "mfma_fp4", "bounded")
        assert e.value.code == epi3.E_CAPACITY
    finally:
        epi3.set_compact_cap(0)
    _, res = _run(epi3, ds, 3, m, "mfma_fp4", "bounded")
    for q in range(4):
        assert_hits_equal_oracle(res[q], *oracle.scan_topk(d.geno, perms[q], 3))


def test_bounded_more_hits_than_triplets(env):
    """k above C(M,3): the sample cannot hold k scores, the batch falls back
    to a plane and returns every triplet."""
    torch, epi3 = env
    d = make_dataset(6, 300, 0.5, 0.05, seed=97)
    perms = make_permutations(d.pheno, 2, seed=98)
    ds = epi3.encode(to_dev(d.geno), d.pheno, layout="masked")
    _, res = _run(epi3, ds, 30, _masks(epi3, perms), "mfma_fp4", "bounded")
    for q in range(2):
        assert len(res[q]) == 20
        assert_hits_equal_oracle(res[q], *oracle.scan_topk(d.geno, perms[q], 30))


@pytest.mark.parametrize("N", [11400, 11600])
def test_bounded_on_both_sides_of_the_one_kernel_limit(env, N):
    """FP4 batches selected by bound count and score in one kernel while the
    log-factorial table fits beside the staging in LDS (up to about 11500
    samples) and in two kernels above: both give the oracle's hits."""
    torch, epi3 = env
    print(f"[case] bounded fp4 N={N}", flush=True)
    d = make_dataset(40, N, 0.45, 0.05, seed=N)
    perms = make_permutations(d.pheno, 3, seed=N + 1)
    ds = epi3.encode(to_dev(d.geno), d.pheno, layout="masked")
    _, res = _run(epi3, ds, 4, _masks(epi3, perms), "mfma_fp4", "bounded")
    for q in range(3):
        assert_hits_equal_oracle(res[q], *oracle.scan_topk(d.geno, perms[q], 4))
