"""Permutation significance end to end: the observed phenotype runs as a job of
the same MASKED batch as its permutations, the p-value comes from hit 0 of
every job, and it must equal the p-value computed from the oracle's lowest
K2 of each phenotype."""
import os

import numpy as np
import pytest

import oracle
from synth import CONFIGS, make_config, make_dataset, make_parity_fixture, make_permutations
from tests.gpu_util import assert_hits_equal_oracle, require_gpu, to_dev

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _p_from_minima(obs, perm_min):
    """p = (1 + #{q : min_q <= observed}) / (P + 1), written out here."""
    return (1 + sum(1 for m in perm_min if m <= obs)) / (len(perm_min) + 1)


def _batch(epi3, d, phenos, k, variant="mfma_fp4"):
    import torch
    ds = epi3.encode(to_dev(d.geno), d.pheno, layout="masked")
    masks = torch.from_numpy(epi3.pack_masks(phenos).view(np.int32)).to("cuda")
    return epi3.BatchScanner(ds, k, masks=masks, variant=variant).run()


@pytest.mark.parametrize("variant", ["mfma", "mfma_fp4"])
def test_pvalue_matches_oracle_minima(env, variant):
    torch, epi3 = env
    d = make_dataset(60, 800, 0.4, 0.05, seed=91)
    perms = make_permutations(d.pheno, 20, seed=92)
    phenos = np.concatenate([d.pheno[None], perms])          # job 0 = observed
    res = _batch(epi3, d, phenos, 3, variant)
    mins = []
    for q in range(len(phenos)):
        ijk, k2, cc = oracle.scan_topk(d.geno, phenos[q], 3)
        assert_hits_equal_oracle(res[q], ijk, k2, cc)
        mins.append(float(k2[0]))
    p = epi3.perm_pvalue(res[0]["k2"][0], [r["k2"][0] for r in res[1:]])
    assert p == _p_from_minima(mins[0], mins[1:])


def test_pvalue_tie_counts_and_all_greater(env):
    """A permutation equal to the observed phenotype ties its minimum and
    counts; with a strong planted triplet every permutation's minimum is
    higher and p = 1 / (P + 1)."""
    torch, epi3 = env
    d = make_parity_fixture(95, M=40, N=2000)
    perms = make_permutations(d.pheno, 9, seed=94)
    phenos = np.concatenate([d.pheno[None], perms, d.pheno[None]])  # last = identity
    res = _batch(epi3, d, phenos, 1)
    mins = [float(oracle.scan_topk(d.geno, ph, 1)[1][0]) for ph in phenos]
    got = [float(r["k2"][0]) for r in res]
    assert got == mins
    assert got[-1] == got[0]                                   # the tie
    p = epi3.perm_pvalue(got[0], got[1:])
    assert p == _p_from_minima(mins[0], mins[1:])
    # the oracle's minima put every real permutation strictly above the observed one
    assert all(m > mins[0] for m in mins[1:-1])
    assert p == 2 / 11                                         # 1 + the identity's tie
    p9 = epi3.perm_pvalue(got[0], got[1:-1])
    assert p9 == _p_from_minima(mins[0], mins[1:-1]) == 1 / 10


def test_cfg4_pvalue_full_size(env):
    """1024 SNPs x 8192 samples: the observed phenotype plus its 64
    permutations in one MASKED batch; p equals the one from the stored oracle
    minima."""
    torch, epi3 = env
    print("[case] cfg4 p-value, 65 jobs", flush=True)
    c = CONFIGS[4]
    d, perms = make_config(4)
    phenos = np.concatenate([d.pheno[None], perms])
    res = _batch(epi3, d, phenos, c["k"])
    z = np.load(os.path.join(GOLDEN, f"oracle_cfg4_observed_top{c['k']}.npz"))
    assert_hits_equal_oracle(res[0], z["ijk"], z["k2"], z["counts"])
    mins = [float(z["k2"][0])]
    for q in range(c["n_perm"]):
        zq = np.load(os.path.join(GOLDEN, f"oracle_cfg4_perm{q:02d}_top{c['k']}.npz"))
        assert_hits_equal_oracle(res[q + 1], zq["ijk"], zq["k2"], zq["counts"])
        mins.append(float(zq["k2"][0]))
    p = epi3.perm_pvalue(res[0]["k2"][0], [r["k2"][0] for r in res[1:]])
    assert p == _p_from_minima(mins[0], mins[1:])
    print(f"[p] cfg4 observed min K2 {mins[0]:.6f}, p = {p:.6f}")
