"""The allocation-free plain scan (epi3_scan_topk_static) against the plain
scan with a caller workspace (epi3_scan + epi3_topk, vector-ALU variant) and
against the oracle: two calls in a row, the second on a smaller data set, so
the second call runs over what the first left in the static workspace."""
import numpy as np
import pytest

import oracle
from synth import make_dataset
from tests.gpu_util import assert_hits_equal_oracle, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _same_hits(a, b):
    assert len(a) == len(b)
    for f in ("i", "j", "k", "k2_f32", "k2", "counts"):
        np.testing.assert_array_equal(a[f], b[f], err_msg=f)


def _check(epi3, M, N, frac, k, seed):
    print(f"static scan: M={M} N={N} k={k} seed={seed}", flush=True)
    d = make_dataset(M, N, frac, 0.05, seed=seed)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    got = epi3.scan_topk_static(ds, k)
    ref = epi3.scan_topk(ds, k, "valu")
    _same_hits(got, ref)
    ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, k)
    assert_hits_equal_oracle(got, ijk, k2, cc)
    return got


def test_static_scan_two_calls_second_smaller(env):
    torch, epi3 = env
    # 230 SNPs (1.99 M triplets, 7.9 MB plane; 2 x 12 workgroup tiles of
    # pivots, ragged last tile), then a smaller data set over the same array
    _check(epi3, 230, 3000, 0.5, 40, seed=5101)
    _check(epi3, 70, 900, 0.4, 15, seed=5102)


def test_static_scan_limits(env):
    torch, epi3 = env
    # more hits asked than triplets exist: all C(5,3) = 10, in order
    d = make_dataset(5, 300, 0.5, 0.05, seed=5103)
    ds = epi3.encode(to_dev(d.geno), d.pheno)
    got = epi3.scan_topk_static(ds, 20)
    ijk, k2, cc = oracle.scan_topk(d.geno, d.pheno, 20)
    assert len(got) == 10
    assert_hits_equal_oracle(got, ijk, k2, cc)
    # a data set whose workspace exceeds the static array is refused before
    # anything is enqueued, and the next call still works
    big = make_dataset(700, 256, 0.5, 0.05, seed=5104)
    dsb = epi3.encode(to_dev(big.geno), big.pheno, values=False)
    assert epi3.n_triplets(700) * 4 > epi3.STATIC_SCRATCH_BYTES
    with pytest.raises(epi3.Epi3Error) as e:
        epi3.scan_topk_static(dsb, 10)
    assert e.value.code == epi3.E_WORKSPACE
    _check(epi3, 40, 500, 0.5, 8, seed=5105)
