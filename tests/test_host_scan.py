"""The host-CPU scan (libepi3_host.so, the paper's fourth CPU approach on
this machine's cores) against the oracle: identical hits (indices, FP64 K2,
all 54 counts) at every instruction-set level this CPU has, any thread
count, ragged sample counts and the degenerate phenotypes; argument and data
errors; the library exports what its header declares and the GPU binding
never loads it."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import oracle
from synth import make_dataset

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def host():
    from paper_2201_10956_amd import host as h
    return h


def _levels(host):
    return list(range(0, host.best_isa() + 1))


def _same_as_oracle(h, geno, pheno, k):
    ijk, k2, cc = oracle.scan_topk(geno, pheno, k)
    got = np.stack([h["i"], h["j"], h["k"]], axis=1).astype(np.int32)
    assert got.shape == ijk.shape
    np.testing.assert_array_equal(got, ijk)
    np.testing.assert_array_equal(h["k2"], k2)
    np.testing.assert_array_equal(h["counts"].astype(np.int64), cc)
    np.testing.assert_array_equal(h["k2_f32"], k2.astype(np.float32))


def test_header_symbols_exported(host):
    src = open(os.path.join(ROOT, "include", "epi3_host.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = sorted(set(re.findall(r"\b(epi3h_\w+)\s*\(", src)))
    assert names == ["epi3h_best_isa", "epi3h_scan_topk"]
    lib = ctypes.CDLL(host.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("M,N,k,frac,seed", [
    (9, 70, 5, 0.4, 1),        # one word per class, ragged
    (40, 300, 20, 0.5, 2),
    (33, 1111, 50, 0.3, 3),    # several words, ragged tail, several vectors
    (20, 64, 2000, 0.5, 4),    # k above C(M,3): every triplet, ordered
    (3, 5, 3, 0.4, 5),         # one triplet
    (25, 1030, 7, 0.05, 6),    # few cases
])
def test_matches_oracle_every_isa(host, M, N, k, frac, seed):
    d = make_dataset(M, N, frac, 0.05, seed=seed)
    for isa in _levels(host):
        h = host.scan_topk(d.geno, d.pheno, k, threads=3, isa=isa)
        _same_as_oracle(h, d.geno, d.pheno, k)


def test_thread_counts_give_identical_bytes(host):
    d = make_dataset(60, 700, 0.45, 0.05, seed=7)
    ref = host.scan_topk(d.geno, d.pheno, 40, threads=1)
    for th in (2, 5, 8):
        assert host.scan_topk(d.geno, d.pheno, 40, threads=th).tobytes() == ref.tobytes()


@pytest.mark.parametrize("case", ["all_controls", "all_cases", "one_case"])
def test_degenerate_phenotypes(host, case):
    d = make_dataset(14, 200, 0.5, 0.05, seed=8)
    ph = np.zeros(200, dtype=np.uint8)
    if case == "all_cases":
        ph[:] = 1
    elif case == "one_case":
        ph[123] = 1
    for isa in _levels(host):
        _same_as_oracle(host.scan_topk(d.geno, ph, 9, isa=isa), d.geno, ph, 9)


def test_constant_snps_and_ties(host):
    """Identical and constant SNPs give equal K2 values: the order falls back
    to (i, j, k) exactly as in the oracle."""
    d = make_dataset(12, 150, 0.5, 0.05, seed=9)
    g = d.geno.copy()
    g[3] = g[7]
    g[5] = 2
    g[6] = 0
    _same_as_oracle(host.scan_topk(g, d.pheno, 220), g, d.pheno, 220)


def test_fewer_than_three_snps(host):
    d = make_dataset(2, 50, 0.5, 0.05, seed=10)
    assert len(host.scan_topk(d.geno, d.pheno, 5)) == 0


def test_errors(host):
    d = make_dataset(6, 40, 0.5, 0.05, seed=11)
    g = d.geno.copy()
    g[2, 17] = 3
    with pytest.raises(host.HostError) as e:
        host.scan_topk(g, d.pheno, 3)
    assert e.value.code == -2
    p = d.pheno.copy()
    p[5] = 2
    with pytest.raises(host.HostError) as e:
        host.scan_topk(d.geno, p, 3)
    assert e.value.code == -3
    with pytest.raises(host.HostError) as e:
        host.scan_topk(d.geno, d.pheno, 0)
    assert e.value.code == -1
    with pytest.raises(host.HostError) as e:
        host.scan_topk(d.geno, d.pheno, 3, isa=7)
    assert e.value.code == -1
    if host.best_isa() < host.ISA_AVX512:
        with pytest.raises(host.HostError) as e:
            host.scan_topk(d.geno, d.pheno, 3, isa=host.ISA_AVX512)
        assert e.value.code == -7


def test_gpu_binding_never_loads_the_host_library():
    """The GPU path has no CPU fallback: importing the GPU binding leaves the
    host library unloaded (checked in a fresh interpreter)."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2201_10956_amd import epi3\n"
            "maps = open('/proc/self/maps').read()\n"
            "assert 'libepi3_host' not in maps, 'host library mapped'\n"
            "assert 'paper_2201_10956_amd.host' not in sys.modules\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
