"""Pins of the CPU oracle against things other than itself.

* brute force: an independent pure-Python tally and exact integer K2
  (ln of Q = prod (r+1) * C(r, r_1)) on tiny inputs;
* invariants: per-class table sums, consistency with independently tallied
  pairwise tables, equivariance under reordering the SNPs;
* closed forms: single-cell data, single-class data, pure rows;
* a library routine: log factorials against math.lgamma;
* a planted signal that must come out on top.
"""
import itertools
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from oracle import brute
from synth import SplitMix64, make_dataset, make_parity_fixture


def tiny(seed, M, N, p_case=0.5):
    u = SplitMix64(seed, 11).uniform(0, M * N + N)
    geno = np.minimum((u[: M * N] * 3).astype(np.uint8), 2).reshape(M, N)
    pheno = (u[M * N:] < p_case).astype(np.uint8)
    return geno, pheno


def _tables_and_k2_vs_brute(lib, seeds=range(40)):
    """Every table of every triplet equals the brute-force tally, K2 equals ln Q."""
    for seed in seeds:
        M = 3 + seed % 6
        N = 1 + (seed * 7) % 48
        geno, pheno = tiny(seed, M, N, p_case=(seed % 5) / 4.0)
        k2, cc = oracle.scan_all(geno, pheno, lib=lib, nthreads=2)
        for x, snps in enumerate(itertools.combinations(range(M), 3)):
            t = brute.table(geno.tolist(), pheno.tolist(), snps)
            assert cc[x].tolist() == t, (seed, snps)
            want = brute.k2_exact(t)
            assert abs(k2[x] - want) <= 1e-12 * max(1.0, abs(want)), (seed, snps, k2[x], want)


def test_tables_and_k2_match_bruteforce():
    _tables_and_k2_vs_brute(oracle.load())


def test_score_list_and_table_agree_with_scan_all():
    geno, pheno = tiny(99, 9, 40)
    k2, cc = oracle.scan_all(geno, pheno)
    ijk = oracle.lex_triplets(9)
    cc2, k22 = oracle.score_list(geno, pheno, ijk)
    assert np.array_equal(cc, cc2)
    assert np.array_equal(k2, k22)
    assert np.array_equal(oracle.table(geno, pheno, *ijk[17]), cc[17])


def test_table_invariants_against_pairwise_tallies():
    d = make_dataset(12, 1000, 0.37, 0.05, seed=5)
    G, ph = d.geno, d.pheno
    n1 = int(ph.sum())
    n0 = ph.size - n1
    k2, cc = oracle.scan_all(G, ph)
    ijk = oracle.lex_triplets(12)

    def pair(x, y):
        out = np.zeros((2, 3, 3), dtype=np.int64)
        for s in range(ph.size):  # plain tally, independent of the oracle's row index
            out[ph[s], G[x, s], G[y, s]] += 1
        return out

    pairs = {xy: pair(*xy) for xy in itertools.combinations(range(12), 2)}
    for x, (i, j, k) in enumerate(ijk):
        t = cc[x].reshape(2, 3, 3, 3)
        assert t[0].sum() == n0 and t[1].sum() == n1
        assert np.array_equal(t.sum(axis=3), pairs[(i, j)])
        assert np.array_equal(t.sum(axis=2), pairs[(i, k)])
        assert np.array_equal(t.sum(axis=1), pairs[(j, k)])


def test_equivariance_under_snp_reordering():
    d = make_dataset(10, 300, 0.5, 0.05, seed=8)
    perm = np.array([7, 2, 9, 0, 4, 1, 8, 3, 6, 5])
    G2 = d.geno[perm]
    inv = np.argsort(perm)
    for (i, j, k) in [(0, 1, 2), (1, 5, 8), (3, 4, 9), (0, 6, 7)]:
        t = oracle.table(d.geno, d.pheno, i, j, k).reshape(2, 3, 3, 3)
        pos = sorted([(inv[i], 'i'), (inv[j], 'j'), (inv[k], 'k')])
        t2 = oracle.table(G2, d.pheno, *[p for p, _ in pos]).reshape(2, 3, 3, 3)
        back = np.transpose(t2, [0] + [1 + [n for _, n in pos].index(a) for a in 'ijk'])
        assert np.array_equal(back, t)
        L = oracle.log_factorial(301)
        a = oracle.k2(t, L)
        b = oracle.k2(t2, L)
        assert abs(a - b) <= 1e-12 * a


def test_log_factorial_against_lgamma():
    L = oracle.log_factorial(70000)
    n = np.arange(L.size)
    ref = np.array([math.lgamma(v + 1.0) for v in n])
    assert L[0] == 0.0 and L[1] == 0.0
    assert np.all(np.abs(L - ref) <= 1e-11 * np.maximum(ref, 1.0))


@pytest.mark.parametrize("N,n1", [(1, 0), (1, 1), (64, 0), (64, 64), (1000, 413), (16384, 8192)])
def test_single_cell_closed_form(N, n1):
    """All samples in one row: K2 = ln((N+1)! / (N0! N1!)); the other 26 rows add ln 1 = 0."""
    G = np.zeros((3, N), dtype=np.uint8)
    G[1] = 2  # any constant genotypes keep every sample in one row
    ph = np.zeros(N, dtype=np.uint8)
    ph[:n1] = 1
    _, k2, cc = oracle.scan_topk(G, ph, 1)
    want = math.lgamma(N + 2) - math.lgamma(N - n1 + 1) - math.lgamma(n1 + 1)
    assert abs(k2[0] - want) <= 1e-12 * max(1.0, want)
    assert cc[0].reshape(2, 27)[:, 9 * 0 + 3 * 2 + 0].tolist() == [N - n1, n1]


def test_single_class_and_pure_rows_closed_form():
    """If every row holds one class only, each row contributes ln(r + 1)."""
    d = make_dataset(6, 500, 0.5, 0.05, seed=3)
    for ph in (np.zeros(500, np.uint8), np.ones(500, np.uint8)):
        k2, cc = oracle.scan_all(d.geno, ph)
        r = cc.sum(axis=1)
        want = np.log(r + 1.0).sum(axis=1)
        assert np.allclose(k2, want, rtol=1e-13, atol=0)
    # pure rows: phenotype is a function of the genotype row of (0, 1, 2)
    row = 9 * d.geno[0].astype(int) + 3 * d.geno[1] + d.geno[2]
    ph = (row % 2).astype(np.uint8)
    t = oracle.table(d.geno, ph, 0, 1, 2)
    assert np.all((t[0] == 0) | (t[1] == 0))
    assert abs(oracle.k2(t, oracle.log_factorial(501)) - np.log(t.sum(axis=0) + 1.0).sum()) < 1e-10


def test_topk_matches_exact_integer_order():
    for seed in range(12):
        M, N = 8 + seed % 3, 24 + seed
        geno, pheno = tiny(1000 + seed, M, N)
        kk = 15
        ijk, k2, cc = oracle.scan_topk(geno, pheno, kk, nthreads=3)
        full = brute.scan(geno.tolist(), pheno.tolist())
        full.sort(key=lambda r: (r[0], r[1]))
        ref = full[:kk]
        # the K2 order is the exact Q order (equal Q: equal up to rounding)
        got_q = [brute.q_value(c.tolist()) for c in cc]
        assert got_q == [q for q, _, _ in ref]
        for x in range(len(ref)):
            assert cc[x].tolist() == brute.table(geno.tolist(), pheno.tolist(), tuple(ijk[x]))
        # where a Q value is unique over all combinations the index must agree
        allq = [r[0] for r in full]
        for x in range(len(ref)):
            if allq.count(ref[x][0]) == 1:
                assert tuple(ijk[x]) == ref[x][1]


def test_topk_edge_sizes():
    geno, pheno = tiny(4, 5, 20)
    ijk, k2, _ = oracle.scan_topk(geno, pheno, 100)
    assert len(ijk) == 10  # C(5,3): k larger than the number of combinations
    ijk, _, _ = oracle.scan_topk(geno[:2], pheno, 5)
    assert len(ijk) == 0   # fewer than three SNPs
    ijk, _, _ = oracle.scan_topk(geno, pheno, 0)
    assert len(ijk) == 0


def test_ties_broken_by_index():
    """Identical SNP rows give identical tables: equal K2 sorted by (i, j, k)."""
    base, pheno = tiny(21, 1, 50)
    G = np.repeat(base, 6, axis=0)
    ijk, k2, _ = oracle.scan_topk(G, pheno, 20)
    assert np.all(k2 == k2[0])
    assert [tuple(x) for x in ijk] == list(itertools.combinations(range(6), 3))


@pytest.mark.parametrize("seed", range(1, 7))
def test_planted_triplet_recovered(seed):
    d = make_parity_fixture(seed)
    ijk, k2, _ = oracle.scan_topk(d.geno, d.pheno, 2)
    assert tuple(ijk[0]) == tuple(d.planted)
    assert k2[1] - k2[0] > 20.0


# ---- second order: pairs of SNPs (9 rows per class) ----

def _pair_tables_and_k2_vs_brute(lib, seeds=range(30)):
    """Every pair table equals the brute-force tally; K2 equals ln Q."""
    for seed in seeds:
        M = 2 + seed % 7
        N = 1 + (seed * 5) % 45
        geno, pheno = tiny(700 + seed, M, N, p_case=(seed % 5) / 4.0)
        k2, cc = oracle.scan_pairs_all(geno, pheno, lib=lib, nthreads=2)
        for x, snps in enumerate(itertools.combinations(range(M), 2)):
            t = brute.table(geno.tolist(), pheno.tolist(), snps)
            assert cc[x].tolist() == t, (seed, snps)
            want = brute.k2_exact(t)
            assert abs(k2[x] - want) <= 1e-12 * max(1.0, abs(want)), (seed, snps, k2[x], want)


def _pair_topk_vs_brute(lib, seeds=range(8)):
    for seed in seeds:
        M, N = 7 + seed % 4, 20 + 3 * seed
        geno, pheno = tiny(800 + seed, M, N)
        ij, k2, cc = oracle.scan_pairs_topk(geno, pheno, 9, lib=lib, nthreads=2)
        full = brute.scan(geno.tolist(), pheno.tolist(), order=2)
        full.sort(key=lambda r: (r[0], r[1]))
        ref = full[:9]
        assert [brute.q_value(c.tolist()) for c in cc] == [q for q, _, _ in ref]
        allq = [r[0] for r in full]
        for x in range(len(ref)):
            assert cc[x].tolist() == brute.table(geno.tolist(), pheno.tolist(), tuple(ij[x]))
            if allq.count(ref[x][0]) == 1:
                assert tuple(ij[x]) == ref[x][1]


def test_pair_tables_and_k2_match_bruteforce():
    _pair_tables_and_k2_vs_brute(oracle.load())


def test_pair_topk_matches_exact_integer_order():
    _pair_topk_vs_brute(oracle.load(), seeds=range(12))


def test_pair_tables_are_margins_of_triplet_tables():
    """Summing a triplet table over one SNP's genotype gives the pair table of
    the other two (ties the pair oracle to the triplet oracle)."""
    d = make_dataset(9, 700, 0.4, 0.05, seed=12)
    _, pcc = oracle.scan_pairs_all(d.geno, d.pheno)
    idx = {tuple(int(v) for v in p): x for x, p in enumerate(oracle.lex_pairs(9))}
    assert len(idx) == 36 and list(idx)[:3] == [(0, 1), (0, 2), (0, 3)]
    for (i, j, k) in [(0, 1, 2), (2, 5, 8), (1, 3, 7), (4, 6, 8)]:
        t = oracle.table(d.geno, d.pheno, i, j, k).reshape(2, 3, 3, 3)
        assert np.array_equal(t.sum(axis=3).reshape(2, 9), pcc[idx[(i, j)]])
        assert np.array_equal(t.sum(axis=2).reshape(2, 9), pcc[idx[(i, k)]])
        assert np.array_equal(t.sum(axis=1).reshape(2, 9), pcc[idx[(j, k)]])
        assert np.array_equal(oracle.pair_table(d.geno, d.pheno, i, j), pcc[idx[(i, j)]])


@pytest.mark.parametrize("N,n1", [(1, 1), (64, 0), (1000, 413), (16384, 8192)])
def test_pair_single_cell_closed_form(N, n1):
    """All samples in one row: K2 = ln((N+1)! / (N0! N1!))."""
    G = np.full((2, N), 1, dtype=np.uint8)
    ph = np.zeros(N, dtype=np.uint8)
    ph[:n1] = 1
    ij, k2, cc = oracle.scan_pairs_topk(G, ph, 1)
    want = math.lgamma(N + 2) - math.lgamma(N - n1 + 1) - math.lgamma(n1 + 1)
    assert abs(k2[0] - want) <= 1e-12 * max(1.0, want)
    assert cc[0][:, 3 * 1 + 1].tolist() == [N - n1, n1]
    assert oracle.k2_rows(cc[0], oracle.log_factorial(N + 1)) == k2[0]


def test_pair_edge_sizes_and_ties():
    geno, pheno = tiny(4, 5, 20)
    ij, _, _ = oracle.scan_pairs_topk(geno, pheno, 100)
    assert len(ij) == 10                     # C(5,2)
    assert len(oracle.scan_pairs_topk(geno[:1], pheno, 5)[0]) == 0
    assert len(oracle.scan_pairs_topk(geno, pheno, 0)[0]) == 0
    base, ph = tiny(21, 1, 50)
    G = np.repeat(base, 5, axis=0)           # identical rows: equal K2, index order
    ij, k2, _ = oracle.scan_pairs_topk(G, ph, 10)
    assert np.all(k2 == k2[0])
    assert [tuple(x) for x in ij] == list(itertools.combinations(range(5), 2))


# ---- fourth order: quads of SNPs (81 rows per class) ----

def _quad_tables_and_k2_vs_brute(lib, seeds=range(12)):
    """Every quad table equals the brute-force tally; K2 equals ln Q."""
    for seed in seeds:
        M = 4 + seed % 3
        N = 1 + (seed * 7) % 40
        geno, pheno = tiny(900 + seed, M, N, p_case=(seed % 5) / 4.0)
        k2, cc = oracle.scan_quads_all(geno, pheno, lib=lib, nthreads=2)
        for x, snps in enumerate(itertools.combinations(range(M), 4)):
            t = brute.table(geno.tolist(), pheno.tolist(), snps)
            assert cc[x].tolist() == t, (seed, snps)
            want = brute.k2_exact(t)
            assert abs(k2[x] - want) <= 1e-12 * max(1.0, abs(want)), (seed, snps, k2[x], want)


def _quad_topk_vs_brute(lib, seeds=range(4)):
    for seed in seeds:
        M, N = 7 + seed % 2, 18 + 4 * seed
        geno, pheno = tiny(950 + seed, M, N)
        q, k2, cc = oracle.scan_quads_topk(geno, pheno, 8, lib=lib, nthreads=2)
        full = brute.scan(geno.tolist(), pheno.tolist(), order=4)
        full.sort(key=lambda r: (r[0], r[1]))
        ref = full[:8]
        assert [brute.q_value(c.tolist()) for c in cc] == [v for v, _, _ in ref]
        allq = [r[0] for r in full]
        for x in range(len(ref)):
            assert cc[x].tolist() == brute.table(geno.tolist(), pheno.tolist(), tuple(q[x]))
            if allq.count(ref[x][0]) == 1:
                assert tuple(q[x]) == ref[x][1]


def test_quad_tables_and_k2_match_bruteforce():
    _quad_tables_and_k2_vs_brute(oracle.load())


def test_quad_topk_matches_exact_integer_order():
    _quad_topk_vs_brute(oracle.load(), seeds=range(8))


def test_quad_tables_are_margins_of_triplet_tables():
    """Summing a quad table over one SNP's genotype gives the triplet table of
    the other three (ties the quad oracle to the triplet oracle)."""
    d = make_dataset(8, 600, 0.45, 0.05, seed=14)
    _, qcc = oracle.scan_quads_all(d.geno, d.pheno)
    quads = [tuple(int(v) for v in q) for q in oracle.lex_quads(8)]
    assert len(quads) == 70 and quads[:2] == [(0, 1, 2, 3), (0, 1, 2, 4)]
    for (i, j, k, l) in [(0, 1, 2, 3), (1, 3, 5, 7), (0, 2, 6, 7), (4, 5, 6, 7)]:
        t = qcc[quads.index((i, j, k, l))].reshape(2, 3, 3, 3, 3)
        for axis, sub in ((4, (i, j, k)), (3, (i, j, l)), (2, (i, k, l)), (1, (j, k, l))):
            want = oracle.table(d.geno, d.pheno, *sub).reshape(2, 27)
            assert np.array_equal(t.sum(axis=axis).reshape(2, 27), want), ((i, j, k, l), sub)
        assert np.array_equal(oracle.quad_table(d.geno, d.pheno, i, j, k, l), t.reshape(2, 81))


@pytest.mark.parametrize("N,n1", [(1, 0), (64, 64), (1000, 413)])
def test_quad_single_cell_closed_form(N, n1):
    """All samples in one row: K2 = ln((N+1)! / (N0! N1!))."""
    G = np.full((4, N), 2, dtype=np.uint8)
    ph = np.zeros(N, dtype=np.uint8)
    ph[:n1] = 1
    q, k2, cc = oracle.scan_quads_topk(G, ph, 1)
    want = math.lgamma(N + 2) - math.lgamma(N - n1 + 1) - math.lgamma(n1 + 1)
    assert abs(k2[0] - want) <= 1e-12 * max(1.0, want)
    assert cc[0][:, 80].tolist() == [N - n1, n1]


def test_quad_edge_sizes_and_ties():
    geno, pheno = tiny(6, 6, 25)
    assert len(oracle.scan_quads_topk(geno, pheno, 100)[0]) == 15   # C(6,4)
    assert len(oracle.scan_quads_topk(geno[:3], pheno, 5)[0]) == 0
    base, ph = tiny(22, 1, 40)
    G = np.repeat(base, 6, axis=0)
    q, k2, _ = oracle.scan_quads_topk(G, ph, 15)
    assert np.all(k2 == k2[0])
    assert [tuple(x) for x in q] == list(itertools.combinations(range(6), 4))


# ---- the pins above must catch plausible mistakes planted in the oracle ----

MUTANTS = {
    "transposed_digits": ("9 * gi[s] + 3 * gj[s] + gk[s]", "9 * gi[s] + gj[s] + 3 * gk[s]"),
    "dropped_plus_one": ("L[r0 + r1 + 1] - (L[r0] + L[r1])", "L[r0 + r1] - (L[r0] + L[r1])"),
    "sign_error": ("L[r0 + r1 + 1] - (L[r0] + L[r1])", "L[r0 + r1 + 1] - L[r0] + L[r1]"),
    "class_swap": ("t[ph[s] * ROWS +", "t[(1 - ph[s]) * ROWS +"),
    "log_index": ("L[n - 1] + log((double)n)", "L[n - 1] + log((double)n + 1.0)"),
    "row_digit_k": ("t[row[s] + gk[s]] += 1;", "t[row[s] + (gk[s] ? 1 : 0)] += 1;"),
    "guard_j": ("for (int32_t j = i + 1; j < M - 1; ++j) {", "for (int32_t j = i; j < M - 1; ++j) {"),
    "pair_digits": ("3 * gi[s] + gj[s]", "gi[s] + 3 * gj[s]"),
    "pair_plus_one": ("L[p0 + p1 + 1] - (L[p0] + L[p1])", "L[p0 + p1] - (L[p0] + L[p1])"),
    "pair_guard": ("for (int32_t j = i + 1; j < M; ++j) {", "for (int32_t j = i; j < M; ++j) {"),
    "pair_offset": ("(int64_t)i * (M - 1) - (int64_t)i * (i - 1) / 2", "(int64_t)i * (M - 1) - (int64_t)i * (i + 1) / 2"),
    "quad_digits": ("27 * gi[s] + 9 * gj[s] + 3 * gk[s] + gl[s]", "27 * gi[s] + 9 * gj[s] + gk[s] + 3 * gl[s]"),
    "quad_guard": ("for (int32_t l = k + 1; l < M; ++l) {", "for (int32_t l = k; l < M; ++l) {"),
    "quad_keep_worse": ("if (nb == topk && !cand4_less(&c, &B[nb - 1])) continue;", "if (nb == topk && cand4_less(&c, &B[nb - 1])) continue;"),
    "quad_offset": ("acc += rest * (rest - 1) * (rest - 2) / 6;", "acc += rest * (rest - 1) / 2;"),
}


def _pin_suite(lib) -> None:
    _tables_and_k2_vs_brute(lib, seeds=range(12))
    for seed in range(6):
        M, N = 8, 30
        geno, pheno = tiny(500 + seed, M, N)
        ijk, k2, cc = oracle.scan_topk(geno, pheno, 10, lib=lib, nthreads=2)
        ref = brute.topk(geno.tolist(), pheno.tolist(), 10)
        assert [brute.q_value(c.tolist()) for c in cc] == [r[0] for r in ref]
        for x in range(len(ref)):
            assert cc[x].tolist() == brute.table(geno.tolist(), pheno.tolist(), tuple(ijk[x]))
    _pair_tables_and_k2_vs_brute(lib, seeds=range(10))
    _pair_topk_vs_brute(lib, seeds=range(3))
    _quad_tables_and_k2_vs_brute(lib, seeds=range(6))
    _quad_topk_vs_brute(lib, seeds=range(2))
    L = oracle.log_factorial(5000, lib=lib)
    assert abs(L[4000] - math.lgamma(4001.0)) < 1e-8


def test_pin_suite_passes_on_oracle():
    _pin_suite(oracle.load())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    """Each planted mistake makes the pin suite fail.  The mutant runs in a
    child interpreter: some mistakes (a loop guard, a rank offset) also write
    outside the caller's output arrays, which must not corrupt this
    process's heap; the child then either fails a pin (exit 3) or is ended by
    the C library's heap checks, and both count as caught."""
    src = open(os.path.join(os.path.dirname(oracle.__file__), "epi3_oracle.c")).read()
    a, b = MUTANTS[name]
    assert src.count(a) >= 1, name
    mut = src.replace(a, b)
    p = tmp_path / "mut.c"
    p.write_text(mut)
    from oracle.build import build_oracle
    lib_path = build_oracle(str(p), str(tmp_path / f"lib_{name}.so"))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (f"import sys\nsys.path.insert(0, {root!r})\n"
            "import oracle\n"
            "from tests.test_oracle_pins import _pin_suite\n"
            f"lib = oracle.load({lib_path!r})\n"
            "try:\n    _pin_suite(lib)\nexcept AssertionError:\n    sys.exit(3)\n"
            "sys.exit(0)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins passed on mutant {name}"
    assert r.returncode == 3 or r.returncode < 0 or r.returncode in (134, 139), (r.returncode, r.stderr[-2000:])
