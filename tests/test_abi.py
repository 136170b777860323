"""The C ABI without a GPU: the library loads, exports every function the
header declares, and its host-only logic (sizes, counts, bounds, tile rules,
argument checks) behaves as documented.  No kernel is launched here."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epi3.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(epi3_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def epi3():
    from paper_2201_10956_amd import epi3 as e
    return e


def test_every_declared_symbol_is_exported(epi3):
    names = _declared()
    assert len(names) >= 20
    lib = ctypes.CDLL(epi3.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(epi3.EXPORTS) == names


def test_counts_and_bounds(epi3):
    assert epi3.n_triplets(0) == 0 and epi3.n_triplets(2) == 0
    assert epi3.n_triplets(3) == 1
    assert epi3.n_triplets(2048) == math.comb(2048, 3)
    assert epi3.n_triplets(100000) == math.comb(100000, 3)
    # e(N) = 32 u L[N + 27], L = log factorial
    for N in (1, 100, 16384):
        want = 32 * 2.0 ** -24 * math.lgamma(N + 28)
        assert epi3.k2_error_bound(N) == pytest.approx(want, rel=1e-12)
    assert epi3.version().startswith("epi3")


def _fake_dataset(epi3, M, N1, N0, layout=0):
    """A struct as epi3_encode fills it; pointers are never dereferenced by
    the size queries."""
    c = epi3.CDataset()
    c.n_snps, c.n_cases, c.n_controls, c.n_samples = M, N1, N0, N1 + N0
    c.layout = layout
    c.snp_stride = (M + 63) // 64 * 64 + 64
    c.byte_stride = (max(N0, N1) + 255) // 256 * 256
    c.words[0], c.words[1] = (N0 + 31) // 32, (N1 + 31) // 32
    for f in ("planes", "bytes", "nibbles", "pairs", "lf64", "lf32", "status"):
        setattr(c, f, 4096)
    return c


def test_encode_bytes(epi3):
    lib = epi3._lib
    assert lib.epi3_encode_bytes(10, 5, 5, 0) > 0
    assert lib.epi3_encode_bytes(10, 0, 0, 0) == epi3.E_INVALID
    assert lib.epi3_encode_bytes(10, 5, 5, 7) == epi3.E_INVALID
    assert lib.epi3_encode_bytes(-1, 5, 5, 0) == epi3.E_INVALID
    # bit planes only: SPLIT with the flag is accepted, MASKED with it is not
    assert lib.epi3_encode_bytes(10, 5, 5, epi3.ENCODE_BITS_ONLY) == lib.epi3_encode_bytes(10, 5, 5, 0)
    assert lib.epi3_encode_bytes(10, 5, 5, 1 | epi3.ENCODE_BITS_ONLY) == epi3.E_INVALID
    # the buffer grows with every dimension
    a = lib.epi3_encode_bytes(100, 500, 500, 0)
    assert lib.epi3_encode_bytes(200, 500, 500, 0) > a
    assert lib.epi3_encode_bytes(100, 5000, 500, 0) > a


def test_workspace_sizes(epi3):
    lib = epi3._lib
    d = _fake_dataset(epi3, 300, 700, 900)
    T = epi3.n_triplets(300)
    v = lib.epi3_workspace_bytes(ctypes.byref(d), 10, epi3.VARIANT_VALU, 0)
    assert v >= 4 * T                      # at least the FP32 score plane
    m = lib.epi3_workspace_bytes(ctypes.byref(d), 10, epi3.VARIANT_MFMA, 0)
    f = lib.epi3_workspace_bytes(ctypes.byref(d), 10, epi3.VARIANT_MFMA_FP4, 0)
    assert m > v and f == m                # plus the corner scratch
    assert lib.epi3_workspace_bytes(ctypes.byref(d), 0, 1, 0) == epi3.E_INVALID
    assert lib.epi3_workspace_bytes(ctypes.byref(d), 10, 9, 0) == epi3.E_INVALID
    big = _fake_dataset(epi3, 30, 70000, 10)
    assert lib.epi3_workspace_bytes(ctypes.byref(big), 10, epi3.VARIANT_MFMA, 0) == \
        epi3.E_UNSUPPORTED
    # the candidate buffers scale with the capacity
    c1 = lib.epi3_workspace_bytes(ctypes.byref(d), 10, 1, 100000)
    assert c1 > v


def test_tile_rules(epi3):
    lib = epi3._lib
    small = _fake_dataset(epi3, 100, 500, 500)
    large = _fake_dataset(epi3, 3000, 20000, 20000)
    try:
        epi3.tile_rules_clear()
        assert lib.epi3_tile_for(ctypes.byref(small), epi3.VARIANT_VALU) == 4
        assert lib.epi3_tile_for(ctypes.byref(large), epi3.VARIANT_VALU) == 8
        assert lib.epi3_tile_for(ctypes.byref(small), epi3.VARIANT_MFMA) == 4
        assert lib.epi3_tile_for(ctypes.byref(large), epi3.VARIANT_MFMA_FP4) == 4
        assert lib.epi3_tile_for(ctypes.byref(large), epi3.VARIANT_AUTO) == epi3.VARIANT_VALU
        # the most specific applicable rule wins
        epi3.tile_rule("valu", 0, 0, 8)
        epi3.tile_rule("valu", 1000, 0, 4)
        epi3.tile_rule("valu", 1000, 50000, 8)
        assert lib.epi3_tile_for(ctypes.byref(small), epi3.VARIANT_VALU) == 8
        assert lib.epi3_tile_for(ctypes.byref(large), epi3.VARIANT_VALU) == 4
        epi3.tile_rule("mfma_fp4", 64, 1000, 8)
        assert lib.epi3_tile_for(ctypes.byref(large), epi3.VARIANT_MFMA_FP4) == 8
        assert lib.epi3_tile_for(ctypes.byref(small), epi3.VARIANT_MFMA_FP4) == 8
        assert lib.epi3_tile_for(ctypes.byref(large), epi3.VARIANT_MFMA) == 4
        # the workspace follows the rules in force when it is sized (the
        # number of tiles, hence of scratch buffers' tiles, depends on JB)
        w2 = lib.epi3_workspace_bytes(ctypes.byref(small), 10, epi3.VARIANT_MFMA, 0)
        epi3.tile_rule("mfma", 0, 0, 2)
        w4 = lib.epi3_workspace_bytes(ctypes.byref(small), 10, epi3.VARIANT_MFMA, 0)
        assert w2 != w4
        # AUTO picks the registered variant, but not where it cannot run
        epi3.tile_rule("auto", 500, 0, "mfma_fp4")
        assert epi3.tile_for(_Wrap(large), "auto") == "mfma_fp4"
        assert epi3.tile_for(_Wrap(small), "auto") == "valu"
        unsup = _fake_dataset(epi3, 3000, 70000, 10)
        assert epi3.tile_for(_Wrap(unsup), "auto") == "valu"
        # invalid tiles are refused
        assert lib.epi3_tile_rule(epi3.VARIANT_VALU, 0, 0, 5) == epi3.E_INVALID
        assert lib.epi3_tile_rule(epi3.VARIANT_MFMA, 0, 0, 16) == epi3.E_INVALID
        assert lib.epi3_tile_rule(epi3.VARIANT_MFMA, 0, 0, 3) == epi3.E_INVALID
        assert lib.epi3_tile_rule(epi3.VARIANT_AUTO, 0, 0, 0) == epi3.E_INVALID
        assert lib.epi3_tile_rule(7, 0, 0, 4) == epi3.E_INVALID
        assert lib.epi3_tile_rule(epi3.VARIANT_VALU, -1, 0, 4) == epi3.E_INVALID
    finally:
        epi3.tile_rules_clear()
        epi3.load_tiles()


def test_pass_bytes_bound_the_scratch(epi3):
    lib = epi3._lib
    d = _fake_dataset(epi3, 2048, 8192, 8192)
    try:
        epi3.set_pass_bytes(0)
        a = lib.epi3_workspace_bytes(ctypes.byref(d), 10, epi3.VARIANT_MFMA, 0)
        epi3.set_pass_bytes(1 << 22)
        b = lib.epi3_workspace_bytes(ctypes.byref(d), 10, epi3.VARIANT_MFMA, 0)
        v = lib.epi3_workspace_bytes(ctypes.byref(d), 10, epi3.VARIANT_VALU, 0)
        assert a - v > (1 << 30) and 0 < b - v <= 2 * (1 << 22) + 256
        assert lib.epi3_set_pass_bytes(-5) == epi3.E_INVALID
    finally:
        epi3.set_pass_bytes(0)


class _Wrap:
    """Stands in for a Dataset in tile_for (only .c is read)."""

    def __init__(self, c):
        self.c = c


def test_perm_pvalue(epi3):
    """p = (1 + #{q: min_q <= obs}) / (Q + 1), counted by hand."""
    import numpy as np
    mins = np.array([5.0, 3.0, 7.5, 3.0, 9.0])
    assert epi3.perm_pvalue(3.0, mins) == pytest.approx(3 / 6)      # two ties count
    assert epi3.perm_pvalue(2.9, mins) == pytest.approx(1 / 6)      # none as low
    assert epi3.perm_pvalue(100.0, mins) == pytest.approx(6 / 6)
    rng = np.random.default_rng(5)
    for _ in range(20):
        m = rng.normal(size=rng.integers(1, 50))
        o = float(rng.normal())
        assert epi3.perm_pvalue(o, m) == (1 + int(np.sum(m <= o))) / (m.size + 1)
    with pytest.raises(epi3.Epi3Error):
        epi3.perm_pvalue(1.0, [])
    with pytest.raises(epi3.Epi3Error):
        epi3.perm_pvalue(float("nan"), [1.0])


def test_compact_cap_sizes_the_workspace(epi3):
    lib = epi3._lib
    d = _fake_dataset(epi3, 300, 700, 900)
    try:
        a = lib.epi3_workspace_bytes(ctypes.byref(d), 10, epi3.VARIANT_VALU, 0)
        epi3.set_compact_cap(1 << 20)
        b = lib.epi3_workspace_bytes(ctypes.byref(d), 10, epi3.VARIANT_VALU, 0)
        assert b - a >= 12 * ((1 << 20) - 65536)
        assert lib.epi3_set_compact_cap(-1) == epi3.E_INVALID
    finally:
        epi3.set_compact_cap(0)


def test_pair_scan_host_side(epi3):
    """Pair counts, the 9-row error bound and the pair workspace queries."""
    lib = epi3._lib
    assert epi3.n_pairs(0) == 0 and epi3.n_pairs(1) == 0 and epi3.n_pairs(2) == 1
    assert epi3.n_pairs(2048) == math.comb(2048, 2)
    for N in (1, 100, 16384):
        want = 14 * 2.0 ** -24 * math.lgamma(N + 10)
        assert epi3.k2_error_bound_pairs(N) == pytest.approx(want, rel=1e-12)
        assert epi3.k2_error_bound_pairs(N) < epi3.k2_error_bound(N)
    d = _fake_dataset(epi3, 300, 700, 900)
    w = lib.epi3_pairs_workspace_bytes(ctypes.byref(d), 10, 0)
    assert w >= 4 * math.comb(300, 2)
    assert lib.epi3_pairs_workspace_bytes(ctypes.byref(d), 10, 100000) > w
    assert lib.epi3_pairs_workspace_bytes(ctypes.byref(d), 0, 0) == epi3.E_INVALID
    m = _fake_dataset(epi3, 300, 700, 900, layout=1)
    assert lib.epi3_pairs_workspace_bytes(ctypes.byref(m), 10, 0) == epi3.E_UNSUPPORTED


def test_quad_scan_host_side(epi3):
    lib = epi3._lib
    assert epi3.n_quads(3) == 0 and epi3.n_quads(4) == 1
    assert epi3.n_quads(256) == math.comb(256, 4)
    assert epi3.n_quads(4096) == math.comb(4096, 4)
    for N in (1, 100, 16384):
        want = 86 * 2.0 ** -24 * math.lgamma(N + 82)
        assert epi3.k2_error_bound_quads(N) == pytest.approx(want, rel=1e-12)
    d = _fake_dataset(epi3, 64, 700, 900)
    w = lib.epi3_quads_workspace_bytes(ctypes.byref(d), 10, 0)
    assert w >= 4 * math.comb(64, 4)
    assert lib.epi3_quads_workspace_bytes(ctypes.byref(d), 0, 0) == epi3.E_INVALID
    m = _fake_dataset(epi3, 64, 700, 900, layout=1)
    assert lib.epi3_quads_workspace_bytes(ctypes.byref(m), 10, 0) == epi3.E_UNSUPPORTED
    big = _fake_dataset(epi3, 5000, 700, 900)
    assert lib.epi3_quads_workspace_bytes(ctypes.byref(big), 10, 0) == epi3.E_UNSUPPORTED


def test_phenotype_batches_limit_sample_count(epi3):
    """Phenotype batches count cells in 16 bits: more than 65535 samples is
    EPI3_E_UNSUPPORTED (checked before anything is launched)."""
    lib = epi3._lib
    ok = _fake_dataset(epi3, 50, 30000, 0, layout=1)
    big = _fake_dataset(epi3, 50, 70000, 0, layout=1)
    for d, want_ok in ((ok, True), (big, False)):
        jobs = (epi3.CJob * 2)()
        for q in range(2):
            jobs[q].d = ctypes.pointer(d)
            jobs[q].case_mask = ctypes.c_void_p(4096)
            jobs[q].k = 5
        r = lib.epi3_batched_workspace_bytes(jobs, 2, epi3.VARIANT_MFMA_FP4, 0)
        assert (r > 0) if want_ok else (r == epi3.E_UNSUPPORTED), r


def test_phenotype_batches_limit_value_plane_bytes(epi3):
    """The phenotype count addresses the value planes (snp_stride x 2 x
    byte_stride bytes) with 32-bit offsets: 33000 SNPs x 65535 samples
    (4.3e9 bytes) is EPI3_E_UNSUPPORTED, 30000 SNPs (3.9e9) is not."""
    lib = epi3._lib
    for M, want_ok in ((30000, True), (33000, False)):
        d = _fake_dataset(epi3, M, 65535, 0, layout=1)
        jobs = (epi3.CJob * 1)()
        jobs[0].d = ctypes.pointer(d)
        jobs[0].case_mask = ctypes.c_void_p(4096)
        jobs[0].k = 5
        r = lib.epi3_batched_workspace_bytes(jobs, 1, epi3.VARIANT_MFMA_FP4, 0)
        assert (r > 0) if want_ok else (r == epi3.E_UNSUPPORTED), (M, r)


def test_bounded_batches_need_no_plane(epi3):
    """A phenotype batch of 1024 SNPs x 8192 samples x 64 masks: selected by
    bound (the default at this size) its workspace does not hold the
    64 x C(1024,3) score plane that plane selection needs; invalid modes are
    refused."""
    lib = epi3._lib
    d = _fake_dataset(epi3, 1024, 8192, 0, layout=1)
    d.byte_stride = 8192
    jobs = (epi3.CJob * 64)()
    for q in range(64):
        jobs[q].d = ctypes.pointer(d)
        jobs[q].case_mask = ctypes.c_void_p(4096)
        jobs[q].k = 10
    T = math.comb(1024, 3)
    try:
        auto = lib.epi3_batched_workspace_bytes(jobs, 64, epi3.VARIANT_MFMA_FP4, 0)
        epi3.set_batch_select("plane")
        plane = lib.epi3_batched_workspace_bytes(jobs, 64, epi3.VARIANT_MFMA_FP4, 0)
        epi3.set_batch_select("bounded")
        bounded = lib.epi3_batched_workspace_bytes(jobs, 64, epi3.VARIANT_MFMA_FP4, 0)
    finally:
        epi3.set_batch_select("auto")
    assert auto == bounded
    assert plane - bounded > 64 * T * 4 * 0.99
    # FP4 batches selected by bound count and score in one kernel: no pass
    # scratch (int8 operands keep the 2 x 4 GiB of corner cells)
    assert bounded < 1 << 30
    try:
        epi3.set_batch_select("bounded")
        int8 = lib.epi3_batched_workspace_bytes(jobs, 64, epi3.VARIANT_MFMA, 0)
    finally:
        epi3.set_batch_select("auto")
    assert int8 - bounded > 7 * (1 << 30)
    assert lib.epi3_set_batch_select(3) == epi3.E_INVALID
    assert lib.epi3_set_batch_select(-1) == epi3.E_INVALID


def test_static_scan_refuses_what_does_not_fit(epi3):
    """epi3_scan_topk_static checks its sizes on the host before it touches a
    device: the score plane of 700 SNPs (57 M triplets) exceeds the static
    workspace; 580 SNPs fit; bad arguments are refused."""
    lib = epi3._lib
    hits = (epi3.CHit * 10)()
    n = ctypes.c_int32(0)
    big = _fake_dataset(epi3, 700, 200, 200)
    rc = lib.epi3_scan_topk_static(ctypes.byref(big), 10, ctypes.cast(hits, ctypes.c_void_p),
                                   ctypes.byref(n), None)
    assert rc == epi3.E_WORKSPACE
    fits = _fake_dataset(epi3, 580, 200, 200)
    assert 0 < lib.epi3_workspace_bytes(ctypes.byref(fits), 10, epi3.VARIANT_VALU, 0) \
        <= epi3.STATIC_SCRATCH_BYTES
    assert lib.epi3_scan_topk_static(ctypes.byref(big), 0, ctypes.cast(hits, ctypes.c_void_p),
                                     ctypes.byref(n), None) == epi3.E_INVALID
    assert lib.epi3_scan_topk_static(ctypes.byref(big), 10, None, ctypes.byref(n), None) == \
        epi3.E_INVALID
    assert "#define EPI3_STATIC_SCRATCH_BYTES (128ll << 20)" in open(HEADER).read()
    assert epi3.STATIC_SCRATCH_BYTES == 128 << 20


def test_scan_select_sizes(epi3):
    """Selecting by bound drops the 4 C(M,3)-byte score plane from a plain
    scan's workspace (matrix-core variants keep a sample plane and a list
    that grow with k, not with C(M,3)); AUTO keeps the plane up to 16 GiB."""
    lib = epi3._lib
    d = _fake_dataset(epi3, 2048, 8192, 8192)
    T = math.comb(2048, 3)
    try:
        assert lib.epi3_set_scan_select(7) == epi3.E_INVALID
        epi3.set_scan_select("plane")
        plane = lib.epi3_workspace_bytes(ctypes.byref(d), 1000, epi3.VARIANT_MFMA_FP4, 0)
        epi3.set_scan_select("auto")
        assert lib.epi3_workspace_bytes(ctypes.byref(d), 1000, epi3.VARIANT_MFMA_FP4, 0) == plane
        epi3.set_scan_select("bounded")
        bounded = lib.epi3_workspace_bytes(ctypes.byref(d), 1000, epi3.VARIANT_MFMA_FP4, 0)
        assert 0 < bounded < plane - 4 * T + (1 << 30)
        # 8192 SNPs: the plane alone would be 366 GB; AUTO selects by bound
        big = _fake_dataset(epi3, 8192, 8192, 8192)
        epi3.set_scan_select("auto")
        b8 = lib.epi3_workspace_bytes(ctypes.byref(big), 1000, epi3.VARIANT_MFMA_FP4, 0)
        assert 0 < b8 < 8 << 30
        # the state and hits sit where epi3_topk looks for them, whatever the variant
        v8 = lib.epi3_workspace_bytes(ctypes.byref(big), 1000, epi3.VARIANT_VALU, 0)
        assert 0 < v8 < b8
        # a data set without value planes keeps the plane under AUTO
        big.bytes = big.nibbles = 0
        assert lib.epi3_workspace_bytes(ctypes.byref(big), 1000, epi3.VARIANT_VALU, 0) > \
            4 * math.comb(8192, 3)
    finally:
        epi3.set_scan_select("auto")


def test_matrix_core_offset_limits(epi3):
    """The matrix-core kernels use 32-bit offsets into the value planes and
    pair tables: shapes beyond them are refused for the matrix-core
    variants, and AUTO counts them on the vector ALU."""
    lib = epi3._lib
    ok = _fake_dataset(epi3, 40000, 8192, 8192)  # 2 x 40064^2 pair entries < 2^32
    assert lib.epi3_workspace_bytes(ctypes.byref(ok), 10, epi3.VARIANT_MFMA_FP4, 0) > 0
    wide = _fake_dataset(epi3, 46400, 8192, 8192)  # 2 x 46464^2 > 2^32
    assert lib.epi3_workspace_bytes(ctypes.byref(wide), 10, epi3.VARIANT_MFMA_FP4, 0) == epi3.E_UNSUPPORTED
    assert lib.epi3_workspace_bytes(ctypes.byref(wide), 10, epi3.VARIANT_MFMA, 0) == epi3.E_UNSUPPORTED
    assert lib.epi3_workspace_bytes(ctypes.byref(wide), 10, epi3.VARIANT_AUTO, 0) == \
        lib.epi3_workspace_bytes(ctypes.byref(wide), 10, epi3.VARIANT_VALU, 0)
    # value planes of 2 x 20032 x 2 x 65536 bytes > 2^32
    deep = _fake_dataset(epi3, 20000, 65535, 65535)
    assert lib.epi3_workspace_bytes(ctypes.byref(deep), 10, epi3.VARIANT_MFMA_FP4, 0) == epi3.E_UNSUPPORTED
    assert lib.epi3_workspace_bytes(ctypes.byref(deep), 10, epi3.VARIANT_VALU, 0) > 0
