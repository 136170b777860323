"""Encode round trip: the bit planes, 0/1 value planes (bytes and E2M1
nibbles), pairwise tables and log-factorial tables that epi3_encode writes
are decoded on the host and compared with the genotypes they came from, for
both layouts; every padding bit, byte, nibble and SNP slot must be zero."""
import numpy as np
import pytest

import oracle
from synth import SplitMix64
from tests.gpu_util import require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _data(seed, M, N, p_case):
    u = SplitMix64(seed, 5).uniform(0, M * N + N)
    geno = np.minimum((u[: M * N] * 3).astype(np.uint8), 2).reshape(M, N)
    pheno = (u[M * N:] < p_case).astype(np.uint8)
    return geno, pheno


def _host(buf, ptr, nbytes):
    off = ptr - buf.data_ptr()
    assert 0 <= off and off + nbytes <= buf.numel()
    return buf[off: off + nbytes].cpu().numpy()


@pytest.mark.parametrize("layout", ["split", "masked"])
@pytest.mark.parametrize("M,N,p", [(1, 1, 1.0), (3, 31, 0.3), (70, 257, 0.5), (130, 1000, 0.0),
                                   (64, 513, 1.0), (200, 4100, 0.37)])
def test_encode_round_trip(env, layout, M, N, p):
    torch, epi3 = env
    print(f"[case] encode {layout} M={M} N={N} p={p}", flush=True)
    geno, pheno = _data(100 * M + N, M, N, p)
    ds = epi3.encode(to_dev(geno), pheno, layout=layout)
    c, buf = ds.c, ds.buf
    torch.cuda.synchronize()
    Mp, S = c.snp_stride, c.byte_stride
    assert Mp >= M + 64 and Mp % 64 == 0
    if layout == "split":
        lists = [np.flatnonzero(pheno == 0), np.flatnonzero(pheno == 1)]
        W = [c.words[0], c.words[1]]
        assert W == [(len(lists[0]) + 31) // 32, (len(lists[1]) + 31) // 32]
        assert (c.n_controls, c.n_cases) == (len(lists[0]), len(lists[1]))
    else:
        lists = [np.arange(N)]
        W = [c.words[0]]
        assert W[0] == (N + 31) // 32
    # list position -> sample index (or -1 for padding), word by word
    pos = np.concatenate([np.concatenate([l, -np.ones(32 * w - len(l), dtype=np.int64)])
                          for l, w in zip(lists, W)])
    Wtot = sum(W)

    # bit planes [word][snp][plane], bit b of word w = list position 32 w + b
    raw = _host(buf, c.planes, Wtot * Mp * 2 * 4)
    bits = np.unpackbits(raw.reshape(Wtot, Mp, 2, 4), axis=-1, bitorder="little")
    bits = bits.reshape(Wtot, Mp, 2, 32).transpose(1, 2, 0, 3).reshape(Mp, 2, Wtot * 32)
    want = np.zeros((Mp, 2, Wtot * 32), dtype=np.uint8)
    real = pos >= 0
    for g in (0, 1):
        want[:M, g, real] = geno[:, pos[real]] == g
    np.testing.assert_array_equal(bits, want)

    # value planes [class][snp][plane][position]: bytes 0/1, nibbles 0x0 / 0x2
    classes = len(lists)
    assert S % 256 == 0 and S >= max(len(l) for l in lists)
    vb = _host(buf, c.bytes, classes * Mp * 2 * S).reshape(classes, Mp, 2, S)
    vn = _host(buf, c.nibbles, classes * Mp * 2 * (S // 2)).reshape(classes, Mp, 2, S // 2)
    nib = np.stack([vn & 0xF, vn >> 4], axis=-1).reshape(classes, Mp, 2, S)
    for cl, lst in enumerate(lists):
        wb = np.zeros((Mp, 2, S), dtype=np.uint8)
        for g in (0, 1):
            wb[:M, g, :len(lst)] = geno[:, lst] == g
        np.testing.assert_array_equal(vb[cl], wb)
        np.testing.assert_array_equal(nib[cl], 2 * wb)

    # pairwise tables [class][x][y][(a, b)] for x, y < M (full square)
    pr = _host(buf, c.pairs, classes * Mp * Mp * 16).view("<i4").reshape(classes, Mp, Mp, 4)
    for cl, lst in enumerate(lists):
        G = geno[:, lst]
        ind = [(G == a).astype(np.int64) for a in (0, 1)]
        for a in (0, 1):
            for b in (0, 1):
                np.testing.assert_array_equal(pr[cl, :M, :M, 2 * a + b], ind[a] @ ind[b].T)

    # log factorials L[0 .. N + 1]: FP64 bit-identical to the oracle's, FP32 its rounding
    L = oracle.log_factorial(N + 1)
    l64 = _host(buf, c.lf64, (N + 2) * 8).view("<f8")
    l32 = _host(buf, c.lf32, (N + 2) * 4).view("<f4")
    np.testing.assert_array_equal(l64, L)
    np.testing.assert_array_equal(l32, L.astype(np.float32))
    assert int(_host(buf, c.status, 4).view("<i4")[0]) == 0


def test_encode_bits_only_has_no_value_planes(env):
    torch, epi3 = env
    geno, pheno = _data(9, 40, 300, 0.5)
    ds = epi3.encode(to_dev(geno), pheno, values=False)
    assert not ds.c.bytes and not ds.c.nibbles
    full = epi3.encode(to_dev(geno), pheno)
    n = ds.c.words[0] + ds.c.words[1]
    a = _host(ds.buf, ds.c.planes, n * ds.c.snp_stride * 8)
    b = _host(full.buf, full.c.planes, n * full.c.snp_stride * 8)
    np.testing.assert_array_equal(a, b)
