"""Helpers shared by the GPU tests (not collected: no test_ prefix)."""
from __future__ import annotations

import numpy as np


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible MI355X; none found")
    from paper_2201_10956_amd import epi3
    return torch, epi3


def to_dev(geno: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(geno)).to("cuda")


def hits_ijk(h) -> np.ndarray:
    return np.stack([h["i"], h["j"], h["k"]], axis=1).astype(np.int32)


def assert_hits_equal_oracle(h, ijk, k2, counts):
    assert len(h) == len(ijk), (len(h), len(ijk))
    np.testing.assert_array_equal(hits_ijk(h), ijk)
    # FP64 K2 evaluated on the device in the same row order: bit-identical
    np.testing.assert_array_equal(h["k2"], k2)
    if counts is not None:
        np.testing.assert_array_equal(h["counts"].astype(np.int64), counts.astype(np.int64))


def assert_k2_close(k2_32, k2_64, N, epi3):
    """FP32 screen vs FP64 oracle: within the error bound e(N) and 1e-4 relative."""
    k2_32 = np.asarray(k2_32, dtype=np.float64)
    diff = np.abs(k2_32 - k2_64)
    e = epi3.k2_error_bound(N)
    assert np.all(diff <= e), (diff.max(), e)
    rel = diff / np.maximum(np.abs(k2_64), 1e-30)
    assert np.all(rel <= 1e-4), rel.max()
    return float(diff.max()), float(rel.max())


def lex_rank(M, i, j, k) -> int:
    """Position of i < j < k < M in lexicographic order of all triplets."""
    from math import comb
    return comb(M, 3) - comb(M - i, 3) + comb(M - 1 - i, 2) - comb(M - j, 2) + (k - j - 1)


def lex_unrank(M, ranks) -> np.ndarray:
    """Inverse of lex_rank by binary search, int32 [n][3]."""
    from math import comb
    out = []
    C = comb(M, 3)
    for r in ranks:
        r = int(r)
        lo, hi = 0, M - 3
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if C - comb(M - mid, 3) <= r:
                lo = mid
            else:
                hi = mid - 1
        i = lo
        r1 = r - (C - comb(M - i, 3))
        lo, hi = i + 1, M - 2
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if comb(M - 1 - i, 2) - comb(M - mid, 2) <= r1:
                lo = mid
            else:
                hi = mid - 1
        j = lo
        k = r1 - (comb(M - 1 - i, 2) - comb(M - j, 2)) + j + 1
        out.append((i, j, k))
    return np.array(out, dtype=np.int32).reshape(-1, 3)
