"""CPU oracle for the three-way epistasis scan (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It never imports the GPU library and the GPU library
never imports it.  The C source (epi3_oracle.c) states what is computed and
which passage of the paper each step follows; `brute` is an independent
pure-Python evaluation used to pin it.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

from .build import LIB, build_oracle

_lib = None


def load(path: Optional[str] = None):
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or LIB
    if not os.path.exists(p):
        build_oracle(out=p)
    lib = ctypes.CDLL(p)
    i32, i64, ptr = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_log_factorial.argtypes = [i32, ptr]
    lib.oracle_table.argtypes = [ptr, i64, ptr, i32, i32, i32, i32, ptr]
    lib.oracle_k2.argtypes = [ptr, ptr]
    lib.oracle_k2.restype = ctypes.c_double
    lib.oracle_scan_topk.argtypes = [ptr, i64, ptr, i32, i32, i32, i32, ptr, ptr, ptr]
    lib.oracle_scan_topk.restype = i32
    lib.oracle_score_list.argtypes = [ptr, i64, ptr, i32, ptr, i64, i32, ptr, ptr]
    lib.oracle_scan_all.argtypes = [ptr, i64, ptr, i32, i32, i32, ptr, ptr]
    lib.oracle_table2.argtypes = [ptr, i64, ptr, i32, i32, i32, ptr]
    lib.oracle_k2_rows.argtypes = [ptr, i32, ptr]
    lib.oracle_k2_rows.restype = ctypes.c_double
    lib.oracle_scan_pairs_all.argtypes = [ptr, i64, ptr, i32, i32, i32, ptr, ptr]
    lib.oracle_scan_pairs_topk.argtypes = [ptr, i64, ptr, i32, i32, i32, i32, ptr, ptr, ptr]
    lib.oracle_scan_pairs_topk.restype = i32
    lib.oracle_table4.argtypes = [ptr, i64, ptr, i32, i32, i32, i32, i32, ptr]
    lib.oracle_scan_quads_all.argtypes = [ptr, i64, ptr, i32, i32, i32, ptr, ptr]
    lib.oracle_scan_quads_topk.argtypes = [ptr, i64, ptr, i32, i32, i32, i32, ptr, ptr, ptr]
    lib.oracle_scan_quads_topk.restype = i32
    if path is None:
        _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _prep(geno, pheno):
    G = np.ascontiguousarray(geno, dtype=np.uint8)
    ph = np.ascontiguousarray(pheno, dtype=np.uint8)
    assert G.ndim == 2 and ph.shape == (G.shape[1],)
    return G, ph


def nthreads_default() -> int:
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def log_factorial(nmax: int, lib=None) -> np.ndarray:
    lib = lib or load()
    L = np.empty(nmax + 1, dtype=np.float64)
    lib.oracle_log_factorial(nmax, _p(L))
    return L


def table(geno, pheno, i: int, j: int, k: int, lib=None) -> np.ndarray:
    """[2][27] int32 frequency table (row 9*g_i + 3*g_j + g_k; 0 = controls)."""
    lib = lib or load()
    G, ph = _prep(geno, pheno)
    t = np.empty((2, 27), dtype=np.int32)
    lib.oracle_table(_p(G), G.shape[1], _p(ph), G.shape[1], i, j, k, _p(t))
    return t


def k2(t: np.ndarray, L: np.ndarray, lib=None) -> float:
    lib = lib or load()
    tt = np.ascontiguousarray(t, dtype=np.int32).reshape(54)
    LL = np.ascontiguousarray(L, dtype=np.float64)
    return float(lib.oracle_k2(_p(tt), _p(LL)))


def scan_topk(geno, pheno, k: int, nthreads: Optional[int] = None, counts: bool = True,
              lib=None) -> Tuple[np.ndarray, np.ndarray, Optional[np.ndarray]]:
    """k lowest (K2, i, j, k): returns (ijk [n][3], k2 [n], tables [n][2][27])."""
    lib = lib or load()
    G, ph = _prep(geno, pheno)
    M, N = G.shape
    ijk = np.zeros((max(k, 0), 3), dtype=np.int32)
    kk = np.zeros(max(k, 0), dtype=np.float64)
    cc = np.zeros((max(k, 0), 2, 27), dtype=np.int32) if counts else None
    n = lib.oracle_scan_topk(_p(G), N, _p(ph), M, N, k, nthreads or nthreads_default(),
                             _p(ijk), _p(kk), _p(cc) if cc is not None else None)
    return ijk[:n], kk[:n], (cc[:n] if cc is not None else None)


def score_list(geno, pheno, ijk, nthreads: Optional[int] = None, lib=None):
    """Tables [n][2][27] and K2 [n] of explicit combinations."""
    lib = lib or load()
    G, ph = _prep(geno, pheno)
    idx = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    n = idx.shape[0]
    cc = np.empty((n, 2, 27), dtype=np.int32)
    kk = np.empty(n, dtype=np.float64)
    lib.oracle_score_list(_p(G), G.shape[1], _p(ph), G.shape[1], _p(idx), n,
                          nthreads or nthreads_default(), _p(cc), _p(kk))
    return cc, kk


def scan_all(geno, pheno, counts: bool = True, nthreads: Optional[int] = None, lib=None):
    """All combinations in lexicographic order: (k2 [T], tables [T][2][27])."""
    lib = lib or load()
    G, ph = _prep(geno, pheno)
    M, N = G.shape
    T = M * (M - 1) * (M - 2) // 6
    kk = np.empty(T, dtype=np.float64)
    cc = np.empty((T, 2, 27), dtype=np.int32) if counts else None
    lib.oracle_scan_all(_p(G), N, _p(ph), M, N, nthreads or nthreads_default(), _p(kk),
                        _p(cc) if cc is not None else None)
    return kk, cc


def lex_triplets(M: int) -> np.ndarray:
    """All (i, j, k), i < j < k < M, in lexicographic order, int32 [T][3]."""
    out = []
    for i in range(M):
        for j in range(i + 1, M):
            ks = np.arange(j + 1, M, dtype=np.int32)
            if ks.size:
                out.append(np.stack([np.full_like(ks, i), np.full_like(ks, j), ks], axis=1))
    return np.concatenate(out) if out else np.zeros((0, 3), dtype=np.int32)


# ---- second order: SNP pairs (9 rows per class, row 3 g_i + g_j) ----

def pair_table(geno, pheno, i: int, j: int, lib=None) -> np.ndarray:
    """[2][9] int32 frequency table of the pair (i, j); 0 = controls."""
    lib = lib or load()
    G, ph = _prep(geno, pheno)
    t = np.empty((2, 9), dtype=np.int32)
    lib.oracle_table2(_p(G), G.shape[1], _p(ph), G.shape[1], i, j, _p(t))
    return t


def k2_rows(t: np.ndarray, L: np.ndarray, lib=None) -> float:
    """Eq. 1 for a [2][rows] table."""
    lib = lib or load()
    tt = np.ascontiguousarray(t, dtype=np.int32)
    rows = tt.size // 2
    LL = np.ascontiguousarray(L, dtype=np.float64)
    return float(lib.oracle_k2_rows(_p(tt.reshape(-1)), rows, _p(LL)))


def scan_pairs_all(geno, pheno, counts: bool = True, nthreads: Optional[int] = None, lib=None):
    """All pairs in lexicographic order: (k2 [C(M,2)], tables [C(M,2)][2][9])."""
    lib = lib or load()
    G, ph = _prep(geno, pheno)
    M, N = G.shape
    P = M * (M - 1) // 2
    kk = np.empty(P, dtype=np.float64)
    cc = np.empty((P, 2, 9), dtype=np.int32) if counts else None
    lib.oracle_scan_pairs_all(_p(G), N, _p(ph), M, N, nthreads or nthreads_default(), _p(kk),
                              _p(cc) if cc is not None else None)
    return kk, cc


def scan_pairs_topk(geno, pheno, k: int, nthreads: Optional[int] = None, counts: bool = True,
                    lib=None):
    """k lowest (K2, i, j): returns (ij [n][2], k2 [n], tables [n][2][9])."""
    lib = lib or load()
    G, ph = _prep(geno, pheno)
    M, N = G.shape
    ij = np.zeros((max(k, 0), 2), dtype=np.int32)
    kk = np.zeros(max(k, 0), dtype=np.float64)
    cc = np.zeros((max(k, 0), 2, 9), dtype=np.int32) if counts else None
    n = lib.oracle_scan_pairs_topk(_p(G), N, _p(ph), M, N, k, nthreads or nthreads_default(),
                                   _p(ij), _p(kk), _p(cc) if cc is not None else None)
    return ij[:n], kk[:n], (cc[:n] if cc is not None else None)


def lex_pairs(M: int) -> np.ndarray:
    """All (i, j), i < j < M, in lexicographic order, int32 [C(M,2)][2]."""
    i, j = np.triu_indices(M, k=1)
    return np.stack([i, j], axis=1).astype(np.int32)


# ---- fourth order: SNP quads (81 rows per class, row 27 g_i + 9 g_j + 3 g_k + g_l) ----

def quad_table(geno, pheno, i: int, j: int, k: int, l: int, lib=None) -> np.ndarray:
    """[2][81] int32 frequency table of the quad (i, j, k, l); 0 = controls."""
    lib = lib or load()
    G, ph = _prep(geno, pheno)
    t = np.empty((2, 81), dtype=np.int32)
    lib.oracle_table4(_p(G), G.shape[1], _p(ph), G.shape[1], i, j, k, l, _p(t))
    return t


def scan_quads_all(geno, pheno, counts: bool = True, nthreads: Optional[int] = None, lib=None):
    """All quads in lexicographic order: (k2 [C(M,4)], tables [C(M,4)][2][81])."""
    lib = lib or load()
    G, ph = _prep(geno, pheno)
    M, N = G.shape
    Q = M * (M - 1) * (M - 2) * (M - 3) // 24
    kk = np.empty(Q, dtype=np.float64)
    cc = np.empty((Q, 2, 81), dtype=np.int32) if counts else None
    lib.oracle_scan_quads_all(_p(G), N, _p(ph), M, N, nthreads or nthreads_default(), _p(kk),
                              _p(cc) if cc is not None else None)
    return kk, cc


def scan_quads_topk(geno, pheno, k: int, nthreads: Optional[int] = None, counts: bool = True,
                    lib=None):
    """k lowest (K2, i, j, k, l): returns (ijkl [n][4], k2 [n], tables [n][2][81])."""
    lib = lib or load()
    G, ph = _prep(geno, pheno)
    M, N = G.shape
    q = np.zeros((max(k, 0), 4), dtype=np.int32)
    kk = np.zeros(max(k, 0), dtype=np.float64)
    cc = np.zeros((max(k, 0), 2, 81), dtype=np.int32) if counts else None
    n = lib.oracle_scan_quads_topk(_p(G), N, _p(ph), M, N, k, nthreads or nthreads_default(),
                                   _p(q), _p(kk), _p(cc) if cc is not None else None)
    return q[:n], kk[:n], (cc[:n] if cc is not None else None)


def lex_quads(M: int) -> np.ndarray:
    """All (i, j, k, l), i < j < k < l < M, in lexicographic order, int32 [C(M,4)][4]."""
    import itertools
    return np.array(list(itertools.combinations(range(M), 4)), dtype=np.int32).reshape(-1, 4)
