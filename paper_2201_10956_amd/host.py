"""ctypes binding of libepi3_host.so, the host-CPU three-way scan.

A measured CPU baseline beside the GPU library (the paper's fourth CPU
approach: class-split bit planes, cache-resident pair planes, vector AND +
POPCNT, OpenMP).  The GPU binding (`epi3`) never imports this module.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "host", "libepi3_host.so")

ISA_BEST, ISA_SCALAR, ISA_AVX2, ISA_AVX512 = -1, 0, 1, 2
ISA_NAMES = {ISA_SCALAR: "scalar popcount", ISA_AVX2: "avx2 nibble-table popcount",
             ISA_AVX512: "avx512 vpopcntq"}
HIT_DTYPE = np.dtype([("i", "<u4"), ("j", "<u4"), ("k", "<u4"), ("k2_f32", "<f4"),
                      ("k2", "<f8"), ("counts", "<u4", (2, 27))])
assert HIT_DTYPE.itemsize == 240


class HostError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with code {code}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2201_10956_amd/build.py")
_lib = ctypes.CDLL(LIB_PATH)
_lib.epi3h_best_isa.restype = ctypes.c_int
_lib.epi3h_best_isa.argtypes = []
_lib.epi3h_scan_topk.restype = ctypes.c_int
_lib.epi3h_scan_topk.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]


def best_isa() -> int:
    """Highest instruction-set level of the counting loop on this CPU."""
    return int(_lib.epi3h_best_isa())


def scan_topk(geno: np.ndarray, pheno: np.ndarray, k: int, threads: int = 0,
              isa: int = ISA_BEST) -> np.ndarray:
    """k lowest-K2 triplets of genotypes `geno` (uint8 [M][N]) and phenotype
    `pheno` (uint8 [N]) on the host cores; a structured array of HIT_DTYPE."""
    g = np.ascontiguousarray(geno, dtype=np.uint8)
    p = np.ascontiguousarray(pheno, dtype=np.uint8)
    if g.ndim != 2 or p.ndim != 1 or p.shape[0] != g.shape[1]:
        raise ValueError("geno must be [M][N] and pheno [N]")
    M, N = g.shape
    n_max = M * (M - 1) * (M - 2) // 6 if M >= 3 else 0
    out = np.zeros(max(1, min(int(k), n_max)) if k > 0 else 1, dtype=HIT_DTYPE)
    n = ctypes.c_int32(0)
    rc = _lib.epi3h_scan_topk(g.ctypes.data, N, p.ctypes.data, M, N, int(k), int(threads),
                              int(isa), out.ctypes.data, ctypes.byref(n))
    if rc != 0:
        raise HostError(rc, "epi3h_scan_topk")
    return out[: n.value].copy()
