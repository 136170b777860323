"""Python binding of libepi3 (ctypes).  Argument marshalling only: device
buffers come from torch, every step of the scan runs in the library's HIP
kernels.  Importing this module fails when libepi3.so has not been built;
there is no fallback."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libepi3.so")

OK, E_INVALID, E_GENOTYPE, E_PHENOTYPE, E_WORKSPACE, E_CAPACITY, E_HIP, E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
LAYOUT_SPLIT, LAYOUT_MASKED = 0, 1
ENCODE_BITS_ONLY = 0x100
VARIANT_AUTO, VARIANT_VALU, VARIANT_MFMA, VARIANT_MFMA_FP4 = 0, 1, 2, 3
_VARIANTS = {"auto": VARIANT_AUTO, "valu": VARIANT_VALU, "mfma": VARIANT_MFMA,
             "mfma_fp4": VARIANT_MFMA_FP4}
_ERRORS = {E_INVALID: "invalid argument", E_GENOTYPE: "genotype byte outside {0,1,2}",
           E_PHENOTYPE: "phenotype byte outside {0,1}", E_WORKSPACE: "workspace too small",
           E_CAPACITY: "candidate capacity exceeded", E_HIP: "HIP runtime error",
           E_UNSUPPORTED: "unsupported variant/layout"}


class Epi3Error(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {_ERRORS.get(code, 'error')} ({code})")
        self.code = code


class CDataset(ctypes.Structure):
    _fields_ = [("n_snps", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("n_cases", ctypes.c_int32), ("n_controls", ctypes.c_int32),
                ("words", ctypes.c_int32 * 2), ("layout", ctypes.c_int32),
                ("snp_stride", ctypes.c_int32), ("byte_stride", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("planes", ctypes.c_void_p), ("bytes", ctypes.c_void_p), ("nibbles", ctypes.c_void_p),
                ("pairs", ctypes.c_void_p), ("lf64", ctypes.c_void_p),
                ("lf32", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class CHit(ctypes.Structure):
    _fields_ = [("i", ctypes.c_uint32), ("j", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("k2_f32", ctypes.c_float), ("k2", ctypes.c_double),
                ("counts", (ctypes.c_uint32 * 27) * 2)]


class CPairHit(ctypes.Structure):
    _fields_ = [("i", ctypes.c_uint32), ("j", ctypes.c_uint32), ("k2_f32", ctypes.c_float),
                ("reserved", ctypes.c_uint32), ("k2", ctypes.c_double),
                ("counts", (ctypes.c_uint32 * 9) * 2)]


class CQuadHit(ctypes.Structure):
    _fields_ = [("i", ctypes.c_uint32), ("j", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("l", ctypes.c_uint32), ("k2_f32", ctypes.c_float), ("reserved", ctypes.c_uint32),
                ("k2", ctypes.c_double), ("counts", (ctypes.c_uint32 * 81) * 2)]


class CJob(ctypes.Structure):
    _fields_ = [("d", ctypes.POINTER(CDataset)), ("case_mask", ctypes.c_void_p),
                ("k", ctypes.c_int32), ("reserved", ctypes.c_int32)]


HIT_DTYPE = np.dtype([("i", "<u4"), ("j", "<u4"), ("k", "<u4"), ("k2_f32", "<f4"),
                      ("k2", "<f8"), ("counts", "<u4", (2, 27))])
assert HIT_DTYPE.itemsize == ctypes.sizeof(CHit) == 240
PAIR_HIT_DTYPE = np.dtype([("i", "<u4"), ("j", "<u4"), ("k2_f32", "<f4"), ("reserved", "<u4"),
                           ("k2", "<f8"), ("counts", "<u4", (2, 9))])
assert PAIR_HIT_DTYPE.itemsize == ctypes.sizeof(CPairHit) == 96
QUAD_HIT_DTYPE = np.dtype([("i", "<u4"), ("j", "<u4"), ("k", "<u4"), ("l", "<u4"),
                           ("k2_f32", "<f4"), ("reserved", "<u4"), ("k2", "<f8"),
                           ("counts", "<u4", (2, 81))])
assert QUAD_HIT_DTYPE.itemsize == ctypes.sizeof(CQuadHit) == 680
assert ctypes.sizeof(CDataset) == 96 and ctypes.sizeof(CJob) == 24


def _load():
    # torch first: the library then binds to the HIP runtime torch already
    # loaded, so device pointers and streams from torch are valid in it
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2201_10956_amd.build "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    P = ctypes.POINTER
    sigs = {
        "epi3_encode_bytes": (i64, [i32, i32, i32, i32]),
        "epi3_encode": (ctypes.c_int, [vp, i64, vp, i32, i32, i32, vp, i64, vp, P(CDataset)]),
        "epi3_workspace_bytes": (i64, [P(CDataset), i32, i32, i64]),
        "epi3_scan": (ctypes.c_int, [P(CDataset), i32, i32, i64, vp, i64, vp]),
        "epi3_topk": (ctypes.c_int, [P(CDataset), i32, i64, vp, vp, P(i32), vp]),
        "epi3_batched_workspace_bytes": (i64, [P(CJob), i32, i32, i64]),
        "epi3_scan_batched": (ctypes.c_int, [P(CJob), i32, i32, i64, vp, i64, vp, vp, vp]),
        "epi3_batched_score_plane": (ctypes.c_int, [P(CJob), i32, i32, i64, vp, i32, P(vp)]),
        "epi3_init": (ctypes.c_int, []),
        "epi3_scan_topk_static": (ctypes.c_int, [P(CDataset), i32, vp, P(i32), vp]),
        "epi3_batched_bound_list": (ctypes.c_int, [P(CJob), i32, i32, i64, vp, i32, P(vp), P(vp),
                                                   P(i64), P(ctypes.c_float), vp]),
        "epi3_set_batch_select": (ctypes.c_int, [i32]),
        "epi3_set_scan_select": (ctypes.c_int, [i32]),
        "epi3_scan_tables": (ctypes.c_int, [P(CDataset), i32, vp, vp, vp, i64, vp]),
        "epi3_score_triplets": (ctypes.c_int, [P(CDataset), vp, i64, vp, vp, vp, vp]),
        "epi3_score_plane": (ctypes.c_int, [P(CDataset), i32, i64, vp, P(vp)]),
        "epi3_k2_error_bound": (ctypes.c_double, [i32]),
        "epi3_n_triplets": (i64, [i32]),
        "epi3_release": (None, []),
        "epi3_timing_enable": (None, [ctypes.c_int]),
        "epi3_timing_query": (ctypes.c_int, [i32, P(ctypes.c_double), P(i64)]),
        "epi3_timing_reset": (None, []),
        "epi3_version": (ctypes.c_char_p, []),
        "epi3_tile_rule": (ctypes.c_int, [i32, i32, i32, i32]),
        "epi3_tile_rules_clear": (None, []),
        "epi3_tile_for": (i32, [P(CDataset), i32]),
        "epi3_set_pass_bytes": (ctypes.c_int, [i64]),
        "epi3_set_compact_cap": (ctypes.c_int, [i64]),
        "epi3_perm_pvalue": (ctypes.c_int, [ctypes.c_double, vp, i32, P(ctypes.c_double)]),
        "epi3_n_pairs": (i64, [i32]),
        "epi3_k2_error_bound_pairs": (ctypes.c_double, [i32]),
        "epi3_pairs_workspace_bytes": (i64, [P(CDataset), i32, i64]),
        "epi3_scan_pairs": (ctypes.c_int, [P(CDataset), i32, i64, vp, i64, vp]),
        "epi3_pairs_topk": (ctypes.c_int, [P(CDataset), i32, i64, vp, vp, P(i32), vp]),
        "epi3_pairs_score_plane": (ctypes.c_int, [P(CDataset), i32, i64, vp, P(vp)]),
        "epi3_n_quads": (i64, [i32]),
        "epi3_k2_error_bound_quads": (ctypes.c_double, [i32]),
        "epi3_quads_workspace_bytes": (i64, [P(CDataset), i32, i64]),
        "epi3_scan_quads": (ctypes.c_int, [P(CDataset), i32, i64, vp, i64, vp]),
        "epi3_quads_topk": (ctypes.c_int, [P(CDataset), i32, i64, vp, vp, P(i32), vp]),
        "epi3_quads_score_plane": (ctypes.c_int, [P(CDataset), i32, i64, vp, P(vp)]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTS = ("epi3_encode_bytes", "epi3_encode", "epi3_workspace_bytes", "epi3_scan", "epi3_topk",
           "epi3_batched_workspace_bytes", "epi3_scan_batched", "epi3_batched_score_plane",
           "epi3_init", "epi3_scan_topk_static", "epi3_scan_tables", "epi3_batched_bound_list",
           "epi3_set_batch_select", "epi3_set_scan_select",
           "epi3_score_triplets", "epi3_score_plane", "epi3_k2_error_bound", "epi3_n_triplets", "epi3_release",
           "epi3_version", "epi3_timing_enable", "epi3_timing_query", "epi3_timing_reset",
           "epi3_tile_rule", "epi3_tile_rules_clear", "epi3_tile_for", "epi3_set_pass_bytes",
           "epi3_perm_pvalue", "epi3_set_compact_cap", "epi3_n_pairs", "epi3_k2_error_bound_pairs",
           "epi3_pairs_workspace_bytes", "epi3_scan_pairs", "epi3_pairs_topk",
           "epi3_pairs_score_plane", "epi3_n_quads", "epi3_k2_error_bound_quads",
           "epi3_quads_workspace_bytes", "epi3_scan_quads", "epi3_quads_topk",
           "epi3_quads_score_plane")
TILES_PATH = os.path.join(_HERE, "tiles.json")


def _check(rc: int, where: str) -> None:
    if rc != OK:
        raise Epi3Error(rc, where)


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _buffer(nbytes: int, device):
    torch = _torch()
    # 256-byte aligned device buffer (torch's caching allocator aligns to >= 512 B)
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


def version() -> str:
    return _lib.epi3_version().decode()


def timing_enable(on: bool = True) -> None:
    _lib.epi3_timing_enable(1 if on else 0)


def timing_reset() -> None:
    _lib.epi3_timing_reset()


def timing_query(which: int = 0):
    """(summed ms, launches) of the count stage (0) or selection (1) since the last reset."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(_lib.epi3_timing_query(which, ctypes.byref(ms), ctypes.byref(n)), "epi3_timing_query")
    return ms.value, n.value


def tile_rule(variant: str, min_snps: int, min_samples: int, tile) -> None:
    """Register a tile rule (for variant "auto", `tile` names the variant)."""
    t = _VARIANTS[tile] if isinstance(tile, str) else int(tile)
    _check(_lib.epi3_tile_rule(_VARIANTS[variant], int(min_snps), int(min_samples), t),
           "epi3_tile_rule")


def tile_rules_clear() -> None:
    _lib.epi3_tile_rules_clear()


def tile_for(ds: "Dataset", variant: str):
    """The tile a scan of ds with `variant` uses (for "auto": the variant's name)."""
    r = int(_lib.epi3_tile_for(ctypes.byref(ds.c), _VARIANTS[variant]))
    _check(r if r < 0 else OK, "epi3_tile_for")
    if variant == "auto":
        return {v: k for k, v in _VARIANTS.items()}[r]
    return r


def set_pass_bytes(nbytes: int) -> None:
    """Scratch bytes per pass buffer of the matrix-core paths (0: default)."""
    _check(_lib.epi3_set_pass_bytes(int(nbytes)), "epi3_set_pass_bytes")


BATCH_SELECT = {"auto": 0, "plane": 1, "bounded": 2}


def set_batch_select(mode: str) -> None:
    """How phenotype batches select: "auto", "plane" (score plane per job) or
    "bounded" (sample pass + bounded list, no plane)."""
    _check(_lib.epi3_set_batch_select(BATCH_SELECT[mode]), "epi3_set_batch_select")


def set_scan_select(mode: str) -> None:
    """How plain scans select: "auto", "plane" (FP32 score plane) or "bounded"
    (sample pass + bounded list, no plane; matrix-core variants)."""
    _check(_lib.epi3_set_scan_select(BATCH_SELECT[mode]), "epi3_set_scan_select")


def set_compact_cap(n: int) -> None:
    """Entries the selection keeps after its first pass (0: default)."""
    _check(_lib.epi3_set_compact_cap(int(n)), "epi3_set_compact_cap")


def load_tiles(path: str = TILES_PATH) -> int:
    """Register the rules of a tile table written by the autotuner; returns how many."""
    import json
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        table = json.load(f)
    for r in table.get("rules", []):
        tile_rule(r["variant"], r["min_snps"], r["min_samples"], r["tile"])
    return len(table.get("rules", []))


def perm_pvalue(observed_k2: float, perm_min_k2) -> float:
    """Family-wise permutation p-value of the observed best K2 given the best
    K2 of each phenotype permutation (hit 0 of each job of a batched scan)."""
    a = np.ascontiguousarray(np.asarray(perm_min_k2, dtype=np.float64))
    p = ctypes.c_double(0.0)
    _check(_lib.epi3_perm_pvalue(float(observed_k2), a.ctypes.data_as(ctypes.c_void_p), a.size,
                                 ctypes.byref(p)), "epi3_perm_pvalue")
    return p.value


def n_triplets(M: int) -> int:
    return int(_lib.epi3_n_triplets(M))


def k2_error_bound(N: int) -> float:
    return float(_lib.epi3_k2_error_bound(N))


@dataclass
class Dataset:
    c: CDataset
    buf: object          # torch uint8 tensor owning the device memory
    geno: object         # keeps the source alive until encode returned

    @property
    def M(self) -> int:
        return self.c.n_snps

    @property
    def N(self) -> int:
        return self.c.n_samples


def encode(geno, pheno, layout: str = "split", stream=None, into: Optional[Dataset] = None,
           values: bool = True) -> Dataset:
    """geno: torch uint8 [M][N] on the GPU (rows may be strided); pheno: host uint8 [N].
    With `into`, the encoding reuses that Dataset's device buffer and struct (same
    addresses, so cached batched graphs stay valid).  values=False (SPLIT only)
    skips the 0/1 value planes that only the matrix-core triplet kernels read."""
    torch = _torch()
    assert geno.dtype == torch.uint8 and geno.dim() == 2 and geno.is_cuda
    assert geno.stride(1) == 1
    ph = np.ascontiguousarray(np.asarray(pheno, dtype=np.uint8))
    M, N = int(geno.shape[0]), int(geno.shape[1])
    lay = LAYOUT_SPLIT if layout == "split" else LAYOUT_MASKED
    if not values:
        lay |= ENCODE_BITS_ONLY
    n1 = int(ph.sum()) if ph.size else 0
    nbytes = _lib.epi3_encode_bytes(M, n1, N - n1, lay)
    _check(int(nbytes) if nbytes < 0 else OK, "epi3_encode_bytes")
    if into is not None and into.buf.numel() >= nbytes:
        buf, c = into.buf, into.c
    else:
        buf, c = _buffer(nbytes, geno.device), CDataset()
    rc = _lib.epi3_encode(ctypes.c_void_p(geno.data_ptr()), geno.stride(0),
                          ph.ctypes.data_as(ctypes.c_void_p), M, N, lay,
                          ctypes.c_void_p(buf.data_ptr()), buf.numel(), _stream(stream),
                          ctypes.byref(c))
    _check(rc, "epi3_encode")
    if into is not None and c is into.c:
        into.geno = geno
        return into
    return Dataset(c=c, buf=buf, geno=geno)


def hits_to_numpy(hits: ctypes.Array, n: int) -> np.ndarray:
    raw = np.frombuffer(hits, dtype=HIT_DTYPE, count=len(hits))
    return raw[:n].copy()


class Scanner:
    """Workspace + calls for repeated plain scans of one data set."""

    def __init__(self, ds: Dataset, k: int, variant: str = "auto", cand_cap: int = 0):
        self.ds, self.k, self.variant, self.cand_cap = ds, int(k), _VARIANTS[variant], int(cand_cap)
        self._alloc()

    def _alloc(self):
        nbytes = _lib.epi3_workspace_bytes(ctypes.byref(self.ds.c), self.k, self.variant,
                                           self.cand_cap)
        _check(int(nbytes) if nbytes < 0 else OK, "epi3_workspace_bytes")
        self.ws = _buffer(nbytes, self.ds.buf.device)
        self.hits = (CHit * max(self.k, 1))()

    def scan(self, stream=None) -> None:
        rc = _lib.epi3_scan(ctypes.byref(self.ds.c), self.k, self.variant, self.cand_cap,
                            ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), _stream(stream))
        _check(rc, "epi3_scan")

    def topk(self, stream=None) -> np.ndarray:
        n = ctypes.c_int32(0)
        rc = _lib.epi3_topk(ctypes.byref(self.ds.c), self.k, self.cand_cap,
                            ctypes.c_void_p(self.ws.data_ptr()), ctypes.cast(self.hits, ctypes.c_void_p),
                            ctypes.byref(n), _stream(stream))
        if rc == E_CAPACITY:
            raise Epi3Error(rc, f"epi3_topk (needs cand_cap >= {n.value})")
        _check(rc, "epi3_topk")
        return hits_to_numpy(self.hits, n.value)

    def run(self, stream=None, retry: bool = True) -> np.ndarray:
        self.scan(stream)
        n = ctypes.c_int32(0)
        rc = _lib.epi3_topk(ctypes.byref(self.ds.c), self.k, self.cand_cap,
                            ctypes.c_void_p(self.ws.data_ptr()), ctypes.cast(self.hits, ctypes.c_void_p),
                            ctypes.byref(n), _stream(stream))
        if rc == E_CAPACITY and retry:
            self.cand_cap = int(n.value)
            self._alloc()
            return self.run(stream, retry=False)
        _check(rc, "epi3_topk")
        return hits_to_numpy(self.hits, n.value)

    def score_plane(self):
        """FP32 K2 of every triplet (lexicographic order): a torch view into the workspace,
        valid after scan()."""
        torch = _torch()
        ptr = ctypes.c_void_p(0)
        rc = _lib.epi3_score_plane(ctypes.byref(self.ds.c), self.k, self.cand_cap,
                                   ctypes.c_void_p(self.ws.data_ptr()), ctypes.byref(ptr))
        _check(rc, "epi3_score_plane")
        off = (ptr.value or 0) - self.ws.data_ptr()
        T = n_triplets(self.ds.M)
        return self.ws[off: off + 4 * T].view(torch.float32)


def n_pairs(M: int) -> int:
    return int(_lib.epi3_n_pairs(int(M)))


def k2_error_bound_pairs(N: int) -> float:
    return float(_lib.epi3_k2_error_bound_pairs(int(N)))


def n_quads(M: int) -> int:
    return int(_lib.epi3_n_quads(int(M)))


def k2_error_bound_quads(N: int) -> float:
    return float(_lib.epi3_k2_error_bound_quads(int(N)))


class _OrderScanner:
    """Workspace + calls for repeated scans of one SPLIT data set at another
    interaction order (pairs or quads)."""
    _names = None  # (workspace_bytes, scan, topk, score_plane) entry points
    _hit = None    # ctypes hit structure
    _dtype = None  # numpy dtype of a hit
    _order = 0

    def __init__(self, ds: Dataset, k: int, cand_cap: int = 0):
        self.ds, self.k, self.cand_cap = ds, int(k), int(cand_cap)
        self._alloc()

    def _fn(self, x):
        return getattr(_lib, self._names[x])

    def _alloc(self):
        nbytes = self._fn(0)(ctypes.byref(self.ds.c), self.k, self.cand_cap)
        _check(int(nbytes) if nbytes < 0 else OK, self._names[0])
        self.ws = _buffer(nbytes, self.ds.buf.device)
        self.hits = (self._hit * max(self.k, 1))()

    def scan(self, stream=None) -> None:
        rc = self._fn(1)(ctypes.byref(self.ds.c), self.k, self.cand_cap,
                         ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), _stream(stream))
        _check(rc, self._names[1])

    def topk(self, stream=None):
        n = ctypes.c_int32(0)
        rc = self._fn(2)(ctypes.byref(self.ds.c), self.k, self.cand_cap,
                         ctypes.c_void_p(self.ws.data_ptr()),
                         ctypes.cast(self.hits, ctypes.c_void_p), ctypes.byref(n), _stream(stream))
        return rc, n.value

    def run(self, stream=None, retry: bool = True) -> np.ndarray:
        self.scan(stream)
        rc, n = self.topk(stream)
        if rc == E_CAPACITY and retry:
            self.cand_cap = int(n)
            self._alloc()
            return self.run(stream, retry=False)
        _check(rc, self._names[2])
        raw = np.frombuffer(self.hits, dtype=self._dtype, count=len(self.hits))
        return raw[:n].copy()

    def score_plane(self):
        """FP32 K2 of every combination (lexicographic order): a torch view into
        the workspace, valid after scan()."""
        torch = _torch()
        ptr = ctypes.c_void_p(0)
        rc = self._fn(3)(ctypes.byref(self.ds.c), self.k, self.cand_cap,
                         ctypes.c_void_p(self.ws.data_ptr()), ctypes.byref(ptr))
        _check(rc, self._names[3])
        off = (ptr.value or 0) - self.ws.data_ptr()
        T = n_pairs(self.ds.M) if self._order == 2 else n_quads(self.ds.M)
        return self.ws[off: off + 4 * T].view(torch.float32)


class PairScanner(_OrderScanner):
    """Second-order scans (pairs of SNPs, 9-row tables)."""
    _names = ("epi3_pairs_workspace_bytes", "epi3_scan_pairs", "epi3_pairs_topk",
              "epi3_pairs_score_plane")
    _hit, _dtype, _order = CPairHit, PAIR_HIT_DTYPE, 2


class QuadScanner(_OrderScanner):
    """Fourth-order scans (quads of SNPs, 81-row tables)."""
    _names = ("epi3_quads_workspace_bytes", "epi3_scan_quads", "epi3_quads_topk",
              "epi3_quads_score_plane")
    _hit, _dtype, _order = CQuadHit, QUAD_HIT_DTYPE, 4


def scan_quads(ds: Dataset, k: int, cand_cap: int = 0, stream=None) -> np.ndarray:
    """The k lowest (K2, i, j, k, l) quads of a SPLIT data set (QUAD_HIT_DTYPE)."""
    return QuadScanner(ds, k, cand_cap).run(stream)


def scan_pairs(ds: Dataset, k: int, cand_cap: int = 0, stream=None) -> np.ndarray:
    """The k lowest (K2, i, j) pairs of a SPLIT data set (structured array, PAIR_HIT_DTYPE)."""
    return PairScanner(ds, k, cand_cap).run(stream)


def scan_topk(ds: Dataset, k: int, variant: str = "auto", cand_cap: int = 0, stream=None):
    return Scanner(ds, k, variant, cand_cap).run(stream)


STATIC_SCRATCH_BYTES = 128 << 20  # EPI3_STATIC_SCRATCH_BYTES


def scan_topk_static(ds: Dataset, k: int, stream=None) -> np.ndarray:
    """Plain vector-ALU scan + top-k in the library's static workspace
    (epi3_scan_topk_static: no device buffer is allocated for the call)."""
    hits = (CHit * max(int(k), 1))()
    n = ctypes.c_int32(0)
    rc = _lib.epi3_scan_topk_static(ctypes.byref(ds.c), int(k), ctypes.cast(hits, ctypes.c_void_p),
                                    ctypes.byref(n), _stream(stream))
    _check(rc, "epi3_scan_topk_static")
    raw = np.frombuffer(hits, dtype=HIT_DTYPE, count=len(hits))
    return raw[:n.value].copy()


def scan_tables(ds: Dataset, variant: str = "auto", counts: bool = True, stream=None):
    """(counts [T][2][27] uint32 or None, k2 [T] float32) as torch tensors, lexicographic order."""
    torch = _torch()
    T = n_triplets(ds.M)
    dev = ds.buf.device
    k2 = torch.empty(max(T, 1), dtype=torch.float32, device=dev)
    cc = torch.empty((max(T, 1), 2, 27), dtype=torch.int32, device=dev) if counts else None
    nbytes = _lib.epi3_workspace_bytes(ctypes.byref(ds.c), 1, _VARIANTS[variant], 0)
    _check(int(nbytes) if nbytes < 0 else OK, "epi3_workspace_bytes")
    ws = _buffer(nbytes, dev)
    rc = _lib.epi3_scan_tables(ctypes.byref(ds.c), _VARIANTS[variant],
                               ctypes.c_void_p(cc.data_ptr()) if cc is not None else None,
                               ctypes.c_void_p(k2.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                               ws.numel(), _stream(stream))
    _check(rc, "epi3_scan_tables")
    torch.cuda.current_stream().synchronize()
    return (cc[:T] if cc is not None else None), k2[:T]


def score_triplets(ds: Dataset, ijk, stream=None):
    """Tables, FP32 and FP64 K2 of explicit triplets (numpy int [n][3])."""
    torch = _torch()
    idx = torch.as_tensor(np.ascontiguousarray(np.asarray(ijk, dtype=np.uint32).reshape(-1, 3)).view(np.int32),
                          device=ds.buf.device)
    n = idx.shape[0]
    dev = ds.buf.device
    cc = torch.empty((max(n, 1), 2, 27), dtype=torch.int32, device=dev)
    kf = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    kd = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    rc = _lib.epi3_score_triplets(ctypes.byref(ds.c), ctypes.c_void_p(idx.data_ptr()), n,
                                  ctypes.c_void_p(cc.data_ptr()), ctypes.c_void_p(kf.data_ptr()),
                                  ctypes.c_void_p(kd.data_ptr()), _stream(stream))
    _check(rc, "epi3_score_triplets")
    torch.cuda.current_stream().synchronize()
    return cc[:n], kf[:n], kd[:n]


def pack_masks(phenos) -> np.ndarray:
    """Host uint8 [Q][N] case indicators -> uint32 [Q][ceil(N/32)] bit masks
    (bit s % 32 of word s / 32 is sample s)."""
    ph = np.ascontiguousarray(np.asarray(phenos, dtype=np.uint8))
    if ph.ndim == 1:
        ph = ph[None]
    Q, N = ph.shape
    W = (N + 31) // 32
    padded = np.zeros((Q, W * 32), dtype=np.uint8)
    padded[:, :N] = ph
    return np.packbits(padded, axis=1, bitorder="little").view("<u4").reshape(Q, W)


class BatchScanner:
    """One batched launch over several jobs.

    split: `datasets` is a list of SPLIT Datasets (each with its own phenotype).
    masked: `datasets` is one MASKED Dataset and `masks` a device uint32 tensor
    [Q][W] of case masks (see pack_masks); job q scans phenotype q."""

    def __init__(self, datasets, k, masks=None, variant: str = "auto", cand_cap: int = 0):
        torch = _torch()
        self.variant, self.cand_cap = _VARIANTS[variant], int(cand_cap)
        if masks is None:
            self.ds_list = list(datasets)
            ks = [int(k)] * len(self.ds_list) if np.isscalar(k) else [int(x) for x in k]
            self.jobs = (CJob * len(self.ds_list))()
            for x, d in enumerate(self.ds_list):
                self.jobs[x].d = ctypes.pointer(d.c)
                self.jobs[x].case_mask = None
                self.jobs[x].k = ks[x]
            device = self.ds_list[0].buf.device
        else:
            ds = datasets
            self.ds_list = [ds]
            assert masks.dtype == torch.int32 or masks.dtype == torch.uint32 or masks.dtype == torch.int64
            self.masks = masks.contiguous()
            Q = int(self.masks.shape[0])
            ks = [int(k)] * Q if np.isscalar(k) else [int(x) for x in k]
            self.jobs = (CJob * Q)()
            row = self.masks.stride(0) * self.masks.element_size()
            for q in range(Q):
                self.jobs[q].d = ctypes.pointer(ds.c)
                self.jobs[q].case_mask = ctypes.c_void_p(self.masks.data_ptr() + q * row)
                self.jobs[q].k = ks[q]
            device = ds.buf.device
        self.ks = ks
        self.device = device
        self._alloc()

    def _alloc(self):
        nbytes = _lib.epi3_batched_workspace_bytes(self.jobs, len(self.jobs), self.variant,
                                                   self.cand_cap)
        _check(int(nbytes) if nbytes < 0 else OK, "epi3_batched_workspace_bytes")
        self.ws = _buffer(nbytes, self.device)
        self.hits = (CHit * sum(self.ks))()
        self.n_out = (ctypes.c_int32 * len(self.jobs))()

    def run(self, stream=None, retry: bool = True):
        rc = _lib.epi3_scan_batched(self.jobs, len(self.jobs), self.variant, self.cand_cap,
                                    ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                    ctypes.cast(self.hits, ctypes.c_void_p),
                                    ctypes.cast(self.n_out, ctypes.c_void_p), _stream(stream))
        if rc == E_CAPACITY and retry:
            need = max(-int(v) for v in self.n_out)
            self.cand_cap = max(self.cand_cap, need)
            self._alloc()
            return self.run(stream, retry=False)
        _check(rc, "epi3_scan_batched")
        out, off = [], 0
        allh = np.frombuffer(self.hits, dtype=HIT_DTYPE, count=sum(self.ks))
        for x, kk in enumerate(self.ks):
            out.append(allh[off: off + int(self.n_out[x])].copy())
            off += kk
        return out

    def bound_list(self, job: int, stream=None):
        """(FP32 scores, lexicographic ranks, bound) of job `job`'s list in a
        batch selected by bound, as numpy arrays in list order."""
        torch = _torch()
        kp, rp = ctypes.c_void_p(0), ctypes.c_void_p(0)
        n, b = ctypes.c_int64(0), ctypes.c_float(0.0)
        rc = _lib.epi3_batched_bound_list(self.jobs, len(self.jobs), self.variant, self.cand_cap,
                                          ctypes.c_void_p(self.ws.data_ptr()), int(job),
                                          ctypes.byref(kp), ctypes.byref(rp), ctypes.byref(n),
                                          ctypes.byref(b), _stream(stream))
        _check(rc, "epi3_batched_bound_list")
        base = self.ws.data_ptr()
        ko, ro, cnt = (kp.value or base) - base, (rp.value or base) - base, int(n.value)
        keys = self.ws[ko: ko + 4 * cnt].view(torch.int32).cpu().numpy().view(np.uint32)
        ranks = self.ws[ro: ro + 8 * cnt].view(torch.int64).cpu().numpy()
        scores = (keys & np.uint32(0x7fffffff)).view(np.float32)
        return scores, ranks, float(b.value)

    def score_plane(self, job: int):
        """FP32 K2 of every triplet of job `job` (lexicographic order): a torch
        view into the workspace, valid after run()."""
        torch = _torch()
        ptr = ctypes.c_void_p(0)
        rc = _lib.epi3_batched_score_plane(self.jobs, len(self.jobs), self.variant, self.cand_cap,
                                           ctypes.c_void_p(self.ws.data_ptr()), int(job),
                                           ctypes.byref(ptr))
        _check(rc, "epi3_batched_score_plane")
        off = (ptr.value or 0) - self.ws.data_ptr()
        T = n_triplets(self.jobs[job].d.contents.n_snps)
        return self.ws[off: off + 4 * T].view(torch.float32)


def init() -> None:
    """Create the library's streams and events now rather than in the first scan."""
    _check(_lib.epi3_init(), "epi3_init")


def release() -> None:
    _lib.epi3_release()


# tuned tile table shipped with the package (written by paper_2201_10956_amd.autotune)
load_tiles()
