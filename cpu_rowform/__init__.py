"""CPU comparator: the row-level PairHMM forward pass with SIMD over each
row's columns and OpenMP threads over pairs (``rowform.c``).

A host baseline stronger than the plain oracle, for the benchmark's report.
It is not part of the GPU library and shares no code with it or with the
oracle; the tests check it against the oracle.  Built with gcc for x86-64
with AVX2 and FMA.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rowform.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "librowform.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O3", "-mavx2", "-mfma", "-fopenmp", "-std=gnu11", "-fPIC",
                        "-shared", _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                raise RuntimeError("librowform.so is not built (cpu_rowform.build())")
            L = ctypes.CDLL(_LIB)
            u8p, u64p = ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_uint64)
            L.rf_forward_pairs.argtypes = [u8p] * 5 + [u64p, u8p, u64p,
                                                       ctypes.POINTER(ctypes.c_uint32),
                                                       ctypes.c_uint64, ctypes.c_int,
                                                       ctypes.POINTER(ctypes.c_double), u8p]
            _lib = L
    return _lib


def forward_pairs(batch, pair_idx=None, threads: int = 0):
    """log10 likelihoods and flags (1 FP32 accepted, 2 FP64) of (a subset of)
    the pairs of a CSR batch dict."""
    L = _load()
    pl = np.ascontiguousarray(batch["pair_list"], dtype=np.uint32).reshape(-1, 2)
    if pair_idx is not None:
        pl = np.ascontiguousarray(pl[np.asarray(pair_idx, dtype=np.int64)])
    u8 = lambda k: np.ascontiguousarray(batch[k], dtype=np.uint8)
    arrs = [u8(k) for k in ("reads", "base_quals", "ins_quals", "del_quals", "gcp", "haplotypes")]
    ro = np.ascontiguousarray(batch["read_offsets"], dtype=np.uint64)
    ho = np.ascontiguousarray(batch["hap_offsets"], dtype=np.uint64)
    out = np.empty(len(pl), np.float64)
    flags = np.empty(len(pl), np.uint8)
    p8 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    p64 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    rc = L.rf_forward_pairs(p8(arrs[0]), p8(arrs[1]), p8(arrs[2]), p8(arrs[3]), p8(arrs[4]),
                            p64(ro), p8(arrs[5]), p64(ho),
                            pl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), len(pl),
                            int(threads), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            p8(flags))
    if rc != 0:
        raise MemoryError("rf_forward_pairs: allocation failed")
    return out, flags
