"""ctypes front end of the FP64 PairHMM oracle (test infrastructure only).

The C source ``phmm_oracle.c`` is compiled with plain gcc, ``-O2
-ffp-contract=off`` (no fused multiply-add, so evaluation orders can be
compared bit for bit).  Every function here follows the paper's Section 2
model (eq. 1-4); see the header of ``phmm_oracle.c`` for the readings taken.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "phmm_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")

NREC = 9  # per-row prior record: pm, px, tMM, tIM, tDM, tMI, tII, tMD, tDD

_lock = threading.Lock()
_lib = None


def lib_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (no GPU code involved)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build_oracle(force=True)
            lib = ctypes.CDLL(_LIB)
            u8p = ctypes.POINTER(ctypes.c_uint8)
            dp = ctypes.POINTER(ctypes.c_double)
            i64p = ctypes.POINTER(ctypes.c_int64)
            u64p = ctypes.POINTER(ctypes.c_uint64)
            u32p = ctypes.POINTER(ctypes.c_uint32)
            ci = ctypes.c_int
            lib.oracle_priors.argtypes = [u8p, u8p, u8p, u8p, ci, dp]
            lib.oracle_forward_probs.argtypes = [dp, u8p, ci, u8p, ci, ci, dp, i64p]
            lib.oracle_forward_antidiag_probs.argtypes = [dp, u8p, ci, u8p, ci, dp]
            lib.oracle_forward_rowform_probs.argtypes = [dp, u8p, ci, u8p, ci, dp]
            lib.oracle_forward_one.argtypes = [u8p, u8p, u8p, u8p, u8p, ci, u8p, ci, ci,
                                               dp, dp, i64p]
            lib.oracle_forward_pairs.argtypes = [u8p, u8p, u8p, u8p, u8p, u64p, ctypes.c_uint32,
                                                 u8p, u64p, ctypes.c_uint32, u32p,
                                                 ctypes.c_uint64, ci, dp]
            for f in ("oracle_priors", "oracle_forward_probs", "oracle_forward_antidiag_probs",
                      "oracle_forward_rowform_probs", "oracle_forward_one",
                      "oracle_forward_pairs"):
                getattr(lib, f).restype = ci
            _lib = lib
    return _lib


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _seq(s):
    if isinstance(s, (bytes, bytearray)):
        return np.frombuffer(bytes(s), dtype=np.uint8)
    if isinstance(s, str):
        return np.frombuffer(s.encode("ascii"), dtype=np.uint8)
    return np.ascontiguousarray(s, dtype=np.uint8)


def priors(bq, iq, dq, gq) -> np.ndarray:
    """Per-row prior records (l x 9) from raw Phred bytes (eq.3 and the
    transition probabilities of Section 2)."""
    lib = _load()
    bq, pb = _u8(bq)
    iq, pi = _u8(iq)
    dq, pd = _u8(dq)
    gq, pg = _u8(gq)
    l = len(bq)
    out = np.zeros((l, NREC), dtype=np.float64)
    rc = lib.oracle_priors(pb, pi, pd, pg, l, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("oracle_priors failed: %d" % rc)
    return out


def forward_probs(pri, read, hap, rescale: bool = False):
    """Row-order forward pass over explicit per-row probabilities.

    Returns (S, E) with L = S * 2**(E - 1020)."""
    lib = _load()
    pri, pp = _f64(pri)
    read, pr = _u8(_seq(read))
    hap, ph = _u8(_seq(hap))
    S = ctypes.c_double(0.0)
    E = ctypes.c_int64(0)
    rc = lib.oracle_forward_probs(pp, pr, len(read), ph, len(hap), int(bool(rescale)),
                                  ctypes.byref(S), ctypes.byref(E))
    if rc != 0:
        raise ValueError("oracle_forward_probs failed: %d" % rc)
    return S.value, E.value


def forward_antidiag_probs(pri, read, hap) -> float:
    lib = _load()
    pri, pp = _f64(pri)
    read, pr = _u8(_seq(read))
    hap, ph = _u8(_seq(hap))
    S = ctypes.c_double(0.0)
    rc = lib.oracle_forward_antidiag_probs(pp, pr, len(read), ph, len(hap), ctypes.byref(S))
    if rc != 0:
        raise ValueError("oracle_forward_antidiag_probs failed: %d" % rc)
    return S.value


def forward_rowform_probs(pri, read, hap) -> float:
    lib = _load()
    pri, pp = _f64(pri)
    read, pr = _u8(_seq(read))
    hap, ph = _u8(_seq(hap))
    S = ctypes.c_double(0.0)
    rc = lib.oracle_forward_rowform_probs(pp, pr, len(read), ph, len(hap), ctypes.byref(S))
    if rc != 0:
        raise ValueError("oracle_forward_rowform_probs failed: %d" % rc)
    return S.value


def forward_one(read, bq, iq, dq, gq, hap, rescale: bool = False):
    """log10 P(read | hap) for one pair from raw Phred bytes.

    Returns (log10L, S, E)."""
    lib = _load()
    read, pr = _u8(_seq(read))
    bq, pb = _u8(bq)
    iq, pi = _u8(iq)
    dq, pd = _u8(dq)
    gq, pg = _u8(gq)
    hap, ph = _u8(_seq(hap))
    out = ctypes.c_double(0.0)
    S = ctypes.c_double(0.0)
    E = ctypes.c_int64(0)
    rc = lib.oracle_forward_one(pr, pb, pi, pd, pg, len(read), ph, len(hap), int(bool(rescale)),
                                ctypes.byref(out), ctypes.byref(S), ctypes.byref(E))
    if rc != 0:
        raise ValueError("oracle_forward_one failed: %d" % rc)
    return out.value, S.value, E.value


def forward_pairs(batch, pair_idx=None, rescale: bool = True) -> np.ndarray:
    """log10 likelihoods of (a subset of) the pairs of a CSR batch dict
    (keys: reads, base_quals, ins_quals, del_quals, gcp, read_offsets,
    haplotypes, hap_offsets, pair_list)."""
    lib = _load()
    pl = np.ascontiguousarray(batch["pair_list"], dtype=np.uint32).reshape(-1, 2)
    if pair_idx is not None:
        pl = np.ascontiguousarray(pl[np.asarray(pair_idx, dtype=np.int64)])
    ro = np.ascontiguousarray(batch["read_offsets"], dtype=np.uint64)
    ho = np.ascontiguousarray(batch["hap_offsets"], dtype=np.uint64)
    arrs = [_u8(batch[k]) for k in ("reads", "base_quals", "ins_quals", "del_quals", "gcp")]
    haps, ph = _u8(batch["haplotypes"])
    out = np.empty(len(pl), dtype=np.float64)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    rc = lib.oracle_forward_pairs(arrs[0][1], arrs[1][1], arrs[2][1], arrs[3][1], arrs[4][1],
                                  ro.ctypes.data_as(u64p), len(ro) - 1, ph,
                                  ho.ctypes.data_as(u64p), len(ho) - 1,
                                  pl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                  len(pl), int(bool(rescale)),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("oracle_forward_pairs failed: %d" % rc)
    return out
