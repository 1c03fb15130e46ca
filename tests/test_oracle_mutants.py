"""The oracle pins must catch plausible mistakes.

Each case copies the oracle's C source, plants one mistake with a textual
edit, compiles the copy with gcc into a temporary directory and runs the
brute-force and closed-form pins against it.  Every planted mistake must be
caught by at least one pin.  Nothing here touches the GPU.
"""
import ctypes
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402

SRC = os.path.join(ROOT, "oracle", "phmm_oracle.c")
GOLDEN = os.path.join(ROOT, "tests", "golden", "exact_small.txt")

MUTANTS = {
    "tIM_replaced_by_tDM": ("double b = pr[P_TIM] * Ip[j - 1];",
                            "double b = pr[P_TDM] * Ip[j - 1];"),
    "diagonal_index": ("double a = pr[P_TMM] * Mp[j - 1];", "double a = pr[P_TMM] * Mp[j];"),
    "insert_uses_tMD": ("Ic[j] = pr[P_TMI] * Mp[j] + pr[P_TII] * Ip[j];",
                        "Ic[j] = pr[P_TMD] * Mp[j] + pr[P_TII] * Ip[j];"),
    "dropped_delete_term": ("Mc[j] = p * ((a + b) + c);", "Mc[j] = p * (a + b);"),
    "delete_from_previous_row": ("Dc[j] = pr[P_TMD] * Mc[j - 1] + pr[P_TDD] * Dc[j - 1];",
                                 "Dc[j] = pr[P_TMD] * Mp[j - 1] + pr[P_TDD] * Dc[j - 1];"),
    "divisor_k_plus_1": ("return ldexp(1.0, 1020) / (double)k;",
                         "return ldexp(1.0, 1020) / (double)(k + 1);"),
    "mismatch_prior_033": ("r[P_PX] = eps / 3.0;", "r[P_PX] = eps * 0.33;"),
    "mismatch_prior_eps": ("r[P_PX] = eps / 3.0;", "r[P_PX] = eps;"),
    "missing_clamp": ("if (tmm < 0.0) tmm = 0.0;", ""),
    "clamp_at_one_minus_ins": ("if (tmm < 0.0) tmm = 0.0;", "if (tmm < 0.0) tmm = 1.0 - tmi;"),
    "final_sum_without_I": ("for (int j = 1; j <= k; ++j) s = s + (Mp[j] + Ip[j]);\n    *S = s;\n    *E = ex;",
                            "for (int j = 1; j <= k; ++j) s = s + Mp[j];\n    *S = s;\n    *E = ex;"),
    "D00_zero": ("Mc[0] = 0.0; Ic[0] = 0.0; Dc[0] = 0.0;\n        for (int j = 1; j <= k; ++j) {\n            double p = emission(pr, r, hap[j - 1]);\n            double a",
                 "Mc[0] = 0.0; Ic[0] = 0.0; Dc[0] = 0.0;\n        if (i == 1) Dp[0] = 0.0;\n        for (int j = 1; j <= k; ++j) {\n            double p = emission(pr, r, hap[j - 1]);\n            double a"),
    "wrong_row_priors_for_delete": ("Dc[j] = pr[P_TMD] * Mc[j - 1]",
                                    "Dc[j] = (i > 1 ? pr[P_TMD - P_NREC] : pr[P_TMD]) * Mc[j - 1]"),
}


def build_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    path = tmp_path / ("m_%s.c" % name)
    # the first occurrence is the row-order pass the pins exercise
    path.write_text(src.replace(old, new, 1))
    so = tmp_path / ("m_%s.so" % name)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared",
                    str(path), "-o", str(so), "-lm"], check=True)
    lib = ctypes.CDLL(str(so))
    P = ctypes.POINTER
    lib.oracle_forward_probs.argtypes = [P(ctypes.c_double), P(ctypes.c_uint8), ctypes.c_int,
                                         P(ctypes.c_uint8), ctypes.c_int, ctypes.c_int,
                                         P(ctypes.c_double), P(ctypes.c_int64)]
    lib.oracle_forward_one.argtypes = [P(ctypes.c_uint8)] * 5 + [ctypes.c_int, P(ctypes.c_uint8),
                                                                 ctypes.c_int, ctypes.c_int,
                                                                 P(ctypes.c_double),
                                                                 P(ctypes.c_double),
                                                                 P(ctypes.c_int64)]
    return lib


def _u8(b):
    a = np.frombuffer(bytes(b), dtype=np.uint8).copy()
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def run_pins(lib):
    """Returns True when every pin passes (i.e. the mistake went unnoticed)."""
    rng = np.random.default_rng(5)
    for _ in range(6):
        l, k = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        read = bytes(np.frombuffer(b"AC", np.uint8)[rng.integers(0, 2, l)])
        hap = bytes(np.frombuffer(b"AC", np.uint8)[rng.integers(0, 2, k)])
        pri = np.column_stack([rng.uniform(a, b, l) for a, b in
                               [(0.55, 0.99), (0.002, 0.15), (0.5, 0.95), (0.3, 0.95),
                                (0.3, 0.95), (0.01, 0.3), (0.05, 0.6), (0.01, 0.3),
                                (0.05, 0.6)]])
        pri = np.ascontiguousarray(pri)
        ra, rp = _u8(read)
        ha, hp = _u8(hap)
        S, E = ctypes.c_double(), ctypes.c_int64()
        lib.oracle_forward_probs(pri.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), rp, l,
                                 hp, k, 0, ctypes.byref(S), ctypes.byref(E))
        got = math.ldexp(S.value, E.value - 1020)
        want = exact.brute_force(pri.tolist(), read, hap)
        if not math.isclose(got, want, rel_tol=1e-12):
            return False
    # closed form of a one-base read from Phred bytes (eq.3)
    out, S, E = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    ra, rp = _u8(b"A")
    args = [_u8(bytes([v])) for v in (20, 45, 45, 10)]
    ha, hp = _u8(b"ACA")
    lib.oracle_forward_one(rp, *[a[1] for a in args], 1, hp, 3, 0, ctypes.byref(out),
                           ctypes.byref(S), ctypes.byref(E))
    want = math.log10(0.9 / 3 * (2 * (1 - 0.01) + 0.01 / 3))
    if abs(out.value - want) >= 1e-12:
        return False
    # exact rational likelihoods from Phred bytes (tests/golden/exact_small.txt),
    # including rows whose T_MI + T_MD exceeds 1 (clamped T_MM)
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        read, hap, bq, iq, dq, gq, lg, _ = line.split()
        ra, rp = _u8(read.encode())
        ha, hp = _u8(hap.encode())
        q = [_u8(bytes(int(x) for x in v.split(","))) for v in (bq, iq, dq, gq)]
        lib.oracle_forward_one(rp, *[a[1] for a in q], len(read), hp, len(hap), 0,
                               ctypes.byref(out), ctypes.byref(S), ctypes.byref(E))
        if not abs(out.value - float(lg)) < 1e-12:
            return False
    return True


def test_unmutated_copy_passes(tmp_path):
    MUTANTS["__none__"] = ("static int is_match", "static int is_match")
    try:
        lib = build_mutant(tmp_path, "__none__")
    finally:
        del MUTANTS["__none__"]
    assert run_pins(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    lib = build_mutant(tmp_path, name)
    assert not run_pins(lib), "pins did not catch mutant %s" % name
