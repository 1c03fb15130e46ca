"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  The oracle (row-order pull recurrences of
the paper's eq.1-4) is checked against independent computations:

P1  brute-force enumeration of every alignment path (tiny inputs)
P2  exact rational path sums over the state DAG (Fractions)
P3  the anti-diagonal evaluation order (bit-exact)
P4  closed form for a one-base read
P5  the ungapped limit (only diagonal paths survive)
P6  the row-level formulation of Section 3.1 (eq.7) evaluated literally
P7  power-of-two rescaling leaves the mantissas untouched
P8  invariants: L <= T_DM_1, L >= weight of the generator's true path,
    L affine in eps_i, alphabet relabelling, determinism
"""
import math
import os
import sys
from fractions import Fraction

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from oracle import exact  # noqa: E402
import synth  # noqa: E402

ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)
TWO1020 = math.ldexp(1.0, 1020)


def rand_seq(rng, n, alphabet=b"ACGT"):
    a = np.frombuffer(alphabet, dtype=np.uint8)
    return bytes(a[rng.integers(0, len(a), n)])


def rand_priors(rng, l, tied=False):
    """Independent random probabilities for each of the 9 per-row values, so
    that a swapped or misplaced prior changes the result."""
    pri = np.empty((l, 9))
    pri[:, 0] = rng.uniform(0.55, 0.99, l)   # pm
    pri[:, 1] = rng.uniform(0.002, 0.15, l)  # px
    pri[:, 2] = rng.uniform(0.5, 0.95, l)    # tMM
    pri[:, 3] = rng.uniform(0.3, 0.95, l)    # tIM
    pri[:, 4] = rng.uniform(0.3, 0.95, l)    # tDM
    pri[:, 5] = rng.uniform(0.01, 0.3, l)    # tMI
    pri[:, 6] = rng.uniform(0.05, 0.6, l)    # tII
    pri[:, 7] = rng.uniform(0.01, 0.3, l)    # tMD
    pri[:, 8] = rng.uniform(0.05, 0.6, l)    # tDD
    if tied:
        pri[:, 8] = pri[:, 6]
        pri[:, 4] = pri[:, 3]
    return pri


def L_from(S, E=0):
    return math.ldexp(S, E - 1020)


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("seed", range(12))
def test_p1_brute_force_enumeration(seed):
    rng = np.random.default_rng(100 + seed)
    l = int(rng.integers(1, 6))
    k = int(rng.integers(1, 6))
    alphabet = b"ACGTN" if seed % 3 == 0 else b"AC"
    read, hap = rand_seq(rng, l, alphabet), rand_seq(rng, k, alphabet)
    pri = rand_priors(rng, l)
    S, E = oracle.forward_probs(pri, read, hap)
    want = exact.brute_force(pri.tolist(), read, hap)
    assert want > 0
    assert L_from(S, E) == pytest.approx(want, rel=1e-12)


def test_p1_enumeration_is_not_trivial():
    # many distinct paths exist even for a 4x4 grid
    assert exact.count_paths(4, 4) > 20
    assert exact.count_paths(5, 6) > exact.count_paths(4, 4)
    assert exact.count_paths(1, 3) == 3


# ---------------------------------------------------------------- P2
def dyadic(rng, lo, hi, bits=12):
    return Fraction(int(rng.integers(int(lo * 2**bits), int(hi * 2**bits))), 2**bits)


@pytest.mark.parametrize("seed,l,k", [(0, 7, 9), (1, 12, 10), (2, 20, 24), (3, 30, 18)])
def test_p2_exact_rational(seed, l, k):
    rng = np.random.default_rng(200 + seed)
    read, hap = rand_seq(rng, l), rand_seq(rng, k)
    ranges = [(0.55, 0.99), (0.002, 0.15), (0.5, 0.95), (0.3, 0.95), (0.3, 0.95),
              (0.01, 0.3), (0.05, 0.6), (0.01, 0.3), (0.05, 0.6)]
    fr = [[dyadic(rng, a, b) for a, b in ranges] for _ in range(l)]
    pri = np.array([[float(x) for x in row] for row in fr])  # exact: dyadic
    S, E = oracle.forward_probs(pri, read, hap)
    want = exact.dag_sum(fr, read, hap)
    assert isinstance(want, Fraction) and want > 0
    rel = abs(Fraction(L_from(S, E)) - want) / want
    assert rel < Fraction(1, 10**13)


def test_p2_dag_sum_equals_enumeration():
    rng = np.random.default_rng(7)
    for _ in range(5):
        l, k = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        read, hap = rand_seq(rng, l), rand_seq(rng, k)
        pri = rand_priors(rng, l).tolist()
        assert exact.dag_sum(pri, read, hap) == pytest.approx(exact.brute_force(pri, read, hap),
                                                              rel=1e-13)


# ---------------------------------------------------------------- P3
@pytest.mark.parametrize("seed", range(6))
def test_p3_antidiagonal_bit_exact(seed):
    rng = np.random.default_rng(300 + seed)
    l, k = int(rng.integers(1, 60)), int(rng.integers(1, 80))
    read, hap = rand_seq(rng, l), rand_seq(rng, k)
    pri = rand_priors(rng, l)
    S, E = oracle.forward_probs(pri, read, hap)
    assert E == 0
    assert oracle.forward_antidiag_probs(pri, read, hap) == S  # bit for bit


# ---------------------------------------------------------------- P4
@pytest.mark.parametrize("seed", range(5))
def test_p4_single_base_read_closed_form(seed):
    rng = np.random.default_rng(400 + seed)
    k = int(rng.integers(1, 40))
    read, hap = rand_seq(rng, 1), rand_seq(rng, k)
    pri = rand_priors(rng, 1)
    n_match = sum(1 for h in hap if h == read[0])
    want = pri[0, 4] / k * (n_match * pri[0, 0] + (k - n_match) * pri[0, 1])
    S, E = oracle.forward_probs(pri, read, hap)
    assert L_from(S, E) == pytest.approx(want, rel=1e-14)


def test_p4_phred_entry_matches_eq3():
    # Q = 20 -> eps = 0.01, gcp 10 -> T_DM = 0.9 ; read 'A' vs hap 'ACA'
    lg, S, E = oracle.forward_one(b"A", [20], [45], [45], [10], b"ACA")
    want = 0.9 / 3 * (2 * (1 - 0.01) + 1 * (0.01 / 3))
    assert lg == pytest.approx(math.log10(want), abs=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_p4_zero_start_gives_zero_likelihood(seed):
    """eq.1-2: row 1 is M(1,j) = P(r_1|h_j) T_DM_1 D(0,j-1), I(1,j) = 0, and
    every later cell descends from row 1, so L = 0 exactly when T_DM_1 = 0
    (gap byte 0 on the first read position), whatever the other rows hold;
    a gap byte of 0 on any other row leaves L > 0."""
    rng = np.random.default_rng(440 + seed)
    l, k = int(rng.integers(1, 30)), int(rng.integers(1, 40))
    read = bytes(rng.choice(np.frombuffer(b"ACGTN", np.uint8), l))
    hap = bytes(rng.choice(np.frombuffer(b"ACGTN", np.uint8), k))
    q = [rng.integers(0, 60, l).astype(np.uint8) for _ in range(3)]
    g = rng.integers(1, 60, l).astype(np.uint8)
    g0 = g.copy()
    g0[0] = 0
    lg, S, E = oracle.forward_one(read, q[0], q[1], q[2], g0, hap)
    assert S == 0.0 and lg == -math.inf
    if l > 1:
        g1 = g.copy()
        g1[int(rng.integers(1, l))] = 0
        lg, S, E = oracle.forward_one(read, q[0], q[1], q[2], g1, hap)
        assert S > 0.0 and math.isfinite(lg)


# ---------------------------------------------------------------- P5
@pytest.mark.parametrize("seed", range(5))
def test_p5_ungapped_limit(seed):
    rng = np.random.default_rng(500 + seed)
    l = int(rng.integers(2, 25))
    k = int(rng.integers(l, l + 30))
    read, hap = rand_seq(rng, l), rand_seq(rng, k)
    pri = rand_priors(rng, l)
    pri[:, 5] = 0.0  # T_MI
    pri[:, 7] = 0.0  # T_MD
    S, E = oracle.forward_probs(pri, read, hap)

    def p(i, j):  # 1-based
        return pri[i - 1, 0] if read[i - 1] == hap[j - 1] else pri[i - 1, 1]
    want = 0.0
    for j0 in range(0, k - l + 1):
        w = pri[0, 4] / k * p(1, j0 + 1)
        for i in range(2, l + 1):
            w *= pri[i - 1, 2] * p(i, j0 + i)
        want += w
    assert L_from(S, E) == pytest.approx(want, rel=1e-13)


# ---------------------------------------------------------------- P6
@pytest.mark.parametrize("seed", range(6))
def test_p6_row_formulation_eq7(seed):
    rng = np.random.default_rng(600 + seed)
    l, k = int(rng.integers(1, 50)), int(rng.integers(1, 70))
    read, hap = rand_seq(rng, l), rand_seq(rng, k)
    pri = rand_priors(rng, l)
    S, _ = oracle.forward_probs(pri, read, hap)
    assert oracle.forward_rowform_probs(pri, read, hap) == pytest.approx(S, rel=1e-12)


# ---------------------------------------------------------------- P7
@pytest.mark.parametrize("seed", range(4))
def test_p7_rescaling_is_exact(seed):
    rng = np.random.default_rng(700 + seed)
    l, k = int(rng.integers(5, 80)), int(rng.integers(5, 120))
    read, hap = rand_seq(rng, l), rand_seq(rng, k)
    pri = rand_priors(rng, l)
    S0, E0 = oracle.forward_probs(pri, read, hap, rescale=False)
    S1, E1 = oracle.forward_probs(pri, read, hap, rescale=True)
    assert E0 == 0 and E1 != 0
    assert S0 > 1e-250  # no underflow in the unrescaled run
    m0, e0 = math.frexp(S0)
    m1, e1 = math.frexp(S1)
    assert m0 == m1  # identical mantissas
    assert e0 == e1 + E1


def test_p7_rescaling_extends_range():
    # i.i.d. 1500 bp pair: log10 L far below the FP64 range of 2^1020 start
    rng = np.random.default_rng(77)
    l, k = 1500, 1600
    read, hap = rand_seq(rng, l), rand_seq(rng, k)
    q = rng.integers(20, 40, l).astype(np.uint8)
    c45 = np.full(l, 45, np.uint8)
    c10 = np.full(l, 10, np.uint8)
    lg_plain, _, _ = oracle.forward_one(read, q, c45, c45, c10, hap, rescale=False)
    lg_res, _, E = oracle.forward_one(read, q, c45, c45, c10, hap, rescale=True)
    assert lg_plain == -math.inf
    assert math.isfinite(lg_res) and lg_res < -700 and E < 0


# ---------------------------------------------------------------- P8
def test_p8_bounds_and_true_path():
    b = synth.generate("one_region", with_cols=True)
    ro, ho = b["read_offsets"], b["hap_offsets"]
    pl = b["pair_list"]
    checked = 0
    for p in range(0, len(pl), 7):
        r, h = pl[p]
        sl = slice(int(ro[r]), int(ro[r + 1]))
        read = b["reads"][sl]
        hap = b["haplotypes"][int(ho[h]):int(ho[h + 1])]
        pri = oracle.priors(b["base_quals"][sl], b["ins_quals"][sl], b["del_quals"][sl],
                            b["gcp"][sl])
        S, E = oracle.forward_probs(pri, read, hap)
        L = L_from(S, E)
        assert 0 < L <= pri[0, 4]
        # the generator drew read r from one hap of the region; its true path
        # is a lower bound of the likelihood against that hap only
        cols = b["cols"][sl]
        if (cols < 0).any():
            continue
        w = exact.path_weight(pri.tolist(), bytes(read), bytes(hap), [int(c) for c in cols])
        if w is not None:
            # cols refer to the source hap; only a lower bound when it is h
            matches = sum(1 for i, c in enumerate(cols) if c > 0 and read[i] == hap[c - 1])
            if matches >= 0.9 * len(read):
                assert L >= w * (1 - 1e-12)
                checked += 1
    assert checked > 5


@pytest.mark.parametrize("seed", range(4))
def test_p8_affine_in_eps(seed):
    rng = np.random.default_rng(800 + seed)
    l, k = int(rng.integers(2, 30)), int(rng.integers(2, 40))
    read, hap = rand_seq(rng, l), rand_seq(rng, k)
    pri = rand_priors(rng, l)
    i = int(rng.integers(0, l))
    vals = []
    eps = [0.01, 0.2, 0.45]
    for e in eps:
        q = pri.copy()
        q[i, 0] = 1 - e
        q[i, 1] = e / 3
        vals.append(L_from(*oracle.forward_probs(q, read, hap)))
    slope1 = (vals[1] - vals[0]) / (eps[1] - eps[0])
    slope2 = (vals[2] - vals[1]) / (eps[2] - eps[1])
    assert slope1 == pytest.approx(slope2, rel=1e-9, abs=1e-300)


def test_p8_monotone_cases():
    rng = np.random.default_rng(81)
    l, k = 12, 15
    hap = b"A" * k
    read = bytearray(rand_seq(rng, l, b"CG"))
    read[5] = ord("A")  # matches every hap base
    base = rng.integers(10, 40, l).astype(np.uint8)
    c45 = np.full(l, 45, np.uint8)
    c10 = np.full(l, 10, np.uint8)
    prev = -math.inf
    for q in range(2, 60, 3):
        bq = base.copy()
        bq[5] = q
        lg, _, _ = oracle.forward_one(bytes(read), bq, c45, c45, c10, hap)
        assert lg >= prev
        prev = lg
    prev = math.inf
    for q in range(2, 60, 3):  # read base 3 (C or G) matches no hap base
        bq = base.copy()
        bq[3] = q
        lg, _, _ = oracle.forward_one(bytes(read), bq, c45, c45, c10, hap)
        assert lg <= prev
        prev = lg


def test_p8_relabelling_bit_exact():
    rng = np.random.default_rng(82)
    l, k = 40, 55
    read, hap = rand_seq(rng, l), rand_seq(rng, k)
    pri = rand_priors(rng, l)
    perm = bytes.maketrans(b"ACGT", b"GTCA")
    a = oracle.forward_probs(pri, read, hap)
    b = oracle.forward_probs(pri, read.translate(perm), hap.translate(perm))
    assert a == b


def test_p8_N_matches_anything():
    q = ([30] * 3, [45] * 3, [45] * 3, [10] * 3)
    # an all-N read matches every haplotype equally well
    a = [oracle.forward_one(b"NNN", *q, h)[0] for h in (b"ACA", b"GGT", b"TCA", b"AAA")]
    assert a[0] == a[1] == a[2] == a[3]
    # an all-N haplotype makes the read content irrelevant
    b = [oracle.forward_one(r, *q, b"NNNN")[0] for r in (b"ACA", b"AGA", b"TTA", b"AAA")]
    assert b[0] == b[1] == b[2] == b[3]
    # and an N column always emits the match prior
    assert oracle.forward_one(b"AAA", *q, b"ANA")[0] == oracle.forward_one(b"AAA", *q, b"AAA")[0]


def test_oracle_rescaled_matches_plain_on_one_region():
    b = synth.generate("one_region")
    idx = np.arange(0, 512, 5)
    plain = oracle.forward_pairs(b, idx, rescale=False)
    resc = oracle.forward_pairs(b, idx, rescale=True)
    assert np.all(np.isfinite(plain))
    np.testing.assert_allclose(resc, plain, rtol=0, atol=1e-11)


def test_golden_exact_small():
    """Exact rational likelihoods of tiny pairs (tests/golden/exact_small.txt,
    written by tests/golden/make_golden.py from the exact path sum)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "exact_small.txt")
    n = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        read, hap, bq, iq, dq, gq, lg, frac = line.split()
        arr = [np.array([int(x) for x in v.split(",")], np.uint8) for v in (bq, iq, dq, gq)]
        got, _, _ = oracle.forward_one(read.encode(), *arr, hap.encode())
        assert got == pytest.approx(float(lg), abs=1e-13)
        num, den = (int(x) for x in frac.split("/"))
        assert got == pytest.approx(math.log10(num) - math.log10(den), abs=1e-12)
        n += 1
    assert n >= 7
