"""Writes tests/golden/exact_small.txt: exact likelihoods of tiny pairs.

Uses only the oracle package's exact path-sum evaluator (Fractions).  Phred
values that are multiples of 10 give exact rational priors (eq.3:
10^(-Q/10) = 1/10, 1/100, ...; gap continuation 10 gives the paper's
T_II = T_DD = 1/10 and T_IM = T_DM = 9/10), so every stored value is the
exact likelihood of the paper's Section 2 model, written as a fraction and
as log10 to 30 significant digits.

Run:  python tests/golden/make_golden.py
"""
import os
import sys
from decimal import Decimal, getcontext
from fractions import Fraction

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import exact  # noqa: E402

CASES = [
    # read, hap, base quals, ins quals, del quals, gcp
    ("A", "ACA", [20], [40], [40], [10]),
    ("AC", "AC", [30, 30], [40, 40], [40, 40], [10, 10]),
    ("ACG", "AGCG", [20, 10, 30], [40, 30, 40], [40, 40, 30], [10, 10, 10]),
    ("GATTA", "GATA", [30, 20, 20, 30, 40], [30] * 5, [30] * 5, [10, 20, 10, 10, 10]),
    ("TTAC", "GTTACA", [10, 20, 30, 40], [40, 40, 40, 40], [40, 40, 40, 40], [10] * 4),
    ("NACG", "ACGN", [20, 20, 20, 20], [30] * 4, [30] * 4, [10] * 4),
    ("CCCCCC", "CCCC", [40] * 6, [10] * 6, [10] * 6, [10] * 6),
    # insertion and/or deletion Phred 0: T_MI or T_MD = 1, so 1 - T_MI - T_MD
    # is negative and T_MM is clamped to 0 on those rows
    ("ACGT", "ACGTA", [20, 30, 20, 10], [0, 40, 40, 30], [40, 0, 40, 30], [10, 10, 10, 20]),
    ("GGA", "GAGA", [30, 30, 30], [0, 0, 10], [0, 20, 0], [10, 10, 10]),
    ("TAC", "TAC", [40, 10, 40], [10, 0, 10], [0, 10, 10], [10, 20, 10]),
]


def prob(q):
    return Fraction(1, 10 ** (q // 10))


def priors(bq, iq, dq, gq):
    rows = []
    for b, i, d, g in zip(bq, iq, dq, gq):
        assert b % 10 == 0 and i % 10 == 0 and d % 10 == 0 and g % 10 == 0
        eps, tmi, tmd, gg = prob(b), prob(i), prob(d), prob(g)
        tmm = max(Fraction(0), 1 - (tmi + tmd))  # clamped at 0 (T_MI + T_MD may exceed 1)
        rows.append([1 - eps, eps / 3, tmm, 1 - gg, 1 - gg, tmi, gg, tmd, gg])
    return rows


def log10_frac(x: Fraction) -> Decimal:
    getcontext().prec = 50
    return (Decimal(x.numerator).ln() - Decimal(x.denominator).ln()) / Decimal(10).ln()


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_small.txt")
    with open(out, "w") as f:
        f.write("# Exact PairHMM likelihoods (paper Section 2, eq.1-4) of tiny pairs.\n")
        f.write("# Written by tests/golden/make_golden.py from the oracle's exact path sum.\n")
        f.write("# read hap bq iq dq gcp log10L numerator/denominator\n")
        for read, hap, bq, iq, dq, gq in CASES:
            L = exact.dag_sum(priors(bq, iq, dq, gq), read.encode(), hap.encode())
            lg = log10_frac(L)
            f.write("%s %s %s %s %s %s %s %d/%d\n" % (
                read, hap, ",".join(map(str, bq)), ",".join(map(str, iq)),
                ",".join(map(str, dq)), ",".join(map(str, gq)),
                format(lg, ".30g"), L.numerator, L.denominator))
    print("wrote", out)


if __name__ == "__main__":
    main()
