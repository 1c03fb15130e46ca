"""Pins of the genotype-likelihood oracle (no GPU): brute force over every
assignment of reads to haplotype copies in exact rational arithmetic, the
VCF genotype order, closed forms far below the FP64 range, and the
degenerate cases.  Also the library's host-side checks of the genotype
call, which run before any device work."""
import itertools
import math
import os
import sys
from fractions import Fraction

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import paper_2606_25738_amd as phmm  # noqa: E402
import synth  # noqa: E402


def brute_force(P):
    """log10 P(reads | a, b) for every genotype a <= b, VCF order: the sum
    over all 2^R ways to draw each read from copy 1 or copy 2 of the
    genotype (each way has probability 1/2^R), products of exact rationals."""
    R, H = len(P), len(P[0]) if P else 0
    out = []
    for b in range(H):
        for a in range(b + 1):
            total = Fraction(0)
            for origin in itertools.product((a, b), repeat=R):
                term = Fraction(1, 2 ** R)
                for r, h in enumerate(origin):
                    term *= P[r][h]
                total += term
            out.append(math.log10(total.numerator) - math.log10(total.denominator))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_matches_brute_force_over_read_origins(seed):
    rng = np.random.default_rng(seed)
    R, H = int(rng.integers(1, 7)), int(rng.integers(1, 6))
    # probabilities k / 2^e, far apart and close together
    P = [[Fraction(int(rng.integers(1, 1000)), 2 ** int(rng.integers(0, 60))) for _ in range(H)]
         for _ in range(R)]
    L = np.array([[math.log10(p.numerator) - math.log10(p.denominator) for p in row] for row in P])
    got = oracle.genotype_region(L)
    want = brute_force(P)
    assert len(got) == H * (H + 1) // 2
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_vcf_genotype_order_and_homozygous_values():
    # one read, three haplotypes: homozygous entries are the read's own values
    L = np.array([[0.0, -1.0, -2.0]])
    gl = oracle.genotype_region(L)
    # (0,0) (0,1) (1,1) (0,2) (1,2) (2,2)
    assert gl[0] == 0.0 and gl[2] == -1.0 and gl[5] == -2.0
    assert gl[1] == pytest.approx(math.log10((1 + 0.1) / 2), abs=1e-15)
    assert gl[3] == pytest.approx(math.log10((1 + 0.01) / 2), abs=1e-15)
    assert gl[4] == pytest.approx(math.log10((0.1 + 0.01) / 2), abs=1e-15)
    assert oracle.best_genotype(gl) == 0


def test_reads_add_up():
    # independent reads: the region's GL is the sum of one-read GLs
    rng = np.random.default_rng(7)
    L = -rng.uniform(0, 50, (9, 4))
    whole = oracle.genotype_region(L)
    parts = sum(oracle.genotype_region(L[r:r + 1]) for r in range(9))
    np.testing.assert_allclose(whole, parts, rtol=1e-14)


def test_far_below_fp64_range():
    # long-read likelihoods: 10^-30000 underflows FP64, the GL must not
    x = -30000.0
    L = np.array([[x, x - 0.5], [x - 0.5, x]] * 3)
    gl = oracle.genotype_region(L)
    het = x + math.log10((1 + 10 ** -0.5) / 2)
    assert gl[0] == 6 * x - 3 * 0.5 and gl[2] == 6 * x - 3 * 0.5
    assert gl[1] == pytest.approx(6 * het, rel=1e-14)
    # a read far better explained by one haplotype: log10(1/2) below it
    gl = oracle.genotype_region(np.array([[-5.0, -900.0]]))
    assert gl[1] == pytest.approx(-5.0 - math.log10(2.0), abs=1e-14)
    assert np.all(np.isfinite(gl))


def test_no_reads_and_ties():
    gl = oracle.genotype_region(np.zeros((0, 4)))
    assert gl.shape == (10,) and np.all(gl == 0.0)
    assert oracle.best_genotype(gl) == 0
    gl = oracle.genotype_region(np.array([[-1.0, -1.0]]))
    assert np.all(gl == -1.0) and oracle.best_genotype(gl) == 0


def test_planted_mistakes_fail_the_pins():
    """Plausible mistakes in the oracle's term (a dropped 1/2, copies
    weighted unevenly, operands from the wrong read) each fail the brute
    force."""
    rng = np.random.default_rng(3)
    P = [[Fraction(int(rng.integers(1, 100)), 2 ** int(rng.integers(0, 20))) for _ in range(3)]
         for _ in range(4)]
    L = np.array([[math.log10(p.numerator) - math.log10(p.denominator) for p in row] for row in P])
    want = np.array(brute_force(P))

    def region(term):
        out = []
        for b in range(3):
            for a in range(b + 1):
                out.append(sum(term(L, r, a, b) for r in range(4)))
        return np.array(out)

    def no_half(L, r, a, b):
        return math.log10(10 ** L[r, a] + 10 ** L[r, b])

    def uneven(L, r, a, b):
        return math.log10(0.75 * 10 ** L[r, a] + 0.25 * 10 ** L[r, b])

    def wrong_read(L, r, a, b):
        return math.log10(0.5 * 10 ** L[r, a] + 0.5 * 10 ** L[(r + 1) % 4, b])

    def right(L, r, a, b):
        return math.log10(0.5 * 10 ** L[r, a] + 0.5 * 10 ** L[r, b])

    np.testing.assert_allclose(region(right), want, atol=1e-12)
    for bad in (no_half, uneven, wrong_read):
        assert np.max(np.abs(region(bad) - want)) > 1e-6, bad.__name__


def test_batch_layout():
    lk, off, R, H = synth.genotype_lk(5, 12, reads=(0, 8), haps=(1, 5))
    gls, best = oracle.genotype_batch(lk, off, R, H)
    for g in range(12):
        o, r, h = int(off[g]), int(R[g]), int(H[g])
        np.testing.assert_array_equal(gls[g], oracle.genotype_region(lk[o:o + r * h].reshape(r, h)))
        assert best[g] == int(np.argmax(gls[g]))


# ---------------------------------------------------------------- host checks of the library

def _expect(match, *args, **kw):
    with pytest.raises(phmm.PhmmError) as e:
        phmm.phmm_genotype_batch(None, *args, **kw)
    assert e.value.code == phmm.PHMM_EINVAL
    assert match in str(e.value), str(e.value)


def test_library_checks_inputs_before_the_context():
    lk = -np.arange(12, dtype=np.float64)
    _expect("NULL ctx", lk, [0, 6], [2, 1], [3, 6])
    _expect("region 1: 0 haplotypes", lk, [0, 6], [2, 1], [3, 0])
    _expect("region 0: 513 haplotypes", lk, [0], [0], [513])
    _expect("region 1: likelihoods [6, +8)", lk, [0, 6], [2, 2], [3, 4])
    _expect("region 0: genotypes [5, +6)", lk, [0], [2], [3], gl_offsets=[5], gl=np.zeros(10))
    bad = lk.copy()
    bad[7] = np.nan
    _expect("region 1: lk[7] is not finite", bad, [0, 6], [2, 1], [3, 6])
    bad[7] = -np.inf
    _expect("lk[7]", bad, [0, 6], [2, 1], [3, 6])
    # a value outside every region is not looked at
    bad = np.concatenate([lk, [np.nan]])
    _expect("NULL ctx", bad, [0, 6], [2, 1], [3, 6])
