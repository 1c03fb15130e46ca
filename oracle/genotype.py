"""Diploid genotype likelihoods from a read x haplotype likelihood matrix:
plain FP64 definition (test infrastructure only: used by the tests, the
smoke check and the benchmark's CPU baseline, never by the library).

Section 1 of the paper places a Bayesian genotyping step after the PairHMM,
which turns the read x haplotype likelihoods of an active region into the
most probable genotype, but does not spell the model out.  The reading taken
here is the diploid mixture model: a genotype is an unordered pair of
haplotypes a <= b, each read comes from either copy with probability 1/2,
and reads are independent, so

    P(reads | a, b) = prod_r ( P(r | a) / 2 + P(r | b) / 2 ),
    GL(a, b)        = sum_r log10( 10^L[r][a] / 2 + 10^L[r][b] / 2 ),

with L[r][h] = log10 P(read r | haplotype h).  Genotypes are listed in the
VCF order for ploidy 2 (index b(b+1)/2 + a).  With a flat prior the maximum
a posteriori genotype is the argmax of GL; ties go to the smaller index.

Each term is evaluated as written after taking the common factor 10^m,
m = max(L[r][a], L[r][b]), out of the sum (an exact identity), so that
likelihoods far below the FP64 range (long reads reach 10^-30000) stay
finite.  Pinned by brute force over every assignment of reads to haplotype
copies in exact rational arithmetic, and by closed forms (tests).
"""
from __future__ import annotations

import math

import numpy as np


def genotype_region(mat) -> np.ndarray:
    """GL of every genotype of one region; mat is the R x H matrix of log10
    likelihoods (float64).  Returns H(H+1)/2 values in VCF order."""
    mat = np.asarray(mat, dtype=np.float64)
    R, H = mat.shape
    out = []
    for b in range(H):
        for a in range(b + 1):
            total = 0.0
            for r in range(R):
                la, lb = float(mat[r, a]), float(mat[r, b])
                m = max(la, lb)
                total += m + math.log10(0.5 * 10.0 ** (la - m) + 0.5 * 10.0 ** (lb - m))
            out.append(total)
    return np.array(out, dtype=np.float64)


def best_genotype(gl) -> int:
    """Index of the largest GL, the smallest index on ties."""
    gl = np.asarray(gl)
    return int(np.argmax(gl)) if gl.size else 0


def genotype_batch(lk, lk_offsets, region_reads, region_haps, regions=None):
    """GL blocks and best genotype per region of a batch (the layout of the
    library's genotype call: region g's matrix is lk[lk_offsets[g] + r*H + h]).
    regions: indices to evaluate (default all).  Returns (list of GL arrays,
    array of best indices)."""
    idx = range(len(region_haps)) if regions is None else regions
    gls, best = [], []
    for g in idx:
        R, H, o = int(region_reads[g]), int(region_haps[g]), int(lk_offsets[g])
        gl = genotype_region(np.asarray(lk[o:o + R * H]).reshape(R, H))
        gls.append(gl)
        best.append(best_genotype(gl))
    return gls, np.array(best, dtype=np.int64)
