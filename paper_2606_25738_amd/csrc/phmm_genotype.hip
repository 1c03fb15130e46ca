// Diploid genotype likelihoods from the read x haplotype likelihood matrix of
// an active region: the Bayesian genotyping stage that consumes the PairHMM
// output (Section 1 names it as the step after the PairHMM).
//
// For a region with R reads, H haplotypes and L[r][h] = log10 P(read r | hap h),
// the genotype made of haplotypes a <= b (a diploid sample: each read comes
// from either copy with probability 1/2) has
//
//   GL(a,b) = sum_r log10( P(r|a)/2 + P(r|b)/2 ),
//
// stored at index b(b+1)/2 + a of the region's genotype block (the genotype
// order of the VCF format for ploidy 2).  best = argmax GL, the smallest
// index on ties: the maximum a posteriori genotype under a flat prior.
//
// Evaluation.  Per read, m = max_h L[r][h] and p[h] = 10^(L[r][h] - m) are
// formed once (H powers per read), so that read r contributes
//   m + log10 f,   f = (p[a] + p[b]) / 2  in (0, 1].
// The factors f of a genotype's reads are multiplied into a mantissa kept in
// [1/2, 1) by frexp, whose exponents are summed as integers:
//   GL = sum_r m + log10(mantissa) + exponent * log10 2,
// one logarithm per genotype instead of one per read, the same value up to
// rounding.  Where a read's p[a] + p[b] underflows (both haplotypes more than
// 290 orders of magnitude below the read's best) its term is added as
//   max(La, Lb) + log10(1 + 10^-|La - Lb|) - log10 2
// instead, so that no likelihood leaves the FP64 range (they reach -3e4 for
// long reads).
//
// Work mapping: one wavefront per region (grid-stride over regions).  The
// powers p of a chunk of whole reads and their maxima m are staged in LDS
// (underflowing terms read L itself, from the cache).  Genotypes are taken 64
// per pass; a pass of rem < 64 genotypes (a small region, or the last pass of
// a larger one) splits the wavefront into 64 / gw groups of gw >= rem lanes
// (gw a power of two), group k taking the reads k, k + 64/gw, ... of every
// genotype, and adds the groups' log-likelihoods at the end.  The arithmetic
// is FP64 (the powers, then a multiply, frexp and two adds per read and
// genotype), so the kernel is bound by VALU issue.
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include <hip/hip_runtime.h>

#include "phmm.h"

namespace phmm {

constexpr int kGtLane = 64;
constexpr uint32_t kGtLds = 1024;    // matrix entries staged per chunk (>= PHMM_GT_MAX_HAPS)
constexpr uint32_t kGtReads = 128;   // reads staged per chunk at most

// b = the largest integer with b(b+1)/2 <= g, a = g - b(b+1)/2.
__device__ inline void genotype_pair(uint32_t g, uint32_t& a, uint32_t& b)
{
    uint32_t t = (uint32_t)((sqrt(8.0 * (double)g + 1.0) - 1.0) * 0.5);
    while ((uint64_t)(t + 1) * (t + 2) / 2 <= g) ++t;
    while ((uint64_t)t * (t + 1) / 2 > g) --t;
    b = t;
    a = g - t * (t + 1) / 2;
}

constexpr double kLog10Of2 = 0.30102999566398119521;
constexpr double kInvLn10 = 0.43429448190325182765;

__global__ __launch_bounds__(kGtLane) void genotype_kernel(
    const double* __restrict__ lk, uint64_t n_lk, const uint64_t* __restrict__ lk_off,
    const uint32_t* __restrict__ n_reads, const uint32_t* __restrict__ n_haps,
    const uint64_t* __restrict__ gl_off, uint32_t n_regions, double* __restrict__ gl,
    uint64_t n_gl, uint32_t* __restrict__ best)
{
    __shared__ double s_p[kGtLds];    // 10^(L - m) of the staged reads
    __shared__ double s_m[kGtReads];  // m per staged read
    const uint32_t lane = threadIdx.x;
    for (uint32_t reg = blockIdx.x; reg < n_regions; reg += gridDim.x) {
        const uint64_t lo = lk_off[reg];
        const uint64_t go = gl_off[reg];
        const uint32_t R = n_reads[reg];
        const uint32_t H = n_haps[reg];
        const uint64_t G = (uint64_t)H * (H + 1) / 2;
        const bool ok = H >= 1 && H <= PHMM_GT_MAX_HAPS && lo <= n_lk &&
                        (uint64_t)R * H <= n_lk - lo && go <= n_gl && G <= n_gl - go;
        if (!ok) {  // block outside the arrays: nothing read or written but best
            if (lane == 0) best[reg] = 0xFFFFFFFFu;
            continue;
        }
        // >= 1 since H <= PHMM_GT_MAX_HAPS <= kGtLds
        const uint32_t rchunk = min(kGtLds / H, kGtReads);
        uint32_t staged_r0 = 0xFFFFFFFFu;     // first read of the chunk in LDS
        double bv = -INFINITY;
        uint32_t bi = 0xFFFFFFFFu;
        for (uint64_t g0 = 0; g0 < G; g0 += kGtLane) {
            // genotypes g0 .. g0 + rem - 1 in this pass, on groups of gw lanes
            const uint32_t rem = (uint32_t)min(G - g0, (uint64_t)kGtLane);
            uint32_t gw = 1;
            while (gw < rem) gw <<= 1;
            const uint32_t groups = kGtLane / gw;
            const uint32_t sub = lane & (gw - 1);
            const uint32_t grp = lane / gw;
            const uint64_t gi = g0 + sub;
            const bool act = sub < rem;
            uint32_t a = 0, b = 0;
            if (act) genotype_pair((uint32_t)gi, a, b);
            double add = 0.0;   // sum of m, and of the underflowing reads' terms
            double mant = 1.0;  // product of the other factors f, in [1/2, 1)
            int ex = 0;         // ... times 2^ex
            for (uint32_t r0 = 0; r0 < R; r0 += rchunk) {
                const uint32_t rn = min(rchunk, R - r0);
                if (staged_r0 != r0) {
                    __syncthreads();
                    const double* src = lk + lo + (uint64_t)r0 * H;
                    for (uint32_t t = lane; t < rn * H; t += kGtLane) s_p[t] = src[t];
                    __syncthreads();
                    for (uint32_t r = lane; r < rn; r += kGtLane) {
                        double m = s_p[r * H];
                        for (uint32_t h = 1; h < H; ++h) m = fmax(m, s_p[r * H + h]);
                        s_m[r] = m;
                    }
                    __syncthreads();
                    for (uint32_t t = lane; t < rn * H; t += kGtLane)
                        s_p[t] = exp10(s_p[t] - s_m[t / H]);
                    __syncthreads();
                    staged_r0 = r0;
                }
                if (act) {
                    const double* row = lk + lo + (uint64_t)r0 * H;
                    for (uint32_t r = grp; r < rn; r += groups) {
                        const double sum = s_p[r * H + a] + s_p[r * H + b];
                        if (sum > 1e-290) {
                            int e;
                            mant = frexp(mant * (0.5 * sum), &e);
                            ex += e;
                            add += s_m[r];
                        } else {
                            const double la = row[r * H + a], lb = row[r * H + b];
                            add += fmax(la, lb) + log1p(exp10(-fabs(la - lb))) * kInvLn10 -
                                   kLog10Of2;
                        }
                    }
                }
            }
            double acc = act ? add + log10(mant) + (double)ex * kLog10Of2 : 0.0;
            for (uint32_t off = gw; off < kGtLane; off <<= 1) acc += __shfl_xor(acc, off, kGtLane);
            if (act && grp == 0) {
                gl[go + gi] = acc;
                if (acc > bv) {
                    bv = acc;
                    bi = (uint32_t)gi;
                }
            }
        }
        // wavefront argmax: larger value, then smaller index
        for (int off = kGtLane / 2; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off, kGtLane);
            const uint32_t oi = __shfl_xor(bi, off, kGtLane);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) best[reg] = bi;
    }
}

int launch_genotype(hipStream_t s, int cus, const double* lk, uint64_t n_lk,
                    const uint64_t* lk_off, const uint32_t* n_reads, const uint32_t* n_haps,
                    const uint64_t* gl_off, uint32_t n_regions, double* gl, uint64_t n_gl,
                    uint32_t* best)
{
    if (n_regions == 0) return 0;
    const uint32_t grid = std::min<uint32_t>(n_regions, (uint32_t)std::max(cus, 1) * 64u);
    hipLaunchKernelGGL(genotype_kernel, dim3(grid), dim3(kGtLane), 0, s, lk, n_lk, lk_off,
                       n_reads, n_haps, gl_off, n_regions, gl, n_gl, best);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace phmm
