// Device helpers for the gfx950 PairHMM kernels: cross-lane moves (DPP),
// the segmented weighted wavefront scan, and small utilities.
#pragma once

#include "phmm_internal.h"

namespace phmm {

// DPP controls of GFX9-family wavefronts (64 lanes = 4 rows of 16).
enum : int {
    kRowShr1 = 0x111,
    kRowShr2 = 0x112,
    kRowShr4 = 0x114,
    kRowShr8 = 0x118,
    kWaveShr1 = 0x138,    // lane L <- lane L-1 across the whole wavefront
    kRowBcast15 = 0x142,  // lane 15 of a row -> every lane of the next row
    kRowBcast31 = 0x143,  // lane 31 -> rows 2 and 3
};

// Lanes whose source is outside the pattern, or whose row is masked off,
// read 0.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ int dpp_i(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROWMASK, 0xf, false);
}
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ float dpp(float x)
{
    return __builtin_bit_cast(float, dpp_i<CTRL, ROWMASK>(__builtin_bit_cast(int, x)));
}
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp(double x)
{
    uint64_t u = __builtin_bit_cast(uint64_t, x);
    int lo = dpp_i<CTRL, ROWMASK>((int)(uint32_t)u);
    int hi = dpp_i<CTRL, ROWMASK>((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Inclusive wavefront sum of ints (no segments).
__device__ __forceinline__ int wave_incl_sum(int x)
{
    x += dpp_i<kRowShr1>(x);
    x += dpp_i<kRowShr2>(x);
    x += dpp_i<kRowShr4>(x);
    x += dpp_i<kRowShr8>(x);
    x += dpp_i<kRowBcast15, 0xa>(x);
    x += dpp_i<kRowBcast31, 0xc>(x);
    return x;
}

// Per-lane multipliers of the segmented first-order linear scan
//   y_L = sum_{q <= L, q in seg(L)} a^(L-q) x_q
// evaluated in 6 DPP steps: four in-row Kogge-Stone steps (distance 1, 2, 4,
// 8) and two row broadcasts (from lane 15 of the previous row, from lane 31).
// Each multiplier is a^distance when the source lane lies in the lane's
// segment and 0 otherwise.
template <typename R>
struct ScanMul {
    R m1, m2, m4, m8, m15, m31;
};

// pw[d] = a^d for d = 0..64 (units of one lane).
template <typename R, typename P>
__device__ __forceinline__ ScanMul<R> make_scan_mul(const P* pw, int lane, int segstart)
{
    ScanMul<R> m;
    const int r = lane >> 4, c = lane & 15;
    m.m1 = (c >= 1 && lane - 1 >= segstart) ? (R)pw[1] : (R)0;
    m.m2 = (c >= 2 && lane - 2 >= segstart) ? (R)pw[2] : (R)0;
    m.m4 = (c >= 4 && lane - 4 >= segstart) ? (R)pw[4] : (R)0;
    m.m8 = (c >= 8 && lane - 8 >= segstart) ? (R)pw[8] : (R)0;
    m.m15 = ((r == 1 || r == 3) && segstart <= 16 * r - 1) ? (R)pw[c + 1] : (R)0;
    m.m31 = (lane >= 32 && segstart <= 31) ? (R)pw[lane - 31] : (R)0;
    return m;
}

template <typename R>
__device__ __forceinline__ ScanMul<R> make_sum_mul(int lane, int segstart)
{
    ScanMul<R> m;
    const int r = lane >> 4, c = lane & 15;
    m.m1 = (c >= 1 && lane - 1 >= segstart) ? (R)1 : (R)0;
    m.m2 = (c >= 2 && lane - 2 >= segstart) ? (R)1 : (R)0;
    m.m4 = (c >= 4 && lane - 4 >= segstart) ? (R)1 : (R)0;
    m.m8 = (c >= 8 && lane - 8 >= segstart) ? (R)1 : (R)0;
    m.m15 = ((r == 1 || r == 3) && segstart <= 16 * r - 1) ? (R)1 : (R)0;
    m.m31 = (lane >= 32 && segstart <= 31) ? (R)1 : (R)0;
    return m;
}

template <typename R>
__device__ __forceinline__ R seg_scan(R x, const ScanMul<R>& m)
{
    x = fmaR(m.m1, dpp<kRowShr1>(x), x);
    x = fmaR(m.m2, dpp<kRowShr2>(x), x);
    x = fmaR(m.m4, dpp<kRowShr4>(x), x);
    x = fmaR(m.m8, dpp<kRowShr8>(x), x);
    x = fmaR(m.m15, dpp<kRowBcast15, 0xa>(x), x);
    x = fmaR(m.m31, dpp<kRowBcast31, 0xc>(x), x);
    return x;
}

// Haplotype columns are held as floats whose IEEE class names the base, so
// one class test against a per-row mask decides match / mismatch:
//   A = +1.0 (+normal)  C = -1.0 (-normal)  G = +0.0  T = -0.0
//   N = +inf (in every mask: matches any read base)  padding = -inf (in none)
// Class-mask bits (v_cmp_class): 3 -normal, 5 -zero, 6 +zero, 8 +normal, 9 +inf.
__device__ __forceinline__ float hap_class_value(uint8_t b)
{
    uint32_t u = b == 'A' ? 0x3f800000u : b == 'C' ? 0xbf800000u : b == 'G' ? 0x00000000u
               : b == 'T' ? 0x80000000u : 0x7f800000u;  // N (and any other byte)
    return __builtin_bit_cast(float, u);
}
__device__ __forceinline__ float hap_pad_value() { return __builtin_bit_cast(float, 0xff800000u); }

// Class mask selecting the haplotype columns that match read base b.
__device__ __forceinline__ int read_class_mask(uint8_t b)
{
    return b == 'A' ? ((1 << 8) | (1 << 9)) : b == 'C' ? ((1 << 3) | (1 << 9))
         : b == 'G' ? ((1 << 6) | (1 << 9)) : b == 'T' ? ((1 << 5) | (1 << 9))
         : 0x3ff;  // N: every column matches
}

__device__ __forceinline__ bool col_match(float hv, int mask)
{
    return __builtin_amdgcn_class(hv, mask);
}

__device__ __forceinline__ uint32_t wave_broadcast0(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// log10 of S * 2^(-scale_exp) with the exponent handled in integers.
__device__ __forceinline__ double log10_scaled(double S, int scale_exp)
{
    if (!(S > 0.0)) return -__builtin_inf();
    int e;
    double m = frexp(S, &e);
    return log10(m) + (double)(e - scale_exp) * 0.30102999566398119521;
}

}  // namespace phmm
