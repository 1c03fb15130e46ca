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
// read 0 (bound_ctrl set: the move needs no zeroed destination when every
// row is enabled).
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ int dpp_i(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROWMASK, 0xf, true);
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

__device__ __forceinline__ double seg_scan(double x, const ScanMul<double>& m)
{
    x = fmaR(m.m1, dpp<kRowShr1>(x), x);
    x = fmaR(m.m2, dpp<kRowShr2>(x), x);
    x = fmaR(m.m4, dpp<kRowShr4>(x), x);
    x = fmaR(m.m8, dpp<kRowShr8>(x), x);
    x = fmaR(m.m15, dpp<kRowBcast15, 0xa>(x), x);
    x = fmaR(m.m31, dpp<kRowBcast31, 0xc>(x), x);
    return x;
}

// FP32: each step is one v_fmac_f32 whose first operand is read through the
// DPP pattern, x += m * x[source lane]; a lane with no source reads 0
// (bound_ctrl) and a lane of a disabled row is not written, so both keep x.
// The leading s_nop gives the two wait states a DPP read needs after the VALU
// write of its source; the trailing one covers a DPP read that follows.
#define PHMM_SCAN_STEP(PAT, BC)                                                      \
    asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %1 " PAT " bank_mask:0xf" BC   \
                 : "+v"(x)                                                           \
                 : "v"(mm))
__device__ __forceinline__ float seg_scan(float x, const ScanMul<float>& m)
{
    float mm = m.m1;
    PHMM_SCAN_STEP("row_shr:1 row_mask:0xf", " bound_ctrl:1");
    mm = m.m2;
    PHMM_SCAN_STEP("row_shr:2 row_mask:0xf", " bound_ctrl:1");
    mm = m.m4;
    PHMM_SCAN_STEP("row_shr:4 row_mask:0xf", " bound_ctrl:1");
    mm = m.m8;
    PHMM_SCAN_STEP("row_shr:8 row_mask:0xf", " bound_ctrl:1");
    mm = m.m15;
    PHMM_SCAN_STEP("row_bcast:15 row_mask:0xa", "");
    mm = m.m31;
    PHMM_SCAN_STEP("row_bcast:31 row_mask:0xc", "");
    asm volatile("s_nop 1" ::: "memory");
    return x;
}
#undef PHMM_SCAN_STEP

// Emission select without compares.  Each haplotype column is an 8-bit
// code with bit b set when a read base of index b matches it (A=0, C=1,
// G=2, T=3) and bit 4 always set; 'N' sets bits 0-3, padding sets only bit 4
// (padding columns never influence real ones).  Four columns share a 32-bit
// register.  A row whose read base has index b (4 for 'N', which matches
// everything) extracts bit 8*n+b as a signed 1-bit field: -1 on a match, 0
// otherwise, and that mask picks pm or px bit-wise (v_bfe_i32 + v_bfi_b32).
__device__ __forceinline__ uint32_t hap_code(uint8_t b)
{
    return b == 'A' ? 0x11u : b == 'C' ? 0x12u : b == 'G' ? 0x14u : b == 'T' ? 0x18u
         : 0x1fu;  // N (and any other byte)
}
constexpr uint32_t kPadCode = 0x10u;

__device__ __forceinline__ int read_base_index(uint8_t b)
{
    return b == 'A' ? 0 : b == 'C' ? 1 : b == 'G' ? 2 : b == 'T' ? 3 : 4;
}

// pm if column n (code word w, bit offset off = 8*(n%4) + base index) matches
__device__ __forceinline__ float emit_sel(uint32_t w, int off, float pm, float px)
{
    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)w, off, 1);
    return __builtin_bit_cast(float, (m & __builtin_bit_cast(uint32_t, pm)) |
                                         (~m & __builtin_bit_cast(uint32_t, px)));
}
// The 32-bit mask is applied to each half of the doubles separately: hipcc
// (ROCm 7.2) drops the upper half of a sign-extended 64-bit bfe mask.
__device__ __forceinline__ double emit_sel(uint32_t w, int off, double pm, double px)
{
    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)w, off, 1);
    const uint64_t a = __builtin_bit_cast(uint64_t, pm), b = __builtin_bit_cast(uint64_t, px);
    const uint32_t lo = (m & (uint32_t)a) | (~m & (uint32_t)b);
    const uint32_t hi = (m & (uint32_t)(a >> 32)) | (~m & (uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------- row recurrence
//
// Per-row coefficients, computed once per read row in FP64 and stored in LDS.
//
// Scaled form (SC): row r keeps J_r = T_IM_{r+1} I_r and M*_r = s_r M_r with
// s_r = T_IM_{r+2} T_MI_{r+1} (T_IM_l = 1 past the last row, s_{l-1} = 1, so
// the last row holds M and I themselves).  Substituting into eq.2:
//
//   M*_r(j) = (s_r p) (T_MM_r / s_{r-1} M*_{r-1}(j-1) + J_{r-1}(j-1)
//                      + T_DM_r T_MD_{r-1} / s_{r-1} S*_{r-1}(j-2))
//   J_r(j)  = M*_{r-1}(j) + T_IM_{r+1} T_II_r / T_IM_r J_{r-1}(j)
//
// where S* is the delete prefix of the scaled row.  Both coefficients that
// would multiply J and M* are 1, so a cell costs two FMAs and a multiply for
// M and one FMA for I.  The scale factors are per row, not cumulative; the
// form needs T_IM_r > 0 and s_r bounded away from 0 (checked per pack, see
// sc_ok).  Otherwise the plain form runs: a = T_MI_r, b = T_II_r, unscaled.
template <typename R>
struct RowRec {
    R pm, px, tmm, cd, a, b, tim, pad;
};

// kScMaxInsQ (the largest insertion Phred byte of the scaled form) keeps
// s_r >= 2^-24 for every gap byte >= 1 (T_IM >= 1 - 10^-0.1), so the scaled
// rows stay within 24 binary orders of the plain ones.

// FP64 coefficient to R.  DITHER (FP32 only): unbiased stochastic rounding
// to one of the two floats around v, chosen by a hash of (row, coefficient).
// Rounding every row's coefficients to nearest gives all rows with the same
// quality bytes the same relative error, which adds up linearly over a long
// read; dithered, the errors are uncorrelated from row to row and their sum
// grows like the square root of the row count.  The hash depends only on the
// row index, so every tile of a pair rounds identically.
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x = (x ^ (x >> 16)) * 0x7feb352du;
    x = (x ^ (x >> 15)) * 0x846ca68bu;
    return x ^ (x >> 16);
}
template <typename R, bool DITHER>
__device__ __forceinline__ R to_coef(double v, int i, int which)
{
    if constexpr (!DITHER || sizeof(R) != 4) {
        return (R)v;
    } else {
        const float f = (float)v;
        const double df = (double)f;
        if (!(v > 0.0) || df == v || !(f < 3.0e38f)) return f;
        const uint32_t u = __builtin_bit_cast(uint32_t, f);
        const float lo = df > v ? __builtin_bit_cast(float, u - 1u) : f;  // v > 0: below is u - 1
        const float hi = df > v ? f : __builtin_bit_cast(float, u + 1u);
        const double r = (double)mix32((uint32_t)i * 8u + (uint32_t)which) * 2.3283064365386963e-10;
        return r * ((double)hi - (double)lo) < v - (double)lo ? hi : lo;
    }
}

template <typename R, bool SC, bool DITHER = false>
__device__ __forceinline__ RowRec<R> make_row_rec(const Batch& B, const double* p64, uint64_t a,
                                                  int i, int l)
{
    const double eps = p64[B.bq[a]];
    const double tmi = p64[B.iq[a]];
    const double tmd = p64[B.dq[a]];
    const double g = p64[B.gq[a]];
    const double tmd_prev = i > 0 ? p64[B.dq[a - 1]] : 0.0;
    double tmm = 1.0 - (tmi + tmd);
    tmm = tmm < 0.0 ? 0.0 : tmm;
    const double pm = 1.0 - eps, px = eps / 3.0, tim = 1.0 - g;
    const double cd = tim * tmd_prev;  // T_DM_i T_MD_{i-1}
    RowRec<R> r;
    if (SC) {
        const double tim1 = i + 1 < l ? 1.0 - p64[B.gq[a + 1]] : 1.0;  // T_IM_{i+1}
        const double tim2 = i + 2 < l ? 1.0 - p64[B.gq[a + 2]] : 1.0;  // T_IM_{i+2}
        const double s = i + 1 < l ? tim2 * p64[B.iq[a + 1]] : 1.0;    // s_i
        const double sp = tim1 * tmi;                                   // s_{i-1}
        r.pm = to_coef<R, DITHER>(s * pm, i, 0);
        r.px = to_coef<R, DITHER>(s * px, i, 1);
        r.tmm = to_coef<R, DITHER>(tmm / sp, i, 2);
        r.cd = to_coef<R, DITHER>(cd / sp, i, 3);
        r.a = (R)1;
        r.b = to_coef<R, DITHER>(tim1 * g / tim, i, 4);
    } else {
        r.pm = to_coef<R, DITHER>(pm, i, 0);
        r.px = to_coef<R, DITHER>(px, i, 1);
        r.tmm = to_coef<R, DITHER>(tmm, i, 2);
        r.cd = to_coef<R, DITHER>(cd, i, 3);
        r.a = to_coef<R, DITHER>(tmi, i, 5);
        r.b = to_coef<R, DITHER>(g, i, 4);
    }
    r.tim = to_coef<R, DITHER>(tim, i, 6);
    r.pad = (R)0;
    return r;
}

// Row 1: M(1,j) = P(r_1|h_j) T_DM_1 C0/k (times s_0 in the scaled form, which
// the record's pm and px carry), I(1,j) = 0.
template <typename R, int N>
__device__ __forceinline__ void row_first(R (&Mo)[N], R (&Io)[N], const uint32_t (&hc)[(N + 3) / 4],
                                          int bidx, const RowRec<R>& c, R minit, R g, R& Vp)
{
    R V = (R)0;
    const R base = c.tim * minit;  // T_DM_1 = T_IM_1
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const R p = emit_sel(hc[n / 4], 8 * (n % 4) + bidx, c.pm, c.px);
        const R m = p * base;
        Mo[n] = m;
        Io[n] = (R)0;
        if (n < N - 1) V = fmaR(g, V, m);
    }
    Vp = V;
}

// Rows 2..l of the row-level recurrence: reads row i-1 from (Mi, Ii) and
// writes row i to (Mo, Io).  T rebuilds S(i-1, .) from the lane's carry C, V
// accumulates the new row's window sum for the next scan.
template <typename R, int N, bool SC>
__device__ __forceinline__ void row_step(const R (&Mi)[N], const R (&Ii)[N], R (&Mo)[N], R (&Io)[N],
                                         const uint32_t (&hc)[(N + 3) / 4], int bidx,
                                         const RowRec<R>& c, R Mleft, R Ileft, R C, R gprev,
                                         R gcur, R& Vp)
{
    R T = C, V = (R)0;
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const R mprev = n == 0 ? Mleft : Mi[n - 1];
        const R iprev = n == 0 ? Ileft : Ii[n - 1];
        const R p = emit_sel(hc[n / 4], 8 * (n % 4) + bidx, c.pm, c.px);
        // The small gap terms are summed first and the dominant match term
        // last, in one FMA with its exact product: added to an already
        // rounded sum, a delete term under half an ulp would be dropped every
        // time, a bias of about -3e-9 per row in FP32 (-1.3e-4 in log10 at
        // 100,000 rows); added to the exact product it rounds without bias.
        const R x = SC ? fmaR(c.tmm, mprev, fmaR(c.cd, T, iprev))
                       : fmaR(c.tmm, mprev, fmaR(c.tim, iprev, c.cd * T));
        const R m = p * x;
        Mo[n] = m;
        Io[n] = SC ? fmaR(c.b, Ii[n], Mi[n]) : fmaR(c.b, Ii[n], c.a * Mi[n]);
        T = fmaR(gprev, T, mprev);
        if (n < N - 1) V = fmaR(gcur, V, m);
    }
    Vp = V;
}

// The lane index, read afresh where it is called: values derived from it
// inside a loop (LDS and global addresses) are then recomputed per iteration
// with a few ALU instructions instead of being hoisted out of the loop and,
// under register pressure, spilled to scratch memory.
__device__ __forceinline__ int lane_here()
{
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
}

// ---------------------------------------------------------------- power-of-two scaling

// Wavefront max of a non-negative int (0 = nothing).
__device__ __forceinline__ int wave_max_int(int x)
{
    x = max(x, dpp_i<kRowShr1>(x));
    x = max(x, dpp_i<kRowShr2>(x));
    x = max(x, dpp_i<kRowShr4>(x));
    x = max(x, dpp_i<kRowShr8>(x));
    x = max(x, dpp_i<kRowBcast15, 0xa>(x));
    x = max(x, dpp_i<kRowBcast31, 0xc>(x));
    return __builtin_amdgcn_readlane(x, 63);
}

__device__ __forceinline__ float maxR(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double maxR(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ int exponent_of(float v) { int e; frexpf(v, &e); return e; }
__device__ __forceinline__ int exponent_of(double v) { int e; frexp(v, &e); return e; }
__device__ __forceinline__ float scale2(float v, int e) { return ldexpf(v, e); }
__device__ __forceinline__ double scale2(double v, int e) { return ldexp(v, e); }

// 2^e as an exact R when it is a normal number of R (|e| within the exponent
// range), so that scaling is one multiply; callers fall back to ldexp outside.
template <typename R>
__device__ __forceinline__ bool pow2_ok(int e)
{
    return sizeof(R) == 4 ? (e >= -126 && e <= 127) : (e >= -1022 && e <= 1023);
}
__device__ __forceinline__ float pow2f(int e) { return __builtin_bit_cast(float, (uint32_t)(e + 127) << 23); }
__device__ __forceinline__ double pow2d(int e)
{
    return __builtin_bit_cast(double, (uint64_t)(e + 1023) << 52);
}
template <typename R>
__device__ __forceinline__ R pow2(int e);
template <>
__device__ __forceinline__ float pow2<float>(int e) { return pow2f(e); }
template <>
__device__ __forceinline__ double pow2<double>(int e) { return pow2d(e); }

__device__ __forceinline__ uint32_t wave_broadcast0(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// log10 of s * 2^(-scale_exp) for a positive normal float s (an FP32 result):
// the mantissa's log2 from the hardware (v_log_f32, error well below 1e-7 on
// [0.5, 1)) plus the exponent.  It needs no polynomial constants, which the
// compiler would otherwise keep in registers across the whole pack.
__device__ __forceinline__ double log10_scaled_f32(float s, int scale_exp)
{
    int e;
    const float m = frexpf(s, &e);
    return ((double)__builtin_amdgcn_logf(m) + (double)(e - scale_exp)) * 0.30102999566398119521;
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
