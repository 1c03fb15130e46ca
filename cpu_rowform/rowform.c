/*
 * CPU comparator: the PairHMM forward pass in the row-level formulation
 * (Section 3.1, eq.5-7) with SIMD over the columns of a row and threads over
 * pairs, as a stronger host baseline than the plain oracle.  It is not part
 * of the GPU library and shares no code with it or with the oracle.
 *
 * Per row i of a pair (read length l, haplotype length k):
 *   M(i,j) = P(r_i|h_j) (T_MM M(i-1,j-1) + T_IM I(i-1,j-1) + T_DM D(i-1,j-1))
 *   I(i,j) = T_MI M(i-1,j) + T_II I(i-1,j)                 (eq.2, both vector loops)
 *   D(i,j) = T_DD D(i,j-1) + T_MD M(i,j-1)                 (first-order recurrence)
 * The Delete row is D(j) = sum_{t<=j} g^(j-t) x(t), x(t) = T_MD M(i,t-1),
 * g = T_DD.  It is evaluated as in the wavefront scan of Section 3.4, with
 * vector loops only: three doubling steps y <- y + g^s y(shifted by s),
 * s = 1, 2, 4, give u(j) = sum_{s<8} g^s x(j-s); then D(j) = g^8 D(j-8) + u(j),
 * a recurrence of distance 8 that vectorises over 8 lanes.
 *
 * Precision policy as on the GPU: FP32 with the start row D(0,j) = 2^120/k;
 * a pair whose FP32 sum is not finite or below 1e-28 is recomputed in FP64
 * from D(0,j) = 1/k with a power-of-two rescaling of the row every 8 rows
 * (exact; the exponents are summed and added back at the end).
 * Priors: raw Phred bytes, 10^(-q/10) from a 256-entry table (eq.3 and the
 * transition definitions of Section 2; mismatch prior eps/3, N matches all).
 * Subnormal values are flushed to zero (FTZ and DAZ in each worker thread):
 * cells below 1.2e-38 in FP32 add less than 1e-10 relative to an accepted
 * sum (>= 1e-28), and subnormal arithmetic is many times slower on x86.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <xmmintrin.h>

#define RF_ACCEPT_MIN 1e-28

static double g_pow10[256];

/* filled when the library is loaded, before any call can read it */
__attribute__((constructor)) static void init_table(void)
{
    for (int q = 0; q < 256; ++q) g_pow10[q] = pow(10.0, -q / 10.0);
}

typedef struct {
    double pm, px, mm, im, dm, mi, ii, md, dd;
} row_prior;

static void priors(const uint8_t* bq, const uint8_t* iq, const uint8_t* dq, const uint8_t* gq,
                   uint32_t l, row_prior* pr)
{
    for (uint32_t i = 0; i < l; ++i) {
        const double e = g_pow10[bq[i]], tmi = g_pow10[iq[i]], tmd = g_pow10[dq[i]];
        const double g = g_pow10[gq[i]];
        double tmm = 1.0 - tmi - tmd;
        if (tmm < 0.0) tmm = 0.0;
        pr[i].pm = 1.0 - e;
        pr[i].px = e / 3.0;
        pr[i].mm = tmm;
        pr[i].im = 1.0 - g;
        pr[i].dm = 1.0 - g;
        pr[i].mi = tmi;
        pr[i].ii = g;
        pr[i].md = tmd;
        pr[i].dd = g;
    }
}

/* One pair in type T.  Eight row arrays of k + 1 entries, each behind 8
 * zeros so that the shifted reads of the Delete scan (index -1 .. -4) see
 * zeros.  Returns log10 L; *ok = 0 when the sum fails the acceptance test. */
#define DEFINE_PAIR(NAME, T, SCALE_LOG2, RESCALE)                                           \
    static double NAME(const uint8_t* read, const uint8_t* hap, uint32_t l, uint32_t k,      \
                       const row_prior* pr, T* buf, int* ok)                                 \
    {                                                                                        \
        const uint32_t w = k + 1 + 8;                                                        \
        T* Mp = buf + 8;                                                                     \
        T* Ip = Mp + w;                                                                      \
        T* Dp = Ip + w;                                                                      \
        T* Mc = Dp + w;                                                                      \
        T* Ic = Mc + w;                                                                      \
        T* Dc = Ic + w;                                                                      \
        T* y = Dc + w;                                                                       \
        T* z = y + w;                                                                        \
        memset(buf, 0, sizeof(T) * (size_t)8 * w);                                           \
        const T d0 = (T)(ldexp(1.0, SCALE_LOG2) / (double)k);                                \
        for (uint32_t j = 0; j <= k; ++j) Dp[j] = d0;                                        \
        long expo = 0;                                                                       \
        for (uint32_t i = 0; i < l; ++i) {                                                   \
            const row_prior* p = &pr[i];                                                     \
            const T pm = (T)p->pm, px = (T)p->px, mm = (T)p->mm, im = (T)p->im;              \
            const T dm = (T)p->dm, mi = (T)p->mi, ii = (T)p->ii, md = (T)p->md;              \
            const T g = (T)p->dd, g2 = g * g, g4 = g2 * g2, g8 = g4 * g4;                     \
            const uint8_t rb = read[i];                                                      \
            T* restrict mc = Mc;                                                             \
            T* restrict ic = Ic;                                                             \
            T* restrict dc = Dc;                                                             \
            T* restrict yy = y;                                                              \
            T* restrict zz = z;                                                              \
            const T* restrict mp = Mp;                                                       \
            const T* restrict ip = Ip;                                                       \
            const T* restrict dp = Dp;                                                       \
            mc[0] = ic[0] = dc[0] = (T)0;                                                    \
            for (uint32_t j = 1; j <= k; ++j) {                                              \
                const uint8_t hb = hap[j - 1];                                               \
                const T e = (rb == hb || rb == 'N' || hb == 'N') ? pm : px;                  \
                mc[j] = e * (mm * mp[j - 1] + im * ip[j - 1] + dm * dp[j - 1]);              \
                ic[j] = mi * mp[j] + ii * ip[j];                                             \
            }                                                                                \
            /* x(j) = T_MD M(i, j-1), j = 1..k; x(0) = 0 */                                  \
            yy[0] = (T)0;                                                                    \
            for (uint32_t j = 1; j <= k; ++j) yy[j] = md * mc[j - 1];                        \
            for (uint32_t j = 0; j <= k; ++j) zz[j] = yy[j] + g * yy[(int)j - 1];           \
            for (uint32_t j = 0; j <= k; ++j) yy[j] = zz[j] + g2 * zz[(int)j - 2];          \
            for (uint32_t j = 0; j <= k; ++j) zz[j] = yy[j] + g4 * yy[(int)j - 4];          \
            for (uint32_t j = 0; j < 8 && j <= k; ++j) dc[j] = zz[j];                        \
            for (uint32_t j = 8; j <= k; ++j) dc[j] = g8 * dc[j - 8] + zz[j];                \
            dc[0] = (T)0;                                                                    \
            if (RESCALE && (i & 7) == 7) {                                                   \
                T mx = (T)0;                                                                 \
                for (uint32_t j = 0; j <= k; ++j) {                                          \
                    mx = Mc[j] > mx ? Mc[j] : mx;                                            \
                    mx = Ic[j] > mx ? Ic[j] : mx;                                            \
                    mx = Dc[j] > mx ? Dc[j] : mx;                                            \
                }                                                                            \
                if (mx > (T)0) {                                                             \
                    int e2;                                                                  \
                    frexp((double)mx, &e2);                                                  \
                    const T f = (T)ldexp(1.0, -e2);                                          \
                    for (uint32_t j = 0; j <= k; ++j) {                                      \
                        Mc[j] *= f;                                                          \
                        Ic[j] *= f;                                                          \
                        Dc[j] *= f;                                                          \
                    }                                                                        \
                    expo += e2;                                                              \
                }                                                                            \
            }                                                                                \
            T* t;                                                                            \
            t = Mp, Mp = Mc, Mc = t;                                                         \
            t = Ip, Ip = Ic, Ic = t;                                                         \
            t = Dp, Dp = Dc, Dc = t;                                                         \
        }                                                                                    \
        double s = 0.0;                                                                      \
        T st = (T)0;                                                                         \
        for (uint32_t j = 1; j <= k; ++j) st += Mp[j] + Ip[j];                               \
        s = (double)st;                                                                      \
        *ok = isfinite(s) && s >= (RESCALE ? 1e-290 : RF_ACCEPT_MIN);                        \
        return log10(s) + (double)expo * log10(2.0) - (SCALE_LOG2) * log10(2.0);             \
    }

DEFINE_PAIR(pair_f32, float, 120, 0)
DEFINE_PAIR(pair_f64, double, 0, 1)

/* out_log10[p] for every pair; out_flags[p] = 1 (FP32 accepted) or 2 (FP64).
 * threads <= 0 uses the OpenMP default.  Returns 0, or -1 on allocation
 * failure. */
int rf_forward_pairs(const uint8_t* reads, const uint8_t* bq, const uint8_t* iq,
                     const uint8_t* dq, const uint8_t* gq, const uint64_t* read_off,
                     const uint8_t* haps, const uint64_t* hap_off, const uint32_t* pairs,
                     uint64_t n_pairs, int threads, double* out_log10, uint8_t* out_flags)
{
    int fail = 0;
#pragma omp parallel num_threads(threads > 0 ? threads : omp_get_max_threads())
    {
        const unsigned int csr = _mm_getcsr();
        _mm_setcsr(csr | 0x8040u); /* flush-to-zero, denormals-are-zero */
        size_t cap = 0;
        double* buf = NULL;
        row_prior* pr = NULL;
        size_t prcap = 0;
#pragma omp for schedule(dynamic, 64)
        for (uint64_t p = 0; p < n_pairs; ++p) {
            const uint32_t r = pairs[2 * p], h = pairs[2 * p + 1];
            const uint64_t r0 = read_off[r], h0 = hap_off[h];
            const uint32_t l = (uint32_t)(read_off[r + 1] - r0);
            const uint32_t k = (uint32_t)(hap_off[h + 1] - h0);
            const size_t need = (size_t)8 * (k + 9);
            if (need > cap || l > prcap) {
                free(buf);
                free(pr);
                cap = need > cap ? 2 * need : cap;
                prcap = l > prcap ? 2 * (size_t)l : prcap;
                buf = (double*)malloc(sizeof(double) * cap);
                pr = (row_prior*)malloc(sizeof(row_prior) * prcap);
                if (!buf || !pr) {
#pragma omp atomic write
                    fail = 1;
                    cap = prcap = 0;
                    continue;
                }
            }
            priors(bq + r0, iq + r0, dq + r0, gq + r0, l, pr);
            int ok = 0;
            double v = pair_f32(reads + r0, haps + h0, l, k, pr, (float*)buf, &ok);
            uint8_t fl = 1;
            if (!ok) {
                v = pair_f64(reads + r0, haps + h0, l, k, pr, buf, &ok);
                fl = 2;
            }
            out_log10[p] = v;
            if (out_flags) out_flags[p] = fl;
        }
        free(buf);
        free(pr);
        _mm_setcsr(csr);
    }
    return fail ? -1 : 0;
}
