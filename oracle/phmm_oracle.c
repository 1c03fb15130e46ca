/*
 * PairHMM forward-algorithm ORACLE — test infrastructure only.
 *
 * This file is a plain, slow, single-threaded FP64 evaluation of what the
 * PairHMM forward algorithm computes.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it; the product library
 * never links or calls it, and it shares no code, header or table with the
 * product (each side computes its own quality->probability values).
 *
 * Build with -ffp-contract=off so every product and sum is rounded on its
 * own and evaluation orders can be compared bit for bit.
 *
 * The model (paper, Section 2 "Background", eq. 1-4):
 *   eq.1  M(i,0)=I(i,0)=D(i,0)=M(0,j)=I(0,j)=0,  D(0,j)=C/k  (C = 2^1020)
 *   eq.2  M(i,j) = P(r_i|h_j) (T_MM_i M(i-1,j-1) + T_IM I(i-1,j-1) + T_DM D(i-1,j-1))
 *         I(i,j) = T_MI_i M(i-1,j) + T_II I(i-1,j)
 *         D(i,j) = T_MD_i M(i,j-1) + T_DD D(i,j-1)
 *   eq.3  P(r_i|h_j) = 1-eps_i on a match, eps_i/3 otherwise,
 *         eps_i = 10^(-Q_i/10)  (Q is raw Phred; the paper's -33 is the
 *         FASTQ character offset, removed by the caller)
 *   eq.4  L = sum_j M(l,j) + I(l,j)
 *
 * Readings taken where the paper is silent or self-contradictory (each is
 * also listed in the design notes):
 *   - D(0,0) = C/k as well (the row-1 initialisation of Section 3.4 gives
 *     M(1,j) = p T_DM C/k for every j including j = 1).
 *   - divisor k = haplotype length (eq.1), not the listings' N.
 *   - mismatch prior exactly eps/3 (eq.3), not 0.33.
 *   - T_MI_i = 10^(-ins_i/10), T_MD_i = 10^(-del_i/10),
 *     T_MM_i = max(0, 1 - (T_MI_i + T_MD_i)); gap continuation
 *     g_i = 10^(-gcp_i/10) per read position gives T_II = T_DD = g_i and
 *     T_IM = T_DM = 1 - g_i (gcp = 10 gives the paper's 0.1 / 0.9).
 *   - row i uses row i's priors for M, I and D of that row.
 *   - the base 'N' in either sequence matches anything.
 *   - result reported as log10 L = log10 S - log10 C (+ E log10 2 when the
 *     optional per-row power-of-two rescaling accumulated exponent E).
 *
 * Per-row rescaling (not in the paper, needed once log10 L falls below the
 * FP64 range, i.e. for long reads): after each row, the row is multiplied by
 * 2^-e where e is the frexp exponent of the row maximum over M, I and D, and
 * e is added to an integer exponent E.  Multiplying by a power of two is
 * exact, so without underflow the rescaled and unrescaled runs carry the
 * same mantissas.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Per-row prior record, in this order. */
enum { P_PM = 0, P_PX, P_TMM, P_TIM, P_TDM, P_TMI, P_TII, P_TMD, P_TDD, P_NREC };

static double phred_to_prob(unsigned q) { return pow(10.0, -(double)q / 10.0); }

/* Priors of eq.3 and the transition probabilities, one record per read row. */
int oracle_priors(const uint8_t* bq, const uint8_t* iq, const uint8_t* dq,
                  const uint8_t* gq, int l, double* out)
{
    if (l < 0 || (l > 0 && (!bq || !iq || !dq || !gq || !out))) return -1;
    for (int i = 0; i < l; ++i) {
        double eps = phred_to_prob(bq[i]);
        double tmi = phred_to_prob(iq[i]);
        double tmd = phred_to_prob(dq[i]);
        double g = phred_to_prob(gq[i]);
        double tmm = 1.0 - (tmi + tmd);
        if (tmm < 0.0) tmm = 0.0;
        double* r = out + (size_t)i * P_NREC;
        r[P_PM] = 1.0 - eps;
        r[P_PX] = eps / 3.0;
        r[P_TMM] = tmm;
        r[P_TIM] = 1.0 - g;
        r[P_TDM] = 1.0 - g;
        r[P_TMI] = tmi;
        r[P_TII] = g;
        r[P_TMD] = tmd;
        r[P_TDD] = g;
    }
    return 0;
}

static int is_match(uint8_t r, uint8_t h) { return r == h || r == 'N' || h == 'N'; }

static double emission(const double* pr, uint8_t r, uint8_t h)
{
    return is_match(r, h) ? pr[P_PM] : pr[P_PX];
}

/* 2^1020 / k, the eq.1 start value of the D row. */
static double start_value(int k) { return ldexp(1.0, 1020) / (double)k; }

/* Row-order forward pass of eq.1-4 in O(k) memory.  On return *S is the
 * final scaled sum of eq.4 and *E the accumulated rescale exponent, so that
 * L = S * 2^E / 2^1020. */
int oracle_forward_probs(const double* pri, const uint8_t* read, int l,
                         const uint8_t* hap, int k, int rescale,
                         double* S, int64_t* E)
{
    if (l <= 0 || k <= 0 || !pri || !read || !hap || !S || !E) return -1;
    size_t n = (size_t)k + 1;
    double* buf = (double*)malloc(sizeof(double) * n * 6);
    if (!buf) return -2;
    double *Mp = buf, *Ip = buf + n, *Dp = buf + 2 * n;
    double *Mc = buf + 3 * n, *Ic = buf + 4 * n, *Dc = buf + 5 * n;
    double d0 = start_value(k);
    for (size_t j = 0; j < n; ++j) { Mp[j] = 0.0; Ip[j] = 0.0; Dp[j] = d0; }
    int64_t ex = 0;
    for (int i = 1; i <= l; ++i) {
        const double* pr = pri + (size_t)(i - 1) * P_NREC;
        uint8_t r = read[i - 1];
        Mc[0] = 0.0; Ic[0] = 0.0; Dc[0] = 0.0;
        for (int j = 1; j <= k; ++j) {
            double p = emission(pr, r, hap[j - 1]);
            double a = pr[P_TMM] * Mp[j - 1];
            double b = pr[P_TIM] * Ip[j - 1];
            double c = pr[P_TDM] * Dp[j - 1];
            Mc[j] = p * ((a + b) + c);
            Ic[j] = pr[P_TMI] * Mp[j] + pr[P_TII] * Ip[j];
            Dc[j] = pr[P_TMD] * Mc[j - 1] + pr[P_TDD] * Dc[j - 1];
        }
        if (rescale) {
            double s = 0.0;
            for (size_t j = 0; j < n; ++j) {
                if (Mc[j] > s) s = Mc[j];
                if (Ic[j] > s) s = Ic[j];
                if (Dc[j] > s) s = Dc[j];
            }
            if (s > 0.0) {
                int e;
                frexp(s, &e);
                if (e > -1000 && e < 1000) {
                    /* 2^-e is a normal double: x * 2^-e is the correctly
                     * rounded value of the same exact product as ldexp. */
                    const double f = ldexp(1.0, -e);
                    for (size_t j = 0; j < n; ++j) {
                        Mc[j] = Mc[j] * f;
                        Ic[j] = Ic[j] * f;
                        Dc[j] = Dc[j] * f;
                    }
                } else {
                    for (size_t j = 0; j < n; ++j) {
                        Mc[j] = ldexp(Mc[j], -e);
                        Ic[j] = ldexp(Ic[j], -e);
                        Dc[j] = ldexp(Dc[j], -e);
                    }
                }
                ex += e;
            }
        }
        double* t;
        t = Mp; Mp = Mc; Mc = t;
        t = Ip; Ip = Ic; Ic = t;
        t = Dp; Dp = Dc; Dc = t;
    }
    double s = 0.0;
    for (int j = 1; j <= k; ++j) s = s + (Mp[j] + Ip[j]);
    *S = s;
    *E = ex;
    free(buf);
    return 0;
}

/* log10 L from the scaled sum: L = S * 2^(E - 1020).  S is split into
 * mantissa and exponent first so the 2^1020 start scale cancels exactly in
 * integer arithmetic instead of in floating point. */
static double to_log10(double S, int64_t E)
{
    if (!(S > 0.0)) return -INFINITY;
    int e;
    double m = frexp(S, &e);
    return log10(m) + (double)((int64_t)e + E - 1020) * log10(2.0);
}

/* Anti-diagonal evaluation order (the prior parallelisation of Section 2):
 * the same cell expressions as above, computed diagonal by diagonal over
 * full matrices.  Without rescaling it must agree bit for bit with the row
 * order. */
int oracle_forward_antidiag_probs(const double* pri, const uint8_t* read, int l,
                                  const uint8_t* hap, int k, double* S)
{
    if (l <= 0 || k <= 0 || !pri || !read || !hap || !S) return -1;
    size_t w = (size_t)k + 1, h = (size_t)l + 1;
    double* M = (double*)calloc(w * h, sizeof(double));
    double* I = (double*)calloc(w * h, sizeof(double));
    double* D = (double*)calloc(w * h, sizeof(double));
    if (!M || !I || !D) { free(M); free(I); free(D); return -2; }
    double d0 = start_value(k);
    for (size_t j = 0; j < w; ++j) D[j] = d0;
    for (int d = 2; d <= l + k; ++d) {
        int ilo = d - k > 1 ? d - k : 1;
        int ihi = d - 1 < l ? d - 1 : l;
        for (int i = ilo; i <= ihi; ++i) {
            int j = d - i;
            const double* pr = pri + (size_t)(i - 1) * P_NREC;
            double p = emission(pr, read[i - 1], hap[j - 1]);
            size_t c = (size_t)i * w + (size_t)j, up = c - w, lf = c - 1, dg = up - 1;
            double a = pr[P_TMM] * M[dg];
            double b = pr[P_TIM] * I[dg];
            double cc = pr[P_TDM] * D[dg];
            M[c] = p * ((a + b) + cc);
            I[c] = pr[P_TMI] * M[up] + pr[P_TII] * I[up];
            D[c] = pr[P_TMD] * M[lf] + pr[P_TDD] * D[lf];
        }
    }
    double s = 0.0;
    for (int j = 1; j <= k; ++j) s = s + (M[(size_t)l * w + j] + I[(size_t)l * w + j]);
    *S = s;
    free(M); free(I); free(D);
    return 0;
}

/* Row-level formulation of Section 3.1 (eq.7) evaluated as written: the D
 * matrix is never formed; each M(i,j), i >= 2, takes the delete term as
 * T_DM_i T_MD_{i-1} sum_{b=1}^{j-2} M(i-1,b) T_DD_{i-1}^{j-2-b}, computed
 * directly in O(k^2) per row.  Row 1 takes its delete term from the start
 * row D(0,j) = C/k of eq.1. */
int oracle_forward_rowform_probs(const double* pri, const uint8_t* read, int l,
                                 const uint8_t* hap, int k, double* S)
{
    if (l <= 0 || k <= 0 || !pri || !read || !hap || !S) return -1;
    size_t n = (size_t)k + 1;
    double* Mp = (double*)calloc(n, sizeof(double));
    double* Ip = (double*)calloc(n, sizeof(double));
    double* Mc = (double*)calloc(n, sizeof(double));
    double* Ic = (double*)calloc(n, sizeof(double));
    double* pw = (double*)calloc(n, sizeof(double));
    if (!Mp || !Ip || !Mc || !Ic || !pw) {
        free(Mp); free(Ip); free(Mc); free(Ic); free(pw); return -2;
    }
    double d0 = start_value(k);
    for (int i = 1; i <= l; ++i) {
        const double* pr = pri + (size_t)(i - 1) * P_NREC;
        uint8_t r = read[i - 1];
        Mc[0] = 0.0; Ic[0] = 0.0;
        if (i == 1) {
            for (int j = 1; j <= k; ++j) {
                double p = emission(pr, r, hap[j - 1]);
                Mc[j] = p * (pr[P_TDM] * d0);
                Ic[j] = 0.0;
            }
        } else {
            const double* pq = pri + (size_t)(i - 2) * P_NREC; /* row i-1 */
            pw[0] = 1.0;
            for (int m = 1; m < k; ++m) pw[m] = pw[m - 1] * pq[P_TDD];
            for (int j = 1; j <= k; ++j) {
                double sum = 0.0;
                for (int b = 1; b <= j - 2; ++b) sum += Mp[b] * pw[j - 2 - b];
                double dterm = pr[P_TDM] * (pq[P_TMD] * sum);
                double p = emission(pr, r, hap[j - 1]);
                Mc[j] = p * ((pr[P_TMM] * Mp[j - 1] + pr[P_TIM] * Ip[j - 1]) + dterm);
                Ic[j] = pr[P_TMI] * Mp[j] + pr[P_TII] * Ip[j];
            }
        }
        double* t;
        t = Mp; Mp = Mc; Mc = t;
        t = Ip; Ip = Ic; Ic = t;
    }
    double s = 0.0;
    for (int j = 1; j <= k; ++j) s = s + (Mp[j] + Ip[j]);
    *S = s;
    free(Mp); free(Ip); free(Mc); free(Ic); free(pw);
    return 0;
}

/* One pair from raw Phred inputs: log10 P(read | hap). */
int oracle_forward_one(const uint8_t* read, const uint8_t* bq, const uint8_t* iq,
                       const uint8_t* dq, const uint8_t* gq, int l,
                       const uint8_t* hap, int k, int rescale,
                       double* out_log10, double* out_S, int64_t* out_E)
{
    if (l <= 0 || k <= 0 || !out_log10) return -1;
    double* pri = (double*)malloc(sizeof(double) * (size_t)l * P_NREC);
    if (!pri) return -2;
    int rc = oracle_priors(bq, iq, dq, gq, l, pri);
    double S = 0.0;
    int64_t E = 0;
    if (rc == 0) rc = oracle_forward_probs(pri, read, l, hap, k, rescale, &S, &E);
    free(pri);
    if (rc != 0) return rc;
    *out_log10 = to_log10(S, E);
    if (out_S) *out_S = S;
    if (out_E) *out_E = E;
    return 0;
}

/* A list of (read, haplotype) pairs over CSR-packed inputs, one after the
 * other.  pair_list holds n_pairs (read index, haplotype index) entries. */
int oracle_forward_pairs(const uint8_t* reads, const uint8_t* bq, const uint8_t* iq,
                         const uint8_t* dq, const uint8_t* gq,
                         const uint64_t* read_offsets, uint32_t n_reads,
                         const uint8_t* haps, const uint64_t* hap_offsets, uint32_t n_haps,
                         const uint32_t* pair_list, uint64_t n_pairs, int rescale,
                         double* out_log10)
{
    for (uint64_t p = 0; p < n_pairs; ++p) {
        uint32_t r = pair_list[2 * p], h = pair_list[2 * p + 1];
        if (r >= n_reads || h >= n_haps) return -1;
        uint64_t r0 = read_offsets[r], r1 = read_offsets[r + 1];
        uint64_t h0 = hap_offsets[h], h1 = hap_offsets[h + 1];
        int rc = oracle_forward_one(reads + r0, bq + r0, iq + r0, dq + r0, gq + r0,
                                    (int)(r1 - r0), haps + h0, (int)(h1 - h0), rescale,
                                    out_log10 + p, NULL, NULL);
        if (rc != 0) return rc;
    }
    return 0;
}
