/*
 * Seeded synthetic PairHMM workloads (reads, qualities, haplotypes, pairs).
 *
 * This module only draws sequences and quality bytes; it holds none of the
 * PairHMM arithmetic.  Both the tests/oracle side and the benchmark use it.
 *
 * Randomness is counter based: every region r of a workload with seed s has
 * its own key mix(s, r), and the t-th draw of that region is
 * splitmix64(key + t * golden).  Any region can therefore be regenerated on
 * its own, and two passes over a region (one to size it, one to fill it)
 * see exactly the same draws.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n_haps_lo, n_haps_hi;      /* haplotypes per region ~ U{lo..hi}           */
    int hap_len_lo, hap_len_hi;    /* base haplotype length ~ U{lo..hi}           */
    int hap_mode;                  /* 0: i.i.d. haplotypes; 1: hap 0 + variants   */
    int var_lo, var_hi;            /* variants per alternative haplotype          */
    double var_snp_frac;           /* fraction of variants that are SNPs          */
    int var_indel_lo, var_indel_hi;
    int reads_mode;                /* 0: fixed count; 1: lognormal                */
    int reads_fixed;
    double reads_mu, reads_sigma;
    int reads_cap;
    int read_len_lo, read_len_hi;  /* read length ~ U{lo..hi}                     */
    int n_len_classes;             /* >0: read length by region class instead     */
    int len_classes[4];
    int regions_per_class;
    double hap_len_factor;         /* >0: hap length = round(factor * read len)   */
    double p_sub, p_indel;
    int indel_lo, indel_hi;
    int q_lo, q_hi, ins_q, del_q, gcp_q;
    int offset_mode;               /* 0: U{0..k-l}; 1: U{0..floor(frac*l)}        */
    double offset_frac;
    /* Mixed streams: a region is "long" with probability long_frac; all its
     * reads then have one length ~ U{long_len_lo..hi}, it has
     * U{long_haps_lo..hi} haplotypes of length round(long_hap_factor * len). */
    double long_frac;
    int long_len_lo, long_len_hi;
    int long_haps_lo, long_haps_hi;
    double long_hap_factor;
} synth_cfg;

typedef struct {
    uint64_t n_haps, hap_bases, n_reads, read_bases, n_pairs;
} synth_sizes;

typedef struct {
    uint64_t key, ctr;
} rng_t;

static uint64_t splitmix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static rng_t rng_for(uint64_t seed, uint64_t region)
{
    rng_t r;
    r.key = splitmix(splitmix(seed * 0xD1B54A32D192ED03ull + 0x8CB92BA72F3D8DD7ull) ^ region);
    r.ctr = 0;
    return r;
}

static uint64_t next_u64(rng_t* r) { return splitmix(r->key + 0x9E3779B97F4A7C15ull * (r->ctr++)); }
static double next_unit(rng_t* r) { return (double)(next_u64(r) >> 11) * 0x1.0p-53; }
static int next_int(rng_t* r, int lo, int hi) /* uniform on {lo..hi} */
{
    if (hi <= lo) return lo;
    uint64_t span = (uint64_t)(hi - lo) + 1;
    return lo + (int)(next_u64(r) % span);
}
static double next_normal(rng_t* r)
{
    double u1 = next_unit(r), u2 = next_unit(r);
    if (u1 < 1e-300) u1 = 1e-300;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

static const uint8_t BASES[4] = {'A', 'C', 'G', 'T'};

static uint8_t other_base(rng_t* r, uint8_t b)
{
    for (;;) {
        uint8_t c = BASES[next_int(r, 0, 3)];
        if (c != b) return c;
    }
}

/* Output buffers of one region (NULL buf => sizing pass). */
typedef struct {
    uint8_t* haps;     /* region's haplotype bases                    */
    uint64_t* hap_off; /* n_haps local start offsets                  */
    uint8_t *reads, *bq, *iq, *dq, *gq;
    uint64_t* read_off;
    int32_t* cols;     /* optional: aligned hap column per read base  */
    uint32_t* pairs;   /* 2 x n_pairs, local indices                  */
} region_out;

static int region_read_len(const synth_cfg* c, rng_t* r, uint64_t region)
{
    if (c->n_len_classes > 0) {
        uint64_t cls = region / (uint64_t)(c->regions_per_class > 0 ? c->regions_per_class : 1);
        if (cls >= (uint64_t)c->n_len_classes) cls = (uint64_t)c->n_len_classes - 1;
        return c->len_classes[cls];
    }
    return next_int(r, c->read_len_lo, c->read_len_hi);
}

/* Generates (or sizes) one region.  All draws happen in the same order in
 * both passes.  Returns 0 or -1 on allocation failure. */
static int gen_region(const synth_cfg* c, uint64_t seed, uint64_t region,
                      region_out* o, synth_sizes* sz)
{
    rng_t r = rng_for(seed, region);
    int fill = o != NULL;
    int is_long = c->long_frac > 0 && next_unit(&r) < c->long_frac;
    int H = is_long ? next_int(&r, c->long_haps_lo, c->long_haps_hi)
                    : next_int(&r, c->n_haps_lo, c->n_haps_hi);
    /* Read length is drawn up front when the haplotype length depends on it. */
    int first_len = is_long ? next_int(&r, c->long_len_lo, c->long_len_hi)
                            : region_read_len(c, &r, region);
    int K = is_long ? (int)llround(c->long_hap_factor * first_len)
          : c->hap_len_factor > 0 ? (int)llround(c->hap_len_factor * first_len)
                                  : next_int(&r, c->hap_len_lo, c->hap_len_hi);
    int maxlen = K + c->var_hi * (c->var_indel_hi > 0 ? c->var_indel_hi : 0) + 8;
    uint8_t* hbuf = (uint8_t*)malloc((size_t)maxlen * (size_t)(H > 0 ? H : 1));
    int* hlen = (int*)malloc(sizeof(int) * (size_t)(H > 0 ? H : 1));
    uint8_t* tmp = (uint8_t*)malloc((size_t)maxlen);
    if (!hbuf || !hlen || !tmp) { free(hbuf); free(hlen); free(tmp); return -1; }
    for (int h = 0; h < H; ++h) {
        uint8_t* dst = hbuf + (size_t)h * maxlen;
        if (h == 0 || c->hap_mode == 0) {
            for (int j = 0; j < K; ++j) dst[j] = BASES[next_int(&r, 0, 3)];
            hlen[h] = K;
            continue;
        }
        memcpy(dst, hbuf, (size_t)hlen[0]);
        int len = hlen[0];
        int nv = next_int(&r, c->var_lo, c->var_hi);
        for (int v = 0; v < nv; ++v) {
            double u = next_unit(&r);
            int pos = next_int(&r, 0, len - 1);
            if (u < c->var_snp_frac) {
                dst[pos] = other_base(&r, dst[pos]);
            } else if (next_unit(&r) < 0.5) { /* insertion before pos */
                int L = next_int(&r, c->var_indel_lo, c->var_indel_hi);
                if (len + L > maxlen) L = maxlen - len;
                memcpy(tmp, dst + pos, (size_t)(len - pos));
                for (int q = 0; q < L; ++q) dst[pos + q] = BASES[next_int(&r, 0, 3)];
                memcpy(dst + pos + L, tmp, (size_t)(len - pos));
                len += L;
            } else { /* deletion at pos */
                int L = next_int(&r, c->var_indel_lo, c->var_indel_hi);
                if (L > len - 1 - pos) L = len - 1 - pos;
                if (L < 0) L = 0;
                memmove(dst + pos, dst + pos + L, (size_t)(len - pos - L));
                len -= L;
            }
        }
        hlen[h] = len;
    }
    int R;
    if (c->reads_mode == 1) {
        double x = exp(c->reads_mu + c->reads_sigma * next_normal(&r));
        R = (int)llround(x);
        if (R < 1) R = 1;
        if (R > c->reads_cap) R = c->reads_cap;
    } else {
        R = c->reads_fixed;
    }
    uint64_t hap_bases = 0;
    for (int h = 0; h < H; ++h) {
        if (fill) {
            o->hap_off[h] = hap_bases;
            memcpy(o->haps + hap_bases, hbuf + (size_t)h * maxlen, (size_t)hlen[h]);
        }
        hap_bases += (uint64_t)hlen[h];
    }
    uint64_t read_bases = 0;
    for (int q = 0; q < R; ++q) {
        int l = (q == 0 || is_long) ? first_len : region_read_len(c, &r, region);
        int src = next_int(&r, 0, H - 1);
        int k = hlen[src];
        const uint8_t* hs = hbuf + (size_t)src * maxlen;
        int off;
        if (c->offset_mode == 1) off = next_int(&r, 0, (int)floor(c->offset_frac * l));
        else off = k >= l ? next_int(&r, 0, k - l) : 0;
        if (fill) o->read_off[q] = read_bases;
        int pos = off, valid = 1;
        int e = 0;
        while (e < l) {
            double u = next_unit(&r);
            if (u < c->p_indel) {
                int ins = next_unit(&r) < 0.5;
                int L = next_int(&r, c->indel_lo, c->indel_hi);
                if (ins) {
                    for (int t = 0; t < L && e < l; ++t, ++e) {
                        uint8_t b = BASES[next_int(&r, 0, 3)];
                        if (fill) {
                            o->reads[read_bases + e] = b;
                            if (o->cols) o->cols[read_bases + e] = valid ? 0 : -1;
                        }
                    }
                    continue;
                }
                pos += L; /* deletion: skip haplotype bases, then emit */
            }
            uint8_t b;
            int col;
            if (pos < k) {
                b = hs[pos];
                if (next_unit(&r) < c->p_sub) b = other_base(&r, b);
                col = pos + 1;
            } else {
                b = BASES[next_int(&r, 0, 3)];
                valid = 0;
                col = -1;
            }
            if (fill) {
                o->reads[read_bases + e] = b;
                if (o->cols) o->cols[read_bases + e] = valid ? col : -1;
            }
            ++pos;
            ++e;
        }
        for (int t = 0; t < l; ++t) {
            uint8_t bq = (uint8_t)next_int(&r, c->q_lo, c->q_hi);
            if (fill) {
                o->bq[read_bases + t] = bq;
                o->iq[read_bases + t] = (uint8_t)c->ins_q;
                o->dq[read_bases + t] = (uint8_t)c->del_q;
                o->gq[read_bases + t] = (uint8_t)c->gcp_q;
            }
        }
        read_bases += (uint64_t)l;
    }
    if (fill) {
        uint64_t p = 0;
        for (int q = 0; q < R; ++q)
            for (int h = 0; h < H; ++h, ++p) {
                o->pairs[2 * p] = (uint32_t)q;
                o->pairs[2 * p + 1] = (uint32_t)h;
            }
    }
    sz->n_haps = (uint64_t)H;
    sz->hap_bases = hap_bases;
    sz->n_reads = (uint64_t)R;
    sz->read_bases = read_bases;
    sz->n_pairs = (uint64_t)R * (uint64_t)H;
    free(hbuf); free(hlen); free(tmp);
    return 0;
}

/* Pass 1: sizes of regions [r0, r0+n). */
int synth_size(const synth_cfg* c, uint64_t seed, uint64_t r0, uint64_t n, synth_sizes* out)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int64_t q = 0; q < (int64_t)n; ++q)
        bad |= gen_region(c, seed, r0 + (uint64_t)q, NULL, out + q) != 0;
    return bad ? -1 : 0;
}

/* Pass 2: fill regions [r0, r0+n) at the global offsets of pass 1.  The
 * prefix arrays hold, per region, the first global hap / hap base / read /
 * read base / pair index.  Offsets written are global; pair entries hold
 * global read and haplotype indices. */
int synth_fill(const synth_cfg* c, uint64_t seed, uint64_t r0, uint64_t n,
               const uint64_t* hap0, const uint64_t* hapb0, const uint64_t* read0,
               const uint64_t* readb0, const uint64_t* pair0,
               uint8_t* haps, uint64_t* hap_off, uint8_t* reads, uint8_t* bq, uint8_t* iq,
               uint8_t* dq, uint8_t* gq, uint64_t* read_off, uint32_t* pairs, int32_t* cols)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int64_t q = 0; q < (int64_t)n; ++q) {
        region_out o;
        synth_sizes sz;
        o.haps = haps + hapb0[q];
        o.hap_off = hap_off + hap0[q];
        o.reads = reads + readb0[q];
        o.bq = bq + readb0[q];
        o.iq = iq + readb0[q];
        o.dq = dq + readb0[q];
        o.gq = gq + readb0[q];
        o.read_off = read_off + read0[q];
        o.cols = cols ? cols + readb0[q] : NULL;
        o.pairs = pairs + 2 * pair0[q];
        /* Offsets are written region-local, then shifted; the closing entry
         * of the whole batch is set by the caller. */
        if (gen_region(c, seed, r0 + (uint64_t)q, &o, &sz) != 0) { bad = 1; continue; }
        for (uint64_t h = 0; h < sz.n_haps; ++h) o.hap_off[h] += hapb0[q];
        for (uint64_t t = 0; t < sz.n_reads; ++t) o.read_off[t] += readb0[q];
        for (uint64_t p = 0; p < sz.n_pairs; ++p) {
            o.pairs[2 * p] += (uint32_t)read0[q];
            o.pairs[2 * p + 1] += (uint32_t)hap0[q];
        }
    }
    return bad ? -1 : 0;
}
