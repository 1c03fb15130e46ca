/* Test driver for the host C code under AddressSanitizer and
 * UndefinedBehaviorSanitizer: reads a batch from raw files in a directory
 * (the CSR arrays of the binding's batch dict), runs either the oracle or the
 * CPU row-form comparator over every pair, and writes the log10 likelihoods
 * to out.bin.  Built with gcc together with exactly one of the two sources
 * (-DUSE_ORACLE or -DUSE_ROWFORM). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#if defined(USE_ORACLE)
int oracle_forward_pairs(const uint8_t* reads, const uint8_t* bq, const uint8_t* iq,
                         const uint8_t* dq, const uint8_t* gq, const uint64_t* read_offsets,
                         uint32_t n_reads, const uint8_t* haps, const uint64_t* hap_offsets,
                         uint32_t n_haps, const uint32_t* pair_list, uint64_t n_pairs,
                         int rescale, double* out_log10);
#elif defined(USE_ROWFORM)
int rf_forward_pairs(const uint8_t* reads, const uint8_t* bq, const uint8_t* iq,
                     const uint8_t* dq, const uint8_t* gq, const uint64_t* read_off,
                     const uint8_t* haps, const uint64_t* hap_off, const uint32_t* pairs,
                     uint64_t n_pairs, int threads, double* out_log10, uint8_t* out_flags);
#else
#error "define USE_ORACLE or USE_ROWFORM"
#endif

/* whole file into an exactly sized heap block, so that any read past the end
 * of an array is a heap overflow the sanitizer reports */
static void* slurp(const char* dir, const char* name, size_t* n)
{
    char path[4096];
    snprintf(path, sizeof path, "%s/%s.bin", dir, name);
    FILE* f = fopen(path, "rb");
    if (!f) { perror(path); exit(2); }
    fseek(f, 0, SEEK_END);
    long sz = ftell(f);
    fseek(f, 0, SEEK_SET);
    void* p = malloc(sz > 0 ? (size_t)sz : 1);
    if (!p || fread(p, 1, (size_t)sz, f) != (size_t)sz) { fprintf(stderr, "read %s\n", path); exit(2); }
    fclose(f);
    *n = (size_t)sz;
    return p;
}

int main(int argc, char** argv)
{
    if (argc != 2) { fprintf(stderr, "usage: %s DIR\n", argv[0]); return 2; }
    const char* d = argv[1];
    size_t nb, nro, nh, nho, npl, t;
    uint8_t* reads = slurp(d, "reads", &nb);
    uint8_t* bq = slurp(d, "base_quals", &t);
    uint8_t* iq = slurp(d, "ins_quals", &t);
    uint8_t* dq = slurp(d, "del_quals", &t);
    uint8_t* gq = slurp(d, "gcp", &t);
    uint64_t* ro = slurp(d, "read_offsets", &nro);
    uint8_t* haps = slurp(d, "haplotypes", &nh);
    uint64_t* ho = slurp(d, "hap_offsets", &nho);
    uint32_t* pl = slurp(d, "pair_list", &npl);
    const uint64_t n_pairs = npl / 8;
    double* out = malloc((n_pairs ? n_pairs : 1) * sizeof(double));
    int rc;
#if defined(USE_ORACLE)
    rc = oracle_forward_pairs(reads, bq, iq, dq, gq, ro, (uint32_t)(nro / 8 - 1), haps, ho,
                              (uint32_t)(nho / 8 - 1), pl, n_pairs, 1, out);
#else
    uint8_t* fl = malloc(n_pairs ? n_pairs : 1);
    rc = rf_forward_pairs(reads, bq, iq, dq, gq, ro, haps, ho, pl, n_pairs, 2, out, fl);
    free(fl);
#endif
    if (rc != 0) { fprintf(stderr, "forward returned %d\n", rc); return 1; }
    char path[4096];
    snprintf(path, sizeof path, "%s/out.bin", d);
    FILE* f = fopen(path, "wb");
    fwrite(out, sizeof(double), n_pairs, f);
    fclose(f);
    free(out); free(reads); free(bq); free(iq); free(dq); free(gq); free(ro); free(haps);
    free(ho); free(pl);
    return 0;
}
