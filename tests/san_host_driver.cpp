// Test driver for the library's host runtime under AddressSanitizer and
// UndefinedBehaviorSanitizer (host code only; the device code is unchanged
// and no device is used).
//   san_host_driver validate DIR : phmm_validate_batch on the batch stored as
//                                  raw files in DIR; prints rc, the longest
//                                  read and haplotype, and the message
//   san_host_driver options      : option checks of phmm_create
// Every input array is an exactly sized heap block, so a read past its end
// is reported.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "phmm.h"

static std::vector<unsigned char> slurp(const char* dir, const char* name)
{
    char path[4096];
    snprintf(path, sizeof path, "%s/%s.bin", dir, name);
    FILE* f = fopen(path, "rb");
    if (!f) { perror(path); exit(2); }
    fseek(f, 0, SEEK_END);
    const long sz = ftell(f);
    fseek(f, 0, SEEK_SET);
    std::vector<unsigned char> v((size_t)sz);
    if (sz > 0 && fread(v.data(), 1, (size_t)sz, f) != (size_t)sz) exit(2);
    fclose(f);
    return v;
}

template <typename T>
static T* heap_copy(const std::vector<unsigned char>& v)
{
    T* p = static_cast<T*>(malloc(v.size() ? v.size() : 1));
    memcpy(p, v.data(), v.size());
    return p;
}

static int validate(const char* d)
{
    const char* names[9] = {"reads", "base_quals", "ins_quals", "del_quals", "gcp",
                            "read_offsets", "haplotypes", "hap_offsets", "pair_list"};
    std::vector<unsigned char> raw[9];
    for (int i = 0; i < 9; ++i) raw[i] = slurp(d, names[i]);
    uint8_t* a[5];
    for (int i = 0; i < 5; ++i) a[i] = heap_copy<uint8_t>(raw[i]);
    uint64_t* ro = heap_copy<uint64_t>(raw[5]);
    uint8_t* haps = heap_copy<uint8_t>(raw[6]);
    uint64_t* ho = heap_copy<uint64_t>(raw[7]);
    uint32_t* pl = heap_copy<uint32_t>(raw[8]);
    const uint32_t n_reads = (uint32_t)(raw[5].size() / 8) - 1, n_haps = (uint32_t)(raw[7].size() / 8) - 1;
    uint32_t ml = 0, mk = 0;
    const int rc = phmm_validate_batch(a[0], a[1], a[2], a[3], a[4], ro, n_reads, haps, ho,
                                       n_haps, pl, raw[8].size() / 8, &ml, &mk);
    printf("%d %u %u %s\n", rc, ml, mk, phmm_last_error());
    for (int i = 0; i < 5; ++i) free(a[i]);
    free(ro);
    free(haps);
    free(ho);
    free(pl);
    return 0;
}

static int options()
{
    struct Case {
        const char* what;
        void (*set)(phmm_options*);
    };
    const Case cases[] = {
        {"precision 7", [](phmm_options* o) { o->precision = 7; }},
        {"accept_min_sum 0", [](phmm_options* o) { o->accept_min_sum = 0.0; }},
        {"accept_min_sum 1e-45", [](phmm_options* o) { o->accept_min_sum = 1e-45; }},
        {"accept_min_sum 1e-31", [](phmm_options* o) { o->accept_min_sum = 1e-31; }},
        {"accept_min_sum nan", [](phmm_options* o) { o->accept_min_sum = NAN; }},
        {"accept_min_sum 1e39", [](phmm_options* o) { o->accept_min_sum = 1e39; }},
        {"force_class 21", [](phmm_options* o) { o->force_class = 21; }},
        {"force_class -2", [](phmm_options* o) { o->force_class = -2; }},
        {"route_diverse_fp64 2", [](phmm_options* o) { o->route_diverse_fp64 = 2; }},
    };
    for (const Case& c : cases) {
        phmm_options o;
        phmm_default_options(&o);
        c.set(&o);
        phmm_ctx* ctx = nullptr;
        const int rc = phmm_create(&ctx, 0, &o);
        printf("%s|%d|%s|%d\n", c.what, rc, phmm_last_error(), ctx == nullptr);
        phmm_destroy(ctx);
    }
    return 0;
}

int main(int argc, char** argv)
{
    if (argc == 3 && !strcmp(argv[1], "validate")) return validate(argv[2]);
    if (argc == 2 && !strcmp(argv[1], "options")) return options();
    fprintf(stderr, "usage: %s validate DIR | options\n", argv[0]);
    return 2;
}
