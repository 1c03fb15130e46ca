// Internal definitions shared by the host runtime and the gfx950 kernels of
// the PairHMM forward library.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace phmm {

// Column classes: a class fixes N, the number of consecutive haplotype
// columns each lane of a wavefront owns in the row-level formulation
// (paper Section 3.2: "each individual thread reads N characters from the
// haplotype and calculates N elements of a M and I row").  A pair of
// haplotype length k occupies ceil(k / N) lanes; pairs of one read are packed
// side by side into one 64-lane wavefront.
// N = 4, 5, ..., 24: odd widths as well as even ones, so that the packer can
// match a read's haplotype lengths more closely (fewer idle lanes).
constexpr int kNumClasses = 21;
__host__ __device__ constexpr int class_n(int c) { return 4 + c; }
__host__ __device__ constexpr int class_of_n(int n) { return n - 4; }
constexpr int kMaxN = 24;
constexpr int kWave = 64;
constexpr uint32_t kShortMaxCols = kWave * kMaxN;  // longer haplotypes use the long kernel
constexpr int kMaxPairsPerPack = 32;                // pair mask is 32 bits
constexpr int kChunk = 256;                         // pairs walked by one packer thread
constexpr int kPackBlock = 256;                     // packer threads per workgroup

// Power table: for class c and gap-continuation Phred byte q, entry m
// (0..64) holds g^(N*m) with g = 10^(-q/10); entry 65 holds g^(N-1).
constexpr int kPowStride = 66;

// Long-pair kernel: one wavefront per tile of 64 lanes x 16 columns; kRing
// rows of boundary records buffered per tile.
constexpr int kRing = 512;

// Long-pair lists: q = 2 * precision + general.  [0] FP32 and [2] FP64 hold
// pairs whose read has one gap byte (>= 1) on every row and insertion bytes
// the scaled row form allows, run by a lean kernel without per-row gap
// changes or the plain form; [1] FP32 and [3] FP64 hold the others (and the
// FP64 pairs whose short-kernel sum underflowed).
constexpr int kLongLists = 4;
__host__ __device__ constexpr int long_list_of(int prec, bool general) { return 2 * prec + (general ? 1 : 0); }

struct Pack {
    uint32_t pair_start;  // first pair (index into pair_list)
    uint32_t npairs;      // consecutive pairs, all of the same read
};

struct Item {             // FP64 rerun item: an FP32 pack and the subset of its pairs
    uint32_t pack;        // global pack index
    uint32_t mask;        // bit s: pair pair_start + s is computed
};

// Pack segments: a pack belongs to one (precision, class) segment, [0] FP32,
// [1] FP64.  The fast FP32 kernel runs the FP32 packs whose read has one gap
// penalty on every row and fits the scaled row form; it defers the others to
// the general FP32 kernel of the class.
constexpr int kSeg = 2 * kNumClasses;
enum KernelKind : int { kFast32 = 0, kGen32 = 1, kAll64 = 2, kNumKernelKinds = 3 };

// Largest insertion Phred byte of the scaled row form (see make_row_rec).
constexpr int kScMaxInsQ = 65;

// Device counters of one call (lives at the start of the workspace).
struct Counters {
    uint32_t pack_cnt[2][kNumClasses];   // [0] FP32 packs, [1] FP64 packs
    uint32_t pack_base[2][kNumClasses];
    uint32_t item_base[kNumClasses];     // rerun items and deferred packs of class k
    uint32_t item_cnt[kNumClasses];      // rerun items queued by the FP32 kernels
    uint32_t defer_cnt[kNumClasses];     // FP32 packs deferred to the general kernel
    uint32_t cursor[kNumKernelKinds][kNumClasses];  // next pack or item of each kernel
    uint32_t n_pend[2];                  // long pairs per precision before routing
    uint32_t n_long[kLongLists];         // long pairs per list (long_list_of)
    uint32_t long_tiles[kLongLists];
    uint32_t long_cursor;
    uint32_t status;                     // 0 or a PHMM_E* code (as uint32); stops the long kernels
    uint32_t bound_err;                  // a long pair in a batch whose bound says none
    uint32_t rerun_pairs;                // counted by the FP64 kernel
    unsigned long long lane_columns;
};

// Everything a kernel needs to find inputs and outputs.
struct Batch {
    const uint8_t* reads;
    const uint8_t* bq;
    const uint8_t* iq;
    const uint8_t* dq;
    const uint8_t* gq;
    const uint64_t* read_off;
    const uint8_t* haps;
    const uint64_t* hap_off;
    const uint32_t* pairs;
    uint64_t n_pairs;
    double* out;
    uint8_t* flags;
};

struct Tables {
    const double* p64;     // 10^(-q/10), q = 0..255
    const double* pw64;    // kNumClasses x 256 x kPowStride
    const float* pw32;     // same, rounded to FP32
};

struct Work {
    Counters* ctr;
    uint32_t* chunk_info;  // per pair (chunk starts only)
    uint32_t* blk_cnt;     // [segment][packer block]: pack count, then offset
    unsigned long long* blk_lanecols;  // per packer block
    uint32_t* chunk_part;  // [segment][scan chunk]: pack count, then offset
    uint32_t n_pack_blocks;
    uint32_t n_scan_chunks;
    Pack* packs;           // pack array, segments per (precision, class)
    Item* items;           // FP64 items, segments per class
    uint32_t* deferred;    // FP32 packs for the general kernel, segments per class
    uint32_t* long_pend[2];            // long pairs per precision, before routing
    uint32_t* long_list[kLongLists];  // long pair indices per list (long_list_of)
    uint32_t* long_pref;   // tile prefix of the list being run (n_long + 1)
    double* long_ring;     // per slot: kRing x 4 records, then the final sum
    uint32_t* long_prog;   // per slot: rows consumed, owner, done
};

// Sets the calling thread's phmm_last_error() message; returns code.
int set_error(int code, const char* msg);

}  // namespace phmm
struct phmm_ctx;
struct phmm_device_batch;
namespace phmm {

// phmm_forward_batch_async's checks and work, launched as a synchronising pass:
// the host reads the device counters between kernel families and launches
// only kernels that have work.  Returns once the last kernels are enqueued;
// the caller waits on the stream for them and for its own copies.
int forward_device_batch_sync(phmm_ctx* c, const phmm_device_batch* db, double* d_out,
                              uint8_t* d_flags, void* d_ws, size_t ws_bytes, hipStream_t s);

// Caps every persistent grid of a context at percent % of a full chip's (the
// long-pair kernels keep at least kMinLongGrid wavefronts).  Call before the
// context's first batch: the workspace layout follows the long grids.
void scale_grids(phmm_ctx* c, int percent);
constexpr int kMinLongGrid = 1024;

struct Policy {
    int precision;          // 0 FP32+rerun, 1 FP64 plain
    int force_class;        // -1 or class index
    int one_pair_per_wave;
    uint32_t fp32_max_rows;
    uint32_t long_fp32_max_rows;
    float accept_min_sum;
    uint32_t watchdog_spins;
    int route_diverse;      // FP32 mode: reads with unrelated haplotypes start in FP64
    int long_haps;          // the batch's length bound admits long pairs (routing runs)
    float cost[2][kNumClasses];  // relative cost of one wavefront-row per class
};

}  // namespace phmm
