/*
 * phmm.h — C ABI of the MI355X (gfx950) PairHMM forward library.
 *
 * The library computes, for every (read, haplotype) pair of a batch, the
 * PairHMM forward likelihood log10 P(read | haplotype) of the model in
 * Section 2 of Graca & Ilic, "Endeavor: Efficient PairHMM for Detection of
 * DNA Variants in Genome-Scale Datasets" (HPDC '26):
 *
 *   eq.1  M(i,0)=I(i,0)=D(i,0)=M(0,j)=I(0,j)=0,  D(0,j) = C/k
 *   eq.2  M(i,j) = P(r_i|h_j)(T_MM_i M(i-1,j-1) + T_IM I(i-1,j-1) + T_DM D(i-1,j-1))
 *         I(i,j) = T_MI_i M(i-1,j) + T_II I(i-1,j)
 *         D(i,j) = T_MD_i M(i,j-1) + T_DD D(i,j-1)
 *   eq.3  P(r_i|h_j) = 1 - eps_i (match) or eps_i/3 (mismatch), eps_i = 10^(-Q_i/10)
 *   eq.4  L = sum_j M(l,j) + I(l,j)
 *
 * evaluated in the row-level formulation of Section 3.1 (eq.5-7): a whole
 * DP row is updated at once and the within-row Delete chain is resolved as
 * a first-order linear recurrence by a wavefront scan (Section 3.4,
 * Algorithm 1).  It also turns a region's read x haplotype likelihoods into
 * diploid genotype likelihoods (phmm_genotype_batch), the step that follows
 * the PairHMM in the pipeline of Section 1.
 *
 * Value conventions
 *   - bases are upper-case ASCII 'A','C','G','T' or 'N'; 'N' in either
 *     sequence matches any base;
 *   - qualities are raw Phred bytes 0..255 (the paper's -33 is the FASTQ
 *     character offset and is removed by the caller);
 *     T_MI_i = 10^(-ins_i/10), T_MD_i = 10^(-del_i/10),
 *     T_MM_i = max(0, 1 - T_MI_i - T_MD_i), g_i = 10^(-gcp_i/10),
 *     T_II_i = T_DD_i = g_i, T_IM_i = T_DM_i = 1 - g_i
 *     (gcp = 10 gives the paper's constants 0.1 / 0.9);
 *   - the start row is D(0,j) = C/k for j = 0..k (also j = 0), k = haplotype
 *     length, and the result is reported with C divided out:
 *     out_log10 = log10 L.
 *
 * Memory and ownership
 *   - the caller owns every buffer; inputs are read-only for the call;
 *   - the synchronous entry points copy host inputs to the device, run, copy
 *     results back and keep no pointer after they return;
 *   - the asynchronous entry point takes device pointers, enqueues all work
 *     on the caller's HIP stream and returns at once; every buffer must stay
 *     alive until the stream has passed the call.
 *
 * Errors
 *   - every entry point returns PHMM_OK or a negative PHMM_E* code;
 *   - the synchronous entry points validate every input on the host before
 *     any device work; on error nothing is written to the outputs and
 *     phmm_last_error() names the first offending index;
 *   - a phmm_ctx is used by one host thread at a time.
 *
 * There is no CPU fallback: without a usable gfx950 device every compute
 * entry point fails with PHMM_EDEVICE.
 */
#ifndef PHMM_H
#define PHMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PHMM_OK 0
#define PHMM_EINVAL (-1)   /* null pointer, empty sequence, base not in ACGTN, offsets not
                              monotone, index out of range, bad option                  */
#define PHMM_ERANGE (-2)   /* read longer than PHMM_MAX_READ or haplotype longer than
                              PHMM_MAX_HAP                                               */
#define PHMM_ENOMEM (-3)   /* device or host allocation failed, or workspace too small   */
#define PHMM_EDEVICE (-4)  /* HIP error, or no gfx950 device                             */
#define PHMM_ETIMEOUT (-5) /* long-pair kernel watchdog fired                            */
#define PHMM_PENDING 1     /* phmm_server_poll: the region has not completed yet         */

#define PHMM_MAX_READ 131072u
#define PHMM_MAX_HAP (1u << 20)

/* out_flags bits (one byte per pair) */
#define PHMM_FLAG_FP32 0x01u     /* FP32 result accepted                           */
#define PHMM_FLAG_RERUN 0x02u    /* FP32 result rejected, recomputed in FP64       */
#define PHMM_FLAG_LONG 0x04u     /* long-pair (multi-wavefront tile) kernel        */
#define PHMM_FLAG_RESCALED 0x08u /* power-of-two rescaling with integer exponent  */
#define PHMM_FLAG_FP64 0x10u     /* computed in FP64                               */

/* Precision policy. */
#define PHMM_FP32_RERUN 0 /* FP32 with scale 2^120/k; pairs whose FP32 scaled sum
                             is below accept_min_sum (or not finite) rerun in FP64 */
#define PHMM_FP64_PLAIN 1 /* every pair in FP64 with scale 2^1020/k                 */

typedef struct phmm_options {
    int precision;          /* PHMM_FP32_RERUN (default) or PHMM_FP64_PLAIN          */
    double accept_min_sum;  /* FP32 acceptance threshold, in [1e-30, 3e38]; default
                               1e-28.  An FP32 result is accepted iff its scaled sum
                               S32 = L * 2^120 (a fixed scale on every row) is
                               finite, > 0 and >= accept_min_sum (1e-28: log10 L >=
                               -64.12); else the pair is recomputed in FP64.  The
                               fixed scale bounds what FP32's range can lose: along
                               a path the weight only falls, so a cell flushed under
                               2^-149 costs the sum at most 2^-149, at most
                               l*k*2^-149 in all, under 1e-5 of an accepted sum for
                               pairs of up to 10^10 cells.  A threshold above 2^120
                               reruns every pair in FP64.                             */
    int force_class;        /* -1: the packer picks columns-per-lane per region;
                               >= 0: force this class index (see phmm_class_n)       */
    int one_pair_per_wave;  /* 1: no packing, every pair gets its own wavefront      */
    uint32_t fp32_max_rows; /* reads longer than this go straight to FP64; default
                               1024.  At the fixed FP32 scale a read with about 1%
                               errors falls under the acceptance threshold from
                               about a thousand bases on (85% of such pairs at 1536
                               bases), so their FP32 pass would be wasted; FP32
                               rounding bias also grows with the row count.          */
    uint32_t long_fp32_max_rows; /* long pairs (haplotype > 64 x 24) with reads up to
                               this many rows run in the FP32 long kernel, the others
                               in the FP64 one; default 0: every long pair in FP64.
                               The long kernels rescale every 8 rows, which no
                               acceptance test can make safe in FP32 (its range holds
                               2^126 below a tile's largest value, and a path that far
                               under, flushed, can carry the sum later): unrelated
                               read/haplotype pairs with costly gaps and reads with a
                               deletion of about 40 bases or more against their
                               haplotype were off by up to thousands of decades.
                               Where neither occurs (reads sampled from their
                               haplotype with small indels, gap bytes of 10 or less,
                               as in the long-read workload) FP32 stays within 3e-5
                               at 100 kbp; reads with a gap byte above 10 keep FP64
                               whatever this limit.  The per-row coefficients are
                               rounded to FP32 stochastically (unbiased, keyed by the
                               row) and each cell adds its gap terms before its
                               match term, so rounding errors do not add up along
                               the read.                                              */
    uint32_t watchdog_spins;/* long kernel: polls of a neighbour tile before giving
                               up with PHMM_ETIMEOUT; 0 = default                     */
    int timing;             /* 1: record per-phase HIP events (phmm_last_timing)     */
    int route_diverse_fp64; /* 1 (default): in PHMM_FP32_RERUN mode, a read whose
                               haplotypes are mutually unrelated (the 4-mer sets of
                               their first 32 bases: none of the run's next three
                               haplotypes shares half of the first one's) runs in FP64
                               directly.  Such a read can match at most one of its
                               haplotypes well, so most of its pairs would fall below
                               the FP32 threshold and be recomputed anyway; 0: every
                               read starts in FP32.  Results are within the same
                               bounds either way; only the work differs.              */
} phmm_options;

/* Fills *opt with the defaults above. */
void phmm_default_options(phmm_options* opt);

typedef struct phmm_ctx phmm_ctx;

/* Creates a context on HIP device `device` (0-based).  Owns a HIP stream,
 * the quality->probability table in device memory and a growable device
 * arena for the synchronous API.  opt == NULL selects the defaults.
 * Errors: PHMM_EINVAL (out == NULL, bad option), PHMM_EDEVICE (no such
 * device, not gfx950, HIP failure). */
int phmm_create(phmm_ctx** out, int device, const phmm_options* opt);

/* Frees everything the context owns.  NULL is ignored. */
void phmm_destroy(phmm_ctx* ctx);

/* Message of the last error on the calling thread ("" if none). */
const char* phmm_last_error(void);

/* Number of column classes and the columns-per-lane N of class c. */
int phmm_num_classes(void);
int phmm_class_n(int c);

/*
 * Batched forward pass (host buffers, synchronous): log10 of the likelihood
 * L of eq.4 for every pair, from the recurrences of eq.1-3 (Section 2),
 * computed in the row-level formulation of Section 3.1 (eq.5-7).
 *
 * reads, base_quals, ins_quals, del_quals, gcp : n_bases bytes each, the
 *     reads one after another; read r is bytes [read_offsets[r],
 *     read_offsets[r+1]) of every one of the five arrays;
 * read_offsets : n_reads + 1 entries, read_offsets[0] = 0, non-decreasing,
 *     each read at least one base and at most PHMM_MAX_READ;
 * haplotypes / hap_offsets / n_haps : the same layout for haplotypes (each
 *     1..PHMM_MAX_HAP bases);
 * pair_list : n_pairs (read index, haplotype index) uint32 pairs, row-major;
 *     pairs of the same read should be adjacent (the packer groups adjacent
 *     pairs of one read into one wavefront);
 * out_log10 : n_pairs doubles, log10 P(read | hap);
 * out_flags : n_pairs bytes of PHMM_FLAG_* bits, or NULL.
 * n_pairs == 0 is valid and does nothing.
 *
 * The host reads the device's counters between kernel families and
 * launches only kernels that have work.  A batch of at most 8192 pairs
 * (unless options.force_class is set) packs every pair in the narrowest
 * column class whose 64 lanes hold its longest short haplotype (one launch
 * per kernel family; the results agree with the cost model's packing to
 * rounding).  A batch of 2^23 pairs or more is
 * split into up to 16 chunks of consecutive pairs; the inputs a chunk needs
 * are copied on a second stream while the chunks before it compute
 * (phmm_last_timing then describes the last chunk's pass).  Inputs need not
 * be pinned; the call returns when the results are in the host buffers.
 */
int phmm_forward_batch(phmm_ctx* ctx,
                       const uint8_t* reads, const uint8_t* base_quals,
                       const uint8_t* ins_quals, const uint8_t* del_quals,
                       const uint8_t* gcp, const uint64_t* read_offsets, uint32_t n_reads,
                       const uint8_t* haplotypes, const uint64_t* hap_offsets,
                       uint32_t n_haps, const uint32_t* pair_list, uint64_t n_pairs,
                       double* out_log10, uint8_t* out_flags);

/*
 * Host-side validation of a batch exactly as phmm_forward_batch performs it
 * (no device needed): returns PHMM_OK or the first error, with
 * phmm_last_error() naming the offending index.  Optionally reports the
 * longest read and haplotype.
 */
int phmm_validate_batch(const uint8_t* reads, const uint8_t* base_quals,
                        const uint8_t* ins_quals, const uint8_t* del_quals,
                        const uint8_t* gcp, const uint64_t* read_offsets, uint32_t n_reads,
                        const uint8_t* haplotypes, const uint64_t* hap_offsets,
                        uint32_t n_haps, const uint32_t* pair_list, uint64_t n_pairs,
                        uint32_t* max_read_len, uint32_t* max_hap_len);

/*
 * One pair, FP64: log10 L of eq.4 (Section 2, eq.1-4; row-level evaluation
 * of Section 3.1) for one read and one haplotype, the plain drop-in for a
 * per-pair caller.  Runs PHMM_FP64_PLAIN on a library-owned default context
 * on device 0 (created on the first call, guarded by a mutex, kept until the
 * process ends).  Arrays hold read_len resp. hap_len bytes (read_len >= 1,
 * hap_len >= 1); the bases and limits are validated as in
 * phmm_forward_batch.  Errors: PHMM_EINVAL (NULL argument, empty sequence,
 * bad base), PHMM_ERANGE, PHMM_EDEVICE.
 */
int phmm_forward_one(const uint8_t* read, const uint8_t* base_quals,
                     const uint8_t* ins_quals, const uint8_t* del_quals,
                     const uint8_t* gcp, uint32_t read_len, const uint8_t* hap,
                     uint32_t hap_len, double* out_log10);

/* Device-resident batch: the fields of phmm_forward_batch as device
 * pointers, plus bounds the caller guarantees (used to size the workspace
 * and to route pairs; the device checks only that no haplotype is longer
 * than 64 x 24 bases when max_hap_len says none is, see
 * phmm_forward_batch_async). */
typedef struct phmm_device_batch {
    const uint8_t* reads;
    const uint8_t* base_quals;
    const uint8_t* ins_quals;
    const uint8_t* del_quals;
    const uint8_t* gcp;
    const uint64_t* read_offsets;
    uint32_t n_reads;
    const uint8_t* haplotypes;
    const uint64_t* hap_offsets;
    uint32_t n_haps;
    const uint32_t* pair_list;
    uint64_t n_pairs;
    uint32_t max_read_len; /* >= every read length in the batch      */
    uint32_t max_hap_len;  /* >= every haplotype length in the batch */
} phmm_device_batch;

/* Device workspace bytes phmm_forward_batch_async needs for a batch of
 * n_pairs pairs within the given length bounds. */
size_t phmm_workspace_bytes(phmm_ctx* ctx, uint64_t n_pairs, uint32_t max_read_len,
                            uint32_t max_hap_len);

/*
 * Stream-ordered forward pass over device-resident inputs: the same
 * likelihoods as phmm_forward_batch (eq.1-4 of Section 2, row-level
 * formulation of Section 3.1, Delete row by the scan of Section 3.4).
 * Packing, FP32 kernels, FP64 reruns and long pairs are all enqueued on
 * hip_stream (a
 * hipStream_t; NULL = the null stream) with no host synchronisation and no
 * allocation.  d_out_log10 (n_pairs doubles) and d_flags (n_pairs bytes, or
 * NULL) are device pointers; d_workspace holds at least
 * phmm_workspace_bytes(...) bytes of device memory.  Only the host-visible
 * fields of *b are checked (null pointers, bounds, workspace size); device
 * contents are trusted.  A batch of at most 8192 pairs is packed in one
 * narrow class chosen from max_hap_len, as in phmm_forward_batch; the
 * launches that only catch exceptions (pairs that do not fit that class,
 * FP32 rejects, and long pairs when max_hap_len <= 64 x 24 and max_read_len
 * <= fp32_max_rows) then get small grids.  Errors
 * detected on the device are reported by phmm_device_status() after the
 * stream has passed the call: PHMM_ETIMEOUT (watchdog), PHMM_ERANGE (a
 * haplotype longer than 64 x 24 bases in a batch whose max_hap_len says
 * there is none; its likelihood is still computed, in FP64).
 */
int phmm_forward_batch_async(phmm_ctx* ctx, const phmm_device_batch* b, double* d_out_log10,
                             uint8_t* d_flags, void* d_workspace, size_t ws_bytes,
                             void* hip_stream);

/*
 * phmm_forward_batch_async replayed from a HIP graph: the same launches and
 * results (bit-identical), captured once per distinct (batch pointers and
 * size, workspace, length bounds, options) and replayed by one
 * hipGraphLaunch on hip_stream afterwards.  The context keeps the graphs of
 * its last four such keys; a new key of the same launch shape updates the
 * least recently used graph's kernel parameters in place, another shape
 * replaces it.  The graph reads the batch through its pointers when it runs,
 * so new contents in the same buffers need no new capture.  The graph holds
 * kernel nodes only (the counters are cleared by a kernel, not a memset).
 * Timing (options.timing) is not recorded on this path.  Same arguments,
 * ownership and errors as phmm_forward_batch_async.
 */
int phmm_forward_batch_graph(phmm_ctx* ctx, const phmm_device_batch* b, double* d_out_log10,
                             uint8_t* d_flags, void* d_workspace, size_t ws_bytes,
                             void* hip_stream);

/*
 * phmm_forward_batch_async without a workspace argument, for callers that
 * cannot allocate device memory: code being captured into a HIP graph, tight
 * serving loops, harnesses that forbid hipMalloc.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); its scratch
 * memory (counters, packs, rerun queues, long lists and the long kernels'
 * ring buffers) is a library-owned static device array of
 * PHMM_NOALLOC_SCRATCH_MIB MiB that each GPU holds from library load until
 * the process ends, looked up once per device by phmm_create.  A batch may
 * hold at most PHMM_NOALLOC_MAX_PAIRS pairs (PHMM_ERANGE beyond); the long
 * kernels run at most 1024 wavefronts each.  Results equal those of
 * phmm_forward_batch_async on the same batch.  The counters the kernels need
 * at zero are cleared by the call's first kernel on the stream.  Every call
 * on one GPU shares that GPU's array, which keeps the last call's contents:
 * calls that overlap on one GPU (other streams, other contexts, other host
 * threads) race and give wrong results; serialise them (one stream, or
 * events).  phmm_device_status / phmm_last_counts do not apply (there is no
 * caller workspace).  Errors: as phmm_forward_batch_async, plus PHMM_ERANGE.
 */
#define PHMM_NOALLOC_SCRATCH_MIB 64u
#define PHMM_NOALLOC_MAX_PAIRS (1u << 19)
int phmm_forward_batch_noalloc(phmm_ctx* ctx, const phmm_device_batch* b, double* d_out_log10,
                               uint8_t* d_flags, void* hip_stream);

/* Synchronises with the stream of the last async call and returns PHMM_OK or
 * the error the device recorded for it: PHMM_ETIMEOUT (long-pair watchdog)
 * or PHMM_ERANGE (a haplotype over 64 x 24 bases in a batch whose
 * max_hap_len is at most that). */
int phmm_device_status(phmm_ctx* ctx, void* d_workspace);

/* Counters of the last call on a workspace (synchronises the stream). */
typedef struct phmm_counts {
    uint64_t packs_fp32;   /* wavefront packs run in FP32              */
    uint64_t packs_fp64;   /* wavefront packs run in FP64 (plain mode) */
    uint64_t rerun_items;  /* FP32 packs with at least one rerun pair  */
    uint64_t rerun_pairs;  /* pairs recomputed in FP64                 */
    uint64_t long_pairs;   /* pairs sent to the long-pair kernels      */
    uint64_t long_tiles;   /* wavefront tiles of the long-pair kernel  */
    uint64_t lane_columns; /* sum over packs of 64*N (occupied cells per row) */
    uint64_t long_pairs_fp32; /* of those, run by the FP32 long kernel */
    uint64_t deferred_packs; /* FP32 packs run by the general FP32 kernel (a read
                                with several gap bytes, a gap byte of 0 or an
                                insertion byte above 65)                     */
} phmm_counts;
int phmm_last_counts(phmm_ctx* ctx, void* d_workspace, phmm_counts* out);

/* Per-phase device times of the last call made with options.timing = 1
 * (milliseconds, from HIP events on the call's stream; synchronises). */
typedef struct phmm_timing {
    float pack_ms;     /* grouping and packing of pairs           */
    float short_ms;    /* short-pair kernels, FP32 or FP64 plain  */
    float rerun_ms;    /* FP64 rerun kernels                      */
    float long_ms;     /* long-pair kernels                       */
    float total_ms;    /* whole call                              */
} phmm_timing;
int phmm_last_timing(phmm_ctx* ctx, phmm_timing* out);

/*
 * Pack-shape tuning.  The packer chooses, for the pairs of each read, the
 * column class N (columns per lane) that minimises (wavefronts needed) x
 * cost[precision][class].  The default cost of a wavefront-row is N + 3 (N
 * cells plus the scan).  phmm_autotune replaces the table of `ctx` by the
 * time (ns) of one wavefront-row of each class's kernel on this device,
 * measured on a synthetic batch in which every pair fills a wavefront exactly
 * (this takes a few tenths of a second and runs on the context's stream;
 * nothing else may use the context meanwhile).  costs / out_costs hold 2 x
 * phmm_num_classes() floats: FP32 kernels first, then FP64.  Errors:
 * PHMM_EINVAL (NULL, non-positive cost), PHMM_EDEVICE.
 */
int phmm_autotune(phmm_ctx* ctx, uint64_t seed, float* out_costs /* NULL ok */);

/* Pack-shape tuning on the caller's own workload: times a sample batch (device
 * buffers as phmm_forward_batch_async, with its workspace and stream) under
 * the context's current cost table and under the family cost = N + a for
 * a in {0, 1, 2, 3, 5, 8, 12, 20} (best of 4 passes after a warm-up each),
 * and keeps the fastest table.  It runs the sample 45 times; results written
 * to the sample's outputs are discarded (a scratch output buffer is allocated
 * for the duration of the call). */
int phmm_autotune_sample(phmm_ctx* ctx, const phmm_device_batch* sample, void* d_workspace,
                         size_t ws_bytes, void* hip_stream, float* out_costs /* NULL ok */);
int phmm_set_class_costs(phmm_ctx* ctx, const float* costs);
int phmm_get_class_costs(phmm_ctx* ctx, float* costs);

/*
 * Genotype likelihoods (the Bayesian genotyping step that follows the
 * PairHMM, Section 1): for each active region, the diploid genotype
 * log-likelihoods from its read x haplotype matrix of log10 P(read | hap).
 *
 * Region g has region_reads[g] = R reads and region_haps[g] = H haplotypes
 * (1 <= H <= PHMM_GT_MAX_HAPS, R may be 0); its matrix is the R x H doubles
 * lk[lk_offsets[g] + r*H + h] (read-major: the order of the pairs a region's
 * reads and haplotypes give in pair_list when each read lists its
 * haplotypes in turn).  For each genotype a <= b the call writes
 *
 *   gl[gl_offsets[g] + b(b+1)/2 + a] = sum_r log10(10^lk[r][a]/2 + 10^lk[r][b]/2)
 *
 * (each read drawn from either haplotype copy with probability 1/2; the
 * genotype order is the VCF one for ploidy 2) and best[g] = the index of the
 * largest of them, the smallest index on ties (the maximum a posteriori
 * genotype under a flat prior).  A region with R = 0 has every entry 0 and
 * best 0.  Each term is evaluated in FP64 relative to the read's largest
 * likelihood, so no likelihood underflows; results agree with the plain sum
 * within 1e-12 relative (the reads of a region may be summed in any order).
 *
 * Host form: every array is a host buffer; lk holds n_lk doubles and gl n_gl.
 * The host checks, before any device work, that each region's matrix lies in
 * [0, n_lk), that its H(H+1)/2 genotypes lie in [0, n_gl), that H is in
 * range and that every lk value the regions use is finite; on error nothing
 * is written and phmm_last_error() names the first offending region or
 * index.  Genotype blocks of different regions must not overlap (not
 * checked: overlapping blocks give unspecified values).  Arguments are checked
 * before the context, so a NULL ctx reports input errors first.
 * Errors: PHMM_EINVAL, PHMM_ENOMEM, PHMM_EDEVICE.
 */
#define PHMM_GT_MAX_HAPS 512u
int phmm_genotype_batch(phmm_ctx* ctx, const double* lk, uint64_t n_lk,
                        const uint64_t* lk_offsets, const uint32_t* region_reads,
                        const uint32_t* region_haps, const uint64_t* gl_offsets,
                        uint32_t n_regions, double* gl, uint64_t n_gl, uint32_t* best);

/*
 * Stream-ordered form: the same arrays as device pointers, enqueued on
 * hip_stream (a hipStream_t, NULL = null stream) without synchronisation or
 * allocation, e.g. straight on the d_out_log10 of phmm_forward_batch_async.
 * Device contents are not checked on the host; the kernel itself skips a
 * region whose matrix or genotype block does not lie within n_lk / n_gl or
 * whose H is 0 or above PHMM_GT_MAX_HAPS, and sets its best to 0xFFFFFFFF
 * (nothing else of it is written).  Non-finite likelihoods give non-finite
 * results.  Errors: PHMM_EINVAL (NULL ctx, NULL array with n_regions > 0),
 * PHMM_EDEVICE (launch failure).
 */
int phmm_genotype_batch_async(phmm_ctx* ctx, const double* d_lk, uint64_t n_lk,
                              const uint64_t* d_lk_offsets, const uint32_t* d_region_reads,
                              const uint32_t* d_region_haps, const uint64_t* d_gl_offsets,
                              uint32_t n_regions, double* d_gl, uint64_t n_gl,
                              uint32_t* d_best, void* hip_stream);

/* Calibration: measures the device's achievable vector FMA rates (FP32
 * scalar FMA and FP64 FMA, TFLOP/s with an FMA counted as two flops) with
 * independent FMA chains in every lane.  Used to state the ALU roofline the
 * kernels are measured against.  Errors: PHMM_EINVAL (NULL output),
 * PHMM_EDEVICE. */
int phmm_vector_peak(int device, double* fp32_tflops, double* fp64_tflops);

/* Calibration: copies `bytes` bytes from device buffer `src` to device buffer
 * `dst` on `stream` (a hipStream_t, NULL = default stream) with a plain
 * vector copy kernel (`copy_calib_kernel`).  Its hardware traffic counters
 * read against the known 2 x bytes give the scale factor applied to the
 * traffic counters of the PairHMM kernels in a profile.  Both pointers and
 * `bytes` must be multiples of 16 and the buffers must not overlap; the call
 * is stream-ordered and does not synchronise.  Errors: PHMM_EINVAL (NULL or
 * misaligned arguments), PHMM_EDEVICE (launch failure). */
int phmm_copy_calib(const void* src, void* dst, uint64_t bytes, void* stream);

/*
 * Serving: a request loop with continuous batching.
 *
 * A server accepts active regions (the reads, haplotypes and pairs of one
 * region, in the layout of phmm_forward_batch) from any host thread and
 * returns each region's log10 likelihoods when they are done.  Regions that
 * arrive while others are on the GPU are batched and launched as lanes free
 * up, so their work overlaps on the device; a region's inputs and results stay
 * resident in device memory for its whole pass.  The results are those of
 * phmm_forward_batch on the region alone, up to the rounding differences a
 * different position in a wavefront may cause (within the FP32 tolerance).
 *
 * Memory: hbm_budget_bytes of device memory (and as much pinned host memory)
 * are divided evenly over the lanes at creation; a lane admits waiting
 * regions in arrival order while the batch layout (inputs, outputs and
 * workspace) fits its share.  A region too large for one lane is rejected at
 * submission with PHMM_ENOMEM.
 *
 * Long regions (a haplotype longer than 64 x 24 columns or a read longer than
 * long_read_min bases) queue apart and run on the long_lanes last lanes when
 * long_lanes > 0.  Each lane's stream is created with a CU mask, which gives
 * it a hardware queue of its own (plain streams share the process's few
 * hardware queues, and a short lane sharing one with a long lane would wait
 * behind its long kernels): the mask holds every compute unit, or with
 * short_cu_percent in 1..99 that share of them for the short lanes and the
 * rest for the long lanes.  If the device refuses a mask the lanes get plain
 * streams and phmm_server_stats reports it.
 */
typedef struct phmm_server phmm_server;

typedef struct phmm_server_options {
    int precision;              /* PHMM_FP32_RERUN (default) or PHMM_FP64_PLAIN        */
    uint32_t lanes;             /* batches in flight, one stream each; 1..16, default 3 */
    uint32_t long_lanes;        /* lanes reserved for long regions (< lanes); default 1 */
    uint64_t hbm_budget_bytes;  /* device bytes for admitted work; default 24 GiB       */
    uint32_t max_batch_regions; /* regions per batch at most; default 8192              */
    uint32_t short_cu_percent;  /* 0 = no CU masks; else the short lanes' CU share      */
    uint32_t long_read_min;     /* a region whose longest read exceeds this many bases
                                   (or whose longest haplotype exceeds 64 x 24 columns)
                                   queues for the long lanes; default 512              */
    uint32_t long_grid_percent; /* the long lanes' persistent grids as a share of a full
                                   chip's, 1..100 (the long-pair kernels keep at least
                                   1024 wavefronts): below 100 a long region's batch
                                   leaves wavefront slots on every compute unit for the
                                   short lanes' kernels.  Default 25: short regions
                                   then never wait for long ones (p99 within 2x of p50
                                   at 0.8x load), at about half the capacity of 100,
                                   where long regions carry 98% of the cells          */
} phmm_server_options;

typedef struct phmm_request_info {
    uint64_t n_pairs, cells;    /* the region's pairs and DP cells                      */
    uint32_t lane, is_long;     /* lane that ran it; 1 if it queued as a long region    */
    uint64_t batch;             /* batch sequence number                                */
    double queue_s;             /* submission to the start of its batch, seconds        */
    double latency_s;           /* submission to completion, seconds                    */
} phmm_request_info;

typedef struct phmm_server_counters {
    uint64_t regions, pairs, cells;  /* completed so far                                 */
    uint64_t batches;                /* batches run                                      */
    uint64_t full_batches;           /* batches that left waiting regions behind (budget
                                        or max_batch_regions reached)                    */
    uint64_t waiting_short, waiting_long;  /* regions queued now                        */
    double lane_busy_s;              /* summed over lanes: batch start to completion     */
    double span_s;                   /* first submission to last completion              */
    int cu_mask_status;              /* 1 CU-masked lane streams, < 0 refused (HIP error,
                                        negated; plain streams instead)                  */
} phmm_server_counters;

void phmm_server_default_options(phmm_server_options* opt);

/* Creates a server on `device` (opt NULL = defaults): allocates the lanes'
 * device and pinned host blocks and starts one worker thread per lane.
 * Errors: PHMM_EINVAL (bad options), PHMM_ENOMEM, PHMM_EDEVICE. */
int phmm_server_create(phmm_server** out, int device, const phmm_server_options* opt);

/* Finishes every submitted region, stops the workers and frees everything.
 * Results not collected are dropped.  NULL is ignored. */
void phmm_server_destroy(phmm_server* srv);

/* Submits one region (arguments as in phmm_forward_batch, n_pairs >= 1);
 * the inputs are validated and copied before it returns, so the caller may
 * reuse its buffers.  *ticket identifies the region in wait/poll.
 * Errors: PHMM_EINVAL / PHMM_ERANGE (validation, as phmm_forward_batch),
 * PHMM_ENOMEM (region larger than one lane's share of the budget). */
int phmm_server_submit(phmm_server* srv, const uint8_t* reads, const uint8_t* base_quals,
                       const uint8_t* ins_quals, const uint8_t* del_quals, const uint8_t* gcp,
                       const uint64_t* read_offsets, uint32_t n_reads,
                       const uint8_t* haplotypes, const uint64_t* hap_offsets, uint32_t n_haps,
                       const uint32_t* pair_list, uint64_t n_pairs, uint64_t* ticket);

/* Blocks until region `ticket` is done, then copies its n_pairs results
 * (out_log10, out_flags; either may be NULL) and its info (may be NULL) and
 * forgets the ticket.  Returns the region's status: PHMM_OK, or the error of
 * its batch (PHMM_EDEVICE, PHMM_ETIMEOUT).  PHMM_EINVAL for an unknown
 * ticket. */
int phmm_server_wait(phmm_server* srv, uint64_t ticket, double* out_log10, uint8_t* out_flags,
                     phmm_request_info* info);

/* As phmm_server_wait, but returns PHMM_PENDING at once if the region is not
 * done yet (the ticket stays valid). */
int phmm_server_poll(phmm_server* srv, uint64_t ticket, double* out_log10, uint8_t* out_flags,
                     phmm_request_info* info);

/* Counters of the server since creation.  Errors: PHMM_EINVAL. */
int phmm_server_stats(phmm_server* srv, phmm_server_counters* stats);

#ifdef __cplusplus
}
#endif
#endif /* PHMM_H */
