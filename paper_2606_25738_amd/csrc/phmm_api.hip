// Host runtime of the PairHMM forward library: contexts, validation,
// workspace layout and the stream-ordered launch sequence behind the C ABI
// declared in include/phmm.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "phmm.h"
#include "phmm_internal.h"

namespace phmm {
void launch_short(int kind, int cls, int grid, hipStream_t s, const Batch& b, const Tables& t,
                  const Work& w, const Policy& p);
const void* short_kernel_ptr(int kind, int cls);
__global__ void reset_kernel(Counters* c);
void launch_pack(hipStream_t s, const Batch& b, const Work& w, const Policy& pol);
uint32_t scan_chunks(uint32_t n_pack_blocks);
void launch_long(hipStream_t s, const int (&grid)[kLongLists], const Batch& b, const Tables& t,
                 const Work& w, const Policy& p);
const void* long_kernel_ptr(int q);
int launch_genotype(hipStream_t s, int cus, const double* lk, uint64_t n_lk,
                    const uint64_t* lk_off, const uint32_t* n_reads, const uint32_t* n_haps,
                    const uint64_t* gl_off, uint32_t n_regions, double* gl, uint64_t n_gl,
                    uint32_t* best);
__host__ __device__ uint32_t long_slots(int grid);
size_t long_ring_slot_bytes();
}  // namespace phmm

using namespace phmm;

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(PHMM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

namespace phmm {
int set_error(int code, const char* msg)
{
    g_err = msg;
    return code;
}
}  // namespace phmm

extern "C" const char* phmm_last_error(void) { return g_err.c_str(); }
extern "C" int phmm_num_classes(void) { return kNumClasses; }
extern "C" int phmm_class_n(int c) { return (c >= 0 && c < kNumClasses) ? class_n(c) : -1; }

extern "C" void phmm_default_options(phmm_options* o)
{
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->precision = PHMM_FP32_RERUN;
    o->accept_min_sum = 1e-28;
    o->force_class = -1;
    o->one_pair_per_wave = 0;
    o->fp32_max_rows = 1024;
    o->long_fp32_max_rows = 0;  // every long pair in FP64 (see phmm.h)
    o->watchdog_spins = 0;
    o->timing = 0;
    o->route_diverse_fp64 = 1;
}

// ---------------------------------------------------------------- context
// Everything one asynchronous pass's launches depend on: the batch's device
// pointers and size, the workspace, the length bounds and the policy (which
// includes the cost table).  Equal keys give identical launch sequences, so a
// captured graph of one is a replay of the other.  Compared bytewise: built
// from a zeroed object so that padding compares equal.
struct GraphKey {
    Batch b;
    const void* ws;
    uint32_t max_hap_len, max_read_len;
    Policy pol;
};
struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
};
constexpr int kGraphSlots = 4;

struct phmm_ctx {
    int device = 0;
    phmm_options opt{};
    hipStream_t stream = nullptr;
    int cus = 0;
    int grid_short[kNumKernelKinds][kNumClasses] = {};  // persistent wavefronts per kernel
    int grid_long[kLongLists] = {};  // persistent wavefronts of each list's long kernel
    double* d_p64 = nullptr;
    double* d_pw64 = nullptr;
    float* d_pw32 = nullptr;
    // synchronous-API arena
    void* arena = nullptr;
    size_t arena_bytes = 0;
    // device counters read back by the synchronising pass (pinned)
    Counters* h_ctr = nullptr;
    // chunked synchronous batches: copy stream, per-chunk events and counters
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_chunk[16] = {};
    Counters* h_chunk = nullptr;
    // timing
    hipEvent_t ev[6] = {};
    bool timed = false;
    // relative cost of one wavefront-row per (precision, class): N + 3 until
    // phmm_autotune or phmm_set_class_costs replaces it
    float cost[2][kNumClasses] = {};
    // phmm_forward_batch_graph: captured launch sets, least recently used
    // replaced first, and the stream they are captured on
    GraphEntry graphs[kGraphSlots];
    uint64_t graph_tick = 0;
    hipStream_t cap_stream = nullptr;
};

static Policy make_policy(const phmm_options& o, const float (&cost)[2][kNumClasses])
{
    Policy p;
    memset(&p, 0, sizeof p);
    p.precision = o.precision;
    p.force_class = o.force_class;
    p.one_pair_per_wave = o.one_pair_per_wave;
    p.fp32_max_rows = o.fp32_max_rows;
    p.long_fp32_max_rows = o.long_fp32_max_rows;
    p.accept_min_sum = (float)o.accept_min_sum;
    p.watchdog_spins = o.watchdog_spins ? o.watchdog_spins : 4000000u;
    p.route_diverse = o.route_diverse_fp64;
    for (int prec = 0; prec < 2; ++prec)
        for (int c = 0; c < kNumClasses; ++c) p.cost[prec][c] = cost[prec][c];
    return p;
}

// Smallest accepted FP32 threshold: ten decades below the default 1e-28 is
// not allowed, two are (see check_options).
constexpr double kAcceptFloor = 1e-30;

static int check_options(const phmm_options& o)
{
    if (o.precision != PHMM_FP32_RERUN && o.precision != PHMM_FP64_PLAIN)
        return fail(PHMM_EINVAL, "options.precision must be PHMM_FP32_RERUN or PHMM_FP64_PLAIN");
    // The FP32 kernels compare the scaled sum with the threshold held as a
    // float.  Below kAcceptFloor an accepted sum could sit so close to
    // FP32's smallest normal numbers that the pair's dominant cells lose
    // precision; above 3e38 the float would overflow.  Any threshold above
    // every possible scaled sum (2^120) reruns every pair in FP64.
    if (!(o.accept_min_sum >= kAcceptFloor) || !(o.accept_min_sum <= 3.0e38))
        return fail(PHMM_EINVAL, "options.accept_min_sum must be in [%g, 3e38]", kAcceptFloor);
    if (o.force_class < -1 || o.force_class >= kNumClasses)
        return fail(PHMM_EINVAL, "options.force_class must be -1 or 0..%d", kNumClasses - 1);
    if (o.route_diverse_fp64 != 0 && o.route_diverse_fp64 != 1)
        return fail(PHMM_EINVAL, "options.route_diverse_fp64 must be 0 or 1");
    return PHMM_OK;
}

static int build_tables(phmm_ctx* c)
{
    std::vector<double> p64(256);
    for (int q = 0; q < 256; ++q) p64[q] = pow(10.0, -(double)q / 10.0);
    std::vector<double> pw64((size_t)kNumClasses * 256 * kPowStride);
    std::vector<float> pw32(pw64.size());
    for (int cls = 0; cls < kNumClasses; ++cls) {
        const int N = class_n(cls);
        for (int q = 0; q < 256; ++q) {
            double* row = &pw64[((size_t)cls * 256 + q) * kPowStride];
            for (int m = 0; m <= 64; ++m) row[m] = pow(p64[q], (double)(N * m));
            row[65] = pow(p64[q], (double)(N - 1));
        }
    }
    for (size_t i = 0; i < pw64.size(); ++i) pw32[i] = (float)pw64[i];
    HIP_TRY(hipMalloc(&c->d_p64, p64.size() * 8));
    HIP_TRY(hipMalloc(&c->d_pw64, pw64.size() * 8));
    HIP_TRY(hipMalloc(&c->d_pw32, pw32.size() * 4));
    HIP_TRY(hipMemcpy(c->d_p64, p64.data(), p64.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d_pw64, pw64.data(), pw64.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d_pw32, pw32.data(), pw32.size() * 4, hipMemcpyHostToDevice));
    return PHMM_OK;
}

extern "C" void phmm_destroy(phmm_ctx* c)
{
    if (!c) return;
    // best-effort teardown: errors here have nowhere to go
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->d_p64);
    (void)hipFree(c->d_pw64);
    (void)hipFree(c->d_pw32);
    (void)hipFree(c->arena);
    if (c->h_ctr) (void)hipHostFree(c->h_ctr);
    if (c->copy_stream) (void)hipStreamSynchronize(c->copy_stream);
    if (c->h_chunk) (void)hipHostFree(c->h_chunk);
    for (auto& e : c->ev_chunk)
        if (e) (void)hipEventDestroy(e);
    if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
    for (auto& g : c->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// ---------------------------------------------------------------- scratch
// Device scratch of phmm_forward_batch_noalloc: the workspace of a batch of
// up to PHMM_NOALLOC_MAX_PAIRS pairs with the long kernels' grids capped at
// kNoAllocLongGrid wavefronts (their ring slots are most of it).  Every GPU
// the library runs on holds its own copy until the process ends; the host
// reaches a device's copy only through the address hipGetSymbolAddress
// returns with that device current (the array's name is a host-side stand-in).
constexpr size_t kScratchBytes = (size_t)PHMM_NOALLOC_SCRATCH_MIB << 20;
// At least the tiles of the longest haplotype (2^20 / 1024 columns), so a
// pair's tiles always fit the resident grid at once.
constexpr int kNoAllocLongGrid = 1024;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static void* g_scratch[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Address of `device`'s scratch array, looked up once per device with that
// device current (the caller has made it current).
static int scratch_for(int device, void** out)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(PHMM_EDEVICE, "device %d beyond the %d the library tracks", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(PHMM_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return PHMM_OK;
}

static int create_impl(phmm_ctx* c, int device)
{
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(PHMM_EDEVICE, "no HIP device %d (%d present)", device, ndev);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(PHMM_EDEVICE, "device %d is %s; this library is built for gfx950 only", device,
                    prop.gcnArchName);
    c->device = device;
    c->cus = prop.multiProcessorCount;
    for (int prec = 0; prec < 2; ++prec)
        for (int cls = 0; cls < kNumClasses; ++cls)
            c->cost[prec][cls] = (float)class_n(cls) + 3.0f;  // row cost ~ N cells + scan
    HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&c->h_ctr), sizeof(Counters), hipHostMallocDefault));
    for (auto& e : c->ev) HIP_TRY(hipEventCreate(&e));
    for (int kind = 0; kind < kNumKernelKinds; ++kind)
        for (int cls = 0; cls < kNumClasses; ++cls) {
            int per_cu = 0;
            HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, short_kernel_ptr(kind, cls), kWave, 0));
            c->grid_short[kind][cls] = std::max(1, per_cu) * c->cus;
        }
    for (int q = 0; q < kLongLists; ++q) {
        int per_cu = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, long_kernel_ptr(q), kWave, 0));
        c->grid_long[q] = std::max(1, per_cu) * c->cus;
    }
    void* sp = nullptr;  // this device's scratch address, for phmm_forward_batch_noalloc
    const int rc = scratch_for(device, &sp);
    if (rc != PHMM_OK) return rc;
    return build_tables(c);
}

void phmm::scale_grids(phmm_ctx* c, int percent)
{
    if (!c || percent <= 0 || percent >= 100) return;
    auto cut = [percent](int g) { return std::max(1, (int)((int64_t)g * percent / 100)); };
    for (auto& kind : c->grid_short)
        for (int& g : kind) g = cut(g);
    // a long pair's tiles must all be resident together once its read is
    // longer than 512 rows per resident wavefront
    for (int& g : c->grid_long) g = std::min(g, std::max(cut(g), kMinLongGrid));
}

extern "C" int phmm_create(phmm_ctx** out, int device, const phmm_options* opt)
{
    if (!out) return fail(PHMM_EINVAL, "phmm_create: out is NULL");
    *out = nullptr;
    phmm_ctx* c = new (std::nothrow) phmm_ctx();
    if (!c) return fail(PHMM_ENOMEM, "phmm_create: out of host memory");
    if (opt) c->opt = *opt;
    else phmm_default_options(&c->opt);
    int rc = check_options(c->opt);
    if (rc == PHMM_OK) rc = create_impl(c, device);
    if (rc != PHMM_OK) {
        std::string keep = g_err;
        phmm_destroy(c);
        g_err = keep;
        return rc;
    }
    *out = c;
    return PHMM_OK;
}

// ---------------------------------------------------------------- workspace
struct Layout {
    size_t ctr, chunk_info, blk_cnt, blk_lc, chunk_part, packs, items, deferred,
        long_pend[2], long_list[kLongLists], long_pref, ring, slot, total;
};

static uint64_t pack_blocks(uint64_t n_pairs) { return (n_pairs + kPackBlock - 1) / kPackBlock; }

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Long-kernel grid of precision q (0 FP32, 1 FP64), capped at long_cap
// wavefronts when long_cap > 0.  The ring slots of the workspace follow the
// grid, so the workspace layout and the launches must use the same cap.
static int long_grid(const phmm_ctx* c, int q, int long_cap)
{
    return long_cap > 0 ? std::min(c->grid_long[q], long_cap) : c->grid_long[q];
}

static Layout layout_for(const phmm_ctx* c, uint64_t n_pairs, int long_cap = 0)
{
    Layout L;
    size_t o = 0;
    const uint64_t n = n_pairs ? n_pairs : 1;
    uint32_t slots = 0;
    for (int q = 0; q < kLongLists; ++q) slots = std::max(slots, long_slots(long_grid(c, q, long_cap)));
    L.ctr = o; o = align256(o + sizeof(Counters));
    L.chunk_info = o; o = align256(o + n * 4);
    L.blk_cnt = o; o = align256(o + pack_blocks(n) * kSeg * 4);
    L.blk_lc = o; o = align256(o + pack_blocks(n) * 8);
    L.chunk_part = o; o = align256(o + (size_t)scan_chunks((uint32_t)pack_blocks(n)) * kSeg * 4);
    L.packs = o; o = align256(o + n * sizeof(Pack));
    L.items = o; o = align256(o + n * sizeof(Item));
    L.deferred = o; o = align256(o + n * 4);
    for (int q = 0; q < 2; ++q) {
        L.long_pend[q] = o;
        o = align256(o + n * 4);
    }
    for (int q = 0; q < kLongLists; ++q) {
        L.long_list[q] = o;
        o = align256(o + n * 4);
    }
    L.long_pref = o; o = align256(o + (n + 1) * 4);
    L.ring = o; o = align256(o + (size_t)slots * long_ring_slot_bytes());
    L.slot = o; o = align256(o + (size_t)slots * 3 * sizeof(uint32_t));
    L.total = o;
    return L;
}

extern "C" size_t phmm_workspace_bytes(phmm_ctx* c, uint64_t n_pairs, uint32_t max_read_len,
                                       uint32_t max_hap_len)
{
    (void)max_read_len;
    (void)max_hap_len;
    if (!c) return 0;
    return layout_for(c, n_pairs).total;
}

static Work work_for(phmm_ctx* c, void* ws, uint64_t n_pairs, int long_cap = 0)
{
    Layout L = layout_for(c, n_pairs, long_cap);
    char* base = static_cast<char*>(ws);
    Work w;
    w.ctr = reinterpret_cast<Counters*>(base + L.ctr);
    w.chunk_info = reinterpret_cast<uint32_t*>(base + L.chunk_info);
    w.blk_cnt = reinterpret_cast<uint32_t*>(base + L.blk_cnt);
    w.blk_lanecols = reinterpret_cast<unsigned long long*>(base + L.blk_lc);
    w.chunk_part = reinterpret_cast<uint32_t*>(base + L.chunk_part);
    w.n_pack_blocks = (uint32_t)pack_blocks(n_pairs ? n_pairs : 1);
    w.n_scan_chunks = scan_chunks(w.n_pack_blocks);
    w.packs = reinterpret_cast<Pack*>(base + L.packs);
    w.items = reinterpret_cast<Item*>(base + L.items);
    w.deferred = reinterpret_cast<uint32_t*>(base + L.deferred);
    for (int q = 0; q < 2; ++q) w.long_pend[q] = reinterpret_cast<uint32_t*>(base + L.long_pend[q]);
    for (int q = 0; q < kLongLists; ++q) w.long_list[q] = reinterpret_cast<uint32_t*>(base + L.long_list[q]);
    w.long_pref = reinterpret_cast<uint32_t*>(base + L.long_pref);
    w.long_ring = reinterpret_cast<double*>(base + L.ring);
    w.long_prog = reinterpret_cast<uint32_t*>(base + L.slot);
    return w;
}

// ---------------------------------------------------------------- launch
// A small batch (at most kSmallBatchPairs pairs) cannot fill the GPU, so its
// time is launches and the longest wavefront, not throughput: unless a class
// is forced, every pack gets the narrowest class whose 64 lanes hold the
// batch's longest short haplotype (max_hap_len, capped at the short limit).
// One class means one launch per kernel family, and a narrow class a short
// row loop.
constexpr uint64_t kSmallBatchPairs = 8192;

static Policy batch_policy(phmm_ctx* c, uint64_t n_pairs, uint32_t max_hap_len)
{
    Policy pol = make_policy(c->opt, c->cost);
    pol.long_haps = max_hap_len > kShortMaxCols ? 1 : 0;
    if (n_pairs <= kSmallBatchPairs && pol.force_class < 0) {
        const uint32_t k = std::max(1u, std::min(max_hap_len, kShortMaxCols));
        const int n = std::max(class_n(0), (int)((k + kWave - 1) / kWave));
        pol.force_class = class_of_n(std::min(n, kMaxN));
    }
    return pol;
}

// Whether class cls can receive packs under pol: with a class forced, only
// that one and the widest (a run whose haplotypes do not fit the forced class
// falls back to the widest).
static bool class_used(const Policy& pol, int cls)
{
    return pol.force_class < 0 || cls == pol.force_class || cls == kNumClasses - 1;
}

static int enqueue(phmm_ctx* c, const Batch& b, void* ws, hipStream_t s, uint32_t max_hap_len,
                   uint32_t max_read_len, int long_cap = 0, bool allow_timing = true)
{
    const Policy pol = batch_policy(c, b.n_pairs, max_hap_len);
    Tables t;
    t.p64 = c->d_p64;
    t.pw64 = c->d_pw64;
    t.pw32 = c->d_pw32;
    const Work w = work_for(c, ws, b.n_pairs, long_cap);
    const bool timed = allow_timing && c->opt.timing != 0;
    if (timed) HIP_TRY(hipEventRecord(c->ev[0], s));
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(256), 0, s, w.ctr);
    if (b.n_pairs > 0) launch_pack(s, b, w, pol);
    if (timed) HIP_TRY(hipEventRecord(c->ev[1], s));
    if (b.n_pairs > 0) {
        // Without reading the device counters the launch set is fixed: every
        // class of every family, even when it has nothing to do.  A launch's
        // cost with no work grows with its workgroup count, so no grid is
        // larger than the batch's pair count (a bound on any class's packs
        // or items), and the general FP32 kernels, which only run packs the
        // fast kernels defer (reads with per-row gap penalties, a gap byte of
        // 0 or an insertion byte above 65), get one wavefront per SIMD.
        const int n_cap = (int)std::min<uint64_t>(b.n_pairs, 1u << 30);
        auto cap = [&](int grid) { return std::min(grid, n_cap); };
        // In a small batch every short pair fits the forced class, so the
        // widest class, the general FP32 kernels, the widest FP64 class and,
        // when no pair can be long, the long kernels only catch exceptions:
        // they get one wavefront per CU (the forced FP64 class, which runs
        // the rejected pairs in FP32 mode, one per SIMD).  Every kernel is a
        // persistent loop over its queue, so any grid completes the same work.
        const bool small = b.n_pairs <= kSmallBatchPairs && c->opt.force_class < 0;
        auto net = [&](int grid, int per_cu) {
            return small ? std::min(grid, per_cu * c->cus) : grid;
        };
        if (pol.precision == PHMM_FP32_RERUN) {
            for (int cls = 0; cls < kNumClasses; ++cls)
                if (class_used(pol, cls))
                    launch_short(kFast32, cls,
                                 cls == pol.force_class ? cap(c->grid_short[kFast32][cls])
                                                        : net(cap(c->grid_short[kFast32][cls]), 1),
                                 s, b, t, w, pol);
            for (int cls = 0; cls < kNumClasses; ++cls)
                if (class_used(pol, cls))
                    launch_short(kGen32, cls,
                                 net(cap(std::min(c->grid_short[kGen32][cls], 4 * c->cus)), 1),
                                 s, b, t, w, pol);
        }
        if (timed) HIP_TRY(hipEventRecord(c->ev[2], s));
        for (int cls = 0; cls < kNumClasses; ++cls)
            if (class_used(pol, cls))
                launch_short(kAll64, cls,
                             cls != pol.force_class ? net(cap(c->grid_short[kAll64][cls]), 1)
                             : pol.precision == PHMM_FP64_PLAIN ? cap(c->grid_short[kAll64][cls])
                                                                : net(cap(c->grid_short[kAll64][cls]), 4),
                             s, b, t, w, pol);
        if (timed) HIP_TRY(hipEventRecord(c->ev[3], s));
        // Lists 0-2 are filled by the routing kernel only, with pairs whose
        // haplotype exceeds the short kernels' reach; list 3 also takes FP64
        // sums that underflowed (and long pairs that contradict the batch's
        // length bound).  Without haplotypes that long only list 3 is
        // launched, with one wavefront per CU in a small batch.
        const bool no_long_haps = max_hap_len <= kShortMaxCols;
        const bool no_long = no_long_haps && max_read_len <= pol.fp32_max_rows;
        int lgrid[kLongLists];
        for (int q = 0; q < kLongLists; ++q) {
            const int g = long_grid(c, q, long_cap);
            lgrid[q] = (no_long_haps && q != kLongLists - 1) ? 0 : small && no_long ? std::min(g, c->cus) : g;
        }
        launch_long(s, lgrid, b, t, w, pol);
    } else if (timed) {
        HIP_TRY(hipEventRecord(c->ev[2], s));
        HIP_TRY(hipEventRecord(c->ev[3], s));
    }
    if (timed) HIP_TRY(hipEventRecord(c->ev[4], s));
    HIP_TRY(hipGetLastError());
    c->timed = timed;
    return PHMM_OK;
}

// The same pass for callers that wait for its end anyway (the synchronous API
// and the serving lanes): the host reads the device counters after the packer
// and after each kernel family, launches only the kernels that have work, and
// gives each a grid no larger than its packs or items.  A persistent launch
// with nothing to do still dispatches every workgroup of its grid (tens of
// microseconds each), which dominates a small batch; the read-backs cost
// about as much as one such launch each.
static int enqueue_sync(phmm_ctx* c, const Batch& b, void* ws, hipStream_t s,
                        uint32_t max_hap_len)
{
    const Policy pol = batch_policy(c, b.n_pairs, max_hap_len);
    Tables t;
    t.p64 = c->d_p64;
    t.pw64 = c->d_pw64;
    t.pw32 = c->d_pw32;
    const Work w = work_for(c, ws, b.n_pairs);
    const bool timed = c->opt.timing != 0;
    Counters* h = c->h_ctr;
    auto fetch = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(h, w.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return PHMM_OK;
    };
    auto capped = [](int grid, uint64_t work) {
        return (int)std::min<uint64_t>((uint64_t)grid, work);
    };
    int rc = PHMM_OK;
    if (timed) HIP_TRY(hipEventRecord(c->ev[0], s));
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(256), 0, s, w.ctr);
    if (b.n_pairs > 0) launch_pack(s, b, w, pol);
    if (timed) HIP_TRY(hipEventRecord(c->ev[1], s));
    if (b.n_pairs > 0) {
        if ((rc = fetch()) != PHMM_OK) return rc;
        if (pol.precision == PHMM_FP32_RERUN) {
            for (int cls = 0; cls < kNumClasses; ++cls)
                if (h->pack_cnt[0][cls] > 0)
                    launch_short(kFast32, cls, capped(c->grid_short[kFast32][cls], h->pack_cnt[0][cls]),
                                 s, b, t, w, pol);
            if ((rc = fetch()) != PHMM_OK) return rc;
            bool deferred = false;
            for (int cls = 0; cls < kNumClasses; ++cls)
                if (h->defer_cnt[cls] > 0) {
                    launch_short(kGen32, cls, capped(c->grid_short[kGen32][cls], h->defer_cnt[cls]), s,
                                 b, t, w, pol);
                    deferred = true;
                }
            if (deferred && (rc = fetch()) != PHMM_OK) return rc;
        }
        if (timed) HIP_TRY(hipEventRecord(c->ev[2], s));
        for (int cls = 0; cls < kNumClasses; ++cls) {
            const uint64_t n = (uint64_t)h->pack_cnt[1][cls] + h->item_cnt[cls];
            if (n > 0) launch_short(kAll64, cls, capped(c->grid_short[kAll64][cls], n), s, b, t, w, pol);
        }
        if (timed) HIP_TRY(hipEventRecord(c->ev[3], s));
        if ((rc = fetch()) != PHMM_OK) return rc;  // FP64 underflow adds long pairs
        int grid[kLongLists];
        for (int q = 0; q < kLongLists; ++q) grid[q] = h->n_long[q] > 0 ? c->grid_long[q] : 0;
        launch_long(s, grid, b, t, w, pol);
    } else if (timed) {
        HIP_TRY(hipEventRecord(c->ev[2], s));
        HIP_TRY(hipEventRecord(c->ev[3], s));
    }
    if (timed) HIP_TRY(hipEventRecord(c->ev[4], s));
    HIP_TRY(hipGetLastError());
    c->timed = timed;
    return PHMM_OK;
}

// Checks a device batch and fills the kernels' view of it.
static int device_batch(phmm_ctx* c, const phmm_device_batch* db, double* d_out, uint8_t* d_flags,
                        void* d_ws, size_t ws_bytes, Batch* b, int long_cap = 0)
{
    if (!c || !db) return fail(PHMM_EINVAL, "phmm_forward_batch_async: ctx or batch is NULL");
    if (db->n_pairs > 0xffffffffull) return fail(PHMM_ERANGE, "n_pairs exceeds 2^32-1");
    if (db->n_pairs > 0 && (!db->reads || !db->base_quals || !db->ins_quals || !db->del_quals ||
                            !db->gcp || !db->read_offsets || !db->haplotypes ||
                            !db->hap_offsets || !db->pair_list || !d_out || !d_ws))
        return fail(PHMM_EINVAL, "phmm_forward_batch_async: NULL device pointer");
    if (db->max_read_len > PHMM_MAX_READ)
        return fail(PHMM_ERANGE, "max_read_len %u exceeds %u", db->max_read_len, PHMM_MAX_READ);
    if (db->max_hap_len > PHMM_MAX_HAP)
        return fail(PHMM_ERANGE, "max_hap_len %u exceeds %u", db->max_hap_len, PHMM_MAX_HAP);
    const size_t need = layout_for(c, db->n_pairs, long_cap).total;
    if (ws_bytes < need) return fail(PHMM_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    b->reads = db->reads;
    b->bq = db->base_quals;
    b->iq = db->ins_quals;
    b->dq = db->del_quals;
    b->gq = db->gcp;
    b->read_off = db->read_offsets;
    b->haps = db->haplotypes;
    b->hap_off = db->hap_offsets;
    b->pairs = db->pair_list;
    b->n_pairs = db->n_pairs;
    b->out = d_out;
    b->flags = d_flags;
    return PHMM_OK;
}

extern "C" int phmm_forward_batch_async(phmm_ctx* c, const phmm_device_batch* db, double* d_out,
                                        uint8_t* d_flags, void* d_ws, size_t ws_bytes,
                                        void* hip_stream)
{
    Batch b;
    const int rc = device_batch(c, db, d_out, d_flags, d_ws, ws_bytes, &b);
    if (rc != PHMM_OK) return rc;
    HIP_TRY(hipSetDevice(c->device));
    return enqueue(c, b, d_ws, static_cast<hipStream_t>(hip_stream), db->max_hap_len,
                   db->max_read_len);
}

extern "C" int phmm_forward_batch_noalloc(phmm_ctx* c, const phmm_device_batch* db,
                                          double* d_out, uint8_t* d_flags, void* hip_stream)
{
    if (!c || !db) return fail(PHMM_EINVAL, "phmm_forward_batch_noalloc: ctx or batch is NULL");
    if (db->n_pairs > PHMM_NOALLOC_MAX_PAIRS)
        return fail(PHMM_ERANGE, "phmm_forward_batch_noalloc: %llu pairs exceed the limit of %u",
                    (unsigned long long)db->n_pairs, PHMM_NOALLOC_MAX_PAIRS);
    const size_t need = layout_for(c, db->n_pairs, kNoAllocLongGrid).total;
    if (need > kScratchBytes)
        return fail(PHMM_ERANGE, "phmm_forward_batch_noalloc: needs %zu bytes of scratch, %zu held",
                    need, kScratchBytes);
    HIP_TRY(hipSetDevice(c->device));
    void* ws = nullptr;
    int rc = scratch_for(c->device, &ws);  // set at phmm_create; no lookup here normally
    if (rc != PHMM_OK) return rc;
    Batch b;
    rc = device_batch(c, db, d_out, d_flags, ws, need, &b, kNoAllocLongGrid);
    if (rc != PHMM_OK) return rc;
    return enqueue(c, b, ws, static_cast<hipStream_t>(hip_stream), db->max_hap_len,
                   db->max_read_len, kNoAllocLongGrid);
}

// The asynchronous pass replayed from a HIP graph.  A context keeps the
// launch sets of its last kGraphSlots distinct (batch, workspace, bounds,
// policy) keys as instantiated graphs; a call with a known key is one
// hipGraphLaunch.  A new key is captured on the context's capture stream
// (the counter reset is a kernel, so the graph holds kernel nodes only) and
// either updated into the least recently used graph, when the launch
// sequence has the same shape, or instantiated in its place.
extern "C" int phmm_forward_batch_graph(phmm_ctx* c, const phmm_device_batch* db, double* d_out,
                                        uint8_t* d_flags, void* d_ws, size_t ws_bytes,
                                        void* hip_stream)
{
    Batch b;
    int rc = device_batch(c, db, d_out, d_flags, d_ws, ws_bytes, &b);
    if (rc != PHMM_OK) return rc;
    HIP_TRY(hipSetDevice(c->device));
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    GraphKey key;
    memset(&key, 0, sizeof key);
    key.b = b;
    key.ws = d_ws;
    key.max_hap_len = db->max_hap_len;
    key.max_read_len = db->max_read_len;
    key.pol = batch_policy(c, b.n_pairs, db->max_hap_len);
    c->timed = false;
    for (GraphEntry& e : c->graphs)
        if (e.exec && memcmp(&e.key, &key, sizeof key) == 0) {
            e.used = ++c->graph_tick;
            HIP_TRY(hipGraphLaunch(e.exec, s));
            return PHMM_OK;
        }
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = enqueue(c, b, d_ws, c->cap_stream, db->max_hap_len, db->max_read_len, 0, false);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
    if (rc != PHMM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (ec != hipSuccess || !g)
        return fail(PHMM_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
    GraphEntry* e = &c->graphs[0];
    for (GraphEntry& x : c->graphs)
        if (x.used < e->used) e = &x;
    bool updated = false;
    if (e->exec) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res;
        if (hipGraphExecUpdate(e->exec, g, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
            updated = true;
        } else {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(e->exec);
            e->exec = nullptr;
        }
    }
    if (!updated) {
        const hipError_t ei = hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            e->exec = nullptr;
            (void)hipGraphDestroy(g);
            return fail(PHMM_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
        }
    }
    (void)hipGraphDestroy(g);
    e->key = key;
    e->used = ++c->graph_tick;
    HIP_TRY(hipGraphLaunch(e->exec, s));
    return PHMM_OK;
}

int phmm::forward_device_batch_sync(phmm_ctx* c, const phmm_device_batch* db, double* d_out,
                              uint8_t* d_flags, void* d_ws, size_t ws_bytes, hipStream_t s)
{
    Batch b;
    const int rc = device_batch(c, db, d_out, d_flags, d_ws, ws_bytes, &b);
    if (rc != PHMM_OK) return rc;
    HIP_TRY(hipSetDevice(c->device));
    return enqueue_sync(c, b, d_ws, s, db->max_hap_len);
}

extern "C" int phmm_device_status(phmm_ctx* c, void* d_ws)
{
    if (!c || !d_ws) return fail(PHMM_EINVAL, "phmm_device_status: NULL argument");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipDeviceSynchronize());
    Counters h;
    HIP_TRY(hipMemcpy(&h, d_ws, sizeof h, hipMemcpyDeviceToHost));
    if (h.status != 0)
        return fail((int)h.status, "device reported error %d%s", (int)h.status,
                    (int)h.status == PHMM_ETIMEOUT ? " (long-pair watchdog)" : "");
    if (h.bound_err != 0)
        return fail(PHMM_ERANGE, "a haplotype longer than %u bases in a batch whose max_hap_len is at most %u",
                    kShortMaxCols, kShortMaxCols);
    return PHMM_OK;
}

extern "C" int phmm_last_counts(phmm_ctx* c, void* d_ws, phmm_counts* out)
{
    if (!c || !d_ws || !out) return fail(PHMM_EINVAL, "phmm_last_counts: NULL argument");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipDeviceSynchronize());
    Counters h;
    HIP_TRY(hipMemcpy(&h, d_ws, sizeof h, hipMemcpyDeviceToHost));
    memset(out, 0, sizeof *out);
    for (int k = 0; k < kNumClasses; ++k) {
        out->packs_fp32 += h.pack_cnt[0][k];
        out->packs_fp64 += h.pack_cnt[1][k];
    }
    out->rerun_items = 0;  // one item per FP32 pack with a rejected pair
    for (int k = 0; k < kNumClasses; ++k) out->rerun_items += h.item_cnt[k];
    out->rerun_pairs = h.rerun_pairs;
    for (int q = 0; q < kLongLists; ++q) {
        out->long_pairs += h.n_long[q];
        out->long_tiles += h.long_tiles[q];
    }
    out->long_pairs_fp32 = (uint64_t)h.n_long[0] + h.n_long[1];
    out->lane_columns = h.lane_columns;
    for (int k = 0; k < kNumClasses; ++k) out->deferred_packs += h.defer_cnt[k];
    return PHMM_OK;
}

extern "C" int phmm_last_timing(phmm_ctx* c, phmm_timing* out)
{
    if (!c || !out) return fail(PHMM_EINVAL, "phmm_last_timing: NULL argument");
    if (!c->timed) return fail(PHMM_EINVAL, "phmm_last_timing: last call was not timed");
    HIP_TRY(hipEventSynchronize(c->ev[4]));
    HIP_TRY(hipEventElapsedTime(&out->pack_ms, c->ev[0], c->ev[1]));
    HIP_TRY(hipEventElapsedTime(&out->short_ms, c->ev[1], c->ev[2]));
    HIP_TRY(hipEventElapsedTime(&out->rerun_ms, c->ev[2], c->ev[3]));
    HIP_TRY(hipEventElapsedTime(&out->long_ms, c->ev[3], c->ev[4]));
    HIP_TRY(hipEventElapsedTime(&out->total_ms, c->ev[0], c->ev[4]));
    return PHMM_OK;
}

// ---------------------------------------------------------------- validation
// Host checks of a batch before any device work.  Large arrays are scanned in
// parallel blocks (up to 16 threads, at least 16 Mi elements each); a scan
// reports the first failing index of the whole array, so the error message is
// the same as a sequential check's.

template <typename F>  // bad(lo, hi): first failing index in [lo, hi), or hi
static uint64_t first_failure(uint64_t n, F bad)
{
    const uint64_t kMinPerThread = 1ull << 24;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const uint64_t nt = std::min<uint64_t>(std::min(16u, hw), std::max<uint64_t>(1, n / kMinPerThread));
    if (nt <= 1) return bad(0, n);
    std::vector<uint64_t> res(nt, n);
    std::vector<std::thread> th;
    const uint64_t per = (n + nt - 1) / nt;
    for (uint64_t t = 0; t < nt; ++t) {
        const uint64_t lo = std::min(n, per * t), hi = std::min(n, lo + per);
        th.emplace_back([&res, &bad, t, lo, hi, n] {
            const uint64_t f = bad(lo, hi);
            res[t] = f < hi ? f : n;
        });
    }
    for (auto& x : th) x.join();
    return *std::min_element(res.begin(), res.end());
}

struct BaseTable {
    uint8_t bad[256];
    BaseTable()
    {
        for (int c = 0; c < 256; ++c)
            bad[c] = !(c == 'A' || c == 'C' || c == 'G' || c == 'T' || c == 'N');
    }
};
static const BaseTable kBases;

// First byte in [lo, hi) that is not one of ACGTN (branch-free per block).
static uint64_t first_non_base(const uint8_t* p, uint64_t lo, uint64_t hi)
{
    for (uint64_t i = lo; i < hi;) {
        const uint64_t e = std::min(hi, i + 4096);
        uint32_t acc = 0;
        for (uint64_t j = i; j < e; ++j) acc |= kBases.bad[p[j]];
        if (acc)
            for (uint64_t j = i; j < e; ++j)
                if (kBases.bad[p[j]]) return j;
        i = e;
    }
    return hi;
}

// CSR offsets: first entry that is empty, not increasing or longer than
// max_len (n when none), and the longest length before it.
static uint64_t check_offsets(const uint64_t* off, uint64_t n, uint64_t max_len, uint32_t* longest)
{
    std::atomic<uint32_t> top{0};
    const uint64_t f = first_failure(n, [&](uint64_t lo, uint64_t hi) {
        uint32_t m = 0;
        uint64_t i = lo;
        for (; i < hi; ++i) {
            if (off[i + 1] <= off[i] || off[i + 1] - off[i] > max_len) break;
            m = std::max(m, (uint32_t)(off[i + 1] - off[i]));
        }
        uint32_t cur = top.load();
        while (m > cur && !top.compare_exchange_weak(cur, m)) {
        }
        return i;
    });
    *longest = top.load();
    return f;
}

static int validate(const uint8_t* reads, const uint8_t* bq, const uint8_t* iq, const uint8_t* dq,
                    const uint8_t* gq, const uint64_t* ro, uint32_t n_reads, const uint8_t* haps,
                    const uint64_t* ho, uint32_t n_haps, const uint32_t* pl, uint64_t n_pairs,
                    double* out, uint32_t* max_l, uint32_t* max_k)
{
    *max_l = 0;
    *max_k = 0;
    if (n_pairs == 0) return PHMM_OK;
    if (!ro || !ho || !pl || !out) return fail(PHMM_EINVAL, "NULL offsets, pair_list or output");
    if (n_reads == 0 || n_haps == 0) return fail(PHMM_EINVAL, "pairs given but no reads or haplotypes");
    if (!reads || !bq || !iq || !dq || !gq || !haps) return fail(PHMM_EINVAL, "NULL sequence or quality array");
    if (ro[0] != 0) return fail(PHMM_EINVAL, "read_offsets[0] = %llu, must be 0", (unsigned long long)ro[0]);
    if (ho[0] != 0) return fail(PHMM_EINVAL, "hap_offsets[0] = %llu, must be 0", (unsigned long long)ho[0]);
    uint64_t r = check_offsets(ro, n_reads, PHMM_MAX_READ, max_l);
    if (r < n_reads) {
        if (ro[r + 1] <= ro[r]) return fail(PHMM_EINVAL, "read %llu is empty or offsets not increasing", (unsigned long long)r);
        return fail(PHMM_ERANGE, "read %llu has %llu bases (max %u)", (unsigned long long)r,
                    (unsigned long long)(ro[r + 1] - ro[r]), PHMM_MAX_READ);
    }
    uint64_t h = check_offsets(ho, n_haps, PHMM_MAX_HAP, max_k);
    if (h < n_haps) {
        if (ho[h + 1] <= ho[h]) return fail(PHMM_EINVAL, "haplotype %llu is empty or offsets not increasing", (unsigned long long)h);
        return fail(PHMM_ERANGE, "haplotype %llu has %llu bases (max %u)", (unsigned long long)h,
                    (unsigned long long)(ho[h + 1] - ho[h]), PHMM_MAX_HAP);
    }
    const uint64_t nb = ro[n_reads], nh = ho[n_haps];
    uint64_t i = first_failure(nb, [&](uint64_t lo, uint64_t hi) { return first_non_base(reads, lo, hi); });
    if (i < nb) return fail(PHMM_EINVAL, "read base %llu is 0x%02x, not one of ACGTN", (unsigned long long)i, reads[i]);
    i = first_failure(nh, [&](uint64_t lo, uint64_t hi) { return first_non_base(haps, lo, hi); });
    if (i < nh) return fail(PHMM_EINVAL, "haplotype base %llu is 0x%02x, not one of ACGTN", (unsigned long long)i, haps[i]);
    const uint64_t p = first_failure(n_pairs, [&](uint64_t lo, uint64_t hi) {
        for (uint64_t q = lo; q < hi; ++q)
            if (pl[2 * q] >= n_reads || pl[2 * q + 1] >= n_haps) return q;
        return hi;
    });
    if (p < n_pairs) {
        if (pl[2 * p] >= n_reads) return fail(PHMM_EINVAL, "pair %llu: read index %u >= %u", (unsigned long long)p, pl[2 * p], n_reads);
        return fail(PHMM_EINVAL, "pair %llu: haplotype index %u >= %u", (unsigned long long)p, pl[2 * p + 1], n_haps);
    }
    return PHMM_OK;
}

extern "C" int phmm_validate_batch(const uint8_t* reads, const uint8_t* bq, const uint8_t* iq,
                                   const uint8_t* dq, const uint8_t* gq, const uint64_t* ro,
                                   uint32_t n_reads, const uint8_t* haps, const uint64_t* ho,
                                   uint32_t n_haps, const uint32_t* pl, uint64_t n_pairs,
                                   uint32_t* max_read_len, uint32_t* max_hap_len)
{
    uint32_t ml = 0, mk = 0;
    double dummy = 0.0;
    if (n_pairs > 0xffffffffull) return fail(PHMM_ERANGE, "n_pairs exceeds 2^32-1");
    int rc = validate(reads, bq, iq, dq, gq, ro, n_reads, haps, ho, n_haps, pl, n_pairs, &dummy,
                      &ml, &mk);
    if (max_read_len) *max_read_len = ml;
    if (max_hap_len) *max_hap_len = mk;
    return rc;
}

static int ensure_arena(phmm_ctx* c, size_t bytes)
{
    if (c->arena_bytes >= bytes) return PHMM_OK;
    if (c->arena) {
        HIP_TRY(hipStreamSynchronize(c->stream));
        HIP_TRY(hipFree(c->arena));
        c->arena = nullptr;
        c->arena_bytes = 0;
    }
    size_t sz = std::max(bytes, c->arena_bytes * 3 / 2);
    if (hipMalloc(&c->arena, sz) != hipSuccess) {
        c->arena = nullptr;
        return fail(PHMM_ENOMEM, "device arena of %zu bytes", sz);
    }
    c->arena_bytes = sz;
    return PHMM_OK;
}

// Synchronous batches of at least 2 * kChunkPairs pairs move their inputs in
// chunks of pairs (at most kMaxChunks) on a copy stream while the chunks
// before them compute on the context's stream.
constexpr uint64_t kChunkPairs = 1ull << 22;
constexpr int kMaxChunks = 16;

// Per chunk of pairs [p0[k], p0[k+1]): one past the largest read and
// haplotype index any pair of chunks 0..k uses, so that chunk k can start
// once those prefixes of the read and haplotype arrays are on the device.
static void chunk_needs(const uint32_t* pl, const std::vector<uint64_t>& p0,
                        std::vector<uint64_t>& need_r, std::vector<uint64_t>& need_h)
{
    const size_t nc = p0.size() - 1;
    need_r.assign(nc, 0);
    need_h.assign(nc, 0);
    std::vector<std::thread> th;
    for (size_t k = 0; k < nc; ++k)
        th.emplace_back([&, k] {
            uint64_t r = 0, h = 0;
            for (uint64_t q = p0[k]; q < p0[k + 1]; ++q) {
                r = std::max<uint64_t>(r, pl[2 * q] + 1ull);
                h = std::max<uint64_t>(h, pl[2 * q + 1] + 1ull);
            }
            need_r[k] = r;
            need_h[k] = h;
        });
    for (auto& x : th) x.join();
    for (size_t k = 1; k < nc; ++k) {
        need_r[k] = std::max(need_r[k], need_r[k - 1]);
        need_h[k] = std::max(need_h[k], need_h[k - 1]);
    }
}

extern "C" int phmm_forward_batch(phmm_ctx* c, const uint8_t* reads, const uint8_t* bq,
                                  const uint8_t* iq, const uint8_t* dq, const uint8_t* gq,
                                  const uint64_t* ro, uint32_t n_reads, const uint8_t* haps,
                                  const uint64_t* ho, uint32_t n_haps, const uint32_t* pl,
                                  uint64_t n_pairs, double* out, uint8_t* flags)
{
    if (!c) return fail(PHMM_EINVAL, "phmm_forward_batch: ctx is NULL");
    if (n_pairs > 0xffffffffull) return fail(PHMM_ERANGE, "n_pairs exceeds 2^32-1");
    uint32_t max_l, max_k;
    int rc = validate(reads, bq, iq, dq, gq, ro, n_reads, haps, ho, n_haps, pl, n_pairs, out,
                      &max_l, &max_k);
    if (rc != PHMM_OK || n_pairs == 0) return rc;
    HIP_TRY(hipSetDevice(c->device));
    const uint64_t nb = ro[n_reads], nh = ho[n_haps];
    const int nchunk = (int)std::min<uint64_t>(kMaxChunks, std::max<uint64_t>(1, n_pairs / kChunkPairs / 2));
    std::vector<uint64_t> p0(nchunk + 1);
    for (int k = 0; k <= nchunk; ++k) p0[k] = n_pairs * (uint64_t)k / (uint64_t)nchunk;
    uint64_t chunk_max = 0;
    for (int k = 0; k < nchunk; ++k) chunk_max = std::max(chunk_max, p0[k + 1] - p0[k]);
    size_t o = 0;
    const size_t o_reads = o; o = align256(o + nb * 5);
    const size_t o_ro = o; o = align256(o + ((size_t)n_reads + 1) * 8);
    const size_t o_haps = o; o = align256(o + nh);
    const size_t o_ho = o; o = align256(o + ((size_t)n_haps + 1) * 8);
    const size_t o_pl = o; o = align256(o + n_pairs * 8);
    const size_t o_out = o; o = align256(o + n_pairs * 8);
    const size_t o_fl = o; o = align256(o + n_pairs);
    const size_t o_ws = o;
    const size_t ws = phmm_workspace_bytes(c, chunk_max, max_l, max_k);
    o += ws;
    rc = ensure_arena(c, o);
    if (rc != PHMM_OK) return rc;
    char* A = static_cast<char*>(c->arena);
    hipStream_t s = c->stream;
    Batch b;
    b.reads = reinterpret_cast<const uint8_t*>(A + o_reads);
    b.bq = b.reads + nb;
    b.iq = b.reads + 2 * nb;
    b.dq = b.reads + 3 * nb;
    b.gq = b.reads + 4 * nb;
    b.read_off = reinterpret_cast<const uint64_t*>(A + o_ro);
    b.haps = reinterpret_cast<const uint8_t*>(A + o_haps);
    b.hap_off = reinterpret_cast<const uint64_t*>(A + o_ho);
    b.pairs = reinterpret_cast<const uint32_t*>(A + o_pl);
    b.n_pairs = n_pairs;
    b.out = reinterpret_cast<double*>(A + o_out);
    b.flags = reinterpret_cast<uint8_t*>(A + o_fl);
    // the byte ranges [b0, b1) of the five read arrays, of the haplotypes and
    // of the pair list, on stream cs
    auto copy_reads = [&](uint64_t b0, uint64_t b1, hipStream_t cs) -> int {
        if (b1 <= b0) return PHMM_OK;
        const uint8_t* src[5] = {reads, bq, iq, dq, gq};
        for (int q = 0; q < 5; ++q)
            HIP_TRY(hipMemcpyAsync(A + o_reads + q * nb + b0, src[q] + b0, b1 - b0,
                                   hipMemcpyHostToDevice, cs));
        return PHMM_OK;
    };
    auto copy_haps = [&](uint64_t b0, uint64_t b1, hipStream_t cs) -> int {
        if (b1 > b0) HIP_TRY(hipMemcpyAsync(A + o_haps + b0, haps + b0, b1 - b0, hipMemcpyHostToDevice, cs));
        return PHMM_OK;
    };
    auto copy_pairs = [&](uint64_t q0, uint64_t q1, hipStream_t cs) -> int {
        if (q1 > q0)
            HIP_TRY(hipMemcpyAsync(A + o_pl + q0 * 8, pl + 2 * q0, (q1 - q0) * 8, hipMemcpyHostToDevice, cs));
        return PHMM_OK;
    };
    if (nchunk == 1) {
        if ((rc = copy_reads(0, nb, s)) != PHMM_OK || (rc = copy_haps(0, nh, s)) != PHMM_OK ||
            (rc = copy_pairs(0, n_pairs, s)) != PHMM_OK)
            return rc;
        HIP_TRY(hipMemcpyAsync(A + o_ro, ro, ((size_t)n_reads + 1) * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(A + o_ho, ho, ((size_t)n_haps + 1) * 8, hipMemcpyHostToDevice, s));
        rc = enqueue_sync(c, b, A + o_ws, s, max_k);
        if (rc != PHMM_OK) return rc;
        HIP_TRY(hipMemcpyAsync(c->h_ctr, A + o_ws, sizeof(Counters), hipMemcpyDeviceToHost, s));
    } else {
        // copies of chunk k+1 (pageable host memory: the host thread stages
        // them) overlap the pass over chunk k, which the context's stream
        // starts once its inputs are on the device
        if (!c->copy_stream) HIP_TRY(hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
        if (!c->h_chunk)
            HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&c->h_chunk), kMaxChunks * sizeof(Counters),
                                  hipHostMallocDefault));
        for (int k = 0; k < nchunk; ++k)
            if (!c->ev_chunk[k]) HIP_TRY(hipEventCreateWithFlags(&c->ev_chunk[k], hipEventDisableTiming));
        std::vector<uint64_t> need_r, need_h;
        chunk_needs(pl, p0, need_r, need_h);
        hipStream_t cs = c->copy_stream;
        HIP_TRY(hipMemcpyAsync(A + o_ro, ro, ((size_t)n_reads + 1) * 8, hipMemcpyHostToDevice, cs));
        HIP_TRY(hipMemcpyAsync(A + o_ho, ho, ((size_t)n_haps + 1) * 8, hipMemcpyHostToDevice, cs));
        uint64_t done_r = 0, done_h = 0;
        for (int k = 0; k < nchunk; ++k) {
            if ((rc = copy_reads(ro[done_r], ro[need_r[k]], cs)) != PHMM_OK ||
                (rc = copy_haps(ho[done_h], ho[need_h[k]], cs)) != PHMM_OK ||
                (rc = copy_pairs(p0[k], p0[k + 1], cs)) != PHMM_OK)
                return rc;
            done_r = std::max(done_r, need_r[k]);
            done_h = std::max(done_h, need_h[k]);
            HIP_TRY(hipEventRecord(c->ev_chunk[k], cs));
            HIP_TRY(hipStreamWaitEvent(s, c->ev_chunk[k], 0));
            Batch bk = b;
            bk.pairs = b.pairs + 2 * p0[k];
            bk.n_pairs = p0[k + 1] - p0[k];
            bk.out = b.out + p0[k];
            bk.flags = b.flags + p0[k];
            rc = enqueue(c, bk, A + o_ws, s, max_k, UINT32_MAX);
            if (rc != PHMM_OK) return rc;
            HIP_TRY(hipMemcpyAsync(c->h_chunk + k, A + o_ws, sizeof(Counters), hipMemcpyDeviceToHost, s));
        }
    }
    HIP_TRY(hipMemcpyAsync(out, b.out, n_pairs * 8, hipMemcpyDeviceToHost, s));
    if (flags) HIP_TRY(hipMemcpyAsync(flags, b.flags, n_pairs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < nchunk; ++k) {
        const uint32_t st = nchunk == 1 ? c->h_ctr->status : c->h_chunk[k].status;
        if (st != 0) return fail((int)st, "device reported error %d", (int)st);
    }
    return PHMM_OK;
}

static std::mutex g_default_mu;
// ---------------------------------------------------------------- genotypes
static int genotype_args(const void* lk, const uint64_t* lo, const uint32_t* nr,
                         const uint32_t* nh, const uint64_t* go, uint32_t n_regions,
                         const void* gl, const uint32_t* best)
{
    if (n_regions == 0) return PHMM_OK;
    if (!lk || !lo || !nr || !nh || !go || !gl || !best)
        return fail(PHMM_EINVAL, "genotype batch: NULL array with %u regions", n_regions);
    return PHMM_OK;
}

extern "C" int phmm_genotype_batch(phmm_ctx* c, const double* lk, uint64_t n_lk,
                                   const uint64_t* lo, const uint32_t* nr, const uint32_t* nh,
                                   const uint64_t* go, uint32_t n_regions, double* gl,
                                   uint64_t n_gl, uint32_t* best)
{
    int rc = genotype_args(lk, lo, nr, nh, go, n_regions, gl, best);
    if (rc != PHMM_OK) return rc;
    for (uint32_t g = 0; g < n_regions; ++g) {
        const uint64_t R = nr[g], H = nh[g], G = H * (H + 1) / 2;
        if (H == 0 || H > PHMM_GT_MAX_HAPS)
            return fail(PHMM_EINVAL, "region %u: %llu haplotypes (1..%u allowed)", g,
                        (unsigned long long)H, PHMM_GT_MAX_HAPS);
        if (lo[g] > n_lk || R * H > n_lk - lo[g])
            return fail(PHMM_EINVAL, "region %u: likelihoods [%llu, +%llu) outside n_lk = %llu",
                        g, (unsigned long long)lo[g], (unsigned long long)(R * H),
                        (unsigned long long)n_lk);
        if (go[g] > n_gl || G > n_gl - go[g])
            return fail(PHMM_EINVAL, "region %u: genotypes [%llu, +%llu) outside n_gl = %llu",
                        g, (unsigned long long)go[g], (unsigned long long)G,
                        (unsigned long long)n_gl);
        for (uint64_t t = 0; t < R * H; ++t)
            if (!std::isfinite(lk[lo[g] + t]))
                return fail(PHMM_EINVAL, "region %u: lk[%llu] is not finite", g,
                            (unsigned long long)(lo[g] + t));
    }
    if (!c) return fail(PHMM_EINVAL, "phmm_genotype_batch: NULL ctx");
    if (n_regions == 0) return PHMM_OK;
    HIP_TRY(hipSetDevice(c->device));
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t b_lk = up(n_lk * 8), b_gl = up(n_gl * 8), b_r8 = up((size_t)n_regions * 8),
                 b_r4 = up((size_t)n_regions * 4);
    rc = ensure_arena(c, b_lk + b_gl + 2 * b_r8 + 3 * b_r4);
    if (rc != PHMM_OK) return rc;
    char* p = static_cast<char*>(c->arena);
    double* d_lk = reinterpret_cast<double*>(p);
    double* d_gl = reinterpret_cast<double*>(p += b_lk);
    uint64_t* d_lo = reinterpret_cast<uint64_t*>(p += b_gl);
    uint64_t* d_go = reinterpret_cast<uint64_t*>(p += b_r8);
    uint32_t* d_nr = reinterpret_cast<uint32_t*>(p += b_r8);
    uint32_t* d_nh = reinterpret_cast<uint32_t*>(p += b_r4);
    uint32_t* d_best = reinterpret_cast<uint32_t*>(p += b_r4);
    hipStream_t s = c->stream;
    HIP_TRY(hipMemcpyAsync(d_lk, lk, n_lk * 8, hipMemcpyHostToDevice, s));
    // entries of gl outside every region's block keep the caller's values
    HIP_TRY(hipMemcpyAsync(d_gl, gl, n_gl * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_lo, lo, (size_t)n_regions * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_go, go, (size_t)n_regions * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_nr, nr, (size_t)n_regions * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_nh, nh, (size_t)n_regions * 4, hipMemcpyHostToDevice, s));
    if (launch_genotype(s, c->cus, d_lk, n_lk, d_lo, d_nr, d_nh, d_go, n_regions, d_gl, n_gl,
                        d_best) != 0)
        return fail(PHMM_EDEVICE, "genotype kernel launch failed");
    HIP_TRY(hipMemcpyAsync(gl, d_gl, n_gl * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(best, d_best, (size_t)n_regions * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PHMM_OK;
}

extern "C" int phmm_genotype_batch_async(phmm_ctx* c, const double* d_lk, uint64_t n_lk,
                                         const uint64_t* d_lo, const uint32_t* d_nr,
                                         const uint32_t* d_nh, const uint64_t* d_go,
                                         uint32_t n_regions, double* d_gl, uint64_t n_gl,
                                         uint32_t* d_best, void* hip_stream)
{
    if (!c) return fail(PHMM_EINVAL, "phmm_genotype_batch_async: NULL ctx");
    const int rc = genotype_args(d_lk, d_lo, d_nr, d_nh, d_go, n_regions, d_gl, d_best);
    if (rc != PHMM_OK) return rc;
    if (n_regions == 0) return PHMM_OK;
    HIP_TRY(hipSetDevice(c->device));
    if (launch_genotype(static_cast<hipStream_t>(hip_stream), c->cus, d_lk, n_lk, d_lo, d_nr,
                        d_nh, d_go, n_regions, d_gl, n_gl, d_best) != 0)
        return fail(PHMM_EDEVICE, "genotype kernel launch failed");
    return PHMM_OK;
}

static phmm_ctx* g_default = nullptr;

extern "C" int phmm_forward_one(const uint8_t* read, const uint8_t* bq, const uint8_t* iq,
                                const uint8_t* dq, const uint8_t* gq, uint32_t read_len,
                                const uint8_t* hap, uint32_t hap_len, double* out_log10)
{
    if (!read || !bq || !iq || !dq || !gq || !hap || !out_log10)
        return fail(PHMM_EINVAL, "phmm_forward_one: NULL argument");
    if (read_len == 0 || hap_len == 0) return fail(PHMM_EINVAL, "phmm_forward_one: empty sequence");
    std::lock_guard<std::mutex> lk(g_default_mu);
    if (!g_default) {
        phmm_options o;
        phmm_default_options(&o);
        o.precision = PHMM_FP64_PLAIN;
        int rc = phmm_create(&g_default, 0, &o);
        if (rc != PHMM_OK) return rc;
    }
    const uint64_t ro[2] = {0, read_len}, ho[2] = {0, hap_len};
    const uint32_t pl[2] = {0, 0};
    return phmm_forward_batch(g_default, read, bq, iq, dq, gq, ro, 1, hap, ho, 1, pl, 1,
                              out_log10, nullptr);
}

// ---------------------------------------------------------------- autotuning
extern "C" int phmm_set_class_costs(phmm_ctx* c, const float* costs)
{
    if (!c || !costs) return fail(PHMM_EINVAL, "phmm_set_class_costs: NULL argument");
    for (int i = 0; i < 2 * kNumClasses; ++i)
        if (!(costs[i] > 0.0f) || !(costs[i] < 1e30f))
            return fail(PHMM_EINVAL, "phmm_set_class_costs: cost %d is not a positive number", i);
    for (int prec = 0; prec < 2; ++prec)
        for (int cls = 0; cls < kNumClasses; ++cls) c->cost[prec][cls] = costs[prec * kNumClasses + cls];
    return PHMM_OK;
}

extern "C" int phmm_get_class_costs(phmm_ctx* c, float* costs)
{
    if (!c || !costs) return fail(PHMM_EINVAL, "phmm_get_class_costs: NULL argument");
    for (int prec = 0; prec < 2; ++prec)
        for (int cls = 0; cls < kNumClasses; ++cls) costs[prec * kNumClasses + cls] = c->cost[prec][cls];
    return PHMM_OK;
}

// Measures the time of one wavefront-row of every (precision, class) kernel
// on a synthetic batch whose pairs fill a wavefront exactly in that class
// (haplotypes of 64 N bases, one pair per pack, reads of 150 bases drawn from
// the haplotypes so that no FP32 result falls under the acceptance
// threshold), and makes those times the packer's cost table.
extern "C" int phmm_autotune(phmm_ctx* c, uint64_t seed, float* out_costs)
{
    if (!c) return fail(PHMM_EINVAL, "phmm_autotune: ctx is NULL");
    HIP_TRY(hipSetDevice(c->device));
    constexpr int kReads = 512, kHaps = 16, kRepeat = 8, kLen = 150;
    const uint64_t n_pairs = (uint64_t)kReads * kHaps * kRepeat;
    uint64_t st = seed * 0x9E3779B97F4A7C15ull + 0xD1B54A32D192ED03ull;
    auto rnd = [&st]() {
        st ^= st << 13; st ^= st >> 7; st ^= st << 17;
        return st;
    };
    static const uint8_t kB[4] = {'A', 'C', 'G', 'T'};
    float measured[2][kNumClasses];
    const phmm_options saved = c->opt;
    int rc = PHMM_OK;
    for (int cls = 0; cls < kNumClasses && rc == PHMM_OK; ++cls) {
        const int k = kWave * class_n(cls);
        // haplotypes: one random sequence and variants of it with a few SNPs
        std::vector<uint8_t> haps((size_t)kHaps * k);
        for (int j = 0; j < k; ++j) haps[j] = kB[rnd() & 3];
        for (int h = 1; h < kHaps; ++h) {
            memcpy(&haps[(size_t)h * k], haps.data(), k);
            for (int v = 0; v < 3; ++v) haps[(size_t)h * k + rnd() % k] = kB[rnd() & 3];
        }
        std::vector<uint64_t> ho(kHaps + 1), ro(kReads + 1);
        for (int h = 0; h <= kHaps; ++h) ho[h] = (uint64_t)h * k;
        std::vector<uint8_t> reads((size_t)kReads * kLen), bq(reads.size()), iq(reads.size(), 45),
            dq(reads.size(), 45), gq(reads.size(), 10);
        for (int r = 0; r < kReads; ++r) {
            ro[r] = (uint64_t)r * kLen;
            const int off = (int)(rnd() % (uint64_t)(k > kLen ? k - kLen : 1));
            for (int i = 0; i < kLen; ++i) {
                const int j = off + i;
                reads[(size_t)r * kLen + i] = j < k ? haps[j] : kB[rnd() & 3];
                bq[(size_t)r * kLen + i] = (uint8_t)(30 + rnd() % 11);
            }
        }
        ro[kReads] = (uint64_t)kReads * kLen;
        std::vector<uint32_t> pl(2 * n_pairs);
        uint64_t p = 0;
        for (int rep = 0; rep < kRepeat; ++rep)
            for (int r = 0; r < kReads; ++r)
                for (int h = 0; h < kHaps; ++h, ++p) {
                    pl[2 * p] = (uint32_t)r;
                    pl[2 * p + 1] = (uint32_t)h;
                }
        std::vector<double> out(n_pairs);
        for (int prec = 0; prec < 2 && rc == PHMM_OK; ++prec) {
            c->opt = saved;
            c->opt.precision = prec == 0 ? PHMM_FP32_RERUN : PHMM_FP64_PLAIN;
            c->opt.force_class = cls;
            c->opt.one_pair_per_wave = 1;
            c->opt.timing = 1;
            float best = 0.f;
            for (int rep = 0; rep < 3 && rc == PHMM_OK; ++rep) {  // first run warms up
                rc = phmm_forward_batch(c, reads.data(), bq.data(), iq.data(), dq.data(), gq.data(),
                                        ro.data(), kReads, haps.data(), ho.data(), kHaps, pl.data(),
                                        n_pairs, out.data(), nullptr);
                float ms = 0.f;
                if (rc == PHMM_OK) {
                    if (hipEventElapsedTime(&ms, c->ev[prec == 0 ? 1 : 2], c->ev[prec == 0 ? 2 : 3]) !=
                        hipSuccess)
                        rc = fail(PHMM_EDEVICE, "phmm_autotune: event timing failed");
                }
                if (rep > 0 && (best == 0.f || ms < best)) best = ms;
            }
            // one pack per pair, kLen rows per pack
            measured[prec][cls] = best / (float)((double)n_pairs * kLen) * 1e6f;  // ns per wave-row
        }
    }
    c->opt = saved;
    if (rc != PHMM_OK) return rc;
    for (int prec = 0; prec < 2; ++prec)
        for (int cls = 0; cls < kNumClasses; ++cls) {
            c->cost[prec][cls] = measured[prec][cls];
            if (out_costs) out_costs[prec * kNumClasses + cls] = measured[prec][cls];
        }
    return PHMM_OK;
}

// Chooses the cost table that runs a sample of the caller's own workload
// fastest: the synthetic per-class measurements above (if phmm_autotune ran)
// and the family N + a for a in {0, 1, 2, 3, 5, 8, 12, 20}, each timed on the
// sample (packing plus the short kernels of the context's precision, best of
// two runs after one warm-up).
extern "C" int phmm_autotune_sample(phmm_ctx* c, const phmm_device_batch* sample, void* d_ws,
                                    size_t ws_bytes, void* hip_stream, float* out_costs)
{
    if (!c || !sample || !d_ws) return fail(PHMM_EINVAL, "phmm_autotune_sample: NULL argument");
    HIP_TRY(hipSetDevice(c->device));
    const float adds[] = {0.f, 1.f, 2.f, 3.f, 5.f, 8.f, 12.f, 20.f};
    constexpr int kCand = 1 + (int)(sizeof(adds) / sizeof(adds[0]));
    float cand[kCand][2][kNumClasses];
    for (int prec = 0; prec < 2; ++prec)
        for (int cls = 0; cls < kNumClasses; ++cls) {
            cand[0][prec][cls] = c->cost[prec][cls];
            for (int a = 0; a < kCand - 1; ++a) cand[a + 1][prec][cls] = (float)class_n(cls) + adds[a];
        }
    const int timing = c->opt.timing;
    c->opt.timing = 1;
    const int prec = c->opt.precision == PHMM_FP32_RERUN ? 0 : 1;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    double* out = nullptr;
    uint8_t* fl = nullptr;
    int rc = PHMM_OK;
    if (hipMalloc(&out, (size_t)(sample->n_pairs ? sample->n_pairs : 1) * 9) != hipSuccess)
        rc = fail(PHMM_ENOMEM, "phmm_autotune_sample: output buffer");
    fl = reinterpret_cast<uint8_t*>(out + (sample->n_pairs ? sample->n_pairs : 1));
    float saved[2][kNumClasses];
    memcpy(saved, c->cost, sizeof saved);
    // the candidates take turns (one pass each per round, a warm-up round
    // first), so that a drift of the clock over the run favours none of them;
    // each keeps its best time over the four timed rounds
    float t_best[kCand] = {};
    for (int rep = 0; rep < 5 && rc == PHMM_OK; ++rep)
        for (int k = 0; k < kCand && rc == PHMM_OK; ++k) {
            memcpy(c->cost, cand[k], sizeof saved);
            rc = phmm_forward_batch_async(c, sample, out, fl, d_ws, ws_bytes, s);
            if (rc != PHMM_OK) break;
            float ms = 0.f;
            if (hipEventSynchronize(c->ev[4]) != hipSuccess ||
                hipEventElapsedTime(&ms, c->ev[0], c->ev[prec == 0 ? 2 : 3]) != hipSuccess)
                rc = fail(PHMM_EDEVICE, "phmm_autotune_sample: event timing failed");
            if (rep > 0 && (t_best[k] == 0.f || ms < t_best[k])) t_best[k] = ms;
        }
    int best = 0;
    for (int k = 1; k < kCand; ++k)
        if (t_best[k] < t_best[best]) best = k;
    if (out) (void)hipFree(out);
    c->opt.timing = timing;
    memcpy(c->cost, rc == PHMM_OK ? cand[best] : saved, sizeof saved);
    if (rc != PHMM_OK) return rc;
    if (out_costs)
        for (int q = 0; q < 2; ++q)
            for (int cls = 0; cls < kNumClasses; ++cls) out_costs[q * kNumClasses + cls] = c->cost[q][cls];
    return PHMM_OK;
}
