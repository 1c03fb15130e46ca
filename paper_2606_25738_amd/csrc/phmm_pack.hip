// Device-side grouping and packing of (read, haplotype) pairs.
//
// Pairs of the same read that are adjacent in the pair list form a run (cut
// every kChunk pairs).  For each run one thread chooses the column class N
// (columns per lane) that minimises the modelled cost waves x cost[N], packs
// the run's pairs greedily into 64-lane wavefronts (ceil(k/N) lanes per
// pair, at most 32 pairs per wavefront) and emits the packs into the segment
// of its (precision, class).  Every pack holds one read, so the per-row
// priors and the read base are uniform across the wavefront.  In FP32 mode a
// run whose haplotypes are mutually unrelated starts in FP64 (most of its
// pairs would be rejected by the FP32 threshold).  Haplotypes
// longer than 64 * kMaxN columns go to one of the long-pair lists (by
// precision, and by whether the read allows the lean long kernel).
//
// Five kernels, no contended global atomics: count (per-block segment pack
// counts from LDS atomics, one greedy pass that sizes all classes at once),
// a two-level scan of the counts (chunk sums, chunk offsets in one workgroup,
// block offsets inside each chunk) and emit (each run writes its packs at
// its block's offset).  Counts and offsets are laid out [segment][block], so
// every scan pass reads and writes contiguous words.
//
// The paper bins pairs by length and runs a dedicated kernel instance per
// sub-warp size (Section 3.2); here the binning key is the column class and
// the packing is done on the device so that a batch never returns to the
// host between packing and compute.
#include "phmm_dev.h"

namespace phmm {

constexpr int kScanChunk = 2048;  // packer blocks per scan chunk (8 per thread)

__global__ void reset_kernel(Counters* c)
{
    uint32_t* w = reinterpret_cast<uint32_t*>(c);
    const int n = (int)(sizeof(Counters) / 4);
    for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0;
}

__device__ __forceinline__ uint32_t hap_len(const Batch& b, uint32_t h)
{
    return (uint32_t)(b.hap_off[h + 1] - b.hap_off[h]);
}

__device__ __forceinline__ bool run_start(const Batch& b, uint64_t p)
{
    return p == 0 || b.pairs[2 * p] != b.pairs[2 * p - 2] || (p % kChunk) == 0;
}

__device__ __forceinline__ uint64_t run_end(const Batch& b, uint64_t p)
{
    const uint32_t r = b.pairs[2 * p];
    uint64_t e = p + 1;
    while (e < b.n_pairs && b.pairs[2 * e] == r && (e % kChunk) != 0) ++e;
    return e;
}

// Greedy packing state of one class: lanes used in the open pack, pairs in
// it, packs so far.  A long pair closes the open pack.
struct Greedy {
    uint32_t used, np, packs;
    __device__ void reset() { used = kWave; np = 0; packs = 0; }
    __device__ void add(uint32_t s, int one_per_wave)
    {
        if (one_per_wave || used + s > (uint32_t)kWave || np == (uint32_t)kMaxPairsPerPack) {
            ++packs;
            used = 0;
            np = 0;
        }
        used += s;
        ++np;
    }
};

// 4-mer presence set (256 bits) of the first kKmerBases bases of haplotype
// h; bases are coded (c >> 1) & 3, which separates A, C, G and T ('N' shares
// G's code, harmless for a similarity estimate).
constexpr uint32_t kKmerBases = 32;
__device__ void kmer_set(const Batch& b, uint32_t h, uint64_t (&m)[4])
{
    m[0] = m[1] = m[2] = m[3] = 0ull;
    const uint8_t* hs = b.haps + b.hap_off[h];
    const uint32_t n = min(hap_len(b, h), kKmerBases);
    uint8_t c[kKmerBases];
#pragma unroll
    for (uint32_t j = 0; j < kKmerBases; ++j) c[j] = j < n ? hs[j] : (uint8_t)0;
    uint32_t code = 0;
#pragma unroll
    for (uint32_t j = 0; j < kKmerBases; ++j) {
        code = ((code << 2) | ((c[j] >> 1) & 3u)) & 255u;
        if (j >= 3 && j < n) {
            const uint64_t bit = 1ull << (code & 63u);
            const uint32_t q = code >> 6;
            m[0] |= q == 0 ? bit : 0ull;
            m[1] |= q == 1 ? bit : 0ull;
            m[2] |= q == 2 ? bit : 0ull;
            m[3] |= q == 3 ? bit : 0ull;
        }
    }
}

// Jaccard index of two 4-mer sets at least 1/2.
__device__ __forceinline__ bool kmer_similar(const uint64_t (&a)[4], const uint64_t (&m)[4])
{
    int both = 0, any = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        both += __popcll(a[q] & m[q]);
        any += __popcll(a[q] | m[q]);
    }
    return 2 * both >= any;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, kWave);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, kWave);
    return ((uint64_t)hi << 32) | lo;
}

// ceil(k / n) for k <= 2^20 and n in [4, 24]: a float estimate with the
// reciprocal of n, then an exact fix-up (no integer division)
__device__ __forceinline__ uint32_t ceil_div_small(uint32_t k, uint32_t n, float rcp)
{
    uint32_t s = (uint32_t)((float)(k + n - 1) * rcp);
    if (s * n < k) ++s;
    if (s > 0 && (s - 1) * n >= k) --s;
    return s;
}

// OR of word(w) over the 4-byte words of the 16-byte-aligned blocks of
// v[0, l) and of byte(x) over the bytes before the first and after the last
// such block.  The kLanes lanes of a group share the scan: lane `sub` takes
// every kLanes-th block (two loads in flight) and every kLanes-th loose byte.
template <int kLanes, typename W, typename B>
__device__ __forceinline__ uint32_t scan_bytes(const uint8_t* v, uint32_t l, int sub, W word, B byte)
{
    const uintptr_t s0 = (uintptr_t)v, s1 = s0 + l;
    const uintptr_t a0 = (s0 + 15u) & ~(uintptr_t)15u, a1 = s1 & ~(uintptr_t)15u;
    uint32_t bad = 0u;
    if (a0 >= a1) {
        for (uint32_t i = (uint32_t)sub; i < l; i += kLanes) bad |= byte(v[i]);
        return bad;
    }
    for (uint32_t i = (uint32_t)sub; i < (uint32_t)(a0 - s0); i += kLanes) bad |= byte(v[i]);
    const uint8_t* t = reinterpret_cast<const uint8_t*>(a1);
    for (uint32_t i = (uint32_t)sub; i < (uint32_t)(s1 - a1); i += kLanes) bad |= byte(t[i]);
    const uint4* V = reinterpret_cast<const uint4*>(a0);
    const uint32_t nb = (uint32_t)((a1 - a0) / 16u);
    for (uint32_t q = (uint32_t)sub; q < nb; q += 2 * kLanes) {
        const uint32_t q2 = q + kLanes;
        const uint4 x = V[q];
        const uint4 y = q2 < nb ? V[q2] : x;
        bad |= word(x.x) | word(x.y) | word(x.z) | word(x.w);
        bad |= word(y.x) | word(y.y) | word(y.z) | word(y.w);
    }
    return bad;
}

// Whether a read needs the general long kernel: a gap byte of 0, more than
// one gap byte, or an insertion byte above kScMaxInsQ on some row.  Words of
// gap bytes are compared with the first byte replicated; a word of insertion
// bytes has one above kScMaxInsQ when its top bit is set or its low seven
// bits plus 127 - kScMaxInsQ carry into it.
template <int kLanes>
__device__ __forceinline__ int read_needs_general(const Batch& b, uint64_t roff, uint32_t l, int sub)
{
    const uint32_t g0 = b.gq[roff];
    if (g0 == 0u) return 1;
    const uint32_t g4 = g0 * 0x01010101u;
    constexpr uint32_t kAdd = (127u - (uint32_t)kScMaxInsQ) * 0x01010101u;
    const uint32_t bad_g = scan_bytes<kLanes>(
        b.gq + roff, l, sub, [g4](uint32_t w) { return w ^ g4; },
        [g0](uint8_t x) { return (uint32_t)(x != g0); });
    const uint32_t bad_i = scan_bytes<kLanes>(
        b.iq + roff, l, sub, [](uint32_t w) { return (((w & 0x7f7f7f7fu) + kAdd) | w) & 0x80808080u; },
        [](uint8_t x) { return (uint32_t)(x > kScMaxInsQ); });
    return (bad_g | bad_i) != 0u;
}

// Whether a read has a gap byte above kLongFp32MaxGap on some row.  A long
// pair has no FP32 acceptance test: its rescaled FP32 sum is accepted
// whatever its value.  FP32 keeps 2^126 between a tile's largest value and
// the smallest it can hold; when gaps are costly (T_II = T_DD = 10^-gcp/10
// small), the diagonals of a read unrelated to its haplotype drift apart by
// more than that, and a diagonal flushed to zero can later carry the sum:
// unrelated pairs of 2-6 kbp were off by up to 1e-1 in log10 at gap byte 20
// and up to 4e1 at 25 (-inf at 60), while every gap byte of 10 or less kept
// them within 6e-6.  Such reads run their long pairs in FP64.
constexpr int kLongFp32MaxGap = 10;

template <int kLanes>
__device__ __forceinline__ int read_gap_over(const Batch& b, uint64_t roff, uint32_t l, int sub)
{
    constexpr uint32_t kAdd = (127u - (uint32_t)kLongFp32MaxGap) * 0x01010101u;
    return scan_bytes<kLanes>(
               b.gq + roff, l, sub,
               [](uint32_t w) { return (((w & 0x7f7f7f7fu) + kAdd) | w) & 0x80808080u; },
               [](uint8_t x) { return (uint32_t)(x > kLongFp32MaxGap); }) != 0u;
}

// Routing of long pairs: one workgroup per pair queued by the count kernel
// scans the pair's read and appends the pair to the lean or the general long
// list of its precision (an FP32 pair whose read has a gap byte above
// kLongFp32MaxGap to the FP64 lists).  A read is scanned once per long pair:
// at most its length in bytes against at least kShortMaxCols cells per row
// of the pair.
constexpr int kRouteBlock = 256;
constexpr int kRouteGrid = 1024;

__global__ __launch_bounds__(kRouteBlock) void long_route_kernel(Batch b, Work w)
{
    const int t = (int)threadIdx.x;
    for (int prec = 0; prec < 2; ++prec) {
        const uint32_t n = w.ctr->n_pend[prec];
        for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {  // workgroup-uniform
            const uint32_t pair = w.long_pend[prec][i];
            const uint32_t r = b.pairs[2 * (uint64_t)pair];
            const uint64_t roff = b.read_off[r];
            const uint32_t l = (uint32_t)(b.read_off[r + 1] - roff);
            const int slow = __syncthreads_or(read_needs_general<kRouteBlock>(b, roff, l, t));
            const int wide = prec == 0 ? __syncthreads_or(read_gap_over<kRouteBlock>(b, roff, l, t)) : 1;
            if (t == 0) {
                const int q = long_list_of(wide ? 1 : 0, slow != 0);
                const uint32_t idx = atomicAdd(&w.ctr->n_long[q], 1u);
                w.long_list[q][idx] = pair;
            }
        }
    }
}

// Pass 1: precision and class per run, pack counts per (segment, block);
// long pairs to the long list.  Each wavefront takes the runs that start in
// its 64 pairs, nine at a time: the 7 lanes 7g .. 7g + 6 size run g, each in
// three of the 21 classes (one greedy pass over the run; the run's
// haplotype lengths are loaded seven at a time, one pair per lane, and
// handed round the group), and the lowest modelled cost waves x cost[class]
// is found across the group.  In FP32 mode a run whose haplotypes are
// mutually unrelated (the 4-mer sets of the first 32 bases of its first short
// haplotype and of up to three more, one set per lane: none shares half of
// the first one's) is packed for FP64.
constexpr int kRunLanes = 7;                           // lanes per run
constexpr int kRunClasses = kNumClasses / kRunLanes;   // classes per lane
constexpr int kRunsPerWave = kWave / kRunLanes;        // runs sized at once
static_assert(kRunClasses * kRunLanes == kNumClasses, "classes split evenly over a run's lanes");


__global__ __launch_bounds__(kPackBlock) void pack_count_kernel(Batch b, Work w, Policy pol)
{
    __shared__ uint32_t cnt[kSeg];
    __shared__ unsigned long long lanecols;
    const int t = (int)threadIdx.x;
    for (int q = t; q < kSeg; q += kPackBlock) cnt[q] = 0u;
    if (t == 0) lanecols = 0ull;
    __syncthreads();
    const int lane = t & (kWave - 1);
    const uint64_t p0 = (uint64_t)blockIdx.x * blockDim.x + (uint64_t)(t - lane);
    const uint64_t mine = p0 + (uint64_t)lane;
    // read of each of the wavefront's pairs, and the run starts among them
    const uint32_t my_r = mine < b.n_pairs ? b.pairs[2 * mine] : 0u;
    const uint32_t left_r = (uint32_t)__shfl((int)my_r, lane > 0 ? lane - 1 : 0, kWave);
    const bool my_start = mine < b.n_pairs &&
                          (mine % kChunk == 0 || my_r != (lane > 0 ? left_r : b.pairs[2 * mine - 2]));
    uint64_t starts = __ballot(my_start);
    const uint64_t all_starts = starts;
    const int g = lane / kRunLanes, sub = lane - g * kRunLanes;  // g = 9: idle lane
    const int lead = g * kRunLanes;
    float rcp[kRunClasses];
#pragma unroll
    for (int i = 0; i < kRunClasses; ++i) rcp[i] = 1.0f / (float)class_n(sub * kRunClasses + i);
    while (starts) {  // wave-uniform
        // the g-th of the next kRunsPerWave run starts
        uint64_t rest = starts;
        for (int j = 0; j < g && rest; ++j) rest &= rest - 1;
        const bool active = g < kRunsPerWave && rest != 0ull;
        const uint64_t p = active ? p0 + (uint64_t)(__ffsll((unsigned long long)rest) - 1) : 0ull;
        for (int j = 0; j < kRunsPerWave && starts; ++j) starts &= starts - 1;
        // the run ends at the next start in the wavefront, else it continues
        // past the wavefront's last pair
        const int pl = active ? (int)(p - p0) : 0;
        const uint32_t r = (uint32_t)__shfl((int)my_r, pl, kWave);
        uint64_t e = p;
        if (active) {
            const uint64_t above = pl < kWave - 1 ? all_starts & (~0ull << (pl + 1)) : 0ull;
            if (above) {
                e = p0 + (uint64_t)(__ffsll((unsigned long long)above) - 1);
            } else {
                e = min(p0 + (uint64_t)kWave, b.n_pairs);
                while (e < b.n_pairs && b.pairs[2 * e] == r && (e % kChunk) != 0) ++e;
            }
        }
        uint32_t l = 0;
        if (active) l = (uint32_t)(b.read_off[r + 1] - b.read_off[r]);
        int prec = (pol.precision == 1 || l > pol.fp32_max_rows) ? 1 : 0;
        const int lprec = (pol.precision == 1 || l > pol.long_fp32_max_rows) ? 1 : 0;
        // this lane's classes sub * kRunClasses + i over the run
        Greedy gr[kRunClasses];
        bool fits[kRunClasses];
#pragma unroll
        for (int i = 0; i < kRunClasses; ++i) {
            gr[i].reset();
            fits[i] = true;
        }
        uint32_t nshort = 0;
        int mylong = 0;  // this lane met a long pair of the run
        uint32_t first_h = 0u, first_k = 0u;  // haplotype and length of pair p + sub
        for (uint64_t base = p; base < e; base += kRunLanes) {
            const uint64_t mine_q = base + (uint64_t)sub;
            const uint32_t mine_h = mine_q < e ? b.pairs[2 * mine_q + 1] : 0u;
            const uint32_t mine_k = mine_q < e ? hap_len(b, mine_h) : 0u;
            if (base == p) {
                first_h = mine_h;
                first_k = mine_k;
            }
            mylong |= mine_k > kShortMaxCols ? 1 : 0;
            const int m = (int)min<uint64_t>((uint64_t)kRunLanes, e - base);
            for (int j = 0; j < m; ++j) {
                const uint32_t k = (uint32_t)__shfl((int)mine_k, lead + j, kWave);
                if (k > kShortMaxCols) {
#pragma unroll
                    for (int i = 0; i < kRunClasses; ++i) {
                        gr[i].used = kWave;
                        gr[i].np = 0;
                    }
                    continue;
                }
                ++nshort;
#pragma unroll
                for (int i = 0; i < kRunClasses; ++i) {
                    const uint32_t N = (uint32_t)class_n(sub * kRunClasses + i);
                    const uint32_t sl = ceil_div_small(k, N, rcp[i]);
                    if (sl > (uint32_t)kWave) fits[i] = false;
                    else gr[i].add(sl, pol.one_pair_per_wave);
                }
            }
        }
        // long pairs of the run wait for routing (lean or general long list).
        // A haplotype beyond the batch's stated length bound (no routing
        // launched) is an error; its pair still goes to the FP64 general
        // list, which every call runs, so that its output is written.
        const int src = active ? lead : lane;
        if (active && mylong) {
            if (!pol.long_haps) w.ctr->bound_err = 1u;
            for (uint64_t base = p; base < e; base += kRunLanes) {
                const uint64_t mine_q = base + (uint64_t)sub;
                if (mine_q < e && hap_len(b, b.pairs[2 * mine_q + 1]) > kShortMaxCols) {
                    uint32_t* cnt = pol.long_haps ? &w.ctr->n_pend[lprec] : &w.ctr->n_long[long_list_of(1, true)];
                    uint32_t* list = pol.long_haps ? w.long_pend[lprec] : w.long_list[long_list_of(1, true)];
                    list[atomicAdd(cnt, 1u)] = (uint32_t)mine_q;
                }
            }
        }
        // unrelated haplotypes: lanes sub = 0..3 take the run's sub-th short
        // haplotype of at least 8 bases: pair p + sub when the pairs p ..
        // p + sub all have one (their lengths are at hand), else by a walk
        const bool check = active && prec == 0 && pol.route_diverse && e - p >= 2;
        const int qual = (p + (uint64_t)sub < e && first_k >= 8u && first_k <= kShortMaxCols) ? 1 : 0;
        int prefix = 1;
        for (int j = 0; j < 4; ++j) {
            const int qj = __shfl(qual, src + j, kWave);
            if (j <= sub) prefix &= qj;
        }
        uint64_t km[4] = {0ull, 0ull, 0ull, 0ull};
        bool have = false;
        if (check && sub < 4 && prefix) {
            kmer_set(b, first_h, km);
            have = true;
        } else if (check && sub < 4) {
            int seen = 0;
            for (uint64_t q = p; q < e; ++q) {
                const uint32_t h = b.pairs[2 * q + 1];
                const uint32_t k = hap_len(b, h);
                if (k > kShortMaxCols || k < 8) continue;
                if (seen == sub) {
                    kmer_set(b, h, km);
                    have = true;
                    break;
                }
                ++seen;
            }
        }
        uint64_t ref[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) ref[q] = shfl64(km[q], src);
        const bool ref_ok = __shfl((int)have, src, kWave) != 0;
        const int cmp = (have && sub > 0 && sub < 4 && ref_ok) ? 1 : 0;
        const int similar = cmp && kmer_similar(ref, km) ? 1 : 0;
        int any_similar = 0, n_compared = 0;
        for (int j = 1; j < 4; ++j) {
            any_similar |= __shfl(similar, src + j, kWave);
            n_compared += __shfl(cmp, src + j, kWave);
        }
        if (check && n_compared > 0 && !any_similar) prec = 1;
        // the class with the lowest modelled cost: first over this lane's
        // classes, then over the group's lanes (first minimum in class order)
        float my_cost = 3.0e38f;
        int my_cls = -1;
        uint32_t my_packs = 0;
#pragma unroll
        for (int i = 0; i < kRunClasses; ++i) {
            const int cls = sub * kRunClasses + i;
            if (!active || nshort == 0 || !fits[i] || (pol.force_class >= 0 && cls != pol.force_class))
                continue;
            const float v = (float)gr[i].packs * pol.cost[prec][cls];
            if (v < my_cost) {
                my_cost = v;
                my_cls = cls;
                my_packs = gr[i].packs;
            }
        }
        float best_cost = 3.0e38f;
        int best = -1;
        uint32_t best_packs = 0;
        for (int j = 0; j < kRunLanes; ++j) {
            const float v = __shfl(my_cost, src + j, kWave);
            const int cl = __shfl(my_cls, src + j, kWave);
            const uint32_t pk = (uint32_t)__shfl((int)my_packs, src + j, kWave);
            if (v < best_cost) {
                best_cost = v;
                best = cl;
                best_packs = pk;
            }
        }
        // forced class too narrow: the widest (held by the group's last lane)
        const uint32_t widest_packs =
            (uint32_t)__shfl((int)gr[kRunClasses - 1].packs, src + kRunLanes - 1, kWave);
        if (active && sub == 0) {
            uint32_t info = 0xffffffffu;
            if (nshort > 0) {
                if (best < 0) {
                    best = kNumClasses - 1;
                    best_packs = widest_packs;
                }
                info = (uint32_t)best | ((uint32_t)prec << 5) | (best_packs << 8);
                atomicAdd(&cnt[prec * kNumClasses + best], best_packs);
                atomicAdd(&lanecols, (unsigned long long)best_packs * kWave * class_n(best));
            }
            w.chunk_info[p] = info;
        }
    }
    __syncthreads();
    for (int q = t; q < kSeg; q += kPackBlock)
        w.blk_cnt[(size_t)q * w.n_pack_blocks + blockIdx.x] = cnt[q];
    if (t == 0) w.blk_lanecols[blockIdx.x] = lanecols;
}

// Block-wide exclusive scan of 256 threads x 8 values (LDS).
__device__ void chunk_scan(uint32_t (&v)[8], uint32_t* lds, uint32_t* total)
{
    const int t = (int)threadIdx.x;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t x = v[j];
        v[j] = s;
        s += x;
    }
    lds[t] = s;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const uint32_t y = t >= d ? lds[t - d] : 0u;
        __syncthreads();
        lds[t] += y;
        __syncthreads();
    }
    const uint32_t excl = lds[t] - s;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] += excl;
    *total = lds[255];
    __syncthreads();
}

// Pass 2a: per (segment, chunk) sums of the block counts; lane columns.
__global__ __launch_bounds__(256) void pack_chunk_sum_kernel(Work w)
{
    __shared__ uint32_t lds[256];
    __shared__ unsigned long long lc[256];
    const uint32_t chunk = blockIdx.x, seg = blockIdx.y;
    const uint32_t b0 = chunk * kScanChunk + threadIdx.x * 8;
    uint32_t v[8];
    unsigned long long l = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t q = b0 + j;
        v[j] = q < w.n_pack_blocks ? w.blk_cnt[(size_t)seg * w.n_pack_blocks + q] : 0u;
        if (seg == 0 && q < w.n_pack_blocks) l += w.blk_lanecols[q];
    }
    uint32_t total;
    chunk_scan(v, lds, &total);
    if (threadIdx.x == 0) w.chunk_part[(size_t)seg * w.n_scan_chunks + chunk] = total;
    if (seg == 0) {
        lc[threadIdx.x] = l;
        __syncthreads();
        for (int d = 128; d > 0; d >>= 1) {
            if ((int)threadIdx.x < d) lc[threadIdx.x] += lc[threadIdx.x + d];
            __syncthreads();
        }
        if (threadIdx.x == 0) atomicAdd(&w.ctr->lane_columns, lc[0]);
    }
}

// Pass 2b (one workgroup): chunk offsets per segment, segment bases of the
// pack array and the capacity of the rerun item lists.  Each wavefront scans
// whole segments (lane t sums a run of consecutive chunks, a shuffle scan
// adds the lanes up), so no barrier is needed until the segment totals.
__global__ __launch_bounds__(1024) void pack_scan_kernel(Work w)
{
    __shared__ uint32_t seg_total[kSeg];
    const int t = (int)threadIdx.x;
    const int lane = t & (kWave - 1);
    const uint32_t n = w.n_scan_chunks;
    const uint32_t per = (n + kWave - 1u) / kWave;
    const uint32_t lo = (uint32_t)lane * per, hi = lo + per < n ? lo + per : n;
    for (int s = t / kWave; s < kSeg; s += (int)blockDim.x / kWave) {
        uint32_t* cp = w.chunk_part + (size_t)s * n;
        uint32_t sum = 0;
        for (uint32_t q = lo; q < hi; ++q) sum += cp[q];
        uint32_t inc = sum;  // inclusive scan of the lane sums
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = __shfl_up(inc, d, kWave);
            if (lane >= d) inc += y;
        }
        uint32_t acc = inc - sum;
        for (uint32_t q = lo; q < hi; ++q) {
            const uint32_t v = cp[q];
            cp[q] = acc;  // becomes the chunk's offset in the segment
            acc += v;
        }
        if (lane == kWave - 1) seg_total[s] = inc;
    }
    __syncthreads();
    if (t == 0) {
        Counters* c = w.ctr;
        uint32_t acc = 0;
        for (int prec = 0; prec < 2; ++prec)
            for (int k = 0; k < kNumClasses; ++k) {
                c->pack_cnt[prec][k] = seg_total[prec * kNumClasses + k];
                c->pack_base[prec][k] = acc;
                acc += seg_total[prec * kNumClasses + k];
            }
        uint32_t acc2 = 0;
        for (int k = 0; k < kNumClasses; ++k) {
            // class k: at most one rerun item, or one deferral, per FP32 pack
            c->item_base[k] = acc2;
            acc2 += c->pack_cnt[0][k];
        }
    }
}

// Pass 2c: block offsets = chunk offset + exclusive scan inside the chunk.
__global__ __launch_bounds__(256) void pack_block_offset_kernel(Work w)
{
    __shared__ uint32_t lds[256];
    const uint32_t chunk = blockIdx.x, seg = blockIdx.y;
    const uint32_t b0 = chunk * kScanChunk + threadIdx.x * 8;
    uint32_t* bc = w.blk_cnt + (size_t)seg * w.n_pack_blocks;
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = b0 + j < w.n_pack_blocks ? bc[b0 + j] : 0u;
    uint32_t total;
    chunk_scan(v, lds, &total);
    const uint32_t base = w.chunk_part[(size_t)seg * w.n_scan_chunks + chunk];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (b0 + j < w.n_pack_blocks) bc[b0 + j] = base + v[j];
}

// Pass 3: write the packs at the block's offset in each segment.
__global__ __launch_bounds__(kPackBlock) void pack_emit_kernel(Batch b, Work w, Policy pol)
{
    __shared__ uint32_t fill[kSeg];
    const int t = (int)threadIdx.x;
    for (int q = t; q < kSeg; q += kPackBlock) fill[q] = 0u;
    __syncthreads();
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + t;
    if (p >= b.n_pairs || !run_start(b, p)) return;
    const uint32_t info = w.chunk_info[p];
    if (info == 0xffffffffu) return;
    const int c = (int)(info & 31u), prec = (int)((info >> 5) & 1u);
    const uint32_t npk = info >> 8;
    const int s = prec * kNumClasses + c;
    const uint32_t slot = w.ctr->pack_base[prec][c] +
                          w.blk_cnt[(size_t)s * w.n_pack_blocks + blockIdx.x] +
                          atomicAdd(&fill[s], npk);
    const uint64_t e = run_end(b, p);
    const uint32_t N = (uint32_t)class_n(c);
    uint32_t written = 0, used = kWave, np = 0;
    uint64_t start = p;
    auto flush = [&]() {
        if (np == 0) return;
        w.packs[slot + written].pair_start = (uint32_t)start;
        w.packs[slot + written].npairs = np;
        ++written;
    };
    for (uint64_t q = p; q < e; ++q) {
        const uint32_t k = hap_len(b, b.pairs[2 * q + 1]);
        if (k > kShortMaxCols) {
            flush();
            used = kWave;
            np = 0;
            continue;
        }
        const uint32_t sl = (k + N - 1) / N;
        if (pol.one_pair_per_wave || used + sl > (uint32_t)kWave ||
            np == (uint32_t)kMaxPairsPerPack) {
            flush();
            used = 0;
            np = 0;
            start = q;
        }
        used += sl;
        ++np;
    }
    flush();
}

void launch_pack(hipStream_t s, const Batch& b, const Work& w, const Policy& pol)
{
    hipLaunchKernelGGL(pack_count_kernel, dim3(w.n_pack_blocks), dim3(kPackBlock), 0, s, b, w, pol);
    if (pol.long_haps)
        hipLaunchKernelGGL(long_route_kernel, dim3((uint32_t)std::min<uint64_t>(b.n_pairs, kRouteGrid)),
                           dim3(kRouteBlock), 0, s, b, w);
    hipLaunchKernelGGL(pack_chunk_sum_kernel, dim3(w.n_scan_chunks, kSeg), dim3(256), 0, s, w);
    hipLaunchKernelGGL(pack_scan_kernel, dim3(1), dim3(1024), 0, s, w);
    hipLaunchKernelGGL(pack_block_offset_kernel, dim3(w.n_scan_chunks, kSeg), dim3(256), 0, s, w);
    hipLaunchKernelGGL(pack_emit_kernel, dim3(w.n_pack_blocks), dim3(kPackBlock), 0, s, b, w, pol);
}

uint32_t scan_chunks(uint32_t n_pack_blocks) { return (n_pack_blocks + kScanChunk - 1) / kScanChunk; }

}  // namespace phmm
