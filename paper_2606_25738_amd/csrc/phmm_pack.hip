// Device-side grouping and packing of (read, haplotype) pairs.
//
// Pairs of the same read that are adjacent in the pair list form a run (cut
// every kChunk pairs).  For each run one thread chooses the column class N
// (columns per lane) that minimises the modelled cost waves x cost[N], packs
// the run's pairs greedily into 64-lane wavefronts (ceil(k/N) lanes per
// pair, at most 32 pairs per wavefront) and emits the packs into the segment
// of its (precision, class).  Every pack holds one read, so the per-row
// priors and the read base are uniform across the wavefront.  Haplotypes
// longer than 64 * kMaxN columns go to the long-pair list.
//
// Three kernels, no contended global atomics: count (per-block per-segment
// pack counts from LDS atomics), scan (segment bases and per-block offsets),
// emit (each run writes its packs at its block's offset).
//
// The paper bins pairs by length and runs a dedicated kernel instance per
// sub-warp size (Section 3.2); here the binning key is the column class and
// the packing is done on the device so that a batch never returns to the
// host between packing and compute.
#include "phmm_dev.h"

namespace phmm {

constexpr int kSeg = 2 * kNumClasses;  // (precision, class) segments

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

// Walks the short pairs of run [p0, p1) at class c exactly as the emitter
// does and returns the number of packs (0 and fits = false if a pair does
// not fit the class).  A long pair closes the current pack.
__device__ uint32_t count_packs(const Batch& b, uint64_t p0, uint64_t p1, int c, int one_per_wave,
                                bool* fits)
{
    const uint32_t N = (uint32_t)class_n(c);
    uint32_t packs = 0, used = kWave, np = 0;
    *fits = true;
    for (uint64_t p = p0; p < p1; ++p) {
        const uint32_t k = hap_len(b, b.pairs[2 * p + 1]);
        if (k > kShortMaxCols) {
            used = kWave;
            np = 0;
            continue;
        }
        const uint32_t s = (k + N - 1) / N;
        if (s > (uint32_t)kWave) { *fits = false; return 0; }
        if (one_per_wave || used + s > (uint32_t)kWave || np == (uint32_t)kMaxPairsPerPack) {
            ++packs;
            used = 0;
            np = 0;
        }
        used += s;
        ++np;
    }
    return packs;
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

// Pass 1: class choice and pack counts per run; long pairs to the long list.
__global__ __launch_bounds__(kPackBlock) void pack_count_kernel(Batch b, Work w, Policy pol)
{
    __shared__ uint32_t cnt[kSeg];
    __shared__ unsigned long long lanecols;
    const int t = (int)threadIdx.x;
    if (t < kSeg) cnt[t] = 0u;
    if (t == 0) lanecols = 0ull;
    __syncthreads();
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + t;
    if (p < b.n_pairs && run_start(b, p)) {
        const uint64_t e = run_end(b, p);
        const uint32_t r = b.pairs[2 * p];
        const uint32_t l = (uint32_t)(b.read_off[r + 1] - b.read_off[r]);
        const int prec = (pol.precision == 1 || l > pol.fp32_max_rows) ? 1 : 0;
        uint32_t nshort = 0;
        for (uint64_t q = p; q < e; ++q) {
            if (hap_len(b, b.pairs[2 * q + 1]) > kShortMaxCols) {
                const uint32_t idx = atomicAdd(&w.ctr->n_long, 1u);
                w.long_list[idx] = (uint32_t)q;
            } else {
                ++nshort;
            }
        }
        uint32_t info = 0xffffffffu;
        if (nshort > 0) {
            int best = -1;
            float best_cost = 0.f;
            uint32_t best_packs = 0;
            for (int c = 0; c < kNumClasses; ++c) {
                if (pol.force_class >= 0 && c != pol.force_class) continue;
                bool fits;
                const uint32_t np = count_packs(b, p, e, c, pol.one_pair_per_wave, &fits);
                if (!fits) continue;
                const float cost = (float)np * pol.cost[prec][c];
                if (best < 0 || cost < best_cost) {
                    best = c;
                    best_cost = cost;
                    best_packs = np;
                }
            }
            if (best < 0) {  // forced class too narrow for this run: use the widest
                bool fits;
                best = kNumClasses - 1;
                best_packs = count_packs(b, p, e, best, pol.one_pair_per_wave, &fits);
            }
            info = (uint32_t)best | ((uint32_t)prec << 4) | (best_packs << 8);
            atomicAdd(&cnt[prec * kNumClasses + best], best_packs);
            atomicAdd(&lanecols, (unsigned long long)best_packs * kWave * class_n(best));
        }
        w.chunk_info[p] = info;
    }
    __syncthreads();
    if (t < kSeg) w.blk_cnt[(size_t)blockIdx.x * kSeg + t] = cnt[t];
    if (t == 0) w.blk_lanecols[blockIdx.x] = lanecols;
}

// Pass 2 (one workgroup): per-segment exclusive scan over the blocks, the
// segment bases of the pack array and the capacity of the rerun item lists.
__global__ __launch_bounds__(1024) void pack_scan_kernel(Work w, uint32_t nblocks)
{
    __shared__ uint32_t part[1024];
    __shared__ uint32_t seg_total[kSeg];
    __shared__ unsigned long long lc[1024];
    const int t = (int)threadIdx.x;
    const uint32_t per = (nblocks + 1023u) / 1024u;
    const uint32_t lo = (uint32_t)t * per, hi = lo + per < nblocks ? lo + per : nblocks;
    for (int s = 0; s < kSeg; ++s) {
        uint32_t sum = 0;
        for (uint32_t q = lo; q < hi; ++q) sum += w.blk_cnt[(size_t)q * kSeg + s];
        part[t] = sum;
        __syncthreads();
        if (t == 0) {
            uint32_t acc = 0;
            for (int q = 0; q < 1024; ++q) {
                const uint32_t v = part[q];
                part[q] = acc;
                acc += v;
            }
            seg_total[s] = acc;
        }
        __syncthreads();
        uint32_t acc = part[t];
        for (uint32_t q = lo; q < hi; ++q) {
            const uint32_t v = w.blk_cnt[(size_t)q * kSeg + s];
            w.blk_cnt[(size_t)q * kSeg + s] = acc;  // becomes the block's offset in the segment
            acc += v;
        }
        __syncthreads();
    }
    unsigned long long sum = 0;
    for (uint32_t q = lo; q < hi; ++q) sum += w.blk_lanecols[q];
    lc[t] = sum;
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
            c->item_base[k] = acc2;  // reruns of class k: at most one item per FP32 pack
            acc2 += c->pack_cnt[0][k];
            c->item_cnt[k] = 0;
            c->cursor32[k] = 0;
            c->cursor64[k] = 0;
        }
        unsigned long long tot = 0;
        for (int q = 0; q < 1024; ++q) tot += lc[q];
        c->lane_columns = tot;
    }
}

// Pass 3: write the packs at the block's offset in each segment.
__global__ __launch_bounds__(kPackBlock) void pack_emit_kernel(Batch b, Work w, Policy pol)
{
    __shared__ uint32_t fill[kSeg];
    const int t = (int)threadIdx.x;
    if (t < kSeg) fill[t] = 0u;
    __syncthreads();
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + t;
    if (p >= b.n_pairs || !run_start(b, p)) return;
    const uint32_t info = w.chunk_info[p];
    if (info == 0xffffffffu) return;
    const int c = (int)(info & 15u), prec = (int)((info >> 4) & 1u);
    const uint32_t npk = info >> 8;
    const int s = prec * kNumClasses + c;
    const uint32_t slot = w.ctr->pack_base[prec][c] + w.blk_cnt[(size_t)blockIdx.x * kSeg + s] +
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

}  // namespace phmm
