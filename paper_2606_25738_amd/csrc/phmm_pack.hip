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
// The paper bins pairs by length and runs a dedicated kernel instance per
// sub-warp size (Section 3.2); here the binning key is the column class and
// the packing is done on the device so that a batch never returns to the
// host between packing and compute.
#include "phmm_dev.h"

namespace phmm {

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

// Greedy packing of the short pairs of run [p0, p1) at class c.
// Returns the number of packs (0 if a pair does not fit the class).
__device__ uint32_t count_packs(const Batch& b, uint32_t p0, uint32_t p1, int c, int one_per_wave,
                                bool* fits)
{
    const uint32_t N = (uint32_t)class_n(c);
    uint32_t packs = 0, used = kWave, np = 0;
    *fits = true;
    for (uint32_t p = p0; p < p1; ++p) {
        uint32_t k = hap_len(b, b.pairs[2 * p + 1]);
        if (k > kShortMaxCols) {  // long pair: closes the current pack
            used = kWave;
            np = 0;
            continue;
        }
        uint32_t s = (k + N - 1) / N;
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
__global__ void pack_plan_kernel(Batch b, Work w, Policy pol)
{
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= b.n_pairs || !run_start(b, p)) return;
    const uint64_t e = run_end(b, p);
    const uint32_t r = b.pairs[2 * p];
    const uint32_t l = (uint32_t)(b.read_off[r + 1] - b.read_off[r]);
    const int prec = (pol.precision == 1 || l > pol.fp32_max_rows) ? 1 : 0;
    uint32_t nshort = 0;
    for (uint64_t q = p; q < e; ++q) {
        if (hap_len(b, b.pairs[2 * q + 1]) > kShortMaxCols) {
            uint32_t idx = atomicAdd(&w.ctr->n_long, 1u);
            w.long_list[idx] = (uint32_t)q;
        } else {
            ++nshort;
        }
    }
    if (nshort == 0) {
        w.chunk_info[p] = 0xffffffffu;
        return;
    }
    int best = -1;
    float best_cost = 0.f;
    uint32_t best_packs = 0;
    for (int c = 0; c < kNumClasses; ++c) {
        if (pol.force_class >= 0 && c != pol.force_class) continue;
        bool fits;
        uint32_t np = count_packs(b, (uint32_t)p, (uint32_t)e, c, pol.one_pair_per_wave, &fits);
        if (!fits) continue;
        float cost = (float)np * pol.cost[prec][c];
        if (best < 0 || cost < best_cost) {
            best = c;
            best_cost = cost;
            best_packs = np;
        }
    }
    if (best < 0) {  // forced class too narrow for this run: use the widest
        bool fits;
        best = kNumClasses - 1;
        best_packs = count_packs(b, (uint32_t)p, (uint32_t)e, best, pol.one_pair_per_wave, &fits);
    }
    w.chunk_info[p] = (uint32_t)best | ((uint32_t)prec << 4) | (best_packs << 8);
    atomicAdd(&w.ctr->pack_cnt[prec][best], best_packs);
    atomicAdd(&w.ctr->lane_columns, (unsigned long long)best_packs * kWave * class_n(best));
}

// Segment bases of the pack array and of the FP64 item lists.
__global__ void pack_layout_kernel(Counters* c)
{
    if (threadIdx.x != 0) return;
    uint32_t acc = 0;
    for (int prec = 0; prec < 2; ++prec)
        for (int k = 0; k < kNumClasses; ++k) {
            c->pack_base[prec][k] = acc;
            acc += c->pack_cnt[prec][k];
            c->pack_fill[prec][k] = 0;
        }
    uint32_t acc2 = 0;
    for (int k = 0; k < kNumClasses; ++k) {
        c->item_base[k] = acc2;
        acc2 += c->pack_cnt[0][k] + c->pack_cnt[1][k];
        c->item_cnt[k] = 0;
        c->cursor32[k] = 0;
        c->cursor64[k] = 0;
    }
}

// Pass 2: write the packs (and, for FP64 packs, their full-mask items).
__global__ void pack_emit_kernel(Batch b, Work w, Policy pol)
{
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= b.n_pairs || !run_start(b, p)) return;
    const uint32_t info = w.chunk_info[p];
    if (info == 0xffffffffu) return;
    const int c = (int)(info & 15u), prec = (int)((info >> 4) & 1u);
    const uint32_t npk = info >> 8;
    const uint64_t e = run_end(b, p);
    const uint32_t N = (uint32_t)class_n(c);
    const uint32_t slot = w.ctr->pack_base[prec][c] + atomicAdd(&w.ctr->pack_fill[prec][c], npk);
    uint32_t written = 0, used = kWave, np = 0, start = 0;
    auto flush = [&]() {
        if (np == 0) return;
        const uint32_t gi = slot + written;
        w.packs[gi].pair_start = start;
        w.packs[gi].npairs = np;
        if (prec == 1) {
            uint32_t it = atomicAdd(&w.ctr->item_cnt[c], 1u);
            w.items[w.ctr->item_base[c] + it].pack = gi;
            w.items[w.ctr->item_base[c] + it].mask = np == 32 ? 0xffffffffu : ((1u << np) - 1u);
        }
        ++written;
    };
    // Packs are built over consecutive short pairs only; a long pair in the
    // middle of a run closes the current pack (its lanes would not be
    // contiguous in pair order otherwise).
    for (uint64_t q = p; q < e; ++q) {
        uint32_t k = hap_len(b, b.pairs[2 * q + 1]);
        if (k > kShortMaxCols) {
            flush();
            used = kWave;
            np = 0;
            continue;
        }
        uint32_t s = (k + N - 1) / N;
        if (pol.one_pair_per_wave || used + s > (uint32_t)kWave || np == (uint32_t)kMaxPairsPerPack) {
            flush();
            used = 0;
            np = 0;
            start = (uint32_t)q;
        }
        used += s;
        ++np;
    }
    flush();
    (void)npk;
}

}  // namespace phmm
