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
// longer than 64 * kMaxN columns go to the long-pair list.
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

// A run whose haplotypes are mutually unrelated: none of the next (up to)
// three short haplotypes after the run's first shares at least half of the
// first one's 4-mers (Jaccard index of the sets below 1/2).  Haplotypes that
// are variants of one locus share almost all of them; unrelated 32-base
// prefixes share about a twentieth.
__device__ bool run_is_diverse(const Batch& b, uint64_t p, uint64_t e)
{
    uint64_t ref[4];
    bool have_ref = false;
    int compared = 0;
    for (uint64_t q = p; q < e && compared < 3; ++q) {
        const uint32_t h = b.pairs[2 * q + 1];
        if (hap_len(b, h) > kShortMaxCols || hap_len(b, h) < 8) continue;
        if (!have_ref) {
            kmer_set(b, h, ref);
            have_ref = true;
            continue;
        }
        uint64_t m[4];
        kmer_set(b, h, m);
        int both = 0, any = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            both += __popcll(ref[w] & m[w]);
            any += __popcll(ref[w] | m[w]);
        }
        if (2 * both >= any) return false;
        ++compared;
    }
    return compared > 0;
}

// Pass 1: precision and class per run, pack counts per (segment, block);
// long pairs to the long list.
__global__ __launch_bounds__(kPackBlock) void pack_count_kernel(Batch b, Work w, Policy pol)
{
    __shared__ uint32_t cnt[kSeg];
    __shared__ unsigned long long lanecols;
    const int t = (int)threadIdx.x;
    for (int q = t; q < kSeg; q += kPackBlock) cnt[q] = 0u;
    if (t == 0) lanecols = 0ull;
    __syncthreads();
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + t;
    if (p < b.n_pairs && run_start(b, p)) {
        const uint64_t e = run_end(b, p);
        const uint32_t r = b.pairs[2 * p];
        const uint32_t l = (uint32_t)(b.read_off[r + 1] - b.read_off[r]);
        int prec = (pol.precision == 1 || l > pol.fp32_max_rows) ? 1 : 0;
        if (prec == 0 && pol.route_diverse && e - p >= 2 && run_is_diverse(b, p, e)) prec = 1;
        const int lprec = (pol.precision == 1 || l > pol.long_fp32_max_rows) ? 1 : 0;
        Greedy g[kNumClasses];
        bool fits[kNumClasses];
#pragma unroll
        for (int c = 0; c < kNumClasses; ++c) {
            g[c].reset();
            fits[c] = true;
        }
        uint32_t nshort = 0;
        for (uint64_t q = p; q < e; ++q) {
            const uint32_t k = hap_len(b, b.pairs[2 * q + 1]);
            if (k > kShortMaxCols) {
                const uint32_t idx = atomicAdd(&w.ctr->n_long[lprec], 1u);
                w.long_list[lprec][idx] = (uint32_t)q;
#pragma unroll
                for (int c = 0; c < kNumClasses; ++c) {
                    g[c].used = kWave;
                    g[c].np = 0;
                }
                continue;
            }
            ++nshort;
#pragma unroll
            for (int c = 0; c < kNumClasses; ++c) {
                const uint32_t s = (k + class_n(c) - 1) / class_n(c);
                if (s > (uint32_t)kWave) fits[c] = false;
                else g[c].add(s, pol.one_pair_per_wave);
            }
        }
        uint32_t info = 0xffffffffu;
        if (nshort > 0) {
            int best = -1;
            float best_cost = 0.f;
#pragma unroll
            for (int c = 0; c < kNumClasses; ++c) {
                if ((pol.force_class >= 0 && c != pol.force_class) || !fits[c]) continue;
                const float cost = (float)g[c].packs * pol.cost[prec][c];
                if (best < 0 || cost < best_cost) {
                    best = c;
                    best_cost = cost;
                }
            }
            if (best < 0) best = kNumClasses - 1;  // forced class too narrow: the widest
            uint32_t packs = 0;
#pragma unroll
            for (int c = 0; c < kNumClasses; ++c)
                if (c == best) packs = g[c].packs;
            info = (uint32_t)best | ((uint32_t)prec << 5) | (packs << 8);
            atomicAdd(&cnt[prec * kNumClasses + best], packs);
            atomicAdd(&lanecols, (unsigned long long)packs * kWave * class_n(best));
        }
        w.chunk_info[p] = info;
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
// pack array and the capacity of the rerun item lists.
__global__ __launch_bounds__(1024) void pack_scan_kernel(Work w)
{
    __shared__ uint32_t part[1024];
    __shared__ uint32_t seg_total[kSeg];
    const int t = (int)threadIdx.x;
    const uint32_t n = w.n_scan_chunks;
    const uint32_t per = (n + 1023u) / 1024u;
    const uint32_t lo = (uint32_t)t * per, hi = lo + per < n ? lo + per : n;
    for (int s = 0; s < kSeg; ++s) {
        uint32_t* cp = w.chunk_part + (size_t)s * n;
        uint32_t sum = 0;
        for (uint32_t q = lo; q < hi; ++q) sum += cp[q];
        part[t] = sum;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const uint32_t y = t >= d ? part[t - d] : 0u;
            __syncthreads();
            part[t] += y;
            __syncthreads();
        }
        uint32_t acc = part[t] - sum;
        for (uint32_t q = lo; q < hi; ++q) {
            const uint32_t v = cp[q];
            cp[q] = acc;  // becomes the chunk's offset in the segment
            acc += v;
        }
        if (t == 1023) seg_total[s] = part[1023];
        __syncthreads();
    }
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
    hipLaunchKernelGGL(pack_chunk_sum_kernel, dim3(w.n_scan_chunks, kSeg), dim3(256), 0, s, w);
    hipLaunchKernelGGL(pack_scan_kernel, dim3(1), dim3(1024), 0, s, w);
    hipLaunchKernelGGL(pack_block_offset_kernel, dim3(w.n_scan_chunks, kSeg), dim3(256), 0, s, w);
    hipLaunchKernelGGL(pack_emit_kernel, dim3(w.n_pack_blocks), dim3(kPackBlock), 0, s, b, w, pol);
}

uint32_t scan_chunks(uint32_t n_pack_blocks) { return (n_pack_blocks + kScanChunk - 1) / kScanChunk; }

}  // namespace phmm
