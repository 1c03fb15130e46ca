// Short-pair PairHMM forward kernel for gfx950: one wavefront per pack (one
// read against up to 32 haplotypes laid side by side over the 64 lanes).
//
// Row-level formulation (paper Section 3.1, eq.5-7).  For read row i the
// whole row of M and I is computed from row i-1 only; the Delete row is not
// stored.  With S(i,j) = sum_{b<=j} T_DD^(j-b) M(i,b) (the unrolled delete
// chain of eq.6, so that D(i,j) = T_MD_i S(i,j-1)):
//
//   M(i,j) = P(r_i|h_j) (T_MM_i M(i-1,j-1) + T_IM_i I(i-1,j-1)
//                        + T_DM_i T_MD_{i-1} S(i-1,j-2))
//   I(i,j) = T_MI_i M(i-1,j) + T_II_i I(i-1,j)
//
// Lane L of a pair's segment owns the N consecutive columns c0+1..c0+N
// (c0 = N * (L - segment start)).  Within a lane S(i-1, .) is rebuilt on the
// fly by a one-FMA-per-column chain started from the lane's carry
// C = S(i-1, c0-1); the carries of all lanes come from one segmented
// first-order linear scan per row over the lanes' weighted window sums
// (paper Section 3.4, Algorithm 1), done with DPP row shifts and row
// broadcasts.  The window of a lane is shifted one column left (it covers
// columns c0..c0+N-1, the first being the left neighbour's last column), so
// the scan yields exactly the exclusive prefix S(i, c0-1) each lane needs and
// no division by T_DD (the paper's T_DD^-1 (T - V) step) is required.
//
// Emission (eq.3): every pack holds one read, so r_i is wavefront-uniform.
// Haplotype columns are held as 8-bit match codes (four per register); the
// row's read-base index selects one bit per column, which picks pm = 1 - eps
// or px = eps / 3 bit-wise, with 'N' on either side matching any base.
//
// Scale: D(0,j) = C0/k with C0 = 2^120 (FP32) or 2^1020 (FP64), eq.1.  The
// FP32 instantiation tests each result against the acceptance threshold and
// queues rejected pairs for the FP64 instantiation (precision policy).
#include <type_traits>

#include "phmm_dev.h"

namespace phmm {

template <typename R>
struct ScaleOf;
template <>
struct ScaleOf<float> {
    static constexpr int exp = 120;
};
template <>
struct ScaleOf<double> {
    static constexpr int exp = 1020;
};

// The FP32 kernels keep the fixed scale 2^120/k on every row, which is what
// makes the acceptance test sound.  Along any path the weight only falls
// (every transition and emission factor is at most 1), and the weight of
// all continuations of a cell is at most 1, so a cell flushed below FP32's
// smallest number (2^-149) takes at most 2^-149 from the scaled sum: with the
// sum at least 1e-28 (2^-93) the l*k cells of a pair lose at most l*k*2^-56
// of it.  Rescaling the rows (bringing a decayed maximum back up) would void
// that bound: a path far under a row's maximum, flushed there, can carry the
// sum later (a read with a 50-base deletion against its haplotype lost 2.2
// decades in FP32 when 64-row windows were rescaled), so reads whose sum
// falls under the threshold are rerun in FP64 instead.

template <typename R>
__device__ __forceinline__ const R* pow_table(const Tables& t, int cls, int gcp);
template <>
__device__ __forceinline__ const float* pow_table<float>(const Tables& t, int cls, int gcp)
{
    return t.pw32 + ((size_t)cls * 256 + gcp) * kPowStride;
}
template <>
__device__ __forceinline__ const double* pow_table<double>(const Tables& t, int cls, int gcp)
{
    return t.pw64 + ((size_t)cls * 256 + gcp) * kPowStride;
}

constexpr int words_for(int n) { return (n + 3) / 4; }

// Waves per SIMD the fast FP32 kernel of a class is compiled for (its
// register budget is 512 / waves VGPRs).  Measured on the genome-scale batch
// with every pair forced into one class: the most waves whose row loop keeps
// all its values in registers wins; spills outside the row loop (a few
// values per pack, class 7 at 5 waves) cost less than the occupancy gains,
// spills inside it cost 5-60%.  Other kernels: no target.
template <typename R, int CLS, int KIND>
constexpr int waves_target()
{
    // N = 4 .. 24
    constexpr int fast_waves[kNumClasses] = {8, 7, 7, 7, 7, 6, 6, 6, 6, 6, 6,
                                             5, 5, 5, 5, 4, 4, 4, 4, 4, 4};
    // FP64: timed per class on the genome-scale batch in plain FP64 at 1
    // (the compiler's choice), 2, 3 and 4 waves; N = 4-8 gain nothing from a
    // target, N = 9-15 run best at 3, N = 16-24 at 2 rather than the one wave
    // per SIMD that 256 VGPRs plus accumulation registers give (the whole
    // plain FP64 pass on that batch: 7.32 s before, 6.55-6.69 s after)
    constexpr int fp64_waves[kNumClasses] = {1, 1, 1, 1, 1, 3, 3, 3, 3, 3, 3,
                                             3, 2, 2, 2, 2, 2, 2, 2, 2, 2};
    return KIND == kFast32 ? fast_waves[CLS] : KIND == kAll64 ? fp64_waves[CLS] : 1;
}

// KIND kFast32 (R = float): walks the FP32 packs of class CLS; a pack whose
// read has more than one gap byte, a gap byte of 0 or an insertion byte
// above the scaled form's limit is deferred to the general FP32 kernel.
// KIND kGen32 (R = float): walks the deferred packs of the class.  Both FP32
// kernels queue pairs under the acceptance threshold as FP64 items.
// KIND kAll64 (R = double): walks the plain FP64 packs of the class, then
// the rerun items.
template <typename R, int CLS, int KIND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(waves_target<R, CLS, KIND>())))
void short_kernel(Batch b, Tables t, Work w, Policy pol)
{
    constexpr int N = class_n(CLS);
    constexpr bool kFP32 = sizeof(R) == 4;
    constexpr bool kFast = KIND == kFast32;
    __shared__ RowRec<R> rec[kWave];
    __shared__ int rinfo[kWave];  // read-base class mask | gcp byte << 16
    __shared__ int sflag[kWave];
    __shared__ uint32_t srej;
    // per pair (lane q < pairs of the pack): first lane | lanes << 8, pair
    // index, bit in the pack mask; per lane: real columns; per lane: its sum
    __shared__ uint32_t pinfo[3][kWave];
    __shared__ int nrl[kWave];
    __shared__ R psum[kWave];

    const int lane = (int)threadIdx.x;
    Counters* ctr = w.ctr;
    uint32_t* cursor = &ctr->cursor[KIND][CLS];
    // FP64: the class's plain FP64 packs first, then the rerun items
    const uint32_t n_plain = ctr->pack_cnt[1][CLS];
    const uint32_t count = KIND == kFast32 ? ctr->pack_cnt[0][CLS]
                         : KIND == kGen32  ? ctr->defer_cnt[CLS]
                                           : n_plain + ctr->item_cnt[CLS];

    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(cursor, 1u);
        it = wave_broadcast0(it);
        if (it >= count) break;
        const int lane = lane_here();  // (one wavefront per workgroup)

        uint32_t pack_gi, mask;
        if (KIND == kFast32 || KIND == kGen32) {
            pack_gi = KIND == kFast32 ? ctr->pack_base[0][CLS] + it
                                      : w.deferred[ctr->item_base[CLS] + it];
            const uint32_t np = w.packs[pack_gi].npairs;
            mask = np == 32 ? 0xffffffffu : ((1u << np) - 1u);
        } else if (it < n_plain) {
            pack_gi = ctr->pack_base[1][CLS] + it;
            const uint32_t np = w.packs[pack_gi].npairs;
            mask = np == 32 ? 0xffffffffu : ((1u << np) - 1u);
        } else {
            const Item itm = w.items[ctr->item_base[CLS] + (it - n_plain)];
            pack_gi = itm.pack;
            mask = itm.mask;
        }
        const uint32_t pair0 = w.packs[pack_gi].pair_start;
        pack_gi = wave_broadcast0(pack_gi);
        mask = wave_broadcast0(mask);
        const bool rerun_item = !kFP32 && it >= n_plain;
        // rerun pairs are counted where they are recomputed (a rare path), so
        // the FP32 kernels touch only the per-class item counter per rejection
        if (rerun_item && lane == 0) atomicAdd(&ctr->rerun_pairs, (uint32_t)__builtin_popcount(mask));

        // ---- read and its gap-continuation profile.  Scaled form possible:
        // T_IM > 0 (gap byte >= 1) and bounded insertion bytes on every row.
        const uint32_t r = b.pairs[2 * (uint64_t)pair0];
        const uint64_t roff = b.read_off[r];
        const int l = (int)(b.read_off[r + 1] - roff);
        const int g0 = b.gq[roff];
        bool varying = false, sc_ok = true;
        for (int i0 = 0; i0 < l; i0 += kWave) {
            const int i = i0 + lane;
            const int gc = i < l ? (int)b.gq[roff + i] : g0;
            const int ic = i < l ? (int)b.iq[roff + i] : 0;
            varying = varying || __ballot(gc != g0) != 0ull;
            sc_ok = sc_ok && __ballot(gc == 0 || ic > kScMaxInsQ) == 0ull;
        }
        if (kFast && (varying || !sc_ok)) {
            if (lane == 0) {
                const uint32_t idx = atomicAdd(&ctr->defer_cnt[CLS], 1u);
                w.deferred[ctr->item_base[CLS] + idx] = pack_gi;
            }
            continue;
        }
        if (kFast) {  // known from here on: one gap byte, scaled form
            varying = false;
            sc_ok = true;
        }

        // ---- segment layout: lanes [start_s, start_s + ceil(k_s/N)) per pair s
        const int nseg = __builtin_popcount(mask);
        uint32_t my_pair = 0, my_k = 0, my_off = 0;
        uint64_t my_h = 0;
        int s_lanes = 0;
        if (lane < nseg) {
            uint32_t m = mask;
            for (int q = 0; q < lane; ++q) m &= m - 1u;
            my_off = (uint32_t)__builtin_ctz(m);
            my_pair = pair0 + my_off;
            const uint32_t h = b.pairs[2 * (uint64_t)my_pair + 1];
            my_h = b.hap_off[h];
            my_k = (uint32_t)(b.hap_off[h + 1] - my_h);
            s_lanes = (int)((my_k + N - 1) / N);
        }
        const int incl = wave_incl_sum(s_lanes);
        const int my_start = incl - s_lanes;
        const int total = __builtin_amdgcn_readlane(incl, 63);
        sflag[lane] = 0;
        __syncthreads();
        if (lane < nseg && my_start < kWave) sflag[my_start] = 1;
        if (lane == 0 && total < kWave) sflag[total] = 1;
        __syncthreads();
        const uint64_t starts = __ballot(sflag[lane] != 0);
        const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const int segstart = 63 - __builtin_clzll(starts & upto);
        const int seg = __builtin_popcountll(starts & upto) - 1;
        const bool real = seg < nseg;
        const int src = real ? seg : 0;
        const uint32_t k = real ? (uint32_t)__shfl((int)my_k, src) : 1u;
        const uint32_t hlo = (uint32_t)__shfl((int)(uint32_t)my_h, src);
        const uint32_t hhi = (uint32_t)__shfl((int)(uint32_t)(my_h >> 32), src);
        const uint64_t hoff = ((uint64_t)hhi << 32) | hlo;
        const int c0 = N * (lane - segstart);
        // what the result step needs after the rows goes to LDS now, so that
        // none of it stays live in registers across the row loop
        if (lane < nseg) {
            pinfo[0][lane] = (uint32_t)my_start | ((uint32_t)s_lanes << 8);
            pinfo[1][lane] = my_pair;
            pinfo[2][lane] = my_off;
        }
        nrl[lane] = real ? max(0, min((int)k - c0, N)) : 0;

        // ---- haplotype columns as 8-bit match codes, four per register
        uint32_t hc[words_for(N)];
#pragma unroll
        for (int q = 0; q < words_for(N); ++q) hc[q] = 0u;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const uint32_t j = (uint32_t)(c0 + n);
            const uint32_t code = (real && j < k) ? hap_code(b.haps[hoff + j]) : kPadCode;
            hc[n / 4] |= code << (8 * (n % 4));
        }

        const R notstart = (lane != segstart) ? (R)1 : (R)0;
        const R minit = real ? (R)(ldexp(1.0, ScaleOf<R>::exp) / (double)k) : (R)0;
        const R* pw = pow_table<R>(t, CLS, g0);
        ScanMul<R> mul = make_scan_mul<R>(pw, lane, segstart);
        R gcur = (R)t.p64[g0], gprev = gcur, gN1 = pw[65];

        R Ma[N], Ia[N], Mb[N], Ib[N];
#pragma unroll
        for (int n = 0; n < N; ++n) { Ma[n] = (R)0; Ia[n] = (R)0; }
        R Mleft = (R)0, Ileft = (R)0, C = (R)0;

        // all rows of the pack; SC selects the scaled form of the rows
        auto run_rows = [&](auto sc_tag) {
            constexpr bool SC = decltype(sc_tag)::value;
            // one row of the recurrence plus the carries for the next row;
            // rows alternate between the (Ma, Ia) and (Mb, Ib) register sets
            auto do_row = [&](int tt, bool first, const R(&Mi)[N], const R(&Ii)[N], R(&Mo)[N],
                              R(&Io)[N]) {
                const RowRec<R> c = rec[tt];
                const int info = __builtin_amdgcn_readfirstlane(rinfo[tt]);
                if (varying) {
                    const int gc = info >> 16;
                    gprev = gcur;
                    gcur = (R)t.p64[gc];
                    const R* pwi = pow_table<R>(t, CLS, gc);
                    mul = make_scan_mul<R>(pwi, lane, segstart);
                    gN1 = pwi[65];
                }
                const int bidx = info & 0xff;
                R Vp;
                if (first)
                    row_first<R, N>(Mo, Io, hc, bidx, c, minit, gcur, Vp);
                else
                    row_step<R, N, SC>(Mi, Ii, Mo, Io, hc, bidx, c, Mleft, Ileft, C, gprev,
                                        gcur, Vp);
                // carries for the next row: left neighbour's last column, and
                // the exclusive scan of the shifted window sums
                Mleft = notstart * dpp<kWaveShr1>(Mo[N - 1]);
                Ileft = notstart * dpp<kWaveShr1>(Io[N - 1]);
                const R vsh = fmaR(gN1, Mleft, Vp);
                C = seg_scan(notstart * dpp<kWaveShr1>(vsh), mul);
            };
            for (int i0 = 0; i0 < l; i0 += kWave) {
                __syncthreads();
                {   // priors of rows i0 .. i0+63 (eq.3 and the transition priors)
                    const int i = i0 + lane;
                    if (i < l) {
                        const uint64_t a = roff + (uint64_t)i;
                        rec[lane] = make_row_rec<R, SC>(b, t.p64, a, i, l);
                        rinfo[lane] = read_base_index(b.reads[a]) | ((int)b.gq[a] << 16);
                    }
                }
                __syncthreads();
                const int nrows = l - i0 < kWave ? l - i0 : kWave;
                int tt = 0;
                for (; tt + 1 < nrows; tt += 2) {
                    do_row(tt, i0 + tt == 0, Ma, Ia, Mb, Ib);
                    do_row(tt + 1, false, Mb, Ib, Ma, Ia);
                }
                if (tt < nrows) {
                    do_row(tt, i0 + tt == 0, Ma, Ia, Mb, Ib);
#pragma unroll
                    for (int n = 0; n < N; ++n) { Ma[n] = Mb[n]; Ia[n] = Ib[n]; }
                }
            }
        };
        if constexpr (kFast) {
            run_rows(std::true_type{});
        } else {
            if (sc_ok)
                run_rows(std::true_type{});
            else
                run_rows(std::false_type{});
        }

        // ---- eq.4: S = sum_j M(l,j) + I(l,j) over the real columns: each
        // lane's partial sum, then one lane per pair adds its segment's lanes
        // in lane order
        {
            const int nreal = nrl[lane];
            R sl = (R)0;
#pragma unroll
            for (int n = 0; n < N; ++n)
                if (n < nreal) sl += Ma[n] + Ia[n];
            psum[lane] = sl;
        }
        __syncthreads();
        bool reject = false;
        uint32_t off = 0;
        if (lane < nseg) {
            const uint32_t pi = pinfo[0][lane];
            const int first = (int)(pi & 0xffu), cnt = (int)(pi >> 8);
            R s = (R)0;
            for (int q = 0; q < cnt; ++q) s += psum[first + q];
            const uint32_t pair = pinfo[1][lane];
            off = pinfo[2][lane];
            const double S = (double)s;
            if (kFP32) {
                // a sum of 0 is rejected whatever the threshold: L > 0 may
                // have underflowed in FP32
                reject = !(S > 0.0) || !(S >= (double)pol.accept_min_sum) || !(S < 3.0e38);
                if (!reject) {
                    b.out[pair] = log10_scaled_f32((float)s, ScaleOf<R>::exp);
                    if (b.flags) b.flags[pair] = 0x01;  // FP32 accepted
                }
            } else {
                // FP64 scaled sums this small would have lost bits to
                // underflow: hand the pair to the rescaling long-pair kernel.
                if (!(S >= 1e-290)) {
                    constexpr int q = long_list_of(1, true);
                    const uint32_t idx = atomicAdd(&ctr->n_long[q], 1u);
                    w.long_list[q][idx] = pair;
                } else {
                    b.out[pair] = log10_scaled(S, ScaleOf<R>::exp);
                    if (b.flags) b.flags[pair] = rerun_item ? (0x02 | 0x10) : 0x10;
                }
            }
        }
        if (kFP32) {
            if (lane == 0) srej = 0u;
            __syncthreads();
            if (reject) atomicOr(&srej, 1u << off);
            __syncthreads();
            const uint32_t rm = srej;
            if (lane == 0 && rm != 0u) {
                const uint32_t idx = atomicAdd(&ctr->item_cnt[CLS], 1u);
                w.items[ctr->item_base[CLS] + idx].pack = pack_gi;
                w.items[ctr->item_base[CLS] + idx].mask = rm;
            }
        }
    }
}

// ---------------------------------------------------------------- launchers
template <int KIND, int CLS>
static void launch_one(int cls, dim3 grid, hipStream_t s, const Batch& b, const Tables& t,
                       const Work& w, const Policy& p)
{
    using R = typename std::conditional<KIND == kAll64, double, float>::type;
    if (cls == CLS) hipLaunchKernelGGL((short_kernel<R, CLS, KIND>), grid, dim3(kWave), 0, s, b, t, w, p);
}

template <int KIND, int... CLS>
static void launch_dispatch(int cls, dim3 grid, hipStream_t s, const Batch& b, const Tables& t,
                            const Work& w, const Policy& p, std::integer_sequence<int, CLS...>)
{
    (launch_one<KIND, CLS>(cls, grid, s, b, t, w, p), ...);
}

void launch_short(int kind, int cls, int grid, hipStream_t s, const Batch& b, const Tables& t,
                  const Work& w, const Policy& p)
{
    const auto seq = std::make_integer_sequence<int, kNumClasses>{};
    if (kind == kFast32) launch_dispatch<kFast32>(cls, dim3(grid), s, b, t, w, p, seq);
    else if (kind == kGen32) launch_dispatch<kGen32>(cls, dim3(grid), s, b, t, w, p, seq);
    else launch_dispatch<kAll64>(cls, dim3(grid), s, b, t, w, p, seq);
}

template <int KIND, int CLS>
static const void* kernel_ptr_one(int cls)
{
    using R = typename std::conditional<KIND == kAll64, double, float>::type;
    return cls == CLS ? reinterpret_cast<const void*>(&short_kernel<R, CLS, KIND>) : nullptr;
}
template <int KIND, int... CLS>
static const void* kernel_ptr(int cls, std::integer_sequence<int, CLS...>)
{
    const void* r = nullptr;
    ((r = r ? r : kernel_ptr_one<KIND, CLS>(cls)), ...);
    return r;
}

const void* short_kernel_ptr(int kind, int cls)
{
    const auto seq = std::make_integer_sequence<int, kNumClasses>{};
    return kind == kFast32 ? kernel_ptr<kFast32>(cls, seq)
         : kind == kGen32  ? kernel_ptr<kGen32>(cls, seq)
                           : kernel_ptr<kAll64>(cls, seq);
}

}  // namespace phmm
