// Long-pair PairHMM forward kernel for gfx950, in FP32 or FP64, with
// power-of-two rescaling.
//
// A pair whose haplotype is too long for one wavefront is cut into tiles of
// 64 lanes x N columns (N = 16).  Each tile is processed
// by one wavefront of a persistent grid; tiles of a pair are handed out in
// column order.  Per row, a tile needs from its left neighbour the row's last
// M and I values and the inclusive delete-chain prefix S(i, c0-1) at its
// first column: this replaces the paper's multi-block extension through
// thread-block clusters and distributed shared memory (Section 3.4, last
// paragraphs), which gfx950 does not have.  The neighbour publishes one
// record per row into a ring buffer in global memory; consumer and producer
// form a skewed pipeline (a look-back of depth one), so the hand-off latency
// is paid once per tile, not once per row.
//
// The row recurrence is the short kernel's (scaled form when the read allows
// it, plain form otherwise); all tiles of a pair use the same per-row
// coefficients, so the records they exchange are in the same units.
//
// Validity without fences: every published value is non-negative, so its
// sign bit carries the parity of the ring lap (row / kRing).  A reader
// accepts a field only when its sign bit matches the lap it expects; the
// owner of a ring slot clears it to -0.  Each field is written and read with
// relaxed agent-scope atomics, so no release/acquire fence is needed per row.
// Ring ownership changes (once per tile) use release/acquire.
//
// Rescaling (not part of the paper, which gives no underflow scheme for its
// long reads): every kRescaleRows rows a tile multiplies its state by 2^-e,
// e the exponent of its largest value, and adds e to an integer exponent E.
// Values handed between tiles carry the producer's exponent and are brought
// into the consumer's scale with ldexp; when a record lies more than
// rebase_bits<R> above the consumer's scale the consumer first rebases to
// it.  The start row is D(0,j) = 1/k; the tiles' last-row sums are combined
// in FP64 with their exponents and the result is log10(S) + E log10(2).
#include <type_traits>

#include "phmm_dev.h"

namespace phmm {

constexpr int kRescaleRows = 8;
constexpr int kNoRec = -(1 << 30);  // no record (all fields 0)

template <typename R>
struct LongGeom;
template <>
struct LongGeom<float> {
    static constexpr int N = 16;
    static constexpr int cls = class_of_n(N);       // short-kernel class with this N (scan tables)
    static constexpr int rebase_bits = 48;          // converted records stay below 2^49
    static constexpr float exp_bias = 8388608.0f;   // 2^23: exponents stored as E + 2^23 (exact)
};
template <>
struct LongGeom<double> {
    static constexpr int N = 16;
    static constexpr int cls = class_of_n(N);
    static constexpr int rebase_bits = 256;
    static constexpr double exp_bias = 1099511627776.0;  // 2^40
};

__host__ __device__ uint32_t long_slots(int grid) { return 2u * (uint32_t)(grid > 0 ? grid : 1); }
__host__ __device__ uint32_t long_tile_cols(bool fp32)
{
    return (uint32_t)(fp32 ? LongGeom<float>::N : LongGeom<double>::N) * kWave;
}

// Ring slot layout (bytes): kRing rows x 4 fields of R, then the tile's final
// (sum, exponent) pair as two doubles at kRingRowBytes.
constexpr size_t kRingRowBytes = (size_t)kRing * 4 * sizeof(double);
constexpr size_t kRingSlotBytes = kRingRowBytes + 4 * sizeof(double);

struct SlotState {
    uint32_t* prog;   // rows the consumer has taken from the ring
    uint32_t* owner;  // item + 1 currently publishing into the ring
    uint32_t* done;   // item + 1 whose ring has been fully consumed
};

__device__ __forceinline__ SlotState slot_state(const Work& w, uint32_t nslot)
{
    SlotState s;
    s.prog = w.long_prog;
    s.owner = w.long_prog + nslot;
    s.done = w.long_prog + 2 * nslot;
    return s;
}

__device__ __forceinline__ char* ring_of(const Work& w, uint32_t slot)
{
    return reinterpret_cast<char*>(w.long_ring) + (size_t)slot * kRingSlotBytes;
}

// Bit patterns of R and the lap parity kept in the sign bit.
template <typename R>
using Bits = typename std::conditional<sizeof(R) == 4, uint32_t, uint64_t>::type;

template <typename R>
__device__ __forceinline__ void st_relaxed(R* p, R v)
{
    __hip_atomic_store(reinterpret_cast<Bits<R>*>(p), __builtin_bit_cast(Bits<R>, v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename R>
__device__ __forceinline__ R ld_relaxed(const R* p)
{
    return __builtin_bit_cast(R, __hip_atomic_load(reinterpret_cast<const Bits<R>*>(p),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
template <int ORDER>
__device__ __forceinline__ uint32_t ld_u32(const uint32_t* p)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)__hip_atomic_load(p, ORDER, __HIP_MEMORY_SCOPE_AGENT));
}
template <int ORDER>
__device__ __forceinline__ void st_u32(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, ORDER, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename R>
__device__ __forceinline__ R with_parity(R v, uint32_t parity)
{
    constexpr int top = 8 * sizeof(R) - 1;
    const Bits<R> u = __builtin_bit_cast(Bits<R>, v) & ~((Bits<R>)1 << top);
    return __builtin_bit_cast(R, u | ((Bits<R>)parity << top));
}
template <typename R>
__device__ __forceinline__ uint32_t parity_of(R v)
{
    return (uint32_t)(__builtin_bit_cast(Bits<R>, v) >> (8 * sizeof(R) - 1));
}
__device__ __forceinline__ float magnitude(float v) { return __builtin_fabsf(v); }
__device__ __forceinline__ double magnitude(double v) { return __builtin_fabs(v); }

__device__ __forceinline__ bool aborted(const Work& w)
{
    return ld_u32<__ATOMIC_RELAXED>(&w.ctr->status) != 0u;
}
__device__ __forceinline__ void raise_timeout(const Work& w)
{
    atomicCAS(&w.ctr->status, 0u, (uint32_t)(-5));  // PHMM_ETIMEOUT
}

// Tile prefix over the long pairs of list `which`, and reset of the ring
// ownership state.
__global__ void long_prefix_kernel(Batch b, Work w, uint32_t nslot, int which, uint32_t tile_cols)
{
    __shared__ uint32_t part[256];
    const uint32_t n = w.ctr->n_long[which];
    const uint32_t* list = w.long_list[which];
    const int t = (int)threadIdx.x;
    const uint32_t per = (n + 255u) / 256u;
    const uint32_t lo = (uint32_t)t * per, hi = lo + per < n ? lo + per : n;
    uint32_t sum = 0;
    for (uint32_t s = lo; s < hi; ++s) {
        const uint32_t pair = list[s];
        const uint32_t h = b.pairs[2 * (uint64_t)pair + 1];
        const uint32_t k = (uint32_t)(b.hap_off[h + 1] - b.hap_off[h]);
        sum += (k + tile_cols - 1) / tile_cols;
    }
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        for (int q = 0; q < 256; ++q) {
            const uint32_t v = part[q];
            part[q] = acc;
            acc += v;
        }
        w.ctr->long_tiles[which] = acc;
        w.ctr->long_cursor = 0;
        w.long_pref[n] = acc;
    }
    __syncthreads();
    uint32_t acc = part[t];
    for (uint32_t s = lo; s < hi; ++s) {
        w.long_pref[s] = acc;
        const uint32_t pair = list[s];
        const uint32_t h = b.pairs[2 * (uint64_t)pair + 1];
        const uint32_t k = (uint32_t)(b.hap_off[h + 1] - b.hap_off[h]);
        acc += (k + tile_cols - 1) / tile_cols;
    }
    for (uint32_t s = (uint32_t)t; s < 3 * nslot; s += 256) w.long_prog[s] = 0u;
}

// Wavefronts of a grid of g that take tiles.  With fewer tiles than
// wavefronts, the first tiles.  Tiles are claimed in arrival order, and the
// first wavefronts to arrive can crowd a few SIMDs (up to 4 tiles on one
// while others hold none); the workgroups with the lowest indices are
// spread over the XCDs and CUs by the dispatcher, so only they take tiles
// and the others leave at once (16 pairs of 64 tiles on a grid of 4096:
// 1368 -> 1600 GCUPS).  With more tiles than wavefronts every wavefront
// stays: cutting the grid to make rounds of equal size helps only when all
// tiles take equally long, and halves the rate of mixed lengths.
__host__ __device__ uint32_t long_active_waves(uint32_t tiles, uint32_t g)
{
    return tiles > 0u && tiles < g ? tiles : g;
}

template <typename R>
__device__ __forceinline__ R rd_lane(R v, int lane);
template <>
__device__ __forceinline__ float rd_lane<float>(float v, int lane)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
template <>
__device__ __forceinline__ double rd_lane<double>(double v, int lane)
{
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// (m1, E1) + (m2, E2) with exponents kept in integers.
__device__ __forceinline__ void acc_add(double& m1, long long& E1, double m2, long long E2)
{
    if (!(m2 > 0.0)) return;
    if (!(m1 > 0.0)) { m1 = m2; E1 = E2; return; }
    if (E1 >= E2) m1 = m1 + ldexp(m2, (int)max(E2 - E1, -2000LL));
    else { m1 = m2 + ldexp(m1, (int)max(E1 - E2, -2000LL)); E1 = E2; }
}

template <typename R>
__device__ __forceinline__ const R* long_pow(const Tables& t, int gcp);
template <>
__device__ __forceinline__ const float* long_pow<float>(const Tables& t, int gcp)
{
    return t.pw32 + ((size_t)LongGeom<float>::cls * 256 + gcp) * kPowStride;
}
template <>
__device__ __forceinline__ const double* long_pow<double>(const Tables& t, int gcp)
{
    return t.pw64 + ((size_t)LongGeom<double>::cls * 256 + gcp) * kPowStride;
}

// Waves per SIMD the kernels are compiled for.  FP32 lean: 4 (128 VGPRs;
// the window records in LDS, spills only per tile), 6-9% faster than at 3
// where its tiles fill the chip.  FP32 general: 3 (168 VGPRs; at 4 its row
// loops spill), 20-24% faster than at the compiler's own choice of 2.  FP64
// lean: 2 (1.4-1.8x the general kernel's rate on 4-16 kbp pairs); FP64
// general: the compiler's choice of 1.
template <typename R, bool GENERAL>
constexpr int long_waves() { return sizeof(R) == 4 ? (GENERAL ? 3 : 4) : (GENERAL ? 1 : 2); }

// List long_list_of(precision of R, GENERAL) in precision R.  The lean
// kernel (GENERAL false) runs pairs whose read has one gap byte (>= 1) and
// the scaled row form on every row, as the packer routed them; the general
// kernel tests each read and runs per-row gap changes and the plain form.
template <typename R, bool GENERAL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(long_waves<R, GENERAL>())))
void long_kernel(Batch b, Tables t, Work w, Policy pol)
{
    constexpr int N = LongGeom<R>::N;
    constexpr uint32_t kTile = (uint32_t)N * kWave;
    constexpr int which = long_list_of(sizeof(R) == 4 ? 0 : 1, GENERAL);
    __shared__ RowRec<R> rec[kWave];
    __shared__ int rinfo[kWave];
    // producer records of the current window, row i0 + q at lane or entry q,
    // in the producer's scale: magnitudes, exponent, and the exponent of the
    // largest field (kNoRec when there is none).  They are read once per
    // kRescaleRows rows: FP32 keeps them in LDS (each lane writes and reads
    // its own entry, no barrier), which frees the registers of a fourth wave
    // per SIMD; FP64 keeps them in registers (in LDS its lean kernel ran
    // 20-25% slower at 16 kbp).
    constexpr bool kWinLds = sizeof(R) == 4;
    __shared__ R winM[kWinLds ? kWave : 1], winI[kWinLds ? kWave : 1], winP[kWinLds ? kWave : 1];
    __shared__ int winE[kWinLds ? kWave : 1], winTop[kWinLds ? kWave : 1];
    const int lane = (int)threadIdx.x;
    const uint32_t nslot = long_slots((int)gridDim.x);
    const SlotState ss = slot_state(w, nslot);
    const uint32_t total = w.ctr->long_tiles[which];
    const uint32_t n_long = w.ctr->n_long[which];
    const uint32_t* list = w.long_list[which];
    const uint32_t spin_limit = pol.watchdog_spins;
    if (blockIdx.x >= long_active_waves(total, gridDim.x)) return;

    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(&w.ctr->long_cursor, 1u);
        it = wave_broadcast0(it);
        if (it >= total || aborted(w)) break;

        // item -> (long pair s, tile)
        uint32_t lo = 0, hi = n_long;  // largest s with long_pref[s] <= it
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (w.long_pref[mid] <= it) lo = mid; else hi = mid;
        }
        const uint32_t s_idx = lo;
        const uint32_t tile = it - w.long_pref[s_idx];
        const uint32_t ntiles = w.long_pref[s_idx + 1] - w.long_pref[s_idx];
        const bool has_prod = tile > 0, has_cons = tile + 1 < ntiles;
        const uint32_t pair = list[s_idx];
        const uint32_t r = b.pairs[2 * (uint64_t)pair], h = b.pairs[2 * (uint64_t)pair + 1];
        const uint64_t roff = b.read_off[r], hoff = b.hap_off[h];
        const int l = (int)(b.read_off[r + 1] - roff);
        const uint32_t k = (uint32_t)(b.hap_off[h + 1] - hoff);
        const uint32_t slot = it % nslot, pslot = (it + nslot - 1) % nslot;
        R* ring = reinterpret_cast<R*>(ring_of(w, slot));
        const R* pring = reinterpret_cast<const R*>(ring_of(w, pslot));
        double* fin = reinterpret_cast<double*>(ring_of(w, slot) + kRingRowBytes);
        const double* pfin = reinterpret_cast<const double*>(ring_of(w, pslot) + kRingRowBytes);

        // ---- take over ring slot `slot` once its previous occupant's ring
        // (item it - nslot) has been read completely
        bool dead = false;
        if (it >= nslot) {
            uint32_t spins = 0;
            while (ld_u32<__ATOMIC_ACQUIRE>(&ss.done[slot]) != it - nslot + 1u) {
                if (++spins > spin_limit) { raise_timeout(w); dead = true; break; }
                if ((spins & 63u) == 0u && aborted(w)) { dead = true; break; }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        if (!dead) {
            if (has_cons) {
                for (int q = lane; q < kRing * 4; q += kWave) st_relaxed(ring + q, (R)-0.0);
                if (lane < 2) st_relaxed(fin + lane, -0.0);
                if (lane == 0) st_u32<__ATOMIC_RELAXED>(&ss.prog[slot], 0u);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                if (lane == 0) st_u32<__ATOMIC_RELEASE>(&ss.owner[slot], it + 1u);
            } else if (lane == 0) {
                st_u32<__ATOMIC_RELEASE>(&ss.done[slot], it + 1u);  // ring unused
            }
        }
        if (has_prod && !dead) {
            uint32_t spins = 0;
            while (ld_u32<__ATOMIC_ACQUIRE>(&ss.owner[pslot]) != it) {
                if (++spins > spin_limit) { raise_timeout(w); dead = true; break; }
                if ((spins & 63u) == 0u && aborted(w)) { dead = true; break; }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        if (__ballot(dead) != 0ull) break;

        // ---- columns of this lane as 8-bit match codes, four per register
        const uint32_t c0 = tile * kTile + (uint32_t)lane * N;
        uint32_t hc[(N + 3) / 4];
#pragma unroll
        for (int q = 0; q < (N + 3) / 4; ++q) hc[q] = 0u;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const uint32_t j = c0 + (uint32_t)n;
            const uint32_t code = j < k ? hap_code(b.haps[hoff + j]) : kPadCode;
            hc[n / 4] |= code << (8 * (n % 4));
        }
        // read profile: scaled row form when every gap byte is >= 1 and every
        // insertion byte within the form's limit (known for the lean kernel)
        const int g0 = b.gq[roff];
        bool sc_ok = true;
        if constexpr (GENERAL) {
            for (int i0 = 0; i0 < l; i0 += kWave) {
                const int i = i0 + lane;
                const int gc = i < l ? (int)b.gq[roff + i] : g0;
                const int ic = i < l ? (int)b.iq[roff + i] : 0;
                sc_ok = sc_ok && __ballot(gc == 0 || ic > kScMaxInsQ) == 0ull;
            }
        }
        const R minit = (R)(1.0 / (double)k);
        const R* pw0 = long_pow<R>(t, g0);
        ScanMul<R> mul = make_scan_mul<R>(pw0, lane, 0);
        R gcur = (R)t.p64[g0], gprev = gcur, gN1 = pw0[65], gN = pw0[1];
        int gc_cur = g0;
        const ScanMul<R> ones = make_sum_mul<R>(lane, 0);

        R Ma[N], Ia[N], Mb[N], Ib[N];
#pragma unroll
        for (int n = 0; n < N; ++n) { Ma[n] = (R)0; Ia[n] = (R)0; Mb[n] = (R)0; Ib[n] = (R)0; }
        R Mleft = (R)0, Ileft = (R)0, C = (R)0;
        int E = 0;
        uint32_t prog_seen = 0;

        auto run_rows = [&](auto sc_tag) {
            constexpr bool SC = decltype(sc_tag)::value;
            R rM = (R)0, rI = (R)0, rP = (R)0;  // window records in registers (FP64)
            int rE = 0, rTop = kNoRec;
            // the current group's records brought to this tile's scale
            R wM = (R)0, wI = (R)0, wP = (R)0;
            // one row: Mp/Ip receive row i (window slot tt) from (Mi, Ii)
            auto do_row = [&](int i, int tt, const R(&Mi)[N], const R(&Ii)[N], R(&Mp)[N],
                              R(&Ip)[N]) -> bool {
                const RowRec<R> c = rec[tt];
                const int info = __builtin_amdgcn_readfirstlane(rinfo[tt]);
                const int gc = info >> 16;
                gprev = gcur;
                if (GENERAL && gc != gc_cur) {  // per-row gap continuation
                    gc_cur = gc;
                    gcur = (R)t.p64[gc];
                    const R* pwi = long_pow<R>(t, gc);
                    mul = make_scan_mul<R>(pwi, lane, 0);
                    gN1 = pwi[65];
                    gN = pwi[1];
                }
                R Vp;
                const int bidx = info & 0xff;
                if (i == 0)
                    row_first<R, N>(Mp, Ip, hc, bidx, c, minit, gcur, Vp);
                else
                    row_step<R, N, SC>(Mi, Ii, Mp, Ip, hc, bidx, c, Mleft, Ileft, C, gprev, gcur,
                                       Vp);
                // lane 0 takes the left neighbour's boundary (zero in the first
                // tile) before the row's delete-chain window sums are formed
                Mleft = dpp<kWaveShr1>(Mp[N - 1]);
                Ileft = dpp<kWaveShr1>(Ip[N - 1]);
                R nbP = (R)0;
                if (has_prod) {
                    const R nbM = rd_lane(wM, tt), nbI = rd_lane(wI, tt);
                    nbP = rd_lane(wP, tt);
                    if (lane == 0) { Mleft = nbM; Ileft = nbI; }
                }
                const R vsh = fmaR(gN1, Mleft, Vp);
                R u = dpp<kWaveShr1>(vsh);
                if (lane == 0) u = nbP;
                C = seg_scan(u, mul);
                if (has_cons) {  // publish row i for the next tile
                    const R P = fmaR(gN, C, vsh);
                    if (i >= kRing && (uint32_t)(i - kRing + 1) > prog_seen) {
                        uint32_t spins = 0;
                        for (;;) {
                            prog_seen = ld_u32<__ATOMIC_RELAXED>(&ss.prog[slot]);
                            if (prog_seen >= (uint32_t)(i - kRing + 1)) break;
                            if (++spins > spin_limit) { raise_timeout(w); dead = true; break; }
                            if ((spins & 63u) == 0u && aborted(w)) { dead = true; break; }
                            __builtin_amdgcn_s_sleep(2);
                        }
                        if (dead) return false;
                    }
                    if (lane == 63) {
                        const uint32_t par = ((uint32_t)i / kRing) & 1u;
                        R* rp = ring + (size_t)((uint32_t)i % kRing) * 4;
                        st_relaxed(rp + 0, with_parity(Mp[N - 1], par));
                        st_relaxed(rp + 1, with_parity(Ip[N - 1], par));
                        st_relaxed(rp + 2, with_parity(P, par));
                        st_relaxed(rp + 3, with_parity((R)((double)E + (double)LongGeom<R>::exp_bias), par));
                    }
                }
                return true;
            };
            // every kRescaleRows rows: bring the row maximum to about 1 (a
            // multiply by an exact power of two, done every time so that the
            // row registers need no merge)
            auto rescale = [&](R(&Mp)[N], R(&Ip)[N]) {
                R mx = maxR(C, maxR(Mleft, Ileft));
#pragma unroll
                for (int n = 0; n < N; ++n) mx = maxR(mx, maxR(Mp[n], Ip[n]));
                const int emax = wave_max_int(mx > (R)0 ? exponent_of(mx) + 4096 : 0);
                int e = emax > 0 ? emax - 4096 : 0;
                if (!pow2_ok<R>(-e)) e = e > 0 ? (sizeof(R) == 4 ? 126 : 1022) : -(sizeof(R) == 4 ? 126 : 1022);
                const R f = pow2<R>(-e);
#pragma unroll
                for (int n = 0; n < N; ++n) {
                    Mp[n] *= f;
                    Ip[n] *= f;
                }
                Mleft *= f;
                Ileft *= f;
                C *= f;
                E += e;
            };
            // Records of window rows tt .. tt+ng-1 to this tile's scale.  Within
            // a tile values fall by T_DD per column away from the alignment
            // band, so a neighbour's boundary can sit far above this tile's
            // own, then negligible, values (a record stays exactly 0 in the
            // neighbour until the band comes within range of its last column):
            // the tile is first rebased to the largest of them when they lie
            // more than rebase_bits above its scale.  Both steps are exact
            // power-of-two scalings over the full exponent range (ldexp), so
            // values far below the new scale flush to 0 and nothing overflows.
            auto take_records = [&](int tt, int ng) {
                int top_e = rTop;
                if constexpr (kWinLds) top_e = winTop[lane_here()];
                const int rel = lane >= tt && lane < tt + ng && top_e != kNoRec ? top_e - E : kNoRec;
                const int top = wave_max_int(rel - kNoRec + 1) - 1 + kNoRec;
                if (top > LongGeom<R>::rebase_bits) {
#pragma unroll
                    for (int n = 0; n < N; ++n) {
                        Ma[n] = scale2(Ma[n], -top);
                        Ia[n] = scale2(Ia[n], -top);
                    }
                    Mleft = scale2(Mleft, -top);
                    Ileft = scale2(Ileft, -top);
                    C = scale2(C, -top);
                    E += top;
                }
                if constexpr (kWinLds) {
                    const int me = lane_here();
                    const int sh = max(min(winE[me] - E, 4000), -4000);
                    wM = scale2(winM[me], sh);
                    wI = scale2(winI[me], sh);
                    wP = scale2(winP[me], sh);
                } else {
                    const int sh = max(min(rE - E, 4000), -4000);
                    wM = scale2(rM, sh);
                    wI = scale2(rI, sh);
                    wP = scale2(rP, sh);
                }
            };
            for (int i0 = 0; i0 < l && !dead; i0 += kWave) {
                __syncthreads();
                {
                    const int i = i0 + lane;
                    if (i < l) {
                        const uint64_t a = roff + (uint64_t)i;
                        rec[lane] = make_row_rec<R, SC, true>(b, t.p64, a, i, l);
                        rinfo[lane] = read_base_index(b.reads[a]) | ((int)b.gq[a] << 16);
                    }
                }
                __syncthreads();
                const int nrows = l - i0 < kWave ? l - i0 : kWave;
                if (has_prod) {
                    // the window of records of rows i0 .. i0 + nrows - 1: one
                    // round trip to L2 serves 64 rows, and the consumer trails
                    // its producer by at least a window
                    if (lane == 0) st_u32<__ATOMIC_RELAXED>(&ss.prog[pslot], (uint32_t)i0);
                    uint32_t spins = 0;
                    R bM = (R)0, bI = (R)0, bP = (R)0, bE = (R)0;
                    for (;;) {
                        const int row = i0 + lane;
                        const uint32_t par = ((uint32_t)row / kRing) & 1u;
                        const R* rp = pring + (size_t)((uint32_t)row % kRing) * 4;
                        bool ok = true;
                        if (lane < nrows) {
                            bM = ld_relaxed(rp + 0);
                            bI = ld_relaxed(rp + 1);
                            bP = ld_relaxed(rp + 2);
                            bE = ld_relaxed(rp + 3);
                            ok = parity_of(bM) == par && parity_of(bI) == par &&
                                 parity_of(bP) == par && parity_of(bE) == par;
                        }
                        if (__ballot(!ok) == 0ull) break;
                        if (++spins > spin_limit) { raise_timeout(w); dead = true; break; }
                        if ((spins & 63u) == 0u && aborted(w)) { dead = true; break; }
                        __builtin_amdgcn_s_sleep(1);
                    }
                    if (__ballot(dead) != 0ull) break;
                    rE = (int)((double)magnitude(bE) - (double)LongGeom<R>::exp_bias);
                    rM = magnitude(bM);
                    rI = magnitude(bI);
                    rP = magnitude(bP);
                    const R mrec = maxR(rM, maxR(rI, rP));
                    rTop = lane < nrows && mrec > (R)0 ? rE + exponent_of(mrec) : kNoRec;
                    if constexpr (kWinLds) {
                        const int me = lane_here();
                        winM[me] = rM;
                        winI[me] = rI;
                        winP[me] = rP;
                        winE[me] = rE;
                        winTop[me] = rTop;
                    }
                }
                int tt = 0;
                // groups of kRescaleRows rows: ping-pong in pairs, rescale at the end
                for (; tt + kRescaleRows <= nrows && !dead; tt += kRescaleRows) {
                    if (has_prod) take_records(tt, kRescaleRows);
#pragma unroll 1
                    for (int q = 0; q < kRescaleRows; q += 2) {
                        if (!do_row(i0 + tt + q, tt + q, Ma, Ia, Mb, Ib)) break;
                        if (!do_row(i0 + tt + q + 1, tt + q + 1, Mb, Ib, Ma, Ia)) break;
                    }
                    if (dead) break;
                    rescale(Ma, Ia);
                }
                // the last rows of the read
                if (tt < nrows && !dead && has_prod) take_records(tt, nrows - tt);
                for (; tt < nrows && !dead; tt += 2) {
                    if (!do_row(i0 + tt, tt, Ma, Ia, Mb, Ib)) break;
                    if (tt + 1 < nrows) {
                        if (!do_row(i0 + tt + 1, tt + 1, Mb, Ib, Ma, Ia)) break;
                    } else {
#pragma unroll
                        for (int n = 0; n < N; ++n) { Ma[n] = Mb[n]; Ia[n] = Ib[n]; }
                    }
                }
            }
        };
        if constexpr (!GENERAL) {
            run_rows(std::true_type{});
        } else {
            if (sc_ok)
                run_rows(std::true_type{});
            else
                run_rows(std::false_type{});
        }
        if (__ballot(dead) != 0ull) break;

        // ---- eq.4 over this tile's real columns, then accumulate along the tiles
        R sp = (R)0;
#pragma unroll
        for (int n = 0; n < N; ++n)
            if (c0 + (uint32_t)n < k) sp += Ma[n] + Ia[n];
        sp = seg_scan(sp, ones);
        double am = (double)rd_lane(sp, 63);
        long long aE = (long long)E;
        if (has_prod) {
            uint32_t spins = 0;
            double fm = 0.0, fe = 0.0;
            for (;;) {
                fm = ld_relaxed(pfin + 0);
                fe = ld_relaxed(pfin + 1);
                const bool ok = parity_of(fm) == 0u && parity_of(fe) == 0u;
                if (__builtin_amdgcn_readfirstlane((int)ok)) break;
                if (++spins > spin_limit) { raise_timeout(w); dead = true; break; }
                if ((spins & 63u) == 0u && aborted(w)) { dead = true; break; }
                __builtin_amdgcn_s_sleep(2);
            }
            if (dead) break;
            fm = rd_lane(fm, 0);
            fe = rd_lane(fe, 0);
            acc_add(am, aE, magnitude(fm), (long long)(magnitude(fe) - 1099511627776.0));
            // the producer's ring has been read completely
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0) st_u32<__ATOMIC_RELEASE>(&ss.done[pslot], it);
        }
        if (has_cons) {
            if (lane == 0) {
                st_relaxed(fin + 0, with_parity(am, 0u));
                st_relaxed(fin + 1, with_parity((double)aE + 1099511627776.0, 0u));
            }
        } else if (lane == 0) {
            double out;
            if (am > 0.0) {
                int e2;
                const double m = frexp(am, &e2);
                out = log10(m) + (double)((long long)e2 + aE) * 0.30102999566398119521;
            } else {
                out = -__builtin_inf();
            }
            b.out[pair] = out;
            // long, rescaled, and the precision
            if (b.flags) b.flags[pair] = (uint8_t)(0x04 | 0x08 | (sizeof(R) == 4 ? 0x01 : 0x10));
        }
    }
}

// Every list in order (long_list_of); a list whose grid is 0 is skipped (the
// caller knows it is empty).  Each list's prefix kernel resets the ring
// ownership state before its long kernel runs.
void launch_long(hipStream_t s, const int (&grid)[kLongLists], const Batch& b, const Tables& t,
                 const Work& w, const Policy& p)
{
    for (int q = 0; q < kLongLists; ++q) {
        if (grid[q] <= 0) continue;
        const bool fp32 = q < 2;
        hipLaunchKernelGGL(long_prefix_kernel, dim3(1), dim3(256), 0, s, b, w, long_slots(grid[q]), q,
                           long_tile_cols(fp32));
        const dim3 g(grid[q]), blk(kWave);
        switch (q) {
        case 0: hipLaunchKernelGGL((long_kernel<float, false>), g, blk, 0, s, b, t, w, p); break;
        case 1: hipLaunchKernelGGL((long_kernel<float, true>), g, blk, 0, s, b, t, w, p); break;
        case 2: hipLaunchKernelGGL((long_kernel<double, false>), g, blk, 0, s, b, t, w, p); break;
        default: hipLaunchKernelGGL((long_kernel<double, true>), g, blk, 0, s, b, t, w, p); break;
        }
    }
}

const void* long_kernel_ptr(int q)
{
    switch (q) {
    case 0: return reinterpret_cast<const void*>(&long_kernel<float, false>);
    case 1: return reinterpret_cast<const void*>(&long_kernel<float, true>);
    case 2: return reinterpret_cast<const void*>(&long_kernel<double, false>);
    default: return reinterpret_cast<const void*>(&long_kernel<double, true>);
    }
}

size_t long_ring_slot_bytes() { return kRingSlotBytes; }

}  // namespace phmm
