// Long-pair PairHMM forward kernel for gfx950 (FP64 with power-of-two
// rescaling).
//
// A pair whose haplotype is too long for one wavefront is cut into tiles of
// kLongTile = 64 lanes x kLongN columns.  Each tile is processed by one
// wavefront of a persistent grid; tiles of a pair are handed out in column
// order.  Per row, a tile needs from its left neighbour the row's last M and
// I values and the inclusive delete-chain prefix S(i, c0-1) at its first
// column: this replaces the paper's multi-block extension through thread-block
// clusters and distributed shared memory (Section 3.4, last paragraphs), which
// gfx950 does not have.  The neighbour publishes one record per row into a
// ring buffer in global memory; consumer and producer form a skewed pipeline
// (a look-back of depth one), so the hand-off latency is paid once per tile,
// not once per row.
//
// Validity without fences: every published value is non-negative, so its
// sign bit carries the parity of the ring lap (row / kRing).  A reader
// accepts a field only when its sign bit matches the lap it expects; the ring
// starts out all -0.0.  Each field is written and read with relaxed
// agent-scope atomics, so no release/acquire fence is needed per row.  Ring
// ownership changes (once per tile) use release/acquire.
//
// Rescaling (not part of the paper, which gives no underflow scheme for its
// long reads): every kRescaleRows rows a tile multiplies its state by 2^-e,
// e the exponent of its largest value, and adds e to an integer exponent E.
// Values handed between tiles carry the producer's exponent and are brought
// into the consumer's scale with ldexp; when a record lies more than
// kRebaseBits above the consumer's scale the consumer first rebases to it.  The start row is D(0,j) = 1/k and the
// result is log10(S) + E log10(2).
#include "phmm_dev.h"

namespace phmm {

constexpr int kRescaleRows = 8;
constexpr long long kRebaseBits = 256;  // rebase when a neighbour's record is this far above
constexpr double kExpBias = 1099511627776.0;  // 2^40: exponents stored as E + 2^40

__host__ __device__ uint32_t long_slots(int grid) { return 2u * (uint32_t)(grid > 0 ? grid : 1); }

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

__device__ __forceinline__ double* ring_of(const Work& w, uint32_t slot)
{
    return w.long_ring + (size_t)slot * (kRing + 1) * 4;
}

__device__ __forceinline__ void st_relaxed(double* p, double v)
{
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), __builtin_bit_cast(uint64_t, v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_relaxed(const double* p)
{
    return __builtin_bit_cast(double, __hip_atomic_load(reinterpret_cast<const uint64_t*>(p),
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

__device__ __forceinline__ double with_parity(double v, uint32_t parity)
{
    uint64_t u = __builtin_bit_cast(uint64_t, v) & 0x7fffffffffffffffull;
    return __builtin_bit_cast(double, u | ((uint64_t)parity << 63));
}
__device__ __forceinline__ uint32_t parity_of(double v)
{
    return (uint32_t)(__builtin_bit_cast(uint64_t, v) >> 63);
}
__device__ __forceinline__ double magnitude(double v) { return __builtin_fabs(v); }

// Sets the device status (first error wins) and returns true if any wave
// already failed.
__device__ __forceinline__ bool aborted(const Work& w)
{
    return ld_u32<__ATOMIC_RELAXED>(&w.ctr->status) != 0u;
}
__device__ __forceinline__ void raise_timeout(const Work& w)
{
    atomicCAS(&w.ctr->status, 0u, (uint32_t)(-5));  // PHMM_ETIMEOUT
}

// Tile prefix over the long pairs, and reset of the ring ownership state.
__global__ void long_prefix_kernel(Batch b, Work w, uint32_t nslot)
{
    __shared__ uint32_t part[256];
    const uint32_t n = w.ctr->n_long;
    const int t = (int)threadIdx.x;
    const uint32_t per = (n + 255u) / 256u;
    const uint32_t lo = (uint32_t)t * per, hi = lo + per < n ? lo + per : n;
    uint32_t sum = 0;
    for (uint32_t s = lo; s < hi; ++s) {
        const uint32_t pair = w.long_list[s];
        const uint32_t h = b.pairs[2 * (uint64_t)pair + 1];
        const uint32_t k = (uint32_t)(b.hap_off[h + 1] - b.hap_off[h]);
        sum += (k + kLongTile - 1) / kLongTile;
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
        w.ctr->long_tiles = acc;
        w.ctr->long_cursor = 0;
        w.long_pref[n] = acc;
    }
    __syncthreads();
    uint32_t acc = part[t];
    for (uint32_t s = lo; s < hi; ++s) {
        w.long_pref[s] = acc;
        const uint32_t pair = w.long_list[s];
        const uint32_t h = b.pairs[2 * (uint64_t)pair + 1];
        const uint32_t k = (uint32_t)(b.hap_off[h + 1] - b.hap_off[h]);
        acc += (k + kLongTile - 1) / kLongTile;
    }
    for (uint32_t s = (uint32_t)t; s < 3 * nslot; s += 256) w.long_prog[s] = 0u;
}

struct LRec {
    double dp, px, tmm, tim, cd, tmi, tii, pm;
};

constexpr int kLongWords = kLongN / 4;

__device__ __forceinline__ void lrow_first(double (&Mo)[kLongN], double (&Io)[kLongN],
                                           const uint32_t (&hc)[kLongWords], int bidx,
                                           const LRec& c, double minit, double g, double& Vp)
{
    double V = 0.0;
    const double base = c.tim * minit;
#pragma unroll
    for (int n = 0; n < kLongN; ++n) {
        const double p = emit_sel(hc[n / 4], 8 * (n % 4) + bidx, c.pm, c.px);
        const double m = p * base;
        Mo[n] = m;
        Io[n] = 0.0;
        if (n < kLongN - 1) V = __builtin_fma(g, V, m);
    }
    Vp = V;
}

__device__ __forceinline__ void lrow_step(const double (&Mi)[kLongN], const double (&Ii)[kLongN],
                                          double (&Mo)[kLongN], double (&Io)[kLongN],
                                          const uint32_t (&hc)[kLongWords], int bidx,
                                          const LRec& c, double Mleft, double Ileft, double C,
                                          double gprev, double gcur, double& Vp)
{
    double T = C, V = 0.0;
#pragma unroll
    for (int n = 0; n < kLongN; ++n) {
        const double mprev = n == 0 ? Mleft : Mi[n - 1];
        const double iprev = n == 0 ? Ileft : Ii[n - 1];
        const double p = emit_sel(hc[n / 4], 8 * (n % 4) + bidx, c.pm, c.px);
        const double x = __builtin_fma(c.cd, T, __builtin_fma(c.tim, iprev, c.tmm * mprev));
        const double m = p * x;
        Mo[n] = m;
        Io[n] = __builtin_fma(c.tii, Ii[n], c.tmi * Mi[n]);
        T = __builtin_fma(gprev, T, mprev);
        if (n < kLongN - 1) V = __builtin_fma(gcur, V, m);
    }
    Vp = V;
}

__device__ __forceinline__ double rd_lane(double v, int lane)
{
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Wavefront max of a non-negative int (0 = nothing).
__device__ __forceinline__ int wave_max_int(int x)
{
    x = max(x, dpp_i<kRowShr1>(x));
    x = max(x, dpp_i<kRowShr2>(x));
    x = max(x, dpp_i<kRowShr4>(x));
    x = max(x, dpp_i<kRowShr8>(x));
    x = max(x, dpp_i<kRowBcast15, 0xa>(x));
    x = max(x, dpp_i<kRowBcast31, 0xc>(x));
    return __builtin_amdgcn_readlane(x, 63);
}

// (m1, E1) + (m2, E2) with exponents kept in integers.
__device__ __forceinline__ void acc_add(double& m1, long long& E1, double m2, long long E2)
{
    if (!(m2 > 0.0)) return;
    if (!(m1 > 0.0)) { m1 = m2; E1 = E2; return; }
    if (E1 >= E2) m1 = m1 + ldexp(m2, (int)max(E2 - E1, -2000LL));
    else { m1 = m2 + ldexp(m1, (int)max(E1 - E2, -2000LL)); E1 = E2; }
}

__global__ __launch_bounds__(64) void long_kernel(Batch b, Tables t, Work w, Policy pol)
{
    constexpr int N = kLongN;
    __shared__ LRec rec[kWave];
    __shared__ int rinfo[kWave];
    const int lane = (int)threadIdx.x;
    const uint32_t nslot = long_slots((int)gridDim.x);
    const SlotState ss = slot_state(w, nslot);
    const uint32_t total = w.ctr->long_tiles;
    const uint32_t n_long = w.ctr->n_long;
    const uint32_t spin_limit = pol.watchdog_spins;

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
        const uint32_t pair = w.long_list[s_idx];
        const uint32_t r = b.pairs[2 * (uint64_t)pair], h = b.pairs[2 * (uint64_t)pair + 1];
        const uint64_t roff = b.read_off[r], hoff = b.hap_off[h];
        const int l = (int)(b.read_off[r + 1] - roff);
        const uint32_t k = (uint32_t)(b.hap_off[h + 1] - hoff);
        const uint32_t slot = it % nslot, pslot = (it + nslot - 1) % nslot;
        double* ring = ring_of(w, slot);
        const double* pring = ring_of(w, pslot);

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
                for (int q = lane; q < (kRing + 1) * 4; q += kWave) st_relaxed(ring + q, -0.0);
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
        const uint32_t c0 = tile * (uint32_t)kLongTile + (uint32_t)lane * N;
        uint32_t hc[kLongWords];
#pragma unroll
        for (int q = 0; q < kLongWords; ++q) hc[q] = 0u;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const uint32_t j = c0 + (uint32_t)n;
            const uint32_t code = j < k ? hap_code(b.haps[hoff + j]) : kPadCode;
            hc[n / 4] |= code << (8 * (n % 4));
        }
        const double minit = 1.0 / (double)k;
        const int g0 = b.gq[roff];
        const double* pw0 = t.pwlong + (size_t)g0 * kPowStride;
        ScanMul<double> mul = make_scan_mul<double>(pw0, lane, 0);
        double gcur = t.p64[g0], gprev = gcur, gN1 = pw0[65], gN = pw0[1];
        const ScanMul<double> ones = make_sum_mul<double>(lane, 0);

        // rows alternate between the (Ma, Ia) and (Mb, Ib) register sets
        double Ma[N], Ia[N], Mb[N], Ib[N];
#pragma unroll
        for (int n = 0; n < N; ++n) { Ma[n] = 0.0; Ia[n] = 0.0; Mb[n] = 0.0; Ib[n] = 0.0; }
        double Mleft = 0.0, Ileft = 0.0, C = 0.0;
        long long E = 0;
        // producer records buffered one per lane: rows rb .. rb+nvalid-1
        double bM = 0.0, bI = 0.0, bP = 0.0, bE = 0.0;
        int rb = 0, nvalid = 0;
        uint32_t prog_seen = 0;

        for (int i0 = 0; i0 < l && !dead; i0 += kWave) {
            __syncthreads();
            {
                const int i = i0 + lane;
                if (i < l) {
                    const uint64_t a = roff + (uint64_t)i;
                    const double eps = t.p64[b.bq[a]];
                    const double tmi = t.p64[b.iq[a]];
                    const double tmd_prev = i > 0 ? t.p64[b.dq[a - 1]] : 0.0;
                    const int gc = b.gq[a];
                    const double g = t.p64[gc];
                    const double tmd = t.p64[b.dq[a]];
                    double tmm = 1.0 - (tmi + tmd);
                    tmm = tmm < 0.0 ? 0.0 : tmm;
                    const double pm = 1.0 - eps, px = eps / 3.0, tim = 1.0 - g;
                    LRec rr;
                    rr.dp = pm - px;
                    rr.px = px;
                    rr.tmm = tmm;
                    rr.tim = tim;
                    rr.cd = tim * tmd_prev;
                    rr.tmi = tmi;
                    rr.tii = g;
                    rr.pm = pm;
                    rec[lane] = rr;
                    rinfo[lane] = read_base_index(b.reads[a]) | (gc << 16);
                }
            }
            __syncthreads();
            const int nrows = l - i0 < kWave ? l - i0 : kWave;
            // one row: Mp/Ip name the register set that receives row i
            auto do_row = [&](int tt, const double(&Mi)[N], const double(&Ii)[N], double(&Mp)[N],
                              double(&Ip)[N]) -> bool {
                const int i = i0 + tt;
                const LRec c = rec[tt];
                const int info = __builtin_amdgcn_readfirstlane(rinfo[tt]);
                const int gc = info >> 16;
                if (gc != g0 || gprev != gcur) {  // per-row gap continuation
                    gprev = gcur;
                    gcur = t.p64[gc];
                    const double* pwi = t.pwlong + (size_t)gc * kPowStride;
                    mul = make_scan_mul<double>(pwi, lane, 0);
                    gN1 = pwi[65];
                    gN = pwi[1];
                }
                double Vp;
                const int bidx = info & 0xff;
                if (i == 0) lrow_first(Mp, Ip, hc, bidx, c, minit, gcur, Vp);
                else lrow_step(Mi, Ii, Mp, Ip, hc, bidx, c, Mleft, Ileft, C, gprev, gcur, Vp);
                double nbM = 0.0, nbI = 0.0, nbP = 0.0;
                if (has_prod) {
                    if (i >= rb + nvalid) {  // refill the record buffer
                        if (lane == 0) st_u32<__ATOMIC_RELAXED>(&ss.prog[pslot], (uint32_t)i);
                        uint32_t spins = 0;
                        for (;;) {
                            const int row = i + lane;
                            const uint32_t par = ((uint32_t)row / kRing) & 1u;
                            const double* rp = pring + (size_t)((uint32_t)row % kRing) * 4;
                            bool ok = false;
                            if (row < l) {
                                bM = ld_relaxed(rp + 0);
                                bI = ld_relaxed(rp + 1);
                                bP = ld_relaxed(rp + 2);
                                bE = ld_relaxed(rp + 3);
                                ok = parity_of(bM) == par && parity_of(bI) == par &&
                                     parity_of(bP) == par && parity_of(bE) == par;
                            }
                            const uint64_t okm = __ballot(ok);
                            const int lead = okm == ~0ull ? 64 : __builtin_ctzll(~okm);
                            if (lead > 0) { rb = i; nvalid = lead; break; }
                            if (++spins > spin_limit) { raise_timeout(w); dead = true; break; }
                            if ((spins & 63u) == 0u && aborted(w)) { dead = true; break; }
                            __builtin_amdgcn_s_sleep(1);
                        }
                        if (dead) return false;
                    }
                    const int q = i - rb;
                    const long long Ep = (long long)(magnitude(rd_lane(bE, q)) - kExpBias);
                    const double rM = magnitude(rd_lane(bM, q)), rI = magnitude(rd_lane(bI, q));
                    const double rP = magnitude(rd_lane(bP, q));
                    // Within a tile values fall by T_DD per column away from the
                    // alignment band, so a neighbour's boundary can sit far above
                    // this tile's scale (this tile's own values are then
                    // negligible).  Rebase before converting so the record stays
                    // representable.
                    const double mrec = fmax(rM, fmax(rI, rP));
                    if (mrec > 0.0) {
                        int er;
                        frexp(mrec, &er);
                        if (Ep + er - E > kRebaseBits) {
                            const long long enew = Ep + er;
                            const double f = ldexp(1.0, (int)max(E - enew, -2000LL));
#pragma unroll
                            for (int n = 0; n < N; ++n) { Mp[n] *= f; Ip[n] *= f; }
                            Vp *= f;
                            E = enew;
                        }
                    }
                    const int sh = (int)max(min(Ep - E, 2000LL), -2000LL);
                    nbM = ldexp(rM, sh);
                    nbI = ldexp(rI, sh);
                    nbP = ldexp(rP, sh);
                }
                Mleft = dpp<kWaveShr1>(Mp[N - 1]);
                Ileft = dpp<kWaveShr1>(Ip[N - 1]);
                if (lane == 0) { Mleft = nbM; Ileft = nbI; }
                const double vsh = __builtin_fma(gN1, Mleft, Vp);
                double u = dpp<kWaveShr1>(vsh);
                if (lane == 0) u = nbP;
                C = seg_scan(u, mul);
                if (has_cons) {  // publish row i for the next tile
                    const double P = __builtin_fma(gN, C, vsh);
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
                        double* rp = ring + (size_t)((uint32_t)i % kRing) * 4;
                        st_relaxed(rp + 0, with_parity(Mp[N - 1], par));
                        st_relaxed(rp + 1, with_parity(Ip[N - 1], par));
                        st_relaxed(rp + 2, with_parity(P, par));
                        st_relaxed(rp + 3, with_parity((double)E + kExpBias, par));
                    }
                }
                if ((i % kRescaleRows) == kRescaleRows - 1) {
                    double mx = C > Mleft ? C : Mleft;
                    mx = mx > Ileft ? mx : Ileft;
#pragma unroll
                    for (int n = 0; n < N; ++n) {
                        mx = mx > Mp[n] ? mx : Mp[n];
                        mx = mx > Ip[n] ? mx : Ip[n];
                    }
                    int ex = 0;
                    if (mx > 0.0) { frexp(mx, &ex); ex += 4096; }
                    const int emax = wave_max_int(ex);
                    if (emax > 0) {
                        const int e = emax - 4096;
                        const double f = ldexp(1.0, -e);
#pragma unroll
                        for (int n = 0; n < N; ++n) { Mp[n] *= f; Ip[n] *= f; }
                        Mleft *= f;
                        Ileft *= f;
                        C *= f;
                        E += e;
                    }
                }
                return true;
            };
            int tt = 0;
            for (; tt + 1 < nrows; tt += 2) {
                if (!do_row(tt, Ma, Ia, Mb, Ib)) break;
                if (!do_row(tt + 1, Mb, Ib, Ma, Ia)) break;
            }
            if (!dead && tt < nrows) {
                if (do_row(tt, Ma, Ia, Mb, Ib)) {
#pragma unroll
                    for (int n = 0; n < N; ++n) { Ma[n] = Mb[n]; Ia[n] = Ib[n]; }
                }
            }
        }
        if (__ballot(dead) != 0ull) break;

        // ---- eq.4 over this tile's real columns, then accumulate along the tiles
        double sp = 0.0;
#pragma unroll
        for (int n = 0; n < N; ++n)
            if (c0 + (uint32_t)n < k) sp += Ma[n] + Ia[n];
        sp = seg_scan(sp, ones);
        double am = rd_lane(sp, 63);
        long long aE = E;
        if (has_prod) {
            uint32_t spins = 0;
            double fm = 0.0, fe = 0.0;
            for (;;) {
                fm = ld_relaxed(pring + (size_t)kRing * 4 + 0);
                fe = ld_relaxed(pring + (size_t)kRing * 4 + 1);
                const bool ok = parity_of(fm) == 0u && parity_of(fe) == 0u;
                if (__builtin_amdgcn_readfirstlane((int)ok)) break;
                if (++spins > spin_limit) { raise_timeout(w); dead = true; break; }
                if ((spins & 63u) == 0u && aborted(w)) { dead = true; break; }
                __builtin_amdgcn_s_sleep(2);
            }
            if (dead) break;
            fm = rd_lane(fm, 0);
            fe = rd_lane(fe, 0);
            acc_add(am, aE, magnitude(fm), (long long)(magnitude(fe) - kExpBias));
            // the producer's ring has been read completely
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0) st_u32<__ATOMIC_RELEASE>(&ss.done[pslot], it);
        }
        if (has_cons) {
            if (lane == 0) {
                st_relaxed(ring + (size_t)kRing * 4 + 0, with_parity(am, 0u));
                st_relaxed(ring + (size_t)kRing * 4 + 1, with_parity((double)aE + kExpBias, 0u));
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
            if (b.flags) b.flags[pair] = 0x04 | 0x08 | 0x10;  // long, rescaled, FP64
        }
    }
}

void launch_long(hipStream_t s, int grid, const Batch& b, const Tables& t, const Work& w,
                 const Policy& p)
{
    hipLaunchKernelGGL(long_prefix_kernel, dim3(1), dim3(256), 0, s, b, w, long_slots(grid));
    hipLaunchKernelGGL(long_kernel, dim3(grid), dim3(kWave), 0, s, b, t, w, p);
}

const void* long_kernel_ptr() { return reinterpret_cast<const void*>(&long_kernel); }

}  // namespace phmm
