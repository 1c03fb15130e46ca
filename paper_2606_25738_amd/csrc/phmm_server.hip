// Serving runtime: a request loop over active regions with continuous
// batching (host code only).
//
// A region (the reads, haplotypes and pairs of one active region) is
// submitted from any host thread and copied at once, so the caller's buffers
// can be reused.  Lanes run batches: each lane owns a HIP stream, a context,
// a device block and a pinned host block of (HBM budget / lanes) bytes.  A
// lane's worker thread takes as many waiting regions as fit its device block
// (admission by HBM budget), lays them out as one batch, copies the inputs
// to the device in one transfer, runs the forward pass stream-ordered, copies
// the results back and completes the regions.  Regions that arrive while a
// batch runs are taken by the next free lane, so batches of several lanes
// overlap on the device; the inputs and results of a batch stay resident in
// its lane's device block for the whole pass.
//
// Regions whose longest haplotype exceeds the short kernel's reach, or whose
// longest read exceeds long_read_min bases, are long regions.  With
// long_lanes > 0 they queue separately and only those lanes take them, so a
// short region never waits behind a long one inside a batch, and the long
// lanes' persistent grids are capped at long_grid_percent of the chip, so a
// long batch leaves wavefront slots on every compute unit for the short
// lanes' kernels.  Optional CU masks give the short lanes and the long lanes
// disjoint compute units instead.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "phmm.h"
#include "phmm_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Request {
    uint64_t ticket = 0;
    bool is_long = false;
    uint64_t rb = 0, hb = 0, nr = 0, nh = 0, np = 0, cells = 0;
    uint32_t max_l = 0, max_k = 0;
    std::vector<uint8_t> seq;       // reads | bq | iq | dq | gq (5 x rb), then haps (hb)
    std::vector<uint64_t> ro, ho;   // local offsets, n + 1 entries
    std::vector<uint32_t> pairs;    // 2 x np, local indices
    std::vector<double> out;
    std::vector<uint8_t> flags;
    int status = 1;                 // 1 pending, 0 done, < 0 error code
    uint32_t lane = 0;
    uint64_t batch = 0;
    Clock::time_point t_submit, t_launch, t_done;
};

// Byte layout of one batch in a lane's blocks (the host block mirrors the
// input part so one transfer moves all inputs).
struct BatchLayout {
    size_t reads, ro, haps, ho, pl, in_end, out, fl, out_end, ctr, ws, total;
};

BatchLayout layout_of(phmm_ctx* ctx, uint64_t rb, uint64_t nr, uint64_t hb, uint64_t nh,
                      uint64_t np, uint32_t max_l, uint32_t max_k)
{
    BatchLayout L;
    size_t o = 0;
    L.reads = o; o = align256(o + 5 * rb);
    L.ro = o; o = align256(o + (nr + 1) * 8);
    L.haps = o; o = align256(o + hb);
    L.ho = o; o = align256(o + (nh + 1) * 8);
    L.pl = o; o = align256(o + np * 8);
    L.in_end = o;
    L.out = o; o = align256(o + np * 8);
    L.fl = o; o = align256(o + np);
    L.out_end = o;
    L.ctr = o; o = align256(o + sizeof(phmm::Counters));  // host copy of the device counters
    L.ws = o; o = align256(o + phmm_workspace_bytes(ctx, np, max_l, max_k));
    L.total = o;
    return L;
}

}  // namespace

struct phmm_server {
    int device = 0;
    phmm_server_options opt{};
    struct Lane {
        hipStream_t stream = nullptr;
        phmm_ctx* ctx = nullptr;
        void* dev = nullptr;
        void* host = nullptr;
        size_t bytes = 0;
        bool is_long = false;
        std::thread worker;
    };
    std::vector<std::unique_ptr<Lane>> lanes;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> q_short, q_long;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> reqs;
    uint64_t next_ticket = 1, next_batch = 1;
    bool stop = false;
    int cu_mask_status = 0;  // 1 lane streams CU-masked, < 0 HIP error while applying
    // statistics
    uint64_t done_regions = 0, done_pairs = 0, done_cells = 0, batches = 0, full_batches = 0;
    double busy_s = 0.0;
    Clock::time_point t_first{}, t_last{};
    bool any = false;

    void worker(Lane* lane, uint32_t lane_id);
};

extern "C" void phmm_server_default_options(phmm_server_options* o)
{
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->precision = PHMM_FP32_RERUN;
    o->lanes = 3;
    o->long_lanes = 1;
    o->hbm_budget_bytes = 24ull << 30;
    o->max_batch_regions = 8192;
    o->short_cu_percent = 0;
    o->long_read_min = 512;
    o->long_grid_percent = 25;
}

void phmm_server::worker(Lane* lane, uint32_t lane_id)
{
    (void)hipSetDevice(device);
    std::deque<std::shared_ptr<Request>>& q = lane->is_long ? q_long : q_short;
    for (;;) {
        std::vector<std::shared_ptr<Request>> batch;
        uint64_t batch_id = 0;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !q.empty(); });
            if (q.empty()) return;  // stopping, and nothing left to run
            std::deque<std::shared_ptr<Request>>& src = q;
            // admission: take waiting regions in order while the batch fits
            uint64_t rb = 0, hb = 0, nr = 0, nh = 0, np = 0;
            uint32_t ml = 0, mk = 0;
            while (!src.empty() && batch.size() < opt.max_batch_regions) {
                const auto& r = src.front();
                const BatchLayout L = layout_of(lane->ctx, rb + r->rb, nr + r->nr, hb + r->hb,
                                                nh + r->nh, np + r->np, std::max(ml, r->max_l),
                                                std::max(mk, r->max_k));
                if (L.total > lane->bytes) break;
                rb += r->rb; hb += r->hb; nr += r->nr; nh += r->nh; np += r->np;
                ml = std::max(ml, r->max_l);
                mk = std::max(mk, r->max_k);
                batch.push_back(r);
                src.pop_front();
            }
            batch_id = next_batch++;
            if (!src.empty()) ++full_batches;
        }
        if (batch.empty()) continue;  // (cannot happen: submit rejects regions over a lane)
        const Clock::time_point t_launch = Clock::now();
        // ---- lay the batch out in the pinned host block
        uint64_t rb = 0, hb = 0, nr = 0, nh = 0, np = 0;
        uint32_t ml = 0, mk = 0;
        for (const auto& r : batch) {
            rb += r->rb; hb += r->hb; nr += r->nr; nh += r->nh; np += r->np;
            ml = std::max(ml, r->max_l);
            mk = std::max(mk, r->max_k);
        }
        const BatchLayout L = layout_of(lane->ctx, rb, nr, hb, nh, np, ml, mk);
        char* H = static_cast<char*>(lane->host);
        char* D = static_cast<char*>(lane->dev);
        uint64_t* ro = reinterpret_cast<uint64_t*>(H + L.ro);
        uint64_t* ho = reinterpret_cast<uint64_t*>(H + L.ho);
        uint32_t* pl = reinterpret_cast<uint32_t*>(H + L.pl);
        uint64_t ob = 0, oh = 0, oread = 0, ohap = 0, opair = 0;
        for (const auto& r : batch) {
            for (int a = 0; a < 5; ++a)
                memcpy(H + L.reads + a * rb + ob, r->seq.data() + a * r->rb, r->rb);
            memcpy(H + L.haps + oh, r->seq.data() + 5 * r->rb, r->hb);
            for (uint64_t i = 0; i < r->nr; ++i) ro[oread + i] = ob + r->ro[i];
            for (uint64_t i = 0; i < r->nh; ++i) ho[ohap + i] = oh + r->ho[i];
            for (uint64_t p = 0; p < r->np; ++p) {
                pl[2 * (opair + p)] = (uint32_t)(oread + r->pairs[2 * p]);
                pl[2 * (opair + p) + 1] = (uint32_t)(ohap + r->pairs[2 * p + 1]);
            }
            ob += r->rb; oh += r->hb; oread += r->nr; ohap += r->nh; opair += r->np;
        }
        ro[nr] = rb;
        ho[nh] = hb;
        // ---- one transfer in, the pass, one transfer out
        int rc = PHMM_OK;
        if (hipMemcpyAsync(D, H, L.in_end, hipMemcpyHostToDevice, lane->stream) != hipSuccess)
            rc = PHMM_EDEVICE;
        phmm_device_batch db;
        db.reads = reinterpret_cast<const uint8_t*>(D + L.reads);
        db.base_quals = db.reads + rb;
        db.ins_quals = db.reads + 2 * rb;
        db.del_quals = db.reads + 3 * rb;
        db.gcp = db.reads + 4 * rb;
        db.read_offsets = reinterpret_cast<const uint64_t*>(D + L.ro);
        db.n_reads = (uint32_t)nr;
        db.haplotypes = reinterpret_cast<const uint8_t*>(D + L.haps);
        db.hap_offsets = reinterpret_cast<const uint64_t*>(D + L.ho);
        db.n_haps = (uint32_t)nh;
        db.pair_list = reinterpret_cast<const uint32_t*>(D + L.pl);
        db.n_pairs = np;
        db.max_read_len = ml;
        db.max_hap_len = mk;
        if (rc == PHMM_OK)
            rc = phmm::forward_device_batch_sync(lane->ctx, &db,
                                                 reinterpret_cast<double*>(D + L.out),
                                                 reinterpret_cast<uint8_t*>(D + L.fl), D + L.ws,
                                                 L.total - L.ws, lane->stream);
        // results and the device counters (they open the workspace) come back
        // in two stream-ordered copies; only this lane's stream is waited on
        if (rc == PHMM_OK &&
            (hipMemcpyAsync(H + L.out, D + L.out, L.out_end - L.out, hipMemcpyDeviceToHost,
                            lane->stream) != hipSuccess ||
             hipMemcpyAsync(H + L.ctr, D + L.ws, sizeof(phmm::Counters), hipMemcpyDeviceToHost,
                            lane->stream) != hipSuccess))
            rc = PHMM_EDEVICE;
        if (hipStreamSynchronize(lane->stream) != hipSuccess && rc == PHMM_OK) rc = PHMM_EDEVICE;
        if (rc == PHMM_OK) {
            const phmm::Counters* c = reinterpret_cast<const phmm::Counters*>(H + L.ctr);
            if (c->status != 0) rc = (int)c->status;
        }
        const Clock::time_point t_done = Clock::now();
        // ---- complete the regions
        const double* out = reinterpret_cast<const double*>(H + L.out);
        const uint8_t* fl = reinterpret_cast<const uint8_t*>(H + L.fl);
        std::lock_guard<std::mutex> lk(mu);
        uint64_t p0 = 0;
        for (const auto& r : batch) {
            if (rc == PHMM_OK) {
                r->out.assign(out + p0, out + p0 + r->np);
                r->flags.assign(fl + p0, fl + p0 + r->np);
            }
            p0 += r->np;
            r->status = rc == PHMM_OK ? 0 : rc;
            r->lane = lane_id;
            r->batch = batch_id;
            r->t_launch = t_launch;
            r->t_done = t_done;
            ++done_regions;
            done_pairs += r->np;
            done_cells += r->cells;
            if (!any || r->t_submit < t_first) t_first = r->t_submit;
            any = true;
        }
        if (t_done > t_last) t_last = t_done;
        ++batches;
        busy_s += std::chrono::duration<double>(t_done - t_launch).count();
        cv_done.notify_all();
    }
}

// Stream of a lane, created with a CU mask so that it gets a hardware queue
// of its own: plain streams share the process's few hardware queues (4 by
// default) in turn with every other stream of the process, and a short lane
// that shares one with the long lane waits behind its long kernels (short
// p99 11 ms and maximum 608 ms at 0.8x load in a process that had created
// four streams before the server; 0.38 and 2 ms with a queue per lane).  The
// mask holds every compute unit, or with short_cu_percent the first pct % of
// them for the short lanes and the rest for the long lanes.
static int make_stream(int device, bool is_long, uint32_t pct, hipStream_t* s, int* status)
{
    const bool split = pct > 0 && pct < 100;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PHMM_EDEVICE;
    const uint32_t ncu = (uint32_t)prop.multiProcessorCount;
    const uint32_t nshort = std::max(1u, std::min(ncu - 1, ncu * pct / 100));
    std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
    for (uint32_t c = 0; c < ncu; ++c) {
        const bool mine = !split || (is_long ? c >= nshort : c < nshort);
        if (mine) mask[c / 32] |= 1u << (c % 32);
    }
    hipError_t e = hipExtStreamCreateWithCUMask(s, (uint32_t)mask.size(), mask.data());
    if (e != hipSuccess) {
        *status = -(int)e;
        return hipStreamCreateWithFlags(s, hipStreamNonBlocking) == hipSuccess ? PHMM_OK
                                                                                : PHMM_EDEVICE;
    }
    *status = 1;
    return PHMM_OK;
}

extern "C" void phmm_server_destroy(phmm_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& l : s->lanes)
        if (l->worker.joinable()) l->worker.join();
    (void)hipSetDevice(s->device);
    for (auto& l : s->lanes) {
        if (l->stream) (void)hipStreamSynchronize(l->stream);
        if (l->ctx) phmm_destroy(l->ctx);
        if (l->dev) (void)hipFree(l->dev);
        if (l->host) (void)hipHostFree(l->host);
        if (l->stream) (void)hipStreamDestroy(l->stream);
    }
    delete s;
}

extern "C" int phmm_server_create(phmm_server** out, int device, const phmm_server_options* opt)
{
    if (!out) return phmm::set_error(PHMM_EINVAL, "phmm_server_create: out is NULL");
    *out = nullptr;
    phmm_server_options o;
    phmm_server_default_options(&o);
    if (opt) o = *opt;
    if (o.lanes == 0 || o.lanes > 16 || o.long_lanes >= o.lanes || o.hbm_budget_bytes < (64ull << 20) ||
        o.max_batch_regions == 0 || o.short_cu_percent > 100 || o.long_read_min == 0 ||
        o.long_grid_percent == 0 || o.long_grid_percent > 100 ||
        (o.precision != PHMM_FP32_RERUN && o.precision != PHMM_FP64_PLAIN))
        return phmm::set_error(PHMM_EINVAL, "phmm_server_create: bad options (lanes 1..16, "
                               "long_lanes < lanes, budget >= 64 MiB, short_cu_percent <= 100, "
                               "long_read_min >= 1, long_grid_percent 1..100)");
    auto* s = new phmm_server();
    s->device = device;
    s->opt = o;
    if (hipSetDevice(device) != hipSuccess) {
        delete s;
        return phmm::set_error(PHMM_EDEVICE, "phmm_server_create: no such HIP device");
    }
    const size_t per_lane = align256(o.hbm_budget_bytes / o.lanes);
    int rc = PHMM_OK;
    for (uint32_t i = 0; i < o.lanes && rc == PHMM_OK; ++i) {
        auto lane = std::make_unique<phmm_server::Lane>();
        lane->is_long = o.long_lanes > 0 && i >= o.lanes - o.long_lanes;
        lane->bytes = per_lane;
        phmm_options co;
        phmm_default_options(&co);
        co.precision = o.precision;
        rc = phmm_create(&lane->ctx, device, &co);  // sets the error message itself
        if (rc == PHMM_OK && lane->is_long) phmm::scale_grids(lane->ctx, (int)o.long_grid_percent);
        if (rc == PHMM_OK) rc = make_stream(device, lane->is_long, o.long_lanes ? o.short_cu_percent : 0,
                                            &lane->stream, &s->cu_mask_status);
        if (rc == PHMM_OK && hipMalloc(&lane->dev, per_lane) != hipSuccess)
            rc = phmm::set_error(PHMM_ENOMEM, "phmm_server_create: device block of a lane");
        if (rc == PHMM_OK && hipHostMalloc(&lane->host, per_lane, hipHostMallocDefault) != hipSuccess)
            rc = phmm::set_error(PHMM_ENOMEM, "phmm_server_create: pinned host block of a lane");
        s->lanes.push_back(std::move(lane));
    }
    if (rc != PHMM_OK) {
        phmm_server_destroy(s);
        return rc;
    }
    for (uint32_t i = 0; i < o.lanes; ++i) {
        phmm_server::Lane* l = s->lanes[i].get();
        l->worker = std::thread([s, l, i] { s->worker(l, i); });
    }
    *out = s;
    return PHMM_OK;
}

extern "C" int phmm_server_submit(phmm_server* s, const uint8_t* reads, const uint8_t* bq,
                                  const uint8_t* iq, const uint8_t* dq, const uint8_t* gq,
                                  const uint64_t* ro, uint32_t n_reads, const uint8_t* haps,
                                  const uint64_t* ho, uint32_t n_haps, const uint32_t* pl,
                                  uint64_t n_pairs, uint64_t* ticket)
{
    if (!s || !ticket) return phmm::set_error(PHMM_EINVAL, "phmm_server_submit: NULL server or ticket");
    if (n_pairs == 0) return phmm::set_error(PHMM_EINVAL, "phmm_server_submit: region without pairs");
    uint32_t ml = 0, mk = 0;
    int rc = phmm_validate_batch(reads, bq, iq, dq, gq, ro, n_reads, haps, ho, n_haps, pl, n_pairs,
                                 &ml, &mk);
    if (rc != PHMM_OK) return rc;
    auto r = std::make_shared<Request>();
    r->rb = ro[n_reads];
    r->hb = ho[n_haps];
    r->nr = n_reads;
    r->nh = n_haps;
    r->np = n_pairs;
    r->max_l = ml;
    r->max_k = mk;
    r->is_long = mk > phmm::kShortMaxCols || ml > s->opt.long_read_min;
    const BatchLayout L = layout_of(s->lanes[0]->ctx, r->rb, r->nr, r->hb, r->nh, r->np, ml, mk);
    if (L.total > s->lanes[0]->bytes)
        return phmm::set_error(PHMM_ENOMEM, "phmm_server_submit: region needs more device memory "
                               "than one lane holds (HBM budget / lanes)");
    r->seq.resize(5 * r->rb + r->hb);
    const uint8_t* arr[5] = {reads, bq, iq, dq, gq};
    for (int a = 0; a < 5; ++a) memcpy(r->seq.data() + a * r->rb, arr[a], r->rb);
    memcpy(r->seq.data() + 5 * r->rb, haps, r->hb);
    r->ro.assign(ro, ro + n_reads + 1);
    r->ho.assign(ho, ho + n_haps + 1);
    r->pairs.assign(pl, pl + 2 * n_pairs);
    uint64_t cells = 0;
    for (uint64_t p = 0; p < n_pairs; ++p)
        cells += (ro[pl[2 * p] + 1] - ro[pl[2 * p]]) * (ho[pl[2 * p + 1] + 1] - ho[pl[2 * p + 1]]);
    r->cells = cells;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return phmm::set_error(PHMM_EINVAL, "phmm_server_submit: server is stopping");
        r->ticket = s->next_ticket++;
        r->t_submit = Clock::now();
        s->reqs[r->ticket] = r;
        (r->is_long && s->opt.long_lanes > 0 ? s->q_long : s->q_short).push_back(r);
        *ticket = r->ticket;
    }
    s->cv_work.notify_all();
    return PHMM_OK;
}

static int finish(phmm_server* s, std::shared_ptr<Request> r, double* out, uint8_t* flags,
                  phmm_request_info* info)
{
    if (r->status == 0) {
        if (out) memcpy(out, r->out.data(), r->np * sizeof(double));
        if (flags) memcpy(flags, r->flags.data(), r->np);
    }
    if (info) {
        info->n_pairs = r->np;
        info->cells = r->cells;
        info->lane = r->lane;
        info->batch = r->batch;
        info->queue_s = std::chrono::duration<double>(r->t_launch - r->t_submit).count();
        info->latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
        info->is_long = r->is_long ? 1 : 0;
    }
    s->reqs.erase(r->ticket);
    return r->status;
}

extern "C" int phmm_server_wait(phmm_server* s, uint64_t ticket, double* out_log10,
                                uint8_t* out_flags, phmm_request_info* info)
{
    if (!s) return phmm::set_error(PHMM_EINVAL, "phmm_server_wait: server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return phmm::set_error(PHMM_EINVAL, "phmm_server_wait: unknown ticket");
    std::shared_ptr<Request> r = it->second;
    s->cv_done.wait(lk, [&] { return r->status != 1; });
    return finish(s, r, out_log10, out_flags, info);
}

extern "C" int phmm_server_poll(phmm_server* s, uint64_t ticket, double* out_log10,
                                uint8_t* out_flags, phmm_request_info* info)
{
    if (!s) return phmm::set_error(PHMM_EINVAL, "phmm_server_poll: server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return phmm::set_error(PHMM_EINVAL, "phmm_server_poll: unknown ticket");
    if (it->second->status == 1) return PHMM_PENDING;
    return finish(s, it->second, out_log10, out_flags, info);
}

extern "C" int phmm_server_stats(phmm_server* s, phmm_server_counters* st)
{
    if (!s || !st) return PHMM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    memset(st, 0, sizeof *st);
    st->regions = s->done_regions;
    st->pairs = s->done_pairs;
    st->cells = s->done_cells;
    st->batches = s->batches;
    st->full_batches = s->full_batches;
    st->waiting_short = s->q_short.size();
    st->waiting_long = s->q_long.size();
    st->lane_busy_s = s->busy_s;
    st->span_s = s->any ? std::chrono::duration<double>(s->t_last - s->t_first).count() : 0.0;
    st->cu_mask_status = s->cu_mask_status;
    return PHMM_OK;
}
