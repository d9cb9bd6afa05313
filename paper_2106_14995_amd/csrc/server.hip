// server.hip -- continuous-batching solve server (C ABI in include/tron.h).
//
// Requests (a batch of instances each, sizes mixed) are queued by any host thread. One
// scheduler thread owned by the server:
//   * admits queued requests in arrival order while they fit the device-memory budget (a
//     preallocated device arena, first-fit) and the in-flight LDS budget, coalescing
//     consecutive requests into one launch group up to a group size cap;
//   * launches each group on one of its streams: one host-to-device copy of the group's
//     packed inputs (from pinned staging), the size-bucketed solve kernels (lane kernels for
//     n <= 8, wavefront kernels above), one device-to-host copy of the outputs, an event;
//   * polls the events of all groups on the device and completes them out of order, freeing
//     their memory at once so the next queued requests are admitted while others still run.
// Requests naming a session keep that session's solution, radius and Cauchy step resident
// in device memory; a later request of the same session can start from them (x0 = NULL).
// The work of different groups overlaps on the GPU through the stream pool.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tron.h"
#include "tron_internal.hpp"

namespace {

using clock_t_ = std::chrono::steady_clock;

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// first-fit allocator over [0, size)
class Arena {
public:
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes ? bytes : 1);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

int wave_nmax_of(int n) { return n <= 16 ? 16 : n <= 32 ? 32 : n <= 64 ? 64 : 128; }

struct Session {
    std::vector<int32_t> n;
    int64_t nsum = 0;
    size_t off = 0, bytes = 0;  // device: x (nsum), state (2 * batch)
    bool valid = false;         // holds a finished solve
    int outstanding = 0;        // requests queued or on the device (at most one)
};

struct Request {
    int64_t ticket = 0;
    int64_t batch = 0, nsum = 0, psum = 0;
    std::vector<int32_t> n;
    std::vector<double> params, lo, hi, x0;
    bool has_x0 = true;
    uint64_t session = 0;
    size_t lds = 0;
    int state = 0;  // 0 queued, 1 on the device, 2 done
    tron_err err = TRON_OK;  // done without a solve: why (the result call reports it)
    bool cancelled = false;  // taken off the queue by tron_server_cancel
    // session placement, copied at admission (the scheduler never reads the session map
    // outside the lock)
    size_t sess_off = 0;
    int64_t sess_nsum = 0;
    bool sess_warm = false;
    clock_t_::time_point t_submit, t_done;
    std::vector<double> x, f;
    std::vector<int32_t> status, iters;
    // placement inside its group
    int64_t b0 = 0, v0 = 0, p0 = 0;
};

// byte layout of a group: inputs first (one upload), then outputs (one download)
struct Layout {
    size_t params, lo, hi, x0, state, nper, poff, voff, index, in_end;
    size_t x, f, status, iters, out_end;
    void build(int64_t B, int64_t nsum, int64_t psum)
    {
        size_t o = 0;
        auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes); return at; };
        params = take(sizeof(double) * psum);
        lo = take(sizeof(double) * nsum);
        hi = take(sizeof(double) * nsum);
        x0 = take(sizeof(double) * nsum);
        state = take(sizeof(double) * 2 * B);
        nper = take(sizeof(int32_t) * B);
        poff = take(sizeof(int64_t) * B);
        voff = take(sizeof(int64_t) * B);
        index = take(sizeof(int32_t) * B);
        in_end = o;
        x = take(sizeof(double) * nsum);
        f = take(sizeof(double) * B);
        status = take(sizeof(int32_t) * B);
        iters = take(sizeof(int32_t) * B);
        out_end = o;
    }
};

struct BucketSeg {
    int nmax, lanes;
    int64_t off, count;
};

struct Group {
    std::vector<Request *> reqs;
    int64_t B = 0, nsum = 0, psum = 0;
    size_t lds = 0;
    Layout lay{};
    size_t dev_off = 0, stage_off = 0, bytes = 0;
    int stream = 0;
    hipEvent_t done = nullptr;
    std::vector<BucketSeg> buckets;
};

}  // namespace

struct tron_server {
    tron_family fam = TRON_FAMILY_QP4;
    tron_server_config cfg{};
    int device = 0;
    char *d_base = nullptr;   // device arena
    char *h_stage = nullptr;  // pinned staging, same size as the device arena
    Arena dev, stage;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;  // free events

    std::mutex mu;
    std::condition_variable cv;      // scheduler wake-up
    std::condition_variable done_cv; // waiters
    std::deque<Request *> queue;
    std::vector<Group *> inflight;
    std::unordered_map<int64_t, std::unique_ptr<Request>> tickets;
    std::unordered_map<uint64_t, Session> sessions;
    size_t session_bytes = 0;  // device arena bytes held by resident sessions
    size_t lds_inflight = 0;
    int64_t next_ticket = 1;
    int64_t done_requests = 0, done_instances = 0;
    int next_stream = 0;
    bool stop = false;
    std::thread worker;
    tron_err worker_err = TRON_OK;
};

namespace {

int64_t param_size(tron_family fam, int n) { return tron_param_size(fam, n); }

size_t request_device_bytes(const Request &r)
{
    Layout l;
    l.build(r.batch, r.nsum, r.psum);
    return l.out_end;
}

// Fill the group's staging inputs, its plan (buckets and index lists) and its offsets.
void stage_group(tron_server *s, Group *g)
{
    char *h = s->h_stage + g->stage_off;
    const Layout &L = g->lay;
    double *params = (double *)(h + L.params), *lo = (double *)(h + L.lo), *hi = (double *)(h + L.hi);
    double *x0 = (double *)(h + L.x0), *state = (double *)(h + L.state);
    int32_t *nper = (int32_t *)(h + L.nper), *index = (int32_t *)(h + L.index);
    int64_t *poff = (int64_t *)(h + L.poff), *voff = (int64_t *)(h + L.voff);
    std::vector<int32_t> all_n;
    all_n.reserve(g->B);
    for (Request *r : g->reqs) {
        std::memcpy(params + r->p0, r->params.data(), sizeof(double) * r->psum);
        std::memcpy(lo + r->v0, r->lo.data(), sizeof(double) * r->nsum);
        std::memcpy(hi + r->v0, r->hi.data(), sizeof(double) * r->nsum);
        if (r->has_x0) std::memcpy(x0 + r->v0, r->x0.data(), sizeof(double) * r->nsum);
        int64_t pa = r->p0, va = r->v0;
        for (int64_t i = 0; i < r->batch; i++) {
            const int ni = r->n[i];
            nper[r->b0 + i] = ni;
            poff[r->b0 + i] = pa;
            voff[r->b0 + i] = va;
            pa += param_size(s->fam, ni);
            va += ni;
            all_n.push_back(ni);
        }
    }
    for (int64_t b = 0; b < 2 * g->B; b++) state[b] = 0.0;  // cold unless a session overwrites it
    // buckets: wave kernels (largest first) then lane kernels of each exact n
    std::vector<std::vector<int32_t>> wave(4), lane(9);
    for (int64_t b = 0; b < g->B; b++) {
        const int ni = all_n[b];
        if (ni <= 8) lane[ni].push_back((int32_t)b);
        else {
            const int w = wave_nmax_of(ni);
            wave[w == 16 ? 0 : w == 32 ? 1 : w == 64 ? 2 : 3].push_back((int32_t)b);
        }
    }
    int64_t off = 0;
    g->buckets.clear();
    for (int w = 3; w >= 0; w--) {
        auto &v = wave[w];
        if (v.empty()) continue;
        std::stable_sort(v.begin(), v.end(), [&](int32_t a, int32_t b) { return all_n[a] > all_n[b]; });
        std::memcpy(index + off, v.data(), sizeof(int32_t) * v.size());
        g->buckets.push_back({16 << w, 64, off, (int64_t)v.size()});
        off += (int64_t)v.size();
    }
    for (int k = 8; k >= 1; k--) {
        auto &v = lane[k];
        if (v.empty()) continue;
        std::memcpy(index + off, v.data(), sizeof(int32_t) * v.size());
        g->buckets.push_back({k, 1, off, (int64_t)v.size()});
        off += (int64_t)v.size();
    }
}

tron_err launch_group(tron_server *s, Group *g)
{
    hipStream_t st = s->streams[g->stream];
    char *d = s->d_base + g->dev_off;
    char *h = s->h_stage + g->stage_off;
    const Layout &L = g->lay;
    HIP_TRY(hipMemcpyAsync(d, h, L.in_end, hipMemcpyHostToDevice, st));
    // sessions: warm start from the resident solution / radius / Cauchy step
    for (Request *r : g->reqs) {
        if (!r->session || !r->sess_warm) continue;
        char *sd = s->d_base + r->sess_off;
        if (!r->has_x0)
            HIP_TRY(hipMemcpyAsync(d + L.x0 + sizeof(double) * r->v0, sd, sizeof(double) * r->nsum,
                                   hipMemcpyDeviceToDevice, st));
        const size_t so = align_up(sizeof(double) * r->sess_nsum);
        HIP_TRY(hipMemcpyAsync(d + L.state + sizeof(double) * r->b0, sd + so, sizeof(double) * r->batch,
                               hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(d + L.state + sizeof(double) * (g->B + r->b0), sd + so + sizeof(double) * r->batch,
                               sizeof(double) * r->batch, hipMemcpyDeviceToDevice, st));
    }
    LaneArgs a{};
    a.params = (const double *)(d + L.params);
    a.lo = (const double *)(d + L.lo);
    a.hi = (const double *)(d + L.hi);
    a.x0 = (const double *)(d + L.x0);
    a.x = (double *)(d + L.x);
    a.f = (double *)(d + L.f);
    a.status = (int32_t *)(d + L.status);
    a.iters = (int32_t *)(d + L.iters);
    a.state = (double *)(d + L.state);
    a.ts = nullptr;
    a.nper = (const int32_t *)(d + L.nper);
    a.poff = (const int64_t *)(d + L.poff);
    a.voff = (const int64_t *)(d + L.voff);
    a.batch = g->B;
    a.n_uniform = 0;
    a.psize = 0;
    a.opt.gtol = s->cfg.opt.gtol;
    a.opt.cg_rtol = s->cfg.opt.cg_rtol;
    a.opt.delta0 = s->cfg.opt.delta0;
    a.opt.max_iter = s->cfg.opt.max_iter;
    a.opt.warm = 1;  // cold instances carry a zero radius, which selects the cold rule
    for (const BucketSeg &b : g->buckets) {
        a.index = (const int32_t *)(d + L.index) + b.off;
        a.count = b.count;
        if (b.lanes == 1) {
            lane_launch_fn fn = mt_lane_launcher(s->fam, b.nmax);
            if (!fn) return mt_fail(TRON_ERR_UNSUPPORTED, "n = %d unsupported", b.nmax);
            fn(a, st);
        } else {
            mt_launch_wave(s->fam, a, b.nmax, st);
        }
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h + L.in_end, d + L.in_end, L.out_end - L.in_end, hipMemcpyDeviceToHost, st));
    for (Request *r : g->reqs) {
        if (!r->session) continue;
        char *sd = s->d_base + r->sess_off;
        const size_t so = align_up(sizeof(double) * r->sess_nsum);
        HIP_TRY(hipMemcpyAsync(sd, d + L.x + sizeof(double) * r->v0, sizeof(double) * r->nsum,
                               hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(sd + so, d + L.state + sizeof(double) * r->b0, sizeof(double) * r->batch,
                               hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(sd + so + sizeof(double) * r->batch, d + L.state + sizeof(double) * (g->B + r->b0),
                               sizeof(double) * r->batch, hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(hipEventRecord(g->done, st));
    return TRON_OK;
}

void complete_group(tron_server *s, Group *g)
{
    const char *h = s->h_stage + g->stage_off;
    const Layout &L = g->lay;
    const double *x = (const double *)(h + L.x), *f = (const double *)(h + L.f);
    const int32_t *status = (const int32_t *)(h + L.status), *iters = (const int32_t *)(h + L.iters);
    const auto now = clock_t_::now();
    for (Request *r : g->reqs) {
        r->x.assign(x + r->v0, x + r->v0 + r->nsum);
        r->f.assign(f + r->b0, f + r->b0 + r->batch);
        r->status.assign(status + r->b0, status + r->b0 + r->batch);
        r->iters.assign(iters + r->b0, iters + r->b0 + r->batch);
        r->t_done = now;
        r->state = 2;
        if (r->session) {
            auto it = s->sessions.find(r->session);
            if (it != s->sessions.end()) {
                it->second.valid = true;
                it->second.outstanding--;
            }
        }
        s->done_requests++;
        s->done_instances += r->batch;
        std::vector<double>().swap(r->params);
        std::vector<double>().swap(r->lo);
        std::vector<double>().swap(r->hi);
        std::vector<double>().swap(r->x0);
    }
    s->dev.release(g->dev_off, g->bytes);
    s->stage.release(g->stage_off, g->bytes);
    s->lds_inflight -= g->lds;
    s->events.push_back(g->done);
    delete g;
}

// Under the lock: take queued requests (in order) into one group if they fit now.
Group *admit_group(tron_server *s)
{
    if (s->queue.empty() || (int)s->inflight.size() >= s->cfg.max_inflight || s->events.empty()) return nullptr;
    Group *g = new Group();
    int64_t B = 0, nsum = 0, psum = 0;
    size_t lds = 0;
    size_t take = 0;
    for (Request *r : s->queue) {
        if (take > 0 && (!s->cfg.coalesce || B + r->batch > s->cfg.max_group_instances)) break;
        Layout l;
        l.build(B + r->batch, nsum + r->nsum, psum + r->psum);
        const size_t need = l.out_end;
        const bool fits_mem = s->dev.used() + need <= s->cfg.hbm_budget;
        const bool fits_lds = s->lds_inflight + lds + r->lds <= s->cfg.lds_budget || (s->lds_inflight == 0 && take == 0);
        if (!fits_mem || !fits_lds) break;
        r->b0 = B;
        r->v0 = nsum;
        r->p0 = psum;
        B += r->batch;
        nsum += r->nsum;
        psum += r->psum;
        lds += r->lds;
        take++;
    }
    if (take == 0) {
        delete g;
        return nullptr;
    }
    g->lay.build(B, nsum, psum);
    g->bytes = g->lay.out_end;
    if (!s->dev.alloc(g->bytes, &g->dev_off)) {
        delete g;
        return nullptr;
    }
    if (!s->stage.alloc(g->bytes, &g->stage_off)) {
        s->dev.release(g->dev_off, g->bytes);
        delete g;
        return nullptr;
    }
    for (size_t i = 0; i < take; i++) {
        Request *r = s->queue.front();
        s->queue.pop_front();
        r->state = 1;
        if (r->session) {
            const Session &ss = s->sessions[r->session];
            r->sess_off = ss.off;
            r->sess_nsum = ss.nsum;
            r->sess_warm = ss.valid;
        }
        g->reqs.push_back(r);
    }
    g->B = B;
    g->nsum = nsum;
    g->psum = psum;
    g->lds = lds;
    s->lds_inflight += lds;
    g->stream = s->next_stream;
    s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
    g->done = s->events.back();
    s->events.pop_back();
    return g;
}

void scheduler(tron_server *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        bool progress = false;
        // complete finished groups (in any order)
        for (size_t i = 0; i < s->inflight.size();) {
            if (hipEventQuery(s->inflight[i]->done) == hipSuccess) {
                complete_group(s, s->inflight[i]);
                s->inflight.erase(s->inflight.begin() + i);
                progress = true;
            } else {
                i++;
            }
        }
        if (progress) s->done_cv.notify_all();
        // admit and launch as many groups as fit now; the group is owned by this thread
        // once admitted, so its staging and launch run without the lock
        for (;;) {
            Group *g = admit_group(s);
            if (!g) break;
            lk.unlock();
            stage_group(s, g);
            const tron_err rc = launch_group(s, g);
            lk.lock();
            if (rc != TRON_OK) s->worker_err = rc;
            s->inflight.push_back(g);
            progress = true;
        }
        // Nothing on the device and the head request still cannot be placed: only resident
        // sessions hold arena memory now (or leave it fragmented), and waiting frees none,
        // so the request fails instead of blocking its waiter forever.
        if (!progress && s->inflight.empty() && !s->queue.empty()) {
            Request *r = s->queue.front();
            s->queue.pop_front();
            r->err = TRON_ERR_BUSY;
            r->state = 2;
            r->t_done = clock_t_::now();
            if (r->session) {
                auto it = s->sessions.find(r->session);
                if (it != s->sessions.end()) it->second.outstanding--;
            }
            s->done_cv.notify_all();
            progress = true;
        }
        if (!progress) {
            if (s->inflight.empty()) s->cv.wait_for(lk, std::chrono::milliseconds(1));
            else {
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            }
        }
    }
}

}  // namespace

extern "C" void tron_server_default_config(tron_server_config *c)
{
    if (!c) return;
    c->hbm_budget = (size_t)1 << 30;
    c->lds_budget = (size_t)256 * 160 * 1024 * 4;
    c->max_inflight = 8;
    c->streams = 4;
    c->coalesce = 1;
    c->max_group_instances = 65536;
    tron_default_options(&c->opt);
}

static void free_server(tron_server *s)
{
    if (!s) return;
    for (hipStream_t q : s->streams) (void)hipStreamDestroy(q);
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    (void)hipFree(s->d_base);
    (void)hipHostFree(s->h_stage);
    delete s;
}

extern "C" tron_err tron_server_create(tron_server **out, tron_family fam, const tron_server_config *cfg)
{
    if (!out) return mt_fail(TRON_ERR_INVALID, "out is null");
    *out = nullptr;
    if (fam != TRON_FAMILY_QP4 && fam != TRON_FAMILY_BR6 && fam != TRON_FAMILY_HS45M)
        return mt_fail(TRON_ERR_INVALID, "unknown family");
    tron_server_config c;
    tron_server_default_config(&c);
    if (cfg) c = *cfg;
    if (c.hbm_budget < (1u << 20) || c.max_inflight < 1 || c.streams < 1 || c.max_group_instances < 1)
        return mt_fail(TRON_ERR_INVALID, "invalid server configuration");
    tron_server *s = new (std::nothrow) tron_server();
    if (!s) return mt_fail(TRON_ERR_NOMEM, "host allocation failed");
    s->fam = fam;
    s->cfg = c;
    (void)hipGetDevice(&s->device);
    mt_prepare_wave_kernels();
    if (hipMalloc(&s->d_base, c.hbm_budget) != hipSuccess) {
        free_server(s);
        return mt_fail(TRON_ERR_NOMEM, "device arena allocation failed");
    }
    if (hipHostMalloc(&s->h_stage, c.hbm_budget, hipHostMallocDefault) != hipSuccess) {
        free_server(s);
        return mt_fail(TRON_ERR_NOMEM, "pinned staging allocation failed");
    }
    s->dev.reset(c.hbm_budget);
    s->stage.reset(c.hbm_budget);
    for (int i = 0; i < c.streams; i++) {
        hipStream_t q;
        if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) {
            free_server(s);
            return mt_fail(TRON_ERR_DEVICE, "stream creation failed");
        }
        s->streams.push_back(q);
    }
    for (int i = 0; i < c.max_inflight; i++) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            free_server(s);
            return mt_fail(TRON_ERR_DEVICE, "event creation failed");
        }
        s->events.push_back(e);
    }
    s->worker = std::thread(scheduler, s);
    *out = s;
    return TRON_OK;
}

extern "C" tron_err tron_server_submit(tron_server *s, int64_t batch, const int32_t *n, const double *params,
                                       const double *lo, const double *hi, const double *x0, uint64_t session,
                                       int64_t *ticket)
{
    if (!s || !ticket || batch < 0 || (batch > 0 && (!n || !lo || !hi))) return mt_fail(TRON_ERR_INVALID, "bad argument");
    auto r = std::make_unique<Request>();
    r->batch = batch;
    r->n.assign(n, n + batch);
    int64_t nsum = 0, psum = 0;
    size_t lds = 0;
    for (int64_t i = 0; i < batch; i++) {
        const int64_t ps = tron_param_size(s->fam, r->n[i]);
        if (ps < 0) return mt_fail(TRON_ERR_INVALID, "instance %lld: n = %d invalid", (long long)i, r->n[i]);
        // the server's launch groups keep every matrix in LDS
        if (r->n[i] > kLdsMaxN)
            return mt_fail(TRON_ERR_UNSUPPORTED, "instance %lld: n = %d above the server's limit of %d",
                           (long long)i, r->n[i], kLdsMaxN);
        if (r->n[i] > 8) lds += mt_wave_lds_bytes(wave_nmax_of(r->n[i]));
        nsum += r->n[i];
        psum += ps;
    }
    if (psum > 0 && !params) return mt_fail(TRON_ERR_INVALID, "params is null");
    r->nsum = nsum;
    r->psum = psum;
    r->lds = lds;
    r->params.assign(params, params + psum);
    r->lo.assign(lo, lo + nsum);
    r->hi.assign(hi, hi + nsum);
    r->has_x0 = x0 != nullptr;
    if (x0) r->x0.assign(x0, x0 + nsum);
    r->session = session;
    const size_t need = request_device_bytes(*r);
    if (need > s->cfg.hbm_budget) return mt_fail(TRON_ERR_BUSY, "request larger than the device budget");
    std::lock_guard<std::mutex> lk(s->mu);
    // resident sessions keep their arena memory until closed: the request must fit next to
    // them (and next to its own session, when it opens one)
    size_t new_session = 0;
    if (session && s->sessions.find(session) == s->sessions.end())
        new_session = align_up(sizeof(double) * nsum) + sizeof(double) * 2 * batch;
    if (need + new_session > s->cfg.hbm_budget - std::min(s->session_bytes, s->cfg.hbm_budget))
        return mt_fail(TRON_ERR_BUSY, "request does not fit in the device budget next to the resident sessions");
    if (session) {
        auto it = s->sessions.find(session);
        if (it == s->sessions.end()) {
            if (!x0) return mt_fail(TRON_ERR_INVALID, "new session needs x0");
            Session ss;
            ss.n = r->n;
            ss.nsum = nsum;
            ss.bytes = new_session;
            if (!s->dev.alloc(ss.bytes, &ss.off)) return mt_fail(TRON_ERR_BUSY, "no device memory for the session");
            s->sessions[session] = ss;
            s->session_bytes += ss.bytes;
        } else if (it->second.n != r->n) {
            return mt_fail(TRON_ERR_INVALID, "session sizes differ");
        } else if (it->second.outstanding > 0) {
            return mt_fail(TRON_ERR_BUSY, "session has a request outstanding");
        } else if (!x0 && !it->second.valid) {
            return mt_fail(TRON_ERR_INVALID, "session has no solution yet");
        }
        s->sessions[session].outstanding++;
    } else if (!x0) {
        return mt_fail(TRON_ERR_INVALID, "x0 is null without a session");
    }
    r->ticket = s->next_ticket++;
    r->t_submit = clock_t_::now();
    *ticket = r->ticket;
    Request *raw = r.get();
    s->tickets[raw->ticket] = std::move(r);
    if (batch == 0) {
        raw->state = 2;
        raw->t_done = raw->t_submit;
        s->done_cv.notify_all();
        return TRON_OK;
    }
    s->queue.push_back(raw);
    s->cv.notify_one();
    return TRON_OK;
}

extern "C" tron_err tron_server_poll(tron_server *s, int64_t ticket, int32_t *state)
{
    if (!s || !state) return mt_fail(TRON_ERR_INVALID, "bad argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return mt_fail(TRON_ERR_INVALID, "unknown ticket");
    *state = it->second->state;
    return s->worker_err;
}

extern "C" tron_err tron_server_wait(tron_server *s, int64_t ticket, double timeout_s)
{
    if (!s) return mt_fail(TRON_ERR_INVALID, "bad argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return mt_fail(TRON_ERR_INVALID, "unknown ticket");
    Request *r = it->second.get();
    auto ready = [&] { return r->state == 2 || s->worker_err != TRON_OK; };
    if (timeout_s < 0) s->done_cv.wait(lk, ready);
    else if (!s->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), ready))
        return mt_fail(TRON_ERR_BUSY, "timed out");
    return s->worker_err;
}

extern "C" tron_err tron_server_result(tron_server *s, int64_t ticket, double *x, double *f, int32_t *status,
                                       int32_t *iters, double *latency_s)
{
    if (!s) return mt_fail(TRON_ERR_INVALID, "bad argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return mt_fail(TRON_ERR_INVALID, "unknown ticket");
    Request *r = it->second.get();
    if (r->state != 2) return mt_fail(TRON_ERR_BUSY, "request not finished");
    if (r->err != TRON_OK) {
        const tron_err e = r->err;
        const bool cancelled = r->cancelled;
        s->tickets.erase(it);
        if (cancelled) return mt_fail(e, "request was cancelled before it reached the device");
        return mt_fail(e, "request could not be admitted: resident sessions leave too little device memory");
    }
    if (x) std::copy(r->x.begin(), r->x.end(), x);
    if (f) std::copy(r->f.begin(), r->f.end(), f);
    if (status) std::copy(r->status.begin(), r->status.end(), status);
    if (iters) std::copy(r->iters.begin(), r->iters.end(), iters);
    if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    s->tickets.erase(it);
    return TRON_OK;
}

extern "C" tron_err tron_server_cancel(tron_server *s, int64_t ticket)
{
    if (!s) return mt_fail(TRON_ERR_INVALID, "bad argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return mt_fail(TRON_ERR_INVALID, "unknown ticket");
    Request *r = it->second.get();
    if (r->state != 0) return mt_fail(TRON_ERR_BUSY, r->state == 1 ? "request is on the device" : "request is finished");
    auto q = std::find(s->queue.begin(), s->queue.end(), r);
    if (q == s->queue.end()) return mt_fail(TRON_ERR_BUSY, "request is being admitted");
    s->queue.erase(q);
    // completed without a solve: waiters wake, the result call reports the cancellation
    // and releases the ticket
    r->cancelled = true;
    r->err = TRON_ERR_BUSY;
    r->state = 2;
    r->t_done = clock_t_::now();
    if (r->session) {
        auto si = s->sessions.find(r->session);
        if (si != s->sessions.end()) si->second.outstanding--;
    }
    s->done_cv.notify_all();
    s->cv.notify_one();
    return TRON_OK;
}

extern "C" tron_err tron_server_close_session(tron_server *s, uint64_t session)
{
    if (!s) return mt_fail(TRON_ERR_INVALID, "bad argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->sessions.find(session);
    if (it == s->sessions.end()) return mt_fail(TRON_ERR_INVALID, "unknown session");
    if (it->second.outstanding > 0) return mt_fail(TRON_ERR_BUSY, "session has a request outstanding");
    s->dev.release(it->second.off, it->second.bytes);
    s->session_bytes -= it->second.bytes;
    s->sessions.erase(it);
    return TRON_OK;
}

extern "C" tron_err tron_server_stats(tron_server *s, int64_t *out4)
{
    if (!s || !out4) return mt_fail(TRON_ERR_INVALID, "bad argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out4[0] = s->done_requests;
    out4[1] = s->done_instances;
    out4[2] = (int64_t)s->dev.used();
    out4[3] = (int64_t)s->lds_inflight;
    return TRON_OK;
}

extern "C" tron_err tron_server_destroy(tron_server *s)
{
    if (!s) return TRON_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (hipStream_t q : s->streams) (void)hipStreamSynchronize(q);
    for (Group *g : s->inflight) {
        s->events.push_back(g->done);
        delete g;
    }
    s->inflight.clear();
    for (Request *r : s->queue) (void)r;
    s->queue.clear();
    s->tickets.clear();
    free_server(s);
    return TRON_OK;
}
