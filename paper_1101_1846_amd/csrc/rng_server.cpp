// rng_server.cpp -- continuous-batching request server over resident stream
// states.  A worker thread admits queued requests while output memory and
// in-flight slots allow, launches each admitted set as one batch (see
// rng_batch.cpp) on one of several HIP streams so that batches overlap on the
// device, and stamps every request's completion from the batch's event.
// Requests on the same stream are served in arrival order: a request whose
// stream is still in flight waits, so every result is the next slice of its
// stream's serial sequence whatever else shares the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_set>
#include <vector>

#include "rng.h"
#include "rng_abi_internal.hpp"

using namespace rngx;
using Clock = std::chrono::steady_clock;

namespace {

// First-fit allocator over one device buffer, 256-byte granules, coalescing.
class PoolAlloc {
  public:
    void reset(uint64_t bytes)
    {
        free_.clear();
        free_[0] = bytes;
        total_ = bytes;
        used_ = 0;
    }
    bool alloc(uint64_t bytes, uint64_t *off)
    {
        bytes = (bytes + 255) & ~(uint64_t)255;
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            uint64_t rest = it->second - bytes, start = it->first + bytes;
            free_.erase(it);
            if (rest) free_[start] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes)
    {
        bytes = (bytes + 255) & ~(uint64_t)255;
        if (bytes == 0) bytes = 256;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t used() const { return used_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t total_ = 0, used_ = 0;
};

struct Req {
    uint64_t stream = 0, length = 0, off = 0;
    int dtype = 0;
    Clock::time_point t_arrive, t_admit, t_launched, t_done;
    bool admitted = false, done = false, released = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    rng_batch_t *batch = nullptr;
    std::vector<uint64_t> tickets;
    bool busy = false;
};

}  // namespace

struct rng_server {
    rng_server_config_t cfg{};
    int device = 0;
    int gens[5] = {};
    uint32_t n_gens = 0;
    std::vector<uint32_t *> pools;    // per generator kind: [words][count]
    std::vector<uint64_t> pool_count;
    char *out_pool = nullptr;
    PoolAlloc alloc;
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<Req> reqs;             // indexed by ticket
    std::deque<uint64_t> pending;      // tickets in arrival order
    std::unordered_set<uint64_t> busy; // streams with a request in flight
    std::thread worker;
    bool stop = false;
    int worker_error = RNG_OK;

    uint64_t completed = 0, batches = 0, batch_requests = 0, samples_done = 0, admission_waits = 0;
    Clock::time_point first_arrival, last_done;
    bool any_arrival = false;
    std::vector<double> lat_us;
    double queue_us = 0, submit_us = 0, device_us = 0;  // sums over completed requests
};

static void worker_loop(rng_server *h)
{
    (void)hipSetDevice(h->device);
    std::vector<rng_request_t> table;
    std::vector<uint64_t> chosen;
    std::unordered_set<uint64_t> in_batch;
    const auto spin = std::chrono::microseconds(h->cfg.idle_spin_us);
    auto last_active = Clock::now();
    while (true) {
        bool progressed = false;
        // completions
        for (auto &s : h->slots) {
            if (!s.busy || hipEventQuery(s.ev) != hipSuccess) continue;
            const auto t = Clock::now();
            std::lock_guard<std::mutex> lk(h->mu);
            for (uint64_t tk : s.tickets) {
                Req &r = h->reqs[tk];
                r.done = true;
                r.t_done = t;
                h->busy.erase(r.stream);
                h->lat_us.push_back(std::chrono::duration<double, std::micro>(t - r.t_arrive).count());
                h->queue_us += std::chrono::duration<double, std::micro>(r.t_admit - r.t_arrive).count();
                h->submit_us += std::chrono::duration<double, std::micro>(r.t_launched - r.t_admit).count();
                h->device_us += std::chrono::duration<double, std::micro>(t - r.t_launched).count();
                h->samples_done += r.length;
                ++h->completed;
                if (h->cfg.auto_release && !r.released) {
                    h->alloc.release(r.off, r.length * 4);
                    r.released = true;
                }
            }
            h->last_done = t;
            s.tickets.clear();
            s.busy = false;
            progressed = true;
            h->cv_done.notify_all();
        }
        // admission into a free slot
        Slot *free_slot = nullptr;
        for (auto &s : h->slots)
            if (!s.busy) {
                free_slot = &s;
                break;
            }
        if (free_slot) {
            chosen.clear();
            in_batch.clear();
            table.clear();
            {
                std::unique_lock<std::mutex> lk(h->mu);
                if (h->stop && h->pending.empty()) break;
                uint64_t samples = 0;
                const auto t_admit = Clock::now();
                for (auto it = h->pending.begin(); it != h->pending.end();) {
                    if (chosen.size() >= h->cfg.max_batch_requests) break;
                    Req &r = h->reqs[*it];
                    if (h->busy.count(r.stream) || in_batch.count(r.stream)) {
                        ++it;  // keeps its stream's order: waits for the earlier request
                        continue;
                    }
                    if (samples + r.length > h->cfg.max_batch_samples) break;
                    uint64_t off;
                    if (!h->alloc.alloc(r.length * 4, &off)) {
                        ++h->admission_waits;
                        break;  // memory full: admit again when outputs are released
                    }
                    r.off = off;
                    r.admitted = true;
                    r.t_admit = t_admit;
                    samples += r.length;
                    in_batch.insert(r.stream);
                    chosen.push_back(*it);
                    it = h->pending.erase(it);
                }
                for (uint64_t tk : chosen) {
                    const Req &r = h->reqs[tk];
                    const uint32_t k = (uint32_t)(r.stream % h->n_gens);
                    const uint64_t idx = r.stream / h->n_gens;
                    rng_request_t q{};
                    q.gen = h->gens[k];
                    q.dtype = r.dtype;
                    q.d_state = h->pools[k] + idx;
                    q.state_stride = h->pool_count[k];
                    q.offset = 0;
                    q.length = r.length;
                    q.d_out = h->out_pool + r.off;
                    table.push_back(q);
                    h->busy.insert(r.stream);
                }
            }
            if (!chosen.empty()) {
                int rc = batch_set_distinct(free_slot->batch, table.data(), (uint32_t)table.size());
                if (!rc) rc = rng_batch_launch(free_slot->batch, free_slot->stream);
                if (!rc && hipEventRecord(free_slot->ev, free_slot->stream) != hipSuccess) rc = RNG_EHIP;
                if (rc) {
                    std::lock_guard<std::mutex> lk(h->mu);
                    h->worker_error = rc;
                    h->stop = true;
                    h->cv_done.notify_all();
                    break;
                }
                const auto t_launched = Clock::now();
                {
                    std::lock_guard<std::mutex> lk(h->mu);
                    for (uint64_t tk : chosen) h->reqs[tk].t_launched = t_launched;
                }
                free_slot->tickets = chosen;
                free_slot->busy = true;
                ++h->batches;
                h->batch_requests += chosen.size();
                progressed = true;
            }
        }
        if (progressed) {
            last_active = Clock::now();
        } else {
            std::unique_lock<std::mutex> lk(h->mu);
            bool inflight = false;
            for (auto &s : h->slots) inflight |= s.busy;
            // Stopping with nothing in flight: every slot was free and still
            // nothing was admitted, so what is pending waits for output memory
            // that no one will release; it is abandoned.
            if (h->stop && !inflight) break;
            if (!inflight && Clock::now() - last_active >= spin) {
                h->cv_work.wait_for(lk, std::chrono::microseconds(200));
            } else {
                lk.unlock();
                std::this_thread::yield();  // keep polling: in-flight events, or new requests while idle
            }
        }
    }
}

extern "C" {

int rng_server_create(const rng_server_config_t *cfg, rng_server_t **out)
{
    if (!cfg || !out) return fail(RNG_EINVAL, "NULL argument");
    if (cfg->n_streams == 0 || cfg->n_gens == 0 || cfg->n_gens > 5) return fail(RNG_EINVAL, "bad stream/generator count");
    if (cfg->inflight == 0 || cfg->inflight > 8) return fail(RNG_EINVAL, "inflight must be 1..8");
    if (cfg->idle_spin_us > 1000000) return fail(RNG_EINVAL, "idle_spin_us above one second");
    if (cfg->max_batch_requests == 0 || cfg->max_batch_samples == 0 || cfg->pool_bytes < 256)
        return fail(RNG_EINVAL, "empty batch or pool limits");
    for (uint32_t k = 0; k < cfg->n_gens; ++k)
        if (check_gen(cfg->gens[k])) return RNG_EINVAL;
    DevTables tab;
    if (int rc = device_tables(&tab)) return rc;
    auto *h = new rng_server();
    h->cfg = *cfg;
    (void)hipGetDevice(&h->device);
    h->n_gens = cfg->n_gens;
    int rc = RNG_OK;
    hipError_t e;
    for (uint32_t k = 0; k < h->n_gens && !rc; ++k) {
        h->gens[k] = cfg->gens[k];
        uint64_t count = (cfg->n_streams + h->n_gens - 1 - k) / h->n_gens;
        uint32_t *p = nullptr;
        if (count) {
            if ((e = hipMalloc((void **)&p, count * gen_words(h->gens[k]) * 4)) != hipSuccess) {
                rc = hip_fail(e, "hipMalloc(resident states)");
                break;
            }
            rc = rng_seed(h->gens[k], cfg->seed + k, 0, count, p, nullptr);
        }
        h->pools.push_back(p);
        h->pool_count.push_back(count);
    }
    if (!rc && (e = hipMalloc((void **)&h->out_pool, cfg->pool_bytes)) != hipSuccess)
        rc = hip_fail(e, "hipMalloc(output pool)");
    h->alloc.reset(cfg->pool_bytes);
    for (uint32_t i = 0; i < cfg->inflight && !rc; ++i) {
        Slot s;
        if ((e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming)) != hipSuccess)
            rc = hip_fail(e, "server stream/event");
        if (!rc) rc = rng_batch_create(cfg->max_batch_requests, cfg->max_batch_samples, &s.batch);
        // every batch picks its chunk length, so that a lone small request
        // still spreads over the device
        if (!rc && s.batch) rc = rng_batch_set_shape(s.batch, 0, 0, RNG_BATCH_CHUNK_AUTO);
        h->slots.push_back(s);
    }
    if (!rc && (e = hipDeviceSynchronize()) != hipSuccess) rc = hip_fail(e, "hipDeviceSynchronize");
    if (rc) {
        rng_server_destroy(h);
        return rc;
    }
    h->worker = std::thread(worker_loop, h);
    *out = h;
    return RNG_OK;
}

int rng_server_destroy(rng_server_t *h)
{
    if (!h) return RNG_OK;
    if (h->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(h->mu);
            h->stop = true;
        }
        h->cv_work.notify_all();
        h->worker.join();
    }
    (void)hipDeviceSynchronize();
    for (auto &s : h->slots) {
        if (s.batch) rng_batch_destroy(s.batch);
        if (s.ev) (void)hipEventDestroy(s.ev);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    for (auto *p : h->pools)
        if (p) (void)hipFree(p);
    if (h->out_pool) (void)hipFree(h->out_pool);
    delete h;
    return RNG_OK;
}

int rng_server_submit(rng_server_t *h, uint64_t stream_id, uint64_t length, int dtype, uint64_t *ticket)
{
    if (!h || !ticket) return fail(RNG_EINVAL, "NULL argument");
    if (stream_id >= h->cfg.n_streams) return fail(RNG_ERANGE, "stream %llu out of range", (unsigned long long)stream_id);
    if (dtype != RNG_U32 && dtype != RNG_F32) return fail(RNG_EINVAL, "dtype %d", dtype);
    if (length == 0 || length > h->cfg.max_batch_samples || length * 4 > h->cfg.pool_bytes)
        return fail(RNG_ERANGE, "length %llu outside (0, batch and pool limits]", (unsigned long long)length);
    {
        std::lock_guard<std::mutex> lk(h->mu);
        if (h->worker_error) return fail(h->worker_error, "server stopped after a launch error");
        Req r;
        r.stream = stream_id;
        r.length = length;
        r.dtype = dtype;
        r.t_arrive = Clock::now();
        if (!h->any_arrival) {
            h->first_arrival = r.t_arrive;
            h->any_arrival = true;
        }
        *ticket = h->reqs.size();
        h->reqs.push_back(r);
        h->pending.push_back(*ticket);
    }
    h->cv_work.notify_one();
    return RNG_OK;
}

int rng_server_poll(rng_server_t *h, uint64_t ticket, int *done, void **d_out)
{
    if (!h || !done) return fail(RNG_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(h->mu);
    if (ticket >= h->reqs.size()) return fail(RNG_EINVAL, "unknown ticket");
    const Req &r = h->reqs[ticket];
    *done = r.done ? 1 : 0;
    if (d_out) *d_out = (r.done && !r.released) ? (void *)(h->out_pool + r.off) : nullptr;
    return r.done ? RNG_OK : RNG_EAGAIN;
}

int rng_server_release(rng_server_t *h, uint64_t ticket)
{
    if (!h) return fail(RNG_EINVAL, "NULL handle");
    {
        std::lock_guard<std::mutex> lk(h->mu);
        if (ticket >= h->reqs.size()) return fail(RNG_EINVAL, "unknown ticket");
        Req &r = h->reqs[ticket];
        if (!r.done) return fail(RNG_EAGAIN, "ticket not complete");
        if (!r.released) {
            h->alloc.release(r.off, r.length * 4);
            r.released = true;
        }
    }
    h->cv_work.notify_one();
    return RNG_OK;
}

int rng_server_drain(rng_server_t *h)
{
    if (!h) return fail(RNG_EINVAL, "NULL handle");
    std::unique_lock<std::mutex> lk(h->mu);
    h->cv_done.wait(lk, [&] { return h->worker_error || h->completed == h->reqs.size(); });
    return h->worker_error ? fail(h->worker_error, "server stopped after a launch error") : RNG_OK;
}

int rng_server_stats(rng_server_t *h, rng_server_stats_t *st)
{
    if (!h || !st) return fail(RNG_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(h->mu);
    std::memset(st, 0, sizeof(*st));
    st->submitted = h->reqs.size();
    st->completed = h->completed;
    st->batches = h->batches;
    st->samples = h->samples_done;
    st->admission_waits = h->admission_waits;
    st->mean_batch_requests = h->batches ? (double)h->batch_requests / h->batches : 0.0;
    if (!h->lat_us.empty()) {
        std::vector<double> v = h->lat_us;
        std::sort(v.begin(), v.end());
        auto q = [&](double p) { return v[std::min(v.size() - 1, (size_t)(p * (v.size() - 1) + 0.5))]; };
        st->p50_us = q(0.50);
        st->p99_us = q(0.99);
        st->max_us = v.back();
        double s = 0;
        for (double x : v) s += x;
        st->mean_us = s / v.size();
        st->mean_queue_us = h->queue_us / v.size();
        st->mean_submit_us = h->submit_us / v.size();
        st->mean_device_us = h->device_us / v.size();
    }
    if (h->any_arrival && h->completed)
        st->wall_s = std::chrono::duration<double>(h->last_done - h->first_arrival).count();
    st->gsamples_per_s = st->wall_s > 0 ? h->samples_done / st->wall_s / 1e9 : 0.0;
    return RNG_OK;
}

int rng_server_reset_stats(rng_server_t *h)
{
    if (!h) return fail(RNG_EINVAL, "NULL handle");
    std::lock_guard<std::mutex> lk(h->mu);
    h->lat_us.clear();
    h->queue_us = h->submit_us = h->device_us = 0;
    h->batches = h->batch_requests = h->admission_waits = 0;
    h->samples_done = 0;
    h->any_arrival = false;
    // completed counts tickets; keep it consistent with reqs for drain()
    return RNG_OK;
}

int rng_server_read_state(rng_server_t *h, uint64_t stream_id, uint32_t *h_state)
{
    if (!h || !h_state) return fail(RNG_EINVAL, "NULL argument");
    if (stream_id >= h->cfg.n_streams) return fail(RNG_ERANGE, "stream out of range");
    const uint32_t k = (uint32_t)(stream_id % h->n_gens);
    const uint64_t idx = stream_id / h->n_gens, S = h->pool_count[k];
    {
        std::lock_guard<std::mutex> lk(h->mu);
        if (h->busy.count(stream_id)) return fail(RNG_EAGAIN, "stream has a request in flight");
    }
    for (int w = 0; w < gen_words(h->gens[k]); ++w) {
        hipError_t e = hipMemcpy(&h_state[w], h->pools[k] + w * S + idx, 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(state)");
    }
    return RNG_OK;
}

int rng_server_replay(rng_server_t *h, const double *t_arrival_s, const uint64_t *stream_ids,
                      const uint64_t *lengths, const int32_t *dtypes, uint64_t n, uint64_t *tickets)
{
    if (!h || (n && (!t_arrival_s || !stream_ids || !lengths || !dtypes))) return fail(RNG_EINVAL, "NULL argument");
    const auto t0 = Clock::now();
    for (uint64_t i = 0; i < n; ++i) {
        const auto due = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(t_arrival_s[i]));
        while (Clock::now() < due) {
        }
        uint64_t tk;
        if (int rc = rng_server_submit(h, stream_ids[i], lengths[i], dtypes[i], &tk)) return rc;
        if (tickets) tickets[i] = tk;
    }
    return rng_server_drain(h);
}

}  // extern "C"
