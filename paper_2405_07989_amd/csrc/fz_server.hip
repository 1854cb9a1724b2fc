// fz_server.hip -- request server of libfz: continuous batching of arriving
// queries on one device.
//
// Queries arrive one at a time (fz_submit, any thread) into a FIFO.  A server
// thread owns max_inflight launch slots, each a stream with its own batch
// buffers.  Whenever a slot is free and queries are waiting, it takes what
// has arrived (up to max_batch queries and the slot's memory budget) and
// queues it as one batch; so a query that arrives while others run starts in
// the next free slot, and batches in different slots overlap on the device.
// A batch is queued in two phases -- count and work tables, then, once
// their totals are back, the cut and the walk -- and the server thread
// starts the second from its poll loop, so it never waits on the device.
// Inside a launch, the wave that finishes a query's last slice writes the
// query's result to pinned host memory and raises its flag; the server
// thread polls the flags and hands each result to fz_wait as soon as it is
// there, without waiting for the rest of the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fz.h"
#include "fz_host.h"
#include "fz_internal.h"

using namespace fzh;
using Clock = std::chrono::steady_clock;

namespace {

constexpr uint32_t kDefaultInflight = 2;
constexpr uint32_t kMaxInflight = 8;
constexpr uint32_t kDefaultMaxBatch = 4096;
constexpr uint64_t kDefaultMemBudget = 8ull << 30;
constexpr uint64_t kDefaultStoreCap = 10000000ull;

struct Request {
    uint64_t ticket = 0;
    fz_query q{};
    std::array<uint32_t, FZ_MAX_D> g{};
    Clock::time_point t_submit;
};

struct Outcome {
    bool ready = false;
    fz_result r{};
};

struct Slot {
    BatchSlot b;
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    bool busy = false;
    std::vector<Request> reqs;
    std::vector<fz_query> qs;
    std::vector<uint8_t> delivered;
    uint32_t left = 0;
    Clock::time_point t_admit, t_walk; // launch of phase 1, of phase 2
};

// Device bytes a query may need in a slot: count and work tables (if it is
// cut), residue table, histogram bins.
uint64_t predicted_bytes(const fz_query &q)
{
    FzPlan P;
    if (make_plan(q.n, q.g, q.d, q.mode, &P)) return 0; // rejected at launch
    uint64_t b = (uint64_t)(2 * P.d - 3) * P.stride * 8 + 2ull * P.B * 8;
    if (q.mode == FZ_MODE_HIST) b += (uint64_t)P.nbins * 8;
    return b;
}

} // namespace

struct fz_server {
    int device = 0;
    int cus = 0;
    uint32_t inflight = kDefaultInflight;
    uint32_t max_batch = kDefaultMaxBatch;
    uint64_t mem_budget = kDefaultMemBudget;
    uint64_t store_cap = kDefaultStoreCap;

    std::mutex mu;
    std::condition_variable cv_work; // the server thread: new requests, stop
    std::condition_variable cv_done; // fz_wait callers
    bool stop = false;
    int sticky = FZ_OK;              // a device failure ends the service
    uint64_t next_ticket = 1;
    std::deque<Request> queue;
    std::unordered_map<uint64_t, Outcome> outcomes;
    std::vector<double> latency_us;
    uint64_t submitted = 0, completed = 0, launches = 0, launched_queries = 0;
    // launch phases summed over finished launches: phase 1 (admission to
    // the walk's launch: tables, totals read back, cut) and phase 2 (walk
    // launch to the launch's last result)
    double phase1_us = 0, phase2_us = 0;
    uint64_t phased = 0;
    void phases_done(const Slot &sl)
    {
        const Clock::time_point now = Clock::now();
        phase1_us += std::chrono::duration<double, std::micro>(sl.t_walk - sl.t_admit).count();
        phase2_us += std::chrono::duration<double, std::micro>(now - sl.t_walk).count();
        ++phased;
    }

    std::vector<Slot> slots;
    std::thread th;

    void deliver(const Request &rq, const fz_result &r);
    void run();
};

// Called with mu held.
void fz_server::deliver(const Request &rq, const fz_result &r)
{
    auto it = outcomes.find(rq.ticket);
    if (it == outcomes.end()) return;
    it->second.r = r;
    it->second.ready = true;
    latency_us.push_back(
        std::chrono::duration<double, std::micro>(Clock::now() - rq.t_submit).count());
    ++completed;
}

void fz_server::run()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // 1. collect finished queries of the busy slots
        bool any_busy = false, delivered_any = false;
        for (Slot &sl : slots) {
            if (!sl.busy) continue;
            if (sl.b.walk_pending) {
                // phase 2 (cut and walk) once the tables and their totals
                // are in
                const hipError_t te = hipEventQuery(sl.b.tables_ev);
                if (te == hipErrorNotReady) {
                    any_busy = true;
                    continue;
                }
                int rc = te == hipSuccess ? FZ_OK : FZ_EDEVICE;
                if (te != hipSuccess) (void)hipGetLastError();
                if (rc == FZ_OK) {
                    lk.unlock();
                    {
                        std::lock_guard<std::mutex> g(g_mu);
                        rc = batch_launch_walk(sl.b);
                    }
                    sl.t_walk = Clock::now();
                    if (rc == FZ_OK && hipEventRecord(sl.done_ev, sl.stream) != hipSuccess) {
                        (void)hipGetLastError();
                        rc = FZ_EDEVICE;
                    }
                    lk.lock();
                }
                if (rc != FZ_OK) {
                    fz_result r{};
                    r.status = rc;
                    r.min_len = UINT64_MAX;
                    for (uint32_t i = 0; i < (uint32_t)sl.reqs.size(); ++i)
                        if (!sl.delivered[i]) deliver(sl.reqs[i], r);
                    if (rc == FZ_EDEVICE) sticky = rc;
                    sl.left = 0;
                    sl.busy = false;
                    sl.reqs.clear();
                    delivered_any = true;
                    continue;
                }
            }
            // the event first: once it has completed, every flag the launch
            // raises is visible to the polls below
            const hipError_t e = hipEventQuery(sl.done_ev);
            for (uint32_t i = 0; i < (uint32_t)sl.reqs.size(); ++i) {
                if (sl.delivered[i]) continue;
                const bool ready = sl.b.qst[i] != FZ_OK ||
                                   __atomic_load_n(&sl.b.h_done[i], __ATOMIC_ACQUIRE) != 0;
                if (!ready) continue;
                fz_result r;
                batch_result(sl.b, sl.qs[i], i, &r);
                deliver(sl.reqs[i], r);
                sl.delivered[i] = 1;
                --sl.left;
                delivered_any = true;
            }
            if (e == hipSuccess) {
                phases_done(sl);
                // a query the completed launch did not finish would be a bug
                // of the walker: report it rather than wait for it
                fz_result r{};
                r.status = FZ_EINTERNAL;
                r.min_len = UINT64_MAX;
                for (uint32_t i = 0; i < (uint32_t)sl.reqs.size(); ++i)
                    if (!sl.delivered[i]) deliver(sl.reqs[i], r);
                sl.left = 0;
                sl.busy = false;
                sl.reqs.clear();
                delivered_any = true;
                continue;
            }
            if (e != hipSuccess && e != hipErrorNotReady) {
                // the launch failed: fail what it still owes, stop serving
                (void)hipGetLastError();
                sticky = FZ_EDEVICE;
                fz_result r{};
                r.status = FZ_EDEVICE;
                r.min_len = UINT64_MAX;
                for (uint32_t i = 0; i < (uint32_t)sl.reqs.size(); ++i)
                    if (!sl.delivered[i]) deliver(sl.reqs[i], r);
                sl.left = 0;
                sl.busy = false;
                sl.reqs.clear();
                delivered_any = true;
                continue;
            }
            any_busy = true;
        }
        if (delivered_any) cv_done.notify_all();

        // 2. a failed device takes no new work
        if (sticky != FZ_OK && !queue.empty()) {
            fz_result r{};
            r.status = sticky;
            r.min_len = UINT64_MAX;
            while (!queue.empty()) {
                deliver(queue.front(), r);
                queue.pop_front();
            }
            cv_done.notify_all();
        }

        // 3. admit: what has arrived goes to a free slot as one batch
        for (Slot &sl : slots) {
            if (queue.empty() || sl.busy) continue;
            std::vector<Request> take;
            uint64_t bytes = 0;
            std::vector<Request> refused;
            while (!queue.empty() && take.size() < max_batch) {
                Request &rq = queue.front();
                rq.q.g = rq.g.data();
                const uint64_t b = predicted_bytes(rq.q);
                if (b > mem_budget) {
                    refused.push_back(rq);
                    queue.pop_front();
                    continue;
                }
                if (bytes + b > mem_budget && !take.empty()) break;
                bytes += b;
                take.push_back(rq);
                queue.pop_front();
            }
            if (!refused.empty()) {
                fz_result r{};
                r.status = FZ_E2BIG;
                r.min_len = UINT64_MAX;
                for (const Request &rq : refused) deliver(rq, r);
                cv_done.notify_all();
            }
            if (take.empty()) continue;
            sl.reqs = std::move(take);
            sl.qs.resize(sl.reqs.size());
            for (size_t i = 0; i < sl.reqs.size(); ++i) {
                sl.qs[i] = sl.reqs[i].q;
                sl.qs[i].g = sl.reqs[i].g.data();
            }
            sl.delivered.assign(sl.reqs.size(), 0);
            sl.left = (uint32_t)sl.reqs.size();
            sl.busy = true;
            sl.t_admit = sl.t_walk = Clock::now();
            ++launches;
            launched_queries += sl.reqs.size();
            lk.unlock();
            int rc;
            {
                std::lock_guard<std::mutex> g(g_mu);
                uint32_t spw, wgcu;
                current_knobs(&spw, &wgcu);
                rc = batch_launch_tables(sl.b, cus, spw, wgcu, sl.qs.data(),
                                         (uint32_t)sl.qs.size(), sl.stream, store_cap, false);
            }
            // the completion event is recorded after phase 2 (poll loop); a
            // batch whose queries were all rejected has no phase 2
            if (rc == FZ_OK && !sl.b.walk_pending &&
                hipEventRecord(sl.done_ev, sl.stream) != hipSuccess) {
                (void)hipGetLastError();
                rc = FZ_EDEVICE;
            }
            lk.lock();
            if (rc != FZ_OK) {
                fz_result r{};
                r.status = rc;
                r.min_len = UINT64_MAX;
                for (const Request &rq : sl.reqs) deliver(rq, r);
                sl.busy = false;
                sl.reqs.clear();
                sl.left = 0;
                if (rc == FZ_EDEVICE) sticky = rc;
                cv_done.notify_all();
            }
            any_busy = any_busy || sl.busy;
        }

        if (stop && queue.empty() && !any_busy) break;
        if (any_busy)
            cv_work.wait_for(lk, std::chrono::microseconds(20));
        else
            cv_work.wait(lk, [&] { return stop || !queue.empty(); });
    }
}

extern "C" {

int fz_server_create(const fz_server_cfg *cfg, fz_server **out)
{
    if (out == nullptr) return FZ_EINVAL;
    *out = nullptr;
    fz_server_cfg c{};
    if (cfg) c = *cfg;
    if (c.max_inflight > kMaxInflight || c.max_batch > 65536) return FZ_EINVAL;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return dev_err_at(e, "hipGetDevice", __LINE__);
    }
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return dev_err_at(e, "hipDeviceGetAttribute", __LINE__);
    }
    fz_server *s = new fz_server;
    s->device = dev;
    s->cus = cus;
    if (c.max_inflight) s->inflight = c.max_inflight;
    if (c.max_batch) s->max_batch = c.max_batch;
    if (c.mem_budget) s->mem_budget = c.mem_budget;
    if (c.max_store_tuples) s->store_cap = c.max_store_tuples;
    s->slots.resize(s->inflight);
    for (Slot &sl : s->slots) {
        sl.b.small_first = true; // latency: a launch's small queries are walked first
        e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            const int rc = dev_err_at(e, "server slot", __LINE__);
            for (Slot &t : s->slots) {
                if (t.done_ev) (void)hipEventDestroy(t.done_ev);
                if (t.stream) (void)hipStreamDestroy(t.stream);
            }
            delete s;
            return rc;
        }
    }
    s->th = std::thread([s] { s->run(); });
    *out = s;
    return FZ_OK;
}

int fz_submit(fz_server *s, const fz_query *q, uint64_t *ticket)
{
    if (s == nullptr || q == nullptr || ticket == nullptr) return FZ_EINVAL;
    Request rq;
    rq.q = *q;
    if (q->g && q->d >= 1 && q->d <= FZ_MAX_D) std::memcpy(rq.g.data(), q->g, q->d * 4);
    else rq.q.d = q->g ? FZ_MAX_D + 1 : 0; // rejected as FZ_EINVAL at admission
    rq.q.g = nullptr;
    rq.t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return FZ_EINVAL;
        rq.ticket = s->next_ticket++;
        s->outcomes.emplace(rq.ticket, Outcome{});
        s->queue.push_back(rq);
        ++s->submitted;
        *ticket = rq.ticket;
    }
    s->cv_work.notify_one();
    return FZ_OK;
}

int fz_wait(fz_server *s, uint64_t ticket, fz_result *r)
{
    if (s == nullptr || r == nullptr) return FZ_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->outcomes.find(ticket);
    if (it == s->outcomes.end()) return FZ_EINVAL;
    s->cv_done.wait(lk, [&] {
        auto f = s->outcomes.find(ticket);
        return f == s->outcomes.end() || f->second.ready;
    });
    it = s->outcomes.find(ticket);
    if (it == s->outcomes.end()) return FZ_EINVAL; // another waiter took it
    *r = it->second.r;
    s->outcomes.erase(it);
    return FZ_OK;
}

int fz_server_stats_read(fz_server *s, fz_server_stats *out, int reset)
{
    if (s == nullptr || out == nullptr) return FZ_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    fz_server_stats st{};
    st.submitted = s->submitted;
    st.completed = s->completed;
    st.launches = s->launches;
    st.mean_batch = s->launches ? (double)s->launched_queries / s->launches : 0.0;
    std::vector<double> v = s->latency_us;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            size_t k = (size_t)std::ceil(p * v.size());
            return v[std::min(v.size() - 1, k ? k - 1 : 0)];
        };
        st.p50_us = pct(0.50);
        st.p99_us = pct(0.99);
        st.max_us = v.back();
        double sum = 0;
        for (double x : v) sum += x;
        st.mean_us = sum / v.size();
    }
    if (s->phased) {
        st.mean_phase1_us = s->phase1_us / s->phased;
        st.mean_phase2_us = s->phase2_us / s->phased;
    }
    if (reset) {
        s->latency_us.clear();
        s->submitted = s->completed = s->launches = s->launched_queries = 0;
        s->phase1_us = s->phase2_us = 0;
        s->phased = 0;
    }
    *out = st;
    return FZ_OK;
}

int fz_server_destroy(fz_server *s)
{
    if (s == nullptr) return FZ_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->th.joinable()) s->th.join();
    (void)hipSetDevice(s->device);
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        sl.b.release();
        if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete s;
    return FZ_OK;
}

} // extern "C"
