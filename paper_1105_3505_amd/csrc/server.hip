// Continuous-batching server over one context.
//
// A worker thread owns the context.  Each scheduling iteration it retires the iterations
// whose evaluation has completed on the device, then admits waiting requests in arrival
// order while the iteration's request and point limits and the memory budget allow, builds
// one forest plan over them on a free stream and enqueues its evaluation there.  Tree
// construction of a new iteration thus runs on the device beside the evaluation of earlier
// ones.  Since every instance of a forest is built and evaluated from its own points only,
// a request's result does not depend on what it was batched with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "api_common.h"
#include "lfmm.h"

using namespace lfmm;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    int64_t n = 0;
    const int32_t* xy = nullptr;
    const double* f = nullptr;
    double* u = nullptr;
    hipEvent_t ready = nullptr;   // recorded on the producer's stream at submit
    size_t footprint = 0;         // 0 until the root box is known
    ~Request() {
        if (ready) (void)hipEventDestroy(ready);
    }
    lfmm_request_stats st{};
    bool done = false;
    bool solo = false;   // served alone after a batch it was in failed to build
};

struct Inflight {
    lfmm_plan* plan = nullptr;
    hipEvent_t done = nullptr;
    int stream = -1;
    size_t footprint = 0;
    std::vector<std::shared_ptr<Request>> reqs;
};

}  // namespace

struct lfmm_server {
    lfmm_ctx* ctx = nullptr;
    lfmm_server_options opt{};
    Clock::time_point t0;
    std::vector<hipStream_t> streams;
    std::vector<bool> stream_busy;
    hipStream_t probe = nullptr;       // extents of newly queued requests
    std::mutex mu;
    std::condition_variable cv_work;   // worker: new request or stop
    std::condition_variable cv_done;   // waiters: a request finished
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> all;
    std::vector<Inflight> inflight;    // worker thread only
    size_t inflight_bytes = 0;         // worker thread only
    uint64_t next_ticket = 1;
    int64_t next_batch = 0;
    bool stop = false;
    std::thread worker;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    void finish(const std::shared_ptr<Request>& r, lfmm_status s, double t) {
        std::lock_guard<std::mutex> lock(mu);
        r->st.status = s;
        r->st.t_done = t;
        r->done = true;
        cv_done.notify_all();
    }

    // retire every iteration whose completion event has fired; returns how many
    int retire() {
        int k = 0;
        for (size_t i = 0; i < inflight.size();) {
            Inflight& it = inflight[i];
            const hipError_t q = hipEventQuery(it.done);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            const double t = now();
            const lfmm_status s = (q == hipSuccess) ? LFMM_OK : LFMM_E_HIP;
            if (q != hipSuccess) (void)hipGetLastError();
            for (auto& r : it.reqs) finish(r, s, t);
            // the evaluation has completed: the plan's memory may go back to the pool
            plan_destroy_completed(it.plan);
            (void)hipEventDestroy(it.done);
            stream_busy[size_t(it.stream)] = false;
            inflight_bytes -= it.footprint;
            inflight.erase(inflight.begin() + long(i));
            ++k;
        }
        return k;
    }

    // footprint bounds of queued requests that lack one: the root bits of each request are
    // measured on the device (after its producer's event), then lfmm_plan_footprint_bytes;
    // a request over the whole budget finishes at once with LFMM_E_NOMEM
    void measure() {
        std::vector<std::shared_ptr<Request>> todo;
        {
            std::lock_guard<std::mutex> lock(mu);
            for (auto& r : queue)
                if (r->footprint == 0) todo.push_back(r);
        }
        if (todo.empty()) return;
        const int32_t K = int32_t(todo.size());
        std::vector<int64_t> n(static_cast<size_t>(K));
        std::vector<const int32_t*> xy(static_cast<size_t>(K));
        std::vector<int32_t> bits(static_cast<size_t>(K), -1);
        for (int32_t k = 0; k < K; ++k) {
            n[size_t(k)] = todo[size_t(k)]->n;
            xy[size_t(k)] = todo[size_t(k)]->xy;
            if (hipStreamWaitEvent(probe, todo[size_t(k)]->ready, 0) != hipSuccess) (void)hipGetLastError();
        }
        if (root_bits_of(ctx, K, n.data(), xy.data(), probe, bits.data()) != LFMM_OK)
            std::fill(bits.begin(), bits.end(), -1);   // unknown: the bound for any extent
        std::vector<std::shared_ptr<Request>> reject;
        {
            std::lock_guard<std::mutex> lock(mu);
            for (int32_t k = 0; k < K; ++k) {
                Request& r = *todo[size_t(k)];
                const int32_t b = bits[size_t(k)] > 31 ? 31 : bits[size_t(k)];
                size_t fp = 0;
                if (lfmm_plan_footprint_bytes(ctx, r.n, 0, b, &fp) != LFMM_OK || fp == 0) fp = ~size_t(0) / 4;
                r.footprint = fp;
                if (fp > opt.hbm_budget_bytes) reject.push_back(todo[size_t(k)]);
            }
            for (auto& r : reject) queue.erase(std::find(queue.begin(), queue.end(), r));
        }
        for (auto& r : reject) finish(r, LFMM_E_NOMEM, now());
    }

    // requests for the next iteration, in arrival order, within the limits
    std::vector<std::shared_ptr<Request>> admit() {
        std::vector<std::shared_ptr<Request>> out;
        std::lock_guard<std::mutex> lock(mu);
        int64_t pts = 0;
        size_t bytes = 0;
        while (!queue.empty() && int32_t(out.size()) < opt.max_batch) {
            const auto& r = queue.front();
            if (r->footprint == 0) break;   // not measured yet
            if (!out.empty() && (r->solo || out.front()->solo)) break;
            if (!out.empty() && pts + r->n > opt.max_batch_points) break;
            if (inflight_bytes + bytes + r->footprint > opt.hbm_budget_bytes) break;
            pts += r->n;
            bytes += r->footprint;
            r->st.t_admit = now();
            out.push_back(r);
            queue.pop_front();
        }
        return out;
    }

    // builds and launches one iteration on stream slot s
    lfmm_status launch(std::vector<std::shared_ptr<Request>>& reqs, int s) {
        const int32_t K = int32_t(reqs.size());
        std::vector<int64_t> sizes(static_cast<size_t>(K));
        std::vector<const int32_t*> xy(static_cast<size_t>(K));
        std::vector<const double*> f(static_cast<size_t>(K));
        std::vector<double*> u(static_cast<size_t>(K));
        size_t bytes = 0;
        for (int32_t k = 0; k < K; ++k) {
            sizes[size_t(k)] = reqs[size_t(k)]->n;
            xy[size_t(k)] = reqs[size_t(k)]->xy;
            f[size_t(k)] = reqs[size_t(k)]->f;
            u[size_t(k)] = reqs[size_t(k)]->u;
            bytes += reqs[size_t(k)]->footprint;
            // the producer's writes of xy and f come first
            if (hipStreamWaitEvent(streams[size_t(s)], reqs[size_t(k)]->ready, 0) != hipSuccess) return LFMM_E_HIP;
        }
        lfmm_plan* plan = nullptr;
        lfmm_status st = lfmm_plan_create_batch(ctx, K, sizes.data(), xy.data(), nullptr, nullptr, streams[size_t(s)],
                                                &plan);
        if (st != LFMM_OK) return st;
        st = lfmm_execute_instances(plan, f.data(), u.data(), streams[size_t(s)]);
        hipEvent_t ev = nullptr;
        if (st == LFMM_OK && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) st = LFMM_E_HIP;
        if (st == LFMM_OK && hipEventRecord(ev, streams[size_t(s)]) != hipSuccess) st = LFMM_E_HIP;
        if (st != LFMM_OK) {
            (void)hipGetLastError();
            if (ev) (void)hipEventDestroy(ev);
            lfmm_plan_destroy(plan);
            return st;
        }
        const int64_t b = next_batch++;
        {
            std::lock_guard<std::mutex> lock(mu);
            for (auto& r : reqs) {
                r->st.batch_id = b;
                r->st.batch_size = K;
            }
        }
        Inflight it;
        it.plan = plan;
        it.done = ev;
        it.stream = s;
        it.footprint = bytes;
        it.reqs = reqs;
        inflight.push_back(std::move(it));
        inflight_bytes += bytes;
        stream_busy[size_t(s)] = true;
        return LFMM_OK;
    }

    void run() {
        (void)hipSetDevice(ctx_device(ctx));
        for (;;) {
            retire();
            measure();
            int free_slot = -1;
            for (size_t s = 0; s < stream_busy.size(); ++s)
                if (!stream_busy[s]) {
                    free_slot = int(s);
                    break;
                }
            std::vector<std::shared_ptr<Request>> reqs;
            if (free_slot >= 0) reqs = admit();
            if (!reqs.empty()) {
                const lfmm_status st = launch(reqs, free_slot);
                if (st != LFMM_OK) {
                    if (reqs.size() == 1) {
                        finish(reqs[0], st, now());
                    } else {
                        // one request may be at fault (say, an extent out of range): put the
                        // batch back at the head of the queue, to be served one by one
                        std::lock_guard<std::mutex> lock(mu);
                        for (auto r = reqs.rbegin(); r != reqs.rend(); ++r) {
                            (*r)->solo = true;
                            queue.push_front(*r);
                        }
                    }
                }
                continue;
            }
            std::unique_lock<std::mutex> lock(mu);
            if (stop && queue.empty() && inflight.empty()) return;
            if (inflight.empty()) {
                cv_work.wait(lock, [&] { return stop || !queue.empty(); });
            } else {
                // device work in flight: poll its completion, wake early for new requests
                cv_work.wait_for(lock, std::chrono::microseconds(20));
            }
        }
    }
};

extern "C" {

lfmm_status lfmm_server_create(lfmm_ctx* ctx, const lfmm_server_options* opt, lfmm_server** out) {
    if (!ctx || !out) return fail(LFMM_E_INVAL, "null argument");
    *out = nullptr;
    // admission reserves a plan's footprint bound, which holds for uniform trees only
    if (ctx_flags(ctx) & LFMM_FLAG_ADAPTIVE)
        return fail(LFMM_E_UNSUPPORTED, "servers build uniform trees (context has LFMM_FLAG_ADAPTIVE)");
    lfmm_server_options o{};
    if (opt) o = *opt;
    if (o.max_batch < 0 || o.max_inflight < 0 || o.max_batch_points < 0)
        return fail(LFMM_E_INVAL, "negative server limit");
    if (o.max_batch == 0) o.max_batch = 256;
    if (o.max_inflight == 0) o.max_inflight = 3;
    if (o.max_batch_points == 0) o.max_batch_points = int64_t(1) << 24;
    if (o.max_inflight > 16) return fail(LFMM_E_INVAL, "max_inflight above 16");
    if (hipSetDevice(ctx_device(ctx)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LFMM_E_HIP, "hipSetDevice failed");
    }
    if (o.hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LFMM_E_HIP, "hipMemGetInfo failed");
        }
        o.hbm_budget_bytes = fr / 2;
    }
    auto srv = std::make_unique<lfmm_server>();
    srv->ctx = ctx;
    srv->opt = o;
    srv->t0 = Clock::now();
    for (int s = 0; s < o.max_inflight; ++s) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            for (hipStream_t x : srv->streams) (void)hipStreamDestroy(x);
            return fail(LFMM_E_HIP, "hipStreamCreate failed");
        }
        srv->streams.push_back(st);
        srv->stream_busy.push_back(false);
    }
    if (hipStreamCreateWithFlags(&srv->probe, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        for (hipStream_t x : srv->streams) (void)hipStreamDestroy(x);
        return fail(LFMM_E_HIP, "hipStreamCreate failed");
    }
    lfmm_server* raw = srv.get();
    srv->worker = std::thread([raw] { raw->run(); });
    ctx_add_server(ctx, raw);
    *out = srv.release();
    return LFMM_OK;
}

lfmm_status lfmm_server_submit(lfmm_server* srv, int64_t n, const int32_t* xy, const double* f, double* u,
                               void* producer_stream, uint64_t* ticket) {
    if (!srv || !ticket || !xy || !f || !u) return fail(LFMM_E_INVAL, "null argument");
    if (n < 1 || n > (int64_t(1) << 30)) return fail(LFMM_E_INVAL, "n must lie in [1, 2^30]");
    auto r = std::make_shared<Request>();
    r->n = n;
    r->xy = xy;
    r->f = f;
    r->u = u;
    {
        // the caller's current device is left as it was
        int prev = -1;
        (void)hipGetDevice(&prev);
        const bool ok = hipSetDevice(ctx_device(srv->ctx)) == hipSuccess &&
                        hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) == hipSuccess &&
                        hipEventRecord(r->ready, reinterpret_cast<hipStream_t>(producer_stream)) == hipSuccess;
        if (prev >= 0) (void)hipSetDevice(prev);
        if (!ok) {
            (void)hipGetLastError();
            return fail(LFMM_E_HIP, "event on the producer stream failed");
        }
    }
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        if (srv->stop) return fail(LFMM_E_INVAL, "server is stopping");
        r->ticket = srv->next_ticket++;
        r->st.t_submit = srv->now();
        r->st.batch_id = -1;
        srv->queue.push_back(r);
        srv->all.emplace(r->ticket, r);
        *ticket = r->ticket;
    }
    srv->cv_work.notify_one();
    return LFMM_OK;
}

lfmm_status lfmm_server_wait(lfmm_server* srv, uint64_t ticket, double timeout_s, lfmm_request_stats* out) {
    if (!srv) return fail(LFMM_E_INVAL, "null server");
    std::unique_lock<std::mutex> lock(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) return fail(LFMM_E_INVAL, "unknown ticket");
    std::shared_ptr<Request> r = it->second;
    auto ready = [&] { return r->done; };
    if (timeout_s < 0) {
        srv->cv_done.wait(lock, ready);
    } else if (!srv->cv_done.wait_for(lock, std::chrono::duration<double>(timeout_s), ready)) {
        return fail(LFMM_E_BUSY, "request not done yet");
    }
    if (out) *out = r->st;
    srv->all.erase(ticket);
    const lfmm_status s = lfmm_status(r->st.status);
    if (s != LFMM_OK) return fail(s, "request failed");
    return LFMM_OK;
}

lfmm_status lfmm_server_destroy(lfmm_server* srv) {
    if (!srv) return LFMM_OK;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
    if (srv->probe) (void)hipStreamDestroy(srv->probe);
    ctx_remove_server(srv->ctx, srv);
    delete srv;
    return LFMM_OK;
}

}  // extern "C"
