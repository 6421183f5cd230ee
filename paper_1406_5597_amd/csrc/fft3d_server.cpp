// fft3d_server.cpp -- the served form: continuous batching of r2c / c2r
// requests under an HBM budget (see include/fft3d.h, "Serving").
//
// One dispatcher thread per server runs a loop over three steps, under the
// server's lock:
//   1. completion: a launched unit whose event has fired completes its
//      requests (their work buffers go back to the arena);
//   2. admission: waiting requests, first come first served, get their
//      outputs and work buffers from the arena while they fit;
//   3. launch: every admitted request is launched at once -- the small ones
//      together through one batched launch per max_batch_items fields, each
//      large one through the single-field path -- on the server stream with
//      the least estimated work in flight, and an event is recorded behind it.
// The loop sleeps on a condition variable when nothing is in flight and polls
// events every few microseconds otherwise.  The server uses only the public
// entry points of the library for the transforms.
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/fft3d.h"
#include "fft3d_arena.hpp"
#include "fft3d_internal.hpp"

namespace {

enum ReqState { kWaiting = 0, kAdmitted, kLaunched, kDone, kFailed };

struct Req {
    fft3d_request r;
    int state = kWaiting;
    fft3d_plan_t plan = nullptr;
    size_t out_bytes = 0, work_bytes = 0;  // per field
    size_t out_off[FFT3D_SERVER_MAX_COMP] = {}, work_off[FFT3D_SERVER_MAX_COMP] = {};
    bool has_out = false, has_work = false;
    double t_arrive = 0, t_admit = 0, t_launch = 0, t_done = 0;
    std::string err;
    int refs = 0;           // threads waiting on it
    bool released = false;  // erased when the last waiter leaves
};

struct Unit {
    hipEvent_t ev = nullptr;
    int stream = 0;
    double load = 0;  // estimated bytes the unit moves
    int64_t token = -1;  // batched launch: its ring token (error bits read at completion)
    std::vector<int64_t> reqs;
};

int fail(int code, const std::string& m)
{
    fft3d::set_last_error(m);
    return code;
}

}  // namespace

struct fft3d_server_s {
    fft3d_server_config cfg{};
    bool no_device = false;
    int device = -1;
    void* base = nullptr;  // the arena's device region (a fake address without a device)
    fft3d::Arena arena;
    std::vector<hipStream_t> streams;
    std::vector<double> stream_load;  // estimated bytes in flight per stream
    std::vector<hipEvent_t> free_events;
    std::map<std::tuple<int64_t, int64_t, int64_t, int>, fft3d_plan_t> plans;
    std::mutex plan_mu;  // plan creation, outside the main lock

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::unordered_map<int64_t, std::unique_ptr<Req>> reqs;
    std::deque<int64_t> waiting;
    std::vector<int64_t> admitted;
    std::list<Unit> inflight;
    int64_t next_id = 1;
    bool stop = false;
    int waiters = 0;  // threads inside fft3d_server_wait
    fft3d_server_counters st{};
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    std::thread th;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void* at(size_t off) const { return static_cast<char*>(base) + off; }

    void release_buffers(Req& q, bool outs, bool works)
    {
        for (int c = 0; c < q.r.ncomp; ++c) {
            if (outs && q.has_out) arena.free(q.out_off[c], q.out_bytes);
            if (works && q.has_work) arena.free(q.work_off[c], q.work_bytes);
        }
        if (outs && q.has_out) st.reserved_bytes -= (size_t)q.r.ncomp * fft3d::Arena::round(q.out_bytes);
        if (works && q.has_work) st.reserved_bytes -= (size_t)q.r.ncomp * fft3d::Arena::round(q.work_bytes);
        if (outs) q.has_out = false;
        if (works) q.has_work = false;
    }

    // All of a request's blocks, or none.
    bool reserve(Req& q)
    {
        int got_o = 0, got_w = 0;
        bool ok = true;
        for (int c = 0; c < q.r.ncomp && ok; ++c) {
            ok = arena.alloc(q.out_bytes, &q.out_off[c]);
            if (ok) ++got_o;
            if (ok && q.work_bytes) {
                ok = arena.alloc(q.work_bytes, &q.work_off[c]);
                if (ok) ++got_w;
            }
        }
        if (!ok) {
            for (int c = 0; c < got_o; ++c) arena.free(q.out_off[c], q.out_bytes);
            for (int c = 0; c < got_w; ++c) arena.free(q.work_off[c], q.work_bytes);
            return false;
        }
        q.has_out = true;
        q.has_work = q.work_bytes > 0;
        st.reserved_bytes += (size_t)q.r.ncomp * fft3d::Arena::round(q.out_bytes);
        if (q.has_work) st.reserved_bytes += (size_t)q.r.ncomp * fft3d::Arena::round(q.work_bytes);
        if (st.reserved_bytes > st.peak_reserved_bytes) st.peak_reserved_bytes = st.reserved_bytes;
        return true;
    }

    hipEvent_t take_event()
    {
        if (no_device) return nullptr;
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }

    void finish(Req& q, bool ok, const std::string& why)
    {
        q.t_done = now();
        q.state = ok ? kDone : kFailed;
        if (!ok) q.err = why;
        release_buffers(q, !ok, true);  // outputs stay until released (unless failed)
        st.in_flight--;
        st.completed++;
    }

    // Launch a group of admitted requests as one unit on the next stream.
    void launch(const std::vector<int64_t>& ids, bool batched)
    {
        Unit u;
        u.reqs = ids;
        for (int64_t id : ids) {
            const Req& q = *reqs[id];
            u.load += (double)q.r.ncomp * (double)(2 * q.out_bytes + q.work_bytes);
        }
        hipStream_t s = nullptr;
        if (!no_device) {
            // the stream with the least work in flight, so that a small
            // request does not queue behind a large one
            size_t best = 0;
            for (size_t i = 1; i < streams.size(); ++i)
                if (stream_load[i] < stream_load[best]) best = i;
            s = streams[best];
            u.stream = (int)best;
            stream_load[best] += u.load;
        }
        const double t = now();
        int rc = FFT3D_OK;
        std::string why;
        if (!no_device) {
            if (batched) {
                std::vector<fft3d_batch_item> items;
                for (int64_t id : ids) {
                    Req& q = *reqs[id];
                    for (int c = 0; c < q.r.ncomp; ++c)
                        items.push_back({q.plan, q.r.dir, q.r.in[c], nullptr, at(q.out_off[c]),
                                         q.has_work ? at(q.work_off[c]) : nullptr});
                }
                rc = fft3d_batch_submit_checked(items.data(), (int)items.size(), s, &u.token);
                // every ring slot in flight: the same items through their own
                // kernels instead (nothing was enqueued; the submit never waits)
                if (rc == FFT3D_ERR_BUSY) {
                    batched = false;
                    rc = fft3d_batch_submit_ex(items.data(), (int)items.size(), FFT3D_BATCH_SEQUENTIAL, s);
                }
            } else {
                for (int64_t id : ids) {
                    Req& q = *reqs[id];
                    for (int c = 0; c < q.r.ncomp && rc == FFT3D_OK; ++c) {
                        if (q.r.dir == FFT3D_R2C) rc = fft3d_r2c(q.plan, q.r.in[c], at(q.out_off[c]), s);
                        else
                            rc = fft3d_c2r(q.plan, const_cast<void*>(q.r.in[c]), at(q.out_off[c]),
                                           q.has_work ? at(q.work_off[c]) : nullptr, s);
                    }
                }
            }
            if (rc != FFT3D_OK) why = fft3d_last_error();
            if (rc == FFT3D_OK) {
                u.ev = take_event();
                if (!u.ev || hipEventRecord(u.ev, s) != hipSuccess) {
                    rc = FFT3D_ERR_HIP;
                    why = "event record failed";
                }
            }
        }
        for (int64_t id : ids) {
            Req& q = *reqs[id];
            q.t_launch = t;
            q.state = kLaunched;
        }
        if (batched) st.batched_launches++;
        else st.single_launches++;
        if (rc != FFT3D_OK) {
            // nothing of this unit is known to run: fail its requests once the
            // stream has drained what was enqueued
            if (!no_device) {
                (void)hipStreamSynchronize(s);
                stream_load[(size_t)u.stream] -= u.load;
            }
            for (int64_t id : ids) finish(*reqs[id], false, why);
            if (u.ev) free_events.push_back(u.ev);
            cv_done.notify_all();
            return;
        }
        inflight.push_back(std::move(u));
    }

    void loop()
    {
        if (!no_device) (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            // 1. completions
            bool any_done = false;
            for (auto it = inflight.begin(); it != inflight.end();) {
                hipError_t e = no_device ? hipSuccess : hipEventQuery(it->ev);
                if (e == hipErrorNotReady) {
                    ++it;
                    continue;
                }
                std::string why = e == hipSuccess ? "" : hipGetErrorString(e);
                if (e == hipSuccess && it->token != -1) {
                    // the batched kernel's error bits (a dependency wait that
                    // ran out, a queue without workgroups): its results are void
                    const int bits = fft3d_batch_check(it->token);
                    if (bits != 0) {
                        e = hipErrorUnknown;
                        why = bits < 0 ? std::string("batched launch: ") + fft3d_last_error()
                                       : "batched launch reported error bits " + std::to_string(bits);
                    }
                }
                for (int64_t id : it->reqs) finish(*reqs[id], e == hipSuccess, why);
                if (it->ev) free_events.push_back(it->ev);
                if (!no_device) stream_load[(size_t)it->stream] -= it->load;
                it = inflight.erase(it);
                any_done = true;
            }
            if (any_done) cv_done.notify_all();
            // 2. admission, first come first served
            while (!waiting.empty()) {
                Req& q = *reqs[waiting.front()];
                if (!reserve(q)) break;
                q.state = kAdmitted;
                q.t_admit = now();
                admitted.push_back(waiting.front());
                waiting.pop_front();
                st.waiting--;
                st.admitted++;
                st.in_flight++;
            }
            // 3. launch everything admitted: small requests batched
            if (!admitted.empty()) {
                std::vector<int64_t> small;
                int fields = 0;
                for (int64_t id : admitted) {
                    Req& q = *reqs[id];
                    if (q.r.n0 * q.r.n1 * q.r.n2 <= cfg.batch_points) {
                        if (fields + q.r.ncomp > cfg.max_batch_items && !small.empty()) {
                            launch(small, true);
                            small.clear();
                            fields = 0;
                        }
                        small.push_back(id);
                        fields += q.r.ncomp;
                    } else {
                        launch({id}, false);
                    }
                }
                if (!small.empty()) launch(small, true);
                admitted.clear();
                continue;  // completions of no_device launches at once
            }
            if (stop && inflight.empty()) {
                // what never fit is dropped
                for (int64_t id : waiting) {
                    Req& q = *reqs[id];
                    q.state = kFailed;
                    q.err = "server stopped";
                    q.t_done = now();
                }
                st.waiting = 0;
                waiting.clear();
                cv_done.notify_all();
                break;
            }
            if (!inflight.empty()) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(10));
                lk.lock();
            } else {
                cv_work.wait(lk);
            }
        }
    }
};

namespace {

fft3d_plan_t plan_for(fft3d_server_s* s, const fft3d_request* r, int* rc)
{
    std::lock_guard<std::mutex> g(s->plan_mu);
    auto key = std::make_tuple(r->n0, r->n1, r->n2, r->dtype);
    auto it = s->plans.find(key);
    if (it != s->plans.end()) return it->second;
    fft3d_plan_t p = nullptr;
    *rc = fft3d_plan_ex(r->n0, r->n1, r->n2, r->dtype, s->no_device ? FFT3D_PLAN_HOST_ONLY : 0, &p);
    if (*rc) return nullptr;
    s->plans[key] = p;
    return p;
}

}  // namespace

extern "C" {

int fft3d_server_create(const fft3d_server_config* cfg, fft3d_server_t* out)
{
    if (!cfg || !out) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_create: NULL argument");
    *out = nullptr;
    if (cfg->budget_bytes < fft3d::Arena::kAlign || cfg->nstreams < 0 || cfg->nstreams > 16 ||
        cfg->batch_points < 0 || cfg->max_batch_items < 0 || (cfg->flags & ~FFT3D_SERVER_NO_DEVICE))
        return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_create: bad configuration");
    std::unique_ptr<fft3d_server_s> s(new (std::nothrow) fft3d_server_s);
    if (!s) return fail(FFT3D_ERR_NOMEM, "fft3d_server_create: out of host memory");
    s->cfg = *cfg;
    if (!s->cfg.nstreams) s->cfg.nstreams = 4;
    if (!s->cfg.batch_points) s->cfg.batch_points = (int64_t)1 << 21;
    if (!s->cfg.max_batch_items) s->cfg.max_batch_items = 192;
    s->no_device = (cfg->flags & FFT3D_SERVER_NO_DEVICE) != 0;
    s->arena.reset(cfg->budget_bytes);
    s->st.budget_bytes = s->arena.size();
    if (s->no_device) {
        s->base = reinterpret_cast<void*>((uintptr_t)1 << 44);
    } else {
        hipError_t e = hipGetDevice(&s->device);
        if (e != hipSuccess) return fail(FFT3D_ERR_HIP, std::string("fft3d_server_create: ") + hipGetErrorString(e));
        // the device's batch ring (allocated once per device)
        if (int rc = fft3d_init()) return rc;
        e = hipMalloc(&s->base, s->arena.size());
        if (e != hipSuccess) {
            s->base = nullptr;
            return fail(FFT3D_ERR_NOMEM, std::string("fft3d_server_create: arena: ") + hipGetErrorString(e));
        }
        for (int i = 0; i < s->cfg.nstreams; ++i) {
            hipStream_t st = nullptr;
            if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) break;
            s->streams.push_back(st);
            s->stream_load.push_back(0.0);
        }
        if (e != hipSuccess) {
            for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
            (void)hipFree(s->base);
            return fail(FFT3D_ERR_HIP, std::string("fft3d_server_create: streams: ") + hipGetErrorString(e));
        }
    }
    fft3d_server_s* raw = s.release();
    raw->th = std::thread([raw] { raw->loop(); });
    *out = raw;
    return FFT3D_OK;
}

int fft3d_server_submit(fft3d_server_t s, const fft3d_request* r, int64_t* id)
{
    if (!s || !r || !id) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_submit: NULL argument");
    *id = 0;
    if ((r->dir != FFT3D_R2C && r->dir != FFT3D_C2R) || r->ncomp < 1 || r->ncomp > FFT3D_SERVER_MAX_COMP ||
        (r->dtype != FFT3D_F32 && r->dtype != FFT3D_F64))
        return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_submit: bad request");
    const int align = r->dtype == FFT3D_F64 ? 16 : 8;
    for (int c = 0; c < r->ncomp; ++c)
        if (!r->in[c] || (uintptr_t)r->in[c] % (uintptr_t)align)
            return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_submit: input missing or misaligned");
    int rc = FFT3D_OK;
    fft3d_plan_t p = plan_for(s, r, &rc);
    if (!p) return fail(rc, std::string("fft3d_server_submit: ") + fft3d_last_error());
    std::unique_ptr<Req> q(new Req);
    q->r = *r;
    q->plan = p;
    const size_t rb = fft3d_real_bytes(p), cb = fft3d_complex_bytes(p);
    q->out_bytes = r->dir == FFT3D_R2C ? cb : rb;
    q->work_bytes = r->dir == FFT3D_C2R ? cb : 0;  // keeps the caller's spectrum intact
    const size_t need = (size_t)r->ncomp * (fft3d::Arena::round(q->out_bytes) + fft3d::Arena::round(q->work_bytes));
    if (need > s->arena.size()) return fail(FFT3D_ERR_BUDGET, "fft3d_server_submit: request larger than the budget");
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_submit: server is stopping");
        q->t_arrive = s->now();
        *id = s->next_id++;
        s->reqs[*id] = std::move(q);
        s->waiting.push_back(*id);
        s->st.submitted++;
        s->st.waiting++;
    }
    s->cv_work.notify_one();
    return FFT3D_OK;
}

int fft3d_server_wait(fft3d_server_t s, int64_t id, double timeout_s)
{
    if (!s) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_wait: NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || it->second->released)
        return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_wait: unknown request");
    Req* q = it->second.get();
    auto done = [q] { return q->state == kDone || q->state == kFailed; };
    s->waiters++;
    q->refs++;
    bool ok = true;
    if (timeout_s < 0) s->cv_done.wait(lk, done);
    else ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
    const bool failed = ok && q->state == kFailed;
    const std::string why = failed ? q->err : std::string();
    if (--q->refs == 0 && q->released) s->reqs.erase(id);
    if (--s->waiters == 0) s->cv_done.notify_all();  // fft3d_server_destroy may wait for this
    if (!ok) return 0;
    if (failed) return fail(FFT3D_ERR_HIP, "fft3d_server_wait: request failed: " + why);
    return 1;
}

int fft3d_server_result(fft3d_server_t s, int64_t id, void** out, double* times)
{
    if (!s) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_result: NULL server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_result: unknown request");
    const Req& q = *it->second;
    if (q.released || q.state != kDone || !q.has_out)
        return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_result: request not completed (or released)");
    if (out)
        for (int c = 0; c < q.r.ncomp; ++c) out[c] = s->at(q.out_off[c]);
    if (times) {
        times[0] = q.t_arrive;
        times[1] = q.t_admit;
        times[2] = q.t_launch;
        times[3] = q.t_done;
    }
    return FFT3D_OK;
}

int fft3d_server_release(fft3d_server_t s, int64_t id)
{
    if (!s) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_release: NULL server");
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_release: unknown request");
        Req& q = *it->second;
        if (q.released) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_release: unknown request");
        if (q.state != kDone && q.state != kFailed)
            return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_release: request not completed");
        s->release_buffers(q, true, true);
        q.released = true;
        if (q.refs == 0) s->reqs.erase(it);
        s->st.released++;
    }
    s->cv_work.notify_one();
    return FFT3D_OK;
}

int fft3d_server_stats(fft3d_server_t s, fft3d_server_counters* st)
{
    if (!s || !st) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_server_stats: NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    *st = s->st;
    return FFT3D_OK;
}

int fft3d_server_destroy(fft3d_server_t s)
{
    if (!s) return FFT3D_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_one();
    if (s->th.joinable()) s->th.join();
    {
        // threads still inside fft3d_server_wait leave before the server goes
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.notify_all();
        s->cv_done.wait(lk, [s] { return s->waiters == 0; });
    }
    for (auto& kv : s->plans) fft3d_plan_destroy(kv.second);
    if (!s->no_device) {
        for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        if (s->base) (void)hipFree(s->base);
    }
    delete s;
    return FFT3D_OK;
}

}  // extern "C"
