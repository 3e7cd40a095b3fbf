// Serving loop: continuous batching of independent space-time heat solves
// on one GPU.
//
// Two threads per server.  The setup thread does everything that allocates
// or frees device memory or runs long on the host: the FP64 setup of a new
// problem shape (sth_setup), the right-hand side (sth_load_rhs) and the
// release of evicted setups.  The scheduler thread admits requests and
// drives every admitted solve one V-cycle at a time on the request's own
// stream (individual launches, speculative cycles guarded by device flags),
// polling one event per request, so the solves of
// different requests overlap on the device and a request that arrives while
// others run starts as soon as a stream and memory are free.  Admission is
// first come, first served, by device footprint against a fixed budget;
// setups are cached by problem description and reused (idle ones are
// evicted least recently used first).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sth.h"
#include "solve_async.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

std::string problem_key(const sth_problem& p) {
    char buf[384];
    std::snprintf(buf, sizeof buf, "%d|%d|%d|%d|%d|%.17g|%.17g|%.17g|%d|%d|%d|%d|%d|%d|%.17g|%d", p.dim, p.n_elem,
                  p.degree, p.n_slabs, p.n_elem_t, p.T, p.theta, p.omega, p.nu_pre, p.nu_post, (int)p.transform_prec,
                  p.coarse_slabs, p.iterate_basis, p.temporal_form, p.space_ratio, p.minres_iters);
    return buf;
}

// a cached setup with its own right-hand side and iterate (the request's
// result is copied out of u when its solve ends)
struct Entry {
    std::string key;
    sth_handle* h = nullptr;
    double* f = nullptr;
    double* u = nullptr;
    size_t bytes = 0;
    size_t vec_len = 0;
    bool busy = false;
    Clock::time_point last_used;
};

enum class St : int { Pending, Setup, Ready, SetupFailed, Running, Finishing, Done };

struct Request {
    long long ticket = 0;
    sth_problem prob{};
    std::vector<double> amp, omega, phase;
    std::vector<int> k;
    double rtol = 0.0;
    int maxit = 0;
    double* u_out = nullptr;
    size_t vec_len = 0, footprint = 0;
    std::string key;
    std::atomic<St> state{St::Pending};
    Entry* entry = nullptr;
    int slot = -1;
    int status = STH_EAGAIN;
    int iters = 0;
    double relres = 0.0;
    bool reused = false;
    std::string msg;
    Clock::time_point t_submit, t_admit, t_ready, t_done;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    hipEvent_t wait = nullptr;      // ev, or the solve's own event (a speculative cycle may follow it)
    Request* req = nullptr;
};

void free_entry(Entry* e) {
    if (e->h) (void)sth_destroy(e->h);
    if (e->f) (void)hipFree(e->f);
    if (e->u) (void)hipFree(e->u);
    e->h = nullptr;
    e->f = e->u = nullptr;
}

}  // namespace

struct sth_server {
    int device = 0;
    size_t budget = 0, resident = 0;
    std::vector<Slot> slots;
    std::list<std::unique_ptr<Entry>> entries;
    std::deque<Request*> pending, setup_q;
    std::vector<std::unique_ptr<Entry>> to_free;    // evicted, released by the setup thread
    std::map<long long, std::unique_ptr<Request>> reqs;
    long long next_ticket = 1;
    int in_flight = 0;                              // admitted and not finished
    bool stop = false;
    bool graphs = false;                            // new setups replay captured iterations
    std::mutex mu;                                  // everything above
    std::condition_variable cv_sched, cv_setup, cv_done;
    std::mutex alloc_mu;                            // device (de)allocation vs graph capture (handles with graphs on)
    hipStream_t setup_st = nullptr;
    std::thread sched, setup;
};

namespace {

// under s->mu: start pending requests while a stream is free and memory fits
void admit(sth_server* s) {
    while (!s->pending.empty()) {
        int free_slot = -1;
        for (size_t i = 0; i < s->slots.size(); ++i)
            if (!s->slots[i].req) {
                free_slot = (int)i;
                break;
            }
        if (free_slot < 0) return;
        Request* r = s->pending.front();
        Entry* e = nullptr;
        for (auto& up : s->entries)
            if (!up->busy && up->key == r->key) {
                e = up.get();
                break;
            }
        if (e) {
            r->reused = true;
        } else {
            while (s->resident + r->footprint > s->budget) {
                auto victim = s->entries.end();
                for (auto it = s->entries.begin(); it != s->entries.end(); ++it)
                    if (!(*it)->busy && (victim == s->entries.end() || (*it)->last_used < (*victim)->last_used))
                        victim = it;
                if (victim == s->entries.end()) break;
                s->resident -= (*victim)->bytes;
                s->to_free.push_back(std::move(*victim));
                s->entries.erase(victim);
            }
            if (!s->to_free.empty()) s->cv_setup.notify_one();
            if (s->resident + r->footprint > s->budget) return;     // wait for running requests
            auto up = std::make_unique<Entry>();
            up->key = r->key;
            up->bytes = r->footprint;
            up->vec_len = r->vec_len;
            e = up.get();
            s->entries.push_back(std::move(up));
            s->resident += r->footprint;
        }
        e->busy = true;
        r->entry = e;
        r->slot = free_slot;
        s->slots[free_slot].req = r;
        r->t_admit = Clock::now();
        r->state = St::Setup;
        s->pending.pop_front();
        s->setup_q.push_back(r);
        ++s->in_flight;
        s->cv_setup.notify_one();
    }
}

// setup thread: new setups, right-hand sides, releases (all allocation here)
int prepare(sth_server* s, Request* r, std::string& msg) {
    Entry* e = r->entry;
    int rc;
    if (!e->h) {
        if ((rc = sth_setup(&r->prob, (void*)s->setup_st, &e->h))) {
            msg = sth_last_error();
            return rc;
        }
        bool graphs;
        {
            std::lock_guard<std::mutex> g(s->mu);
            graphs = s->graphs;
        }
        if (graphs && (rc = sth_use_graphs(e->h, 1))) {
            msg = sth_last_error();
            return rc;
        }
        if (hipMalloc((void**)&e->f, e->vec_len * sizeof(double)) != hipSuccess ||
            hipMalloc((void**)&e->u, e->vec_len * sizeof(double)) != hipSuccess) {
            msg = "device allocation of the request vectors failed";
            return STH_ENOMEM;
        }
    }
    sth_rhs_modes m{(int)r->amp.size(), r->amp.data(), r->k.data(), r->omega.data(), r->phase.data()};
    if ((rc = sth_load_rhs(e->h, &m, e->f, (void*)s->setup_st))) {
        msg = sth_last_error();
        return rc;
    }
    if (hipMemsetAsync(e->u, 0, e->vec_len * sizeof(double), s->setup_st) != hipSuccess ||
        hipStreamSynchronize(s->setup_st) != hipSuccess) {
        msg = "clearing the initial guess failed";
        return STH_EHIP;
    }
    return STH_OK;
}

void setup_main(sth_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_setup.wait(lk, [&] { return s->stop || !s->setup_q.empty() || !s->to_free.empty(); });
        if (!s->to_free.empty()) {
            auto victims = std::move(s->to_free);
            s->to_free.clear();
            lk.unlock();
            {
                std::lock_guard<std::mutex> g(s->alloc_mu);
                for (auto& v : victims) free_entry(v.get());
            }
            lk.lock();
            continue;
        }
        if (s->setup_q.empty()) {
            if (s->stop) return;
            continue;
        }
        Request* r = s->setup_q.front();
        s->setup_q.pop_front();
        lk.unlock();
        std::string msg;
        int rc;
        {
            std::lock_guard<std::mutex> g(s->alloc_mu);
            rc = prepare(s, r, msg);
        }
        lk.lock();
        r->t_ready = Clock::now();
        if (rc) {
            r->status = rc;
            r->msg = msg;
            r->state = St::SetupFailed;
        } else {
            r->state = St::Ready;
        }
        s->cv_sched.notify_one();
    }
}

// under s->mu: the request is over (its stream has no pending work)
void finalize(sth_server* s, Request* r) {
    Entry* e = r->entry;
    if (e) {
        if (!e->h) {                    // setup never completed: drop the reservation
            for (auto it = s->entries.begin(); it != s->entries.end(); ++it)
                if (it->get() == e) {
                    s->resident -= e->bytes;
                    s->to_free.push_back(std::move(*it));
                    s->entries.erase(it);
                    s->cv_setup.notify_one();
                    break;
                }
        } else {
            e->busy = false;
            e->last_used = Clock::now();
        }
    }
    s->slots[r->slot].req = nullptr;
    r->t_done = Clock::now();
    --s->in_flight;
    r->state = St::Done;
    s->cv_done.notify_all();
}

// Advances one request whose stream work may have completed; returns true
// if it made progress.  Runs on the scheduler thread without s->mu.
bool advance(sth_server* s, Slot& sl, Request* r, bool* over) {
    *over = false;
    Entry* e = r->entry;
    St st = r->state.load();
    if (st == St::SetupFailed) {
        *over = true;
        return true;
    }
    if (st == St::Running || st == St::Finishing) {
        hipError_t q = hipEventQuery(sl.wait ? sl.wait : sl.ev);
        if (q == hipErrorNotReady) return false;
        if (q != hipSuccess) {
            r->status = STH_EHIP;
            r->msg = std::string("stream work failed: ") + hipGetErrorString(q);
            (void)hipStreamSynchronize(sl.st);
            *over = true;
            return true;
        }
    }
    int rc = STH_OK;
    if (st == St::Ready || st == St::Running) {
        const bool locked = s->alloc_mu.try_lock();
        sth::solve_allow_capture(e->h, locked);
        bool more = true;
        if (st == St::Ready)
            rc = sth::solve_begin(e->h, e->f, e->u, r->rtol, r->maxit, sl.st);
        else
            rc = sth::solve_continue(e->h, &more);
        if (locked) s->alloc_mu.unlock();
        if (rc == STH_OK && !more) {
            if (hipMemcpyAsync(r->u_out, e->u, e->vec_len * sizeof(double), hipMemcpyDeviceToDevice, sl.st) !=
                hipSuccess)
                rc = STH_EHIP;
            else
                st = St::Finishing;
        } else if (rc == STH_OK) {
            st = St::Running;
        }
        if (rc == STH_OK && hipEventRecord(sl.ev, sl.st) != hipSuccess) rc = STH_EHIP;
        sl.wait = sl.ev;
        if (rc == STH_OK && st == St::Running) {
            hipEvent_t w = sth::solve_wait_event(e->h);
            if (w) sl.wait = w;
        }
        if (rc) {
            r->status = rc;
            r->msg = sth_last_error();
            (void)hipStreamSynchronize(sl.st);
            *over = true;
            return true;
        }
        r->state = st;
        return true;
    }
    if (st == St::Finishing) {
        r->status = sth::solve_result(e->h, &r->iters, &r->relres);
        r->msg = r->status ? sth_last_error() : "";
        *over = true;
        return true;
    }
    return false;
}

void sched_main(sth_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    std::vector<std::pair<int, Request*>> work;
    for (;;) {
        admit(s);
        work.clear();
        bool gpu_busy = false;
        for (size_t i = 0; i < s->slots.size(); ++i) {
            Request* r = s->slots[i].req;
            if (!r) continue;
            St st = r->state.load();
            if (st == St::Ready || st == St::SetupFailed || st == St::Running || st == St::Finishing)
                work.emplace_back((int)i, r);
            if (st == St::Running || st == St::Finishing) gpu_busy = true;
        }
        if (s->stop && s->in_flight == 0 && s->pending.empty()) return;
        bool progressed = false;
        if (!work.empty()) {
            lk.unlock();
            std::vector<Request*> over;
            for (auto& w : work) {
                bool done = false;
                progressed |= advance(s, s->slots[w.first], w.second, &done);
                if (done) over.push_back(w.second);
            }
            lk.lock();
            for (Request* r : over) finalize(s, r);
        }
        if (!progressed) {
            // poll in-flight GPU work closely; otherwise sleep until notified
            if (gpu_busy)
                s->cv_sched.wait_for(lk, std::chrono::microseconds(20));
            else
                s->cv_sched.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

void fill_stats(const Request* r, sth_request_stats* out) {
    if (!out) return;
    std::memset(out, 0, sizeof(*out));
    out->status = r->status;
    out->iters = r->iters;
    out->relres = r->relres;
    out->queue_ms = ms_between(r->t_submit, r->t_admit);
    out->setup_ms = ms_between(r->t_admit, r->t_ready);
    out->solve_ms = ms_between(r->t_ready, r->t_done);
    out->latency_ms = ms_between(r->t_submit, r->t_done);
    out->footprint_bytes = r->footprint;
    out->setup_reused = r->reused ? 1 : 0;
    std::snprintf(out->message, sizeof out->message, "%s", r->msg.c_str());
}

}  // namespace

extern "C" {

int sth_server_create(size_t hbm_budget_bytes, int max_active, sth_server** out) {
    if (!out || hbm_budget_bytes == 0 || max_active < 1 || max_active > 64) return STH_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return STH_ENODEV;
    auto* s = new sth_server();
    s->budget = hbm_budget_bytes;
    (void)hipGetDevice(&s->device);
    bool ok = hipStreamCreateWithFlags(&s->setup_st, hipStreamNonBlocking) == hipSuccess;
    s->slots.resize(max_active);
    for (auto& sl : s->slots) {
        ok = ok && hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
        for (auto& sl : s->slots) {
            if (sl.ev) (void)hipEventDestroy(sl.ev);
            if (sl.st) (void)hipStreamDestroy(sl.st);
        }
        if (s->setup_st) (void)hipStreamDestroy(s->setup_st);
        delete s;
        return STH_EHIP;
    }
    s->setup = std::thread(setup_main, s);
    s->sched = std::thread(sched_main, s);
    *out = s;
    return STH_OK;
}

int sth_server_submit(sth_server* s, const sth_problem* p, const sth_rhs_modes* rhs, double rtol, int maxit,
                      double* u_out, long long* ticket) {
    if (!s || !p || !rhs || !u_out || !ticket || !(rtol >= 0) || maxit < 0) return STH_EINVAL;
    if (rhs->n_modes < 0 || (rhs->n_modes > 0 && (!rhs->amp || !rhs->k || !rhs->omega || !rhs->phase)))
        return STH_EINVAL;
    size_t ws = 0;
    int rc = sth_workspace_bytes(p, &ws);
    if (rc) return rc;
    auto r = std::make_unique<Request>();
    r->prob = *p;
    r->vec_len = sth_problem_vector_len(p);
    r->footprint = ws + 2 * r->vec_len * sizeof(double);
    if (r->footprint > s->budget) return STH_ENOMEM;
    const int M = rhs->n_modes;
    r->amp.assign(rhs->amp, rhs->amp + M);
    r->omega.assign(rhs->omega, rhs->omega + M);
    r->phase.assign(rhs->phase, rhs->phase + M);
    r->k.assign(rhs->k, rhs->k + (size_t)M * p->dim);
    r->rtol = rtol;
    r->maxit = maxit;
    r->u_out = u_out;
    r->key = problem_key(*p);
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return STH_EINVAL;
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->pending.push_back(r.get());
    s->reqs[r->ticket] = std::move(r);
    s->cv_sched.notify_one();
    return STH_OK;
}

int sth_server_poll(sth_server* s, long long ticket, sth_request_stats* stats) {
    if (!s) return STH_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return STH_EINVAL;
    if (it->second->state.load() != St::Done) return STH_EAGAIN;
    fill_stats(it->second.get(), stats);
    s->reqs.erase(it);
    return STH_OK;
}

int sth_server_wait(sth_server* s, long long ticket, sth_request_stats* stats) {
    if (!s) return STH_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return STH_EINVAL;
    Request* r = it->second.get();
    s->cv_done.wait(lk, [&] { return r->state.load() == St::Done; });
    fill_stats(r, stats);
    s->reqs.erase(ticket);
    return STH_OK;
}

int sth_server_use_graphs(sth_server* s, int enable) {
    if (!s) return STH_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    s->graphs = enable != 0;
    return STH_OK;
}

int sth_server_resident(sth_server* s, size_t* bytes, int* setups) {
    if (!s) return STH_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    if (bytes) *bytes = s->resident;
    if (setups) *setups = (int)s->entries.size();
    return STH_OK;
}

int sth_server_destroy(sth_server* s) {
    if (!s) return STH_OK;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->in_flight == 0 && s->pending.empty(); });
        s->stop = true;
        s->cv_sched.notify_all();
        s->cv_setup.notify_all();
    }
    s->sched.join();
    s->setup.join();
    for (auto& v : s->to_free) free_entry(v.get());
    for (auto& e : s->entries) free_entry(e.get());
    for (auto& sl : s->slots) {
        (void)hipStreamSynchronize(sl.st);
        (void)hipEventDestroy(sl.ev);
        (void)hipStreamDestroy(sl.st);
    }
    (void)hipStreamDestroy(s->setup_st);
    delete s;
    return STH_OK;
}

}  // extern "C"
