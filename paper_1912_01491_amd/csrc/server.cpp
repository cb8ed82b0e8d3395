// Serving: a request loop that admits Lindbladians of different N by device
// memory footprint, keeps each request's Q and K resident while it runs, and
// batches propagations of same-shape requests.
//
// Structure:
//   * a FIFO of submitted requests (thread-safe submit from any thread);
//   * `slots` worker threads, each with its own HIP stream and library
//     context (workspace pre-sized for the largest N at creation);
//   * admission: a free slot takes the queue head if its footprint fits in the
//     remaining budget (head-of-line order is kept: a head that does not fit
//     waits for memory to be released), then also takes up to max_batch-1
//     further queued dense requests with the same (N, B, dt, steps,
//     precision) that fit, and runs them as one batch: one preparation per
//     request, then a single batched RK4 integration (one launch per stage for
//     all of them);
//   * per-request buffers (Q, K, CSR arrays) come from the stream-ordered
//     allocator of the slot's stream and are released when the batch ends.
// Requests arriving while others run are admitted as soon as a slot and
// memory are free, so their work overlaps on the device. Every kernel used
// here is deterministic for a fixed launch configuration and the tile choice
// does not depend on the batch size, so a request's result is the same alone
// and in a mix.
//
// Resident systems: lindblad_server_register prepares a Lindbladian's Q and K
// once (on a registration context of its own) and keeps them until released;
// LB_REQ_SYSTEM requests on it only carry states. A slot that takes such a
// request also takes the queued requests on the same system (same dt, steps,
// precision) up to LB_SYSTEM_BATCH states, packs their states into one block
// and integrates the block with one pass over Q per stage. Dense systems always
// run the 16-state matrix-core path (a single state is padded with a zero
// state) with the default tile for 16 states, so every state column is summed
// in the same order whatever shares the pass; the CSR kernel treats states
// independently anyway.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "lb_internal.h"

namespace {

double now_s() {
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

struct System {
    int64_t id = 0;
    int kind = LB_REQ_DENSE;
    int N = 0, precision = LB_FP64;
    int64_t M = 0, ldq = 0, nnz = 0;
    void *Q = nullptr, *Q32 = nullptr, *K = nullptr;  // dense
    void *rp = nullptr, *col = nullptr, *val = nullptr;  // sparse (K shared)
    size_t bytes = 0;
    int refs = 0;  // queued or running requests
    bool released = false;
};

struct Ticket {
    lb_request req;
    int64_t id = 0;
    size_t footprint = 0;
    System* sys = nullptr;
    int status = 1;  // 1 = pending, 0 = ok, < 0 = error
    bool done = false;
    double t_submit = 0, t_start = 0, t_end = 0;
};

void system_free(System* y) {
    void* ps[] = {y->Q, y->Q32, y->K, y->rp, y->col, y->val};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    delete y;
}

}  // namespace

struct lb_server {
    int device = 0;
    size_t budget = 0, used = 0, peak = 0;
    int max_batch = 1;
    int max_N = 0;
    std::mutex mu;
    std::condition_variable cv_work;  // slots wait for admissible work
    std::condition_variable cv_done;  // waiters wait for completions
    std::deque<Ticket*> queue;
    std::map<int64_t, Ticket*> tickets;
    int64_t next_id = 1;
    int64_t completed = 0, batches = 0, batched_requests = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<lb_ctx*> ctxs;
    std::vector<hipStream_t> streams;
    // resident systems
    std::map<int64_t, System*> systems;
    int64_t next_system = 1;
    size_t registered = 0;          // bytes held by registered systems
    std::mutex reg_mu;              // serializes registrations (one context)
    lb_ctx* reg_ctx = nullptr;
    hipStream_t reg_stream = nullptr;
};

static size_t dense_q_bytes(int N, int precision) {
    const int64_t M = (int64_t)N * N - 1;
    const int64_t ldq = lb_default_ldq(M);
    size_t b = sizeof(double) * (size_t)M * ldq + sizeof(double) * M;
    if (precision == LB_FP32) b += sizeof(float) * (size_t)M * ldq;
    return b;
}

// Upper estimate of the CSR storage for bounded-degree operators (the dimer
// stores about 7.5 N^2 entries).
static size_t sparse_q_bytes(int N) {
    const int64_t M = (int64_t)N * N - 1;
    return (size_t)(24 * (int64_t)N * N) * (sizeof(int64_t) + sizeof(double)) + sizeof(int64_t) * (M + 1) +
           sizeof(double) * M;
}

// Staging of a system batch's states: input and output blocks of up to
// LB_SYSTEM_BATCH states.
static size_t system_stage_bytes(int64_t M) { return sizeof(double) * 2 * (size_t)LB_SYSTEM_BATCH * M; }

static size_t footprint(const lb_request& r, const System* y) {
    if (r.kind == LB_REQ_SYSTEM) return system_stage_bytes(y->M);
    return r.kind == LB_REQ_DENSE ? dense_q_bytes(r.N, r.precision) : sparse_q_bytes(r.N);
}

static bool same_shape(const lb_request& a, const lb_request& b) {
    return a.kind == LB_REQ_DENSE && b.kind == LB_REQ_DENSE && a.N == b.N && a.B == b.B && a.dt == b.dt &&
           a.steps == b.steps && a.precision == b.precision;
}

static bool same_system_pass(const lb_request& a, const lb_request& b) {
    return a.kind == LB_REQ_SYSTEM && b.kind == LB_REQ_SYSTEM && a.system == b.system && a.dt == b.dt &&
           a.steps == b.steps && a.precision == b.precision;
}

// One pass over a registered system for the states of every request in `batch`.
static int run_system_batch(lb_server* s, int slot, std::vector<Ticket*>& batch) {
    lb_ctx* c = s->ctxs[slot];
    hipStream_t st = s->streams[slot];
    System* y = batch[0]->sys;
    const lb_request& r0 = batch[0]->req;
    const int64_t M = y->M;
    int Btot = 0;
    for (Ticket* t : batch) Btot += t->req.B;
    const int Brun = (y->kind == LB_REQ_DENSE && Btot < 2) ? 2 : Btot;
    void* X = nullptr;
    if (hipMallocAsync(&X, sizeof(double) * (size_t)Brun * M, st) != hipSuccess) {
        (void)hipGetLastError();
        return lb_fail(LB_ERR_OOM, "server staging allocation failed");
    }
    int rc = LB_OK;
    double* Xd = (double*)X;
    int64_t off = 0;
    for (Ticket* t : batch) {
        if (hipMemcpyAsync(Xd + off, t->req.V0, sizeof(double) * (size_t)t->req.B * M, hipMemcpyDeviceToDevice,
                           st) != hipSuccess)
            rc = lb_fail(LB_ERR_DEVICE, "copy of the initial states failed");
        off += (int64_t)t->req.B * M;
    }
    if (!rc && Brun > Btot && hipMemsetAsync(Xd + off, 0, sizeof(double) * (size_t)(Brun - Btot) * M, st) != hipSuccess)
        rc = lb_fail(LB_ERR_DEVICE, "clearing the padding state failed");
    if (!rc) {
        if (y->kind == LB_REQ_DENSE) {
            const lb_tile tile = lb_default_tile(M, 16, r0.precision, 1);
            lb_prop_sys ps{(const double*)y->Q, (const float*)y->Q32, (const double*)y->K, Xd};
            rc = lb_impl_propagate(c, 1, M, &ps, y->ldq, Brun, r0.dt, r0.steps, r0.precision, &tile);
        } else {
            rc = lb_impl_propagate_csr(c, M, (const int64_t*)y->rp, (const int64_t*)y->col, (const double*)y->val,
                                       (const double*)y->K, Xd, Brun, r0.dt, r0.steps);
        }
    }
    off = 0;
    for (Ticket* t : batch) {
        if (!rc && hipMemcpyAsync(t->req.Vout, Xd + off, sizeof(double) * (size_t)t->req.B * M,
                                  hipMemcpyDeviceToDevice, st) != hipSuccess)
            rc = lb_fail(LB_ERR_DEVICE, "copy of the results failed");
        off += (int64_t)t->req.B * M;
    }
    (void)hipFreeAsync(X, st);
    hipError_t e = hipStreamSynchronize(st);
    if (!rc && e != hipSuccess) rc = lb_fail(LB_ERR_DEVICE, "slot stream: %s", hipGetErrorString(e));
    return rc;
}

static int run_batch(lb_server* s, int slot, std::vector<Ticket*>& batch) {
    if (batch[0]->req.kind == LB_REQ_SYSTEM) return run_system_batch(s, slot, batch);
    lb_ctx* c = s->ctxs[slot];
    hipStream_t st = s->streams[slot];
    const lb_request& r0 = batch[0]->req;
    const int N = r0.N;
    const int64_t M = (int64_t)N * N - 1;
    int rc = LB_OK;
    std::vector<void*> allocs;
    auto dalloc = [&](size_t bytes, void** p) -> int {
        hipError_t e = hipMallocAsync(p, bytes, st);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return lb_fail(LB_ERR_OOM, "server allocation of %zu bytes failed", bytes);
        }
        allocs.push_back(*p);
        return LB_OK;
    };
    if (r0.kind == LB_REQ_DENSE) {
        const int64_t ldq = lb_default_ldq(M);
        const int R = (int)batch.size();
        std::vector<lb_prop_sys> sys(R);
        for (int i = 0; i < R && !rc; ++i) {
            const lb_request& r = batch[i]->req;
            void *Q = nullptr, *K = nullptr, *Q32 = nullptr;
            rc = dalloc(sizeof(double) * (size_t)M * ldq, &Q);
            if (!rc) rc = dalloc(sizeof(double) * M, &K);
            if (!rc && r.precision == LB_FP32) rc = dalloc(sizeof(float) * (size_t)M * ldq, &Q32);
            if (!rc) rc = lb_impl_prepare_dense(c, N, r.H, r.gamma, (double*)Q, ldq, (double*)K);
            if (!rc && r.precision == LB_FP32) rc = lb_impl_q_to_f32(c, M, (double*)Q, ldq, (float*)Q32);
            if (!rc && hipMemcpyAsync(r.Vout, r.V0, sizeof(double) * (size_t)r.B * M, hipMemcpyDeviceToDevice, st) !=
                           hipSuccess)
                rc = lb_fail(LB_ERR_DEVICE, "copy of the initial states failed");
            sys[i] = lb_prop_sys{(const double*)Q, (const float*)Q32, (const double*)K, r.Vout};
        }
        if (!rc) rc = lb_impl_propagate(c, R, M, sys.data(), ldq, r0.B, r0.dt, r0.steps, r0.precision, nullptr);
    } else {
        const lb_request& r = r0;
        int64_t nnz = 0;
        rc = lb_impl_sparse(c, N, &r.Hs, r.P, r.rates, r.L, &nnz, nullptr, nullptr, nullptr, nullptr);
        void *rp = nullptr, *col = nullptr, *val = nullptr, *K = nullptr;
        if (!rc) rc = dalloc(sizeof(int64_t) * (M + 1), &rp);
        if (!rc) rc = dalloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1), &col);
        if (!rc) rc = dalloc(sizeof(double) * (nnz > 0 ? nnz : 1), &val);
        if (!rc) rc = dalloc(sizeof(double) * M, &K);
        if (!rc)
            rc = lb_impl_sparse(c, N, &r.Hs, r.P, r.rates, r.L, &nnz, (int64_t*)rp, (int64_t*)col, (double*)val,
                                (double*)K);
        if (!rc && hipMemcpyAsync(r.Vout, r.V0, sizeof(double) * (size_t)r.B * M, hipMemcpyDeviceToDevice, st) !=
                       hipSuccess)
            rc = lb_fail(LB_ERR_DEVICE, "copy of the initial states failed");
        if (!rc)
            rc = lb_impl_propagate_csr(c, M, (const int64_t*)rp, (const int64_t*)col, (const double*)val,
                                       (const double*)K, r.Vout, r.B, r.dt, r.steps);
    }
    for (void* p : allocs) (void)hipFreeAsync(p, st);
    hipError_t e = hipStreamSynchronize(st);
    if (!rc && e != hipSuccess) rc = lb_fail(LB_ERR_DEVICE, "slot stream: %s", hipGetErrorString(e));
    return rc;
}

static void worker(lb_server* s, int slot) {
    (void)hipSetDevice(s->device);
    for (;;) {
        std::vector<Ticket*> batch;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                if (!s->queue.empty()) {
                    Ticket* h = s->queue.front();
                    if (s->used + h->footprint <= s->budget) break;
                }
                if (s->stop && s->queue.empty()) return;
                s->cv_work.wait(lk);
            }
            Ticket* h = s->queue.front();
            s->queue.pop_front();
            s->used += h->footprint;
            batch.push_back(h);
            if (h->req.kind == LB_REQ_SYSTEM) {
                int states = h->req.B;
                for (auto it = s->queue.begin(); it != s->queue.end() && (int)batch.size() < s->max_batch;) {
                    Ticket* t = *it;
                    if (same_system_pass(h->req, t->req) && states + t->req.B <= LB_SYSTEM_BATCH &&
                        s->used + t->footprint <= s->budget) {
                        s->used += t->footprint;
                        states += t->req.B;
                        batch.push_back(t);
                        it = s->queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            } else if (h->req.kind == LB_REQ_DENSE) {
                for (auto it = s->queue.begin(); it != s->queue.end() && (int)batch.size() < s->max_batch;) {
                    Ticket* t = *it;
                    if (same_shape(h->req, t->req) && s->used + t->footprint <= s->budget) {
                        s->used += t->footprint;
                        batch.push_back(t);
                        it = s->queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            if (s->used > s->peak) s->peak = s->used;
            const double t0 = now_s();
            for (Ticket* t : batch) t->t_start = t0;
            s->batches += 1;
            if (batch.size() > 1) s->batched_requests += (int64_t)batch.size();
        }
        const int rc = run_batch(s, slot, batch);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            const double t1 = now_s();
            for (Ticket* t : batch) {
                t->status = rc;
                t->done = true;
                t->t_end = t1;
                s->used -= t->footprint;
                s->completed += 1;
                if (System* y = t->sys) {
                    if (--y->refs == 0 && y->released) {
                        s->used -= y->bytes;
                        s->registered -= y->bytes;
                        s->systems.erase(y->id);
                        system_free(y);
                    }
                }
            }
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

extern "C" {

int lindblad_server_create(int device, size_t hbm_budget_bytes, int max_slots, int max_batch, int max_N,
                           lb_server** out) {
    if (!out) return lb_fail(LB_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 64) return lb_fail(LB_ERR_INVALID_ARG, "max_slots must be in [1, 64]");
    if (max_batch < 1 || max_batch > 64) return lb_fail(LB_ERR_INVALID_ARG, "max_batch must be in [1, 64]");
    if (max_N < 2 || max_N > LB_MAX_N) return lb_fail(LB_ERR_INVALID_ARG, "max_N out of range");
    if (hbm_budget_bytes == 0) return lb_fail(LB_ERR_INVALID_ARG, "zero budget");
    lb_server* s = new lb_server();
    s->device = device;
    s->budget = hbm_budget_bytes;
    s->max_batch = max_batch;
    s->max_N = max_N;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) {
        delete s;
        return lb_fail(LB_ERR_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    }
    // keep released pool memory cached so that per-request allocations are cheap
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    for (int i = 0; i < max_slots; ++i) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        lb_ctx* c = nullptr;
        int rc = e == hipSuccess ? lb_create(&c, device, st) : LB_ERR_DEVICE;
        if (rc) {
            if (e == hipSuccess) (void)hipStreamDestroy(st);
            for (size_t k = 0; k < s->ctxs.size(); ++k) {
                lb_destroy(s->ctxs[k]);
                (void)hipStreamDestroy(s->streams[k]);
            }
            delete s;
            return lb_fail(LB_ERR_DEVICE, "slot %d creation failed", i);
        }
        s->streams.push_back(st);
        s->ctxs.push_back(c);
    }
    // pre-size every slot's workspace for the largest systems it may run
    {
        const int64_t M = (int64_t)max_N * max_N - 1;
        const int64_t Mp = (M + 15) / 16 * 16;
        const size_t prep = sizeof(double) * 2 * (size_t)max_N * M + (size_t)64 * max_N * max_N;
        const size_t prop = (size_t)max_batch * (size_t)(24 + 4) * Mp * 16 * sizeof(double);
        const size_t sp = (size_t)(8 + 2 * LB_REQ_MAX_JUMPS) * max_N * max_N * 16 + (size_t)48 * M;
        size_t want = prep > prop ? prep : prop;
        want = want > sp ? want : sp;
        for (auto* c : s->ctxs) (void)lb_ws_reserve(c, want);
    }
    e = hipStreamCreateWithFlags(&s->reg_stream, hipStreamNonBlocking);
    if (e != hipSuccess || lb_create(&s->reg_ctx, device, s->reg_stream) != LB_OK) {
        if (e == hipSuccess) (void)hipStreamDestroy(s->reg_stream);
        for (size_t k = 0; k < s->ctxs.size(); ++k) {
            lb_destroy(s->ctxs[k]);
            (void)hipStreamDestroy(s->streams[k]);
        }
        delete s;
        return lb_fail(LB_ERR_DEVICE, "registration context creation failed");
    }
    for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(worker, s, i);
    *out = s;
    return LB_OK;
}

static int submit_system(lb_server* s, const lb_request* r, int64_t* ticket) {
    if (!r->V0 || !r->Vout || r->B < 1 || r->B > LB_SYSTEM_BATCH || r->steps < 0 || !(r->dt == r->dt))
        return lb_fail(LB_ERR_INVALID_ARG, "bad states (1 <= B <= %d) / steps / dt", LB_SYSTEM_BATCH);
    Ticket* t = new Ticket();
    t->req = *r;
    t->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->systems.find(r->system);
        if (it == s->systems.end() || it->second->released) {
            delete t;
            return lb_fail(LB_ERR_INVALID_ARG, "unknown or released system %lld", (long long)r->system);
        }
        System* y = it->second;
        if (r->precision != LB_FP64 && !(r->precision == LB_FP32 && y->Q32)) {
            delete t;
            return lb_fail(LB_ERR_INVALID_ARG, "system %lld has no FP32 copy", (long long)r->system);
        }
        t->sys = y;
        t->req.N = y->N;
        t->footprint = footprint(t->req, y);
        if (t->footprint + s->registered > s->budget) {
            delete t;
            return lb_fail(LB_ERR_ADMISSION, "no budget left for the states of a request");
        }
        y->refs += 1;
        t->id = s->next_id++;
        s->tickets[t->id] = t;
        s->queue.push_back(t);
    }
    *ticket = t->id;
    s->cv_work.notify_all();
    return LB_OK;
}

int lindblad_server_submit(lb_server* s, const lb_request* r, int64_t* ticket) {
    if (!s || !r || !ticket) return lb_fail(LB_ERR_INVALID_ARG, "null argument");
    if (r->kind == LB_REQ_SYSTEM) return submit_system(s, r, ticket);
    if (r->N < 2 || r->N > s->max_N) return lb_fail(LB_ERR_INVALID_ARG, "N=%d outside [2, %d]", r->N, s->max_N);
    if (r->kind != LB_REQ_DENSE && r->kind != LB_REQ_SPARSE) return lb_fail(LB_ERR_INVALID_ARG, "unknown kind");
    if (!r->V0 || !r->Vout || r->B < 1 || r->B > 64 || r->steps < 0 || !(r->dt == r->dt))
        return lb_fail(LB_ERR_INVALID_ARG, "bad states / steps / dt");
    if (r->kind == LB_REQ_DENSE && (!r->H || !r->gamma)) return lb_fail(LB_ERR_INVALID_ARG, "dense request needs H and gamma");
    if (r->kind == LB_REQ_DENSE && r->precision != LB_FP64 && r->precision != LB_FP32)
        return lb_fail(LB_ERR_INVALID_ARG, "unknown precision");
    if (r->kind == LB_REQ_SPARSE && (r->P < 0 || r->P > LB_REQ_MAX_JUMPS || !r->Hs.rowptr))
        return lb_fail(LB_ERR_INVALID_ARG, "sparse request needs H and at most %d jump operators", LB_REQ_MAX_JUMPS);
    const size_t fp = footprint(*r, nullptr);
    if (fp > s->budget)
        return lb_fail(LB_ERR_ADMISSION, "request footprint %zu bytes exceeds the server budget %zu", fp, s->budget);
    Ticket* t = new Ticket();
    t->req = *r;
    t->footprint = fp;
    t->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        t->id = s->next_id++;
        s->tickets[t->id] = t;
        s->queue.push_back(t);
    }
    *ticket = t->id;
    s->cv_work.notify_all();
    return LB_OK;
}

int lindblad_server_register(lb_server* s, const lb_request* r, int64_t* system) {
    if (!s || !r || !system) return lb_fail(LB_ERR_INVALID_ARG, "null argument");
    if (r->N < 2 || r->N > s->max_N) return lb_fail(LB_ERR_INVALID_ARG, "N=%d outside [2, %d]", r->N, s->max_N);
    if (r->kind == LB_REQ_DENSE) {
        if (!r->H || !r->gamma) return lb_fail(LB_ERR_INVALID_ARG, "dense system needs H and gamma");
        if (r->precision != LB_FP64 && r->precision != LB_FP32) return lb_fail(LB_ERR_INVALID_ARG, "unknown precision");
    } else if (r->kind == LB_REQ_SPARSE) {
        if (r->P < 0 || r->P > LB_REQ_MAX_JUMPS || !r->Hs.rowptr)
            return lb_fail(LB_ERR_INVALID_ARG, "sparse system needs H and at most %d jump operators", LB_REQ_MAX_JUMPS);
    } else {
        return lb_fail(LB_ERR_INVALID_ARG, "a system is registered from a dense or sparse description");
    }
    std::lock_guard<std::mutex> rl(s->reg_mu);
    lb_ctx* c = s->reg_ctx;
    hipStream_t st = s->reg_stream;
    int rc = lb_use_device(c);
    if (rc) return rc;
    System* y = new System();
    y->kind = r->kind;
    y->N = r->N;
    y->precision = r->kind == LB_REQ_DENSE ? r->precision : LB_FP64;
    y->M = (int64_t)r->N * r->N - 1;
    const int64_t M = y->M;
    // footprint: dense from the shape; sparse after the count phase
    if (r->kind == LB_REQ_DENSE) {
        y->ldq = lb_default_ldq(M);
        y->bytes = sizeof(double) * ((size_t)M * y->ldq + M) +
                   (y->precision == LB_FP32 ? sizeof(float) * (size_t)M * y->ldq : 0);
    } else {
        rc = lb_impl_sparse(c, r->N, &r->Hs, r->P, r->rates, r->L, &y->nnz, nullptr, nullptr, nullptr, nullptr);
        if (rc) {
            delete y;
            return rc;
        }
        y->bytes = sizeof(int64_t) * (M + 1) + (sizeof(int64_t) + sizeof(double)) * (size_t)std::max<int64_t>(y->nnz, 1) +
                   sizeof(double) * M;
    }
    {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->registered + y->bytes > s->budget) {
            delete y;
            return lb_fail(LB_ERR_ADMISSION, "system of %zu bytes does not fit next to %zu registered bytes (budget %zu)",
                           y->bytes, s->registered, s->budget);
        }
        s->cv_done.wait(lk, [&] { return s->used + y->bytes <= s->budget; });
        s->used += y->bytes;
        s->registered += y->bytes;
        if (s->used > s->peak) s->peak = s->used;
    }
    auto dalloc = [&](size_t bytes, void** p) -> int {
        if (hipMalloc(p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return lb_fail(LB_ERR_OOM, "system allocation of %zu bytes failed", bytes);
        }
        return LB_OK;
    };
    if (r->kind == LB_REQ_DENSE) {
        rc = dalloc(sizeof(double) * (size_t)M * y->ldq, &y->Q);
        if (!rc) rc = dalloc(sizeof(double) * M, &y->K);
        if (!rc && y->precision == LB_FP32) rc = dalloc(sizeof(float) * (size_t)M * y->ldq, &y->Q32);
        if (!rc) rc = lb_impl_prepare_dense(c, r->N, r->H, r->gamma, (double*)y->Q, y->ldq, (double*)y->K);
        if (!rc && y->Q32) rc = lb_impl_q_to_f32(c, M, (const double*)y->Q, y->ldq, (float*)y->Q32);
    } else {
        rc = dalloc(sizeof(int64_t) * (M + 1), &y->rp);
        if (!rc) rc = dalloc(sizeof(int64_t) * (size_t)std::max<int64_t>(y->nnz, 1), &y->col);
        if (!rc) rc = dalloc(sizeof(double) * (size_t)std::max<int64_t>(y->nnz, 1), &y->val);
        if (!rc) rc = dalloc(sizeof(double) * M, &y->K);
        if (!rc)
            rc = lb_impl_sparse(c, r->N, &r->Hs, r->P, r->rates, r->L, &y->nnz, (int64_t*)y->rp, (int64_t*)y->col,
                                (double*)y->val, (double*)y->K);
    }
    hipError_t e = hipStreamSynchronize(st);
    if (!rc && e != hipSuccess) rc = lb_fail(LB_ERR_DEVICE, "registration stream: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc) {
        s->used -= y->bytes;
        s->registered -= y->bytes;
        system_free(y);
        s->cv_work.notify_all();
        return rc;
    }
    y->id = s->next_system++;
    s->systems[y->id] = y;
    *system = y->id;
    return LB_OK;
}

int lindblad_server_release(lb_server* s, int64_t system) {
    if (!s) return lb_fail(LB_ERR_INVALID_ARG, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->systems.find(system);
        if (it == s->systems.end() || it->second->released)
            return lb_fail(LB_ERR_INVALID_ARG, "unknown or released system %lld", (long long)system);
        System* y = it->second;
        y->released = true;
        if (y->refs == 0) {
            s->used -= y->bytes;
            s->registered -= y->bytes;
            s->systems.erase(it);
            system_free(y);
        }
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    return LB_OK;
}

int lindblad_server_poll(lb_server* s, int64_t ticket, int* done) {
    if (!s || !done) return lb_fail(LB_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return lb_fail(LB_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    *done = it->second->done ? 1 : 0;
    return LB_OK;
}

int lindblad_server_wait(lb_server* s, int64_t ticket) {
    if (!s) return lb_fail(LB_ERR_INVALID_ARG, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return lb_fail(LB_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    Ticket* t = it->second;
    s->cv_done.wait(lk, [&] { return t->done; });
    return t->status;
}

int lindblad_server_times(lb_server* s, int64_t ticket, double* t_submit, double* t_start, double* t_end) {
    if (!s) return lb_fail(LB_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return lb_fail(LB_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    if (t_submit) *t_submit = it->second->t_submit;
    if (t_start) *t_start = it->second->t_start;
    if (t_end) *t_end = it->second->t_end;
    return LB_OK;
}

int lindblad_server_stats(lb_server* s, int64_t* completed, size_t* peak_bytes, int64_t* batches,
                          int64_t* batched_requests) {
    if (!s) return lb_fail(LB_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (completed) *completed = s->completed;
    if (peak_bytes) *peak_bytes = s->peak;
    if (batches) *batches = s->batches;
    if (batched_requests) *batched_requests = s->batched_requests;
    return LB_OK;
}

int lindblad_server_destroy(lb_server* s) {
    if (!s) return LB_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& w : s->workers) w.join();
    for (size_t k = 0; k < s->ctxs.size(); ++k) {
        lb_destroy(s->ctxs[k]);
        (void)hipStreamDestroy(s->streams[k]);
    }
    lb_destroy(s->reg_ctx);
    (void)hipStreamDestroy(s->reg_stream);
    for (auto& kv : s->systems) system_free(kv.second);
    for (auto& kv : s->tickets) delete kv.second;
    delete s;
    return LB_OK;
}

}  // extern "C"
