// Serving: a request loop that admits Lindbladians of different N by device
// memory footprint, keeps each request's Q and K resident while it runs, and
// batches propagations of same-shape requests.
//
// Structure (the queue, admission and worker threads are the device-free
// scheduling core in serve_sched.h; this file is its device side and the C API):
//   * a FIFO of submitted requests (thread-safe submit from any thread);
//   * `slots` worker threads, each with its own HIP stream and library
//     context (workspace pre-sized for the largest N at creation);
//   * admission: a free slot takes the queue head if its footprint fits in the
//     remaining budget (head-of-line order is kept: a head that does not fit
//     waits for memory to be released; one that can never fit next to the
//     registered systems is failed), then the queued requests that can share
//     its batch: those with the same inputs (the same H, gamma or CSR arrays,
//     dt, steps, precision) join a group that is prepared once and whose states
//     are packed into one block of at most 16, and dense requests with the same
//     (N, dt, steps, precision) on other inputs open further groups, up to
//     max_batch; the batch is integrated with one launch per stage for all its
//     groups;
//   * per-request buffers (Q, K, CSR arrays) come from the stream-ordered
//     allocator of the slot's stream and are released when the batch ends.
// Requests arriving while others run are admitted as soon as a slot and
// memory are free, so their work overlaps on the device. Every kernel used
// here is deterministic for a fixed launch configuration, dense blocks always
// run the 16-state matrix-core path with its default tile (a request of more
// than 16 states runs alone on the path of its size) and the CSR kernel treats
// states independently, so a request's result is the same alone and in a mix.
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
#include <mutex>
#include <vector>

#include "lb_internal.h"
#include "serve_sched.h"

using lb_sched::System;
using lb_sched::Ticket;

namespace {

void system_free(System* y) {
    void* ps[] = {y->Q, y->Q32, y->K, y->rp, y->col, y->val};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    delete y;
}

}  // namespace

struct lb_server;

// The device side of the serving loop: one library context and stream per
// slot; the scheduling core calls run() on the slot's worker thread.
struct ServerExec : lb_sched::Executor {
    lb_server* s = nullptr;
    void thread_init(int slot) override;
    int run(int slot, std::vector<Ticket*>& batch) override;
    void free_system(System* y) override { system_free(y); }
};

struct lb_server {
    int device = 0;
    size_t budget = 0;
    int max_batch = 1;
    int max_N = 0;
    lb_sched::Core* core = nullptr;
    ServerExec exec;
    std::vector<lb_ctx*> ctxs;
    std::vector<hipStream_t> streams;
    std::mutex reg_mu;  // serializes registrations (one context)
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

// Share of a request's states in the state block of its group: a group's block
// holds at most LB_SYSTEM_BATCH states (a larger request runs alone).
static size_t request_stage_bytes(int N, int B) {
    const int64_t M = (int64_t)N * N - 1;
    return sizeof(double) * (size_t)std::max(B, LB_SYSTEM_BATCH) * M;
}

// Staging of a system batch's states: input and output blocks of up to
// LB_SYSTEM_BATCH states.
static size_t system_stage_bytes(int64_t M) { return sizeof(double) * 2 * (size_t)LB_SYSTEM_BATCH * M; }

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
    // groups: one preparation each; their requests' states packed into one block
    int G = 0;
    for (Ticket* t : batch) G = std::max(G, t->group + 1);
    std::vector<int> gstates(G, 0);
    std::vector<const lb_request*> rep(G, nullptr);
    for (Ticket* t : batch) {
        gstates[t->group] += t->req.B;
        if (!rep[t->group]) rep[t->group] = &t->req;
    }
    const bool solo = G == 1 && gstates[0] > LB_SYSTEM_BATCH;
    // dense blocks: at least 2 states, the same count in every group (padding
    // states are zero); sparse blocks: the group's states
    int Brun = 2;
    for (int g = 0; g < G; ++g) Brun = std::max(Brun, gstates[g]);
    if (r0.kind == LB_REQ_SPARSE) Brun = gstates[0];
    std::vector<double*> X(G, nullptr);
    for (int g = 0; g < G && !rc; ++g) {
        void* p = nullptr;
        rc = dalloc(sizeof(double) * (size_t)Brun * M, &p);
        X[g] = (double*)p;
    }
    std::vector<int64_t> off(batch.size(), 0);
    {
        std::vector<int64_t> fill(G, 0);
        for (size_t i = 0; i < batch.size() && !rc; ++i) {
            const lb_request& r = batch[i]->req;
            const int g = batch[i]->group;
            off[i] = fill[g];
            if (hipMemcpyAsync(X[g] + fill[g], r.V0, sizeof(double) * (size_t)r.B * M, hipMemcpyDeviceToDevice,
                               st) != hipSuccess)
                rc = lb_fail(LB_ERR_DEVICE, "copy of the initial states failed");
            fill[g] += (int64_t)r.B * M;
        }
        for (int g = 0; g < G && !rc; ++g)
            if (fill[g] < (int64_t)Brun * M &&
                hipMemsetAsync(X[g] + fill[g], 0, sizeof(double) * (size_t)((int64_t)Brun * M - fill[g]), st) !=
                    hipSuccess)
                rc = lb_fail(LB_ERR_DEVICE, "clearing the padding states failed");
    }
    if (r0.kind == LB_REQ_DENSE) {
        const int64_t ldq = lb_default_ldq(M);
        std::vector<lb_prop_sys> sys(G);
        for (int g = 0; g < G && !rc; ++g) {
            const lb_request& r = *rep[g];
            void *Q = nullptr, *K = nullptr, *Q32 = nullptr;
            rc = dalloc(sizeof(double) * (size_t)M * ldq, &Q);
            if (!rc) rc = dalloc(sizeof(double) * M, &K);
            if (!rc && r.precision == LB_FP32) rc = dalloc(sizeof(float) * (size_t)M * ldq, &Q32);
            if (!rc) rc = lb_impl_prepare_dense(c, N, r.H, r.gamma, (double*)Q, ldq, (double*)K);
            if (!rc && r.precision == LB_FP32) rc = lb_impl_q_to_f32(c, M, (double*)Q, ldq, (float*)Q32);
            sys[g] = lb_prop_sys{(const double*)Q, (const float*)Q32, (const double*)K, X[g]};
        }
        // the 16-state matrix-core path with its default tile whatever the
        // batch holds, so that every state column is summed in the same order
        const lb_tile tile = lb_default_tile(M, 16, r0.precision, 1);
        if (!rc) rc = lb_impl_propagate(c, G, M, sys.data(), ldq, Brun, r0.dt, r0.steps, r0.precision,
                                        solo ? nullptr : &tile);
    } else {
        const lb_request& r = r0;
        int64_t nnz = 0;
        if (!rc) rc = lb_impl_sparse(c, N, &r.Hs, r.P, r.rates, r.L, &nnz, nullptr, nullptr, nullptr, nullptr);
        void *rp = nullptr, *col = nullptr, *val = nullptr, *K = nullptr;
        if (!rc) rc = dalloc(sizeof(int64_t) * (M + 1), &rp);
        if (!rc) rc = dalloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1), &col);
        if (!rc) rc = dalloc(sizeof(double) * (nnz > 0 ? nnz : 1), &val);
        if (!rc) rc = dalloc(sizeof(double) * M, &K);
        if (!rc)
            rc = lb_impl_sparse(c, N, &r.Hs, r.P, r.rates, r.L, &nnz, (int64_t*)rp, (int64_t*)col, (double*)val,
                                (double*)K);
        if (!rc)
            rc = lb_impl_propagate_csr(c, M, (const int64_t*)rp, (const int64_t*)col, (const double*)val,
                                       (const double*)K, X[0], Brun, r.dt, r.steps);
    }
    for (size_t i = 0; i < batch.size() && !rc; ++i) {
        const lb_request& r = batch[i]->req;
        if (hipMemcpyAsync(r.Vout, X[batch[i]->group] + off[i], sizeof(double) * (size_t)r.B * M,
                           hipMemcpyDeviceToDevice, st) != hipSuccess)
            rc = lb_fail(LB_ERR_DEVICE, "copy of the results failed");
    }
    for (void* p : allocs) (void)hipFreeAsync(p, st);
    hipError_t e = hipStreamSynchronize(st);
    if (!rc && e != hipSuccess) rc = lb_fail(LB_ERR_DEVICE, "slot stream: %s", hipGetErrorString(e));
    return rc;
}

void ServerExec::thread_init(int slot) {
    (void)slot;
    (void)hipSetDevice(s->device);
}

int ServerExec::run(int slot, std::vector<Ticket*>& batch) { return run_batch(s, slot, batch); }

static void server_free(lb_server* s) {
    for (size_t k = 0; k < s->ctxs.size(); ++k) {
        lb_destroy(s->ctxs[k]);
        (void)hipStreamDestroy(s->streams[k]);
    }
    if (s->reg_ctx) lb_destroy(s->reg_ctx);
    if (s->reg_stream) (void)hipStreamDestroy(s->reg_stream);
    delete s;
}

static int sched_fail(int rc, const char* why) { return rc ? lb_fail(rc, "%s", why ? why : "serving error") : rc; }

extern "C" {

int lindblad_server_create(int device, size_t hbm_budget_bytes, int max_slots, int max_batch, int max_N,
                           lb_server** out) {
    if (!out) return lb_fail(LB_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 64) return lb_fail(LB_ERR_INVALID_ARG, "max_slots must be in [1, 64]");
    if (max_batch < 1 || max_batch > 64) return lb_fail(LB_ERR_INVALID_ARG, "max_batch must be in [1, 64]");
    if (max_N < 2 || max_N > LB_MAX_N) return lb_fail(LB_ERR_INVALID_ARG, "max_N out of range");
    if (hbm_budget_bytes == 0) return lb_fail(LB_ERR_INVALID_ARG, "zero budget");
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return lb_fail(LB_ERR_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    lb_server* s = new lb_server();
    s->device = device;
    s->budget = hbm_budget_bytes;
    s->max_batch = max_batch;
    s->max_N = max_N;
    s->exec.s = s;
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
            server_free(s);
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
    if (e != hipSuccess) s->reg_stream = nullptr;
    if (e != hipSuccess || lb_create(&s->reg_ctx, device, s->reg_stream) != LB_OK) {
        server_free(s);
        return lb_fail(LB_ERR_DEVICE, "registration context creation failed");
    }
    s->core = new lb_sched::Core(hbm_budget_bytes, max_batch);
    s->core->start(max_slots, &s->exec);
    *out = s;
    return LB_OK;
}

int lindblad_server_submit(lb_server* s, const lb_request* r, int64_t* ticket) {
    if (!s || !r || !ticket) return lb_fail(LB_ERR_INVALID_ARG, "null argument");
    const char* why = nullptr;
    if (r->kind == LB_REQ_SYSTEM) {
        if (!r->V0 || !r->Vout || r->B < 1 || r->B > LB_SYSTEM_BATCH || r->steps < 0 || !(r->dt == r->dt))
            return lb_fail(LB_ERR_INVALID_ARG, "bad states (1 <= B <= %d) / steps / dt", LB_SYSTEM_BATCH);
        return sched_fail(s->core->submit_system(*r, ticket, &why), why);
    }
    if (r->N < 2 || r->N > s->max_N) return lb_fail(LB_ERR_INVALID_ARG, "N=%d outside [2, %d]", r->N, s->max_N);
    if (r->kind != LB_REQ_DENSE && r->kind != LB_REQ_SPARSE) return lb_fail(LB_ERR_INVALID_ARG, "unknown kind");
    if (!r->V0 || !r->Vout || r->B < 1 || r->B > 64 || r->steps < 0 || !(r->dt == r->dt))
        return lb_fail(LB_ERR_INVALID_ARG, "bad states / steps / dt");
    if (r->kind == LB_REQ_DENSE && (!r->H || !r->gamma)) return lb_fail(LB_ERR_INVALID_ARG, "dense request needs H and gamma");
    if (r->kind == LB_REQ_DENSE && r->precision != LB_FP64 && r->precision != LB_FP32)
        return lb_fail(LB_ERR_INVALID_ARG, "unknown precision");
    if (r->kind == LB_REQ_SPARSE && (r->P < 0 || r->P > LB_REQ_MAX_JUMPS || !r->Hs.rowptr))
        return lb_fail(LB_ERR_INVALID_ARG, "sparse request needs H and at most %d jump operators", LB_REQ_MAX_JUMPS);
    const size_t stage = request_stage_bytes(r->N, r->B);
    const size_t fp = (r->kind == LB_REQ_DENSE ? dense_q_bytes(r->N, r->precision) : sparse_q_bytes(r->N)) + stage;
    return sched_fail(s->core->submit(*r, fp, stage, ticket, &why), why);
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
    y->stage_bytes = system_stage_bytes(y->M);
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
    const char* why = nullptr;
    rc = s->core->reserve_system(y->bytes, &why);
    if (rc) {
        delete y;
        return sched_fail(rc, why);
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
    if (rc) {
        const size_t bytes = y->bytes;
        system_free(y);
        s->core->cancel_reservation(bytes);
        return rc;
    }
    *system = s->core->commit_system(y);
    return LB_OK;
}

int lindblad_server_release(lb_server* s, int64_t system) {
    if (!s) return lb_fail(LB_ERR_INVALID_ARG, "null server");
    const char* why = nullptr;
    const int rc = s->core->release(system, &why);
    return rc ? lb_fail(rc, "%s %lld", why, (long long)system) : LB_OK;
}

int lindblad_server_poll(lb_server* s, int64_t ticket, int* done) {
    if (!s || !done) return lb_fail(LB_ERR_INVALID_ARG, "null argument");
    if (s->core->poll(ticket, done)) return lb_fail(LB_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    return LB_OK;
}

int lindblad_server_wait(lb_server* s, int64_t ticket) {
    if (!s) return lb_fail(LB_ERR_INVALID_ARG, "null server");
    bool known = false;
    const int rc = s->core->wait(ticket, &known);
    if (!known) return lb_fail(LB_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    if (rc == LB_ERR_ADMISSION) return lb_fail(rc, "request %lld can no longer fit next to the registered systems",
                                               (long long)ticket);
    if (rc == LB_ERR_CANCELLED) return lb_fail(rc, "request %lld was cancelled", (long long)ticket);
    return rc;
}

int lindblad_server_times(lb_server* s, int64_t ticket, double* t_submit, double* t_start, double* t_end) {
    if (!s) return lb_fail(LB_ERR_INVALID_ARG, "null server");
    if (s->core->times(ticket, t_submit, t_start, t_end))
        return lb_fail(LB_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    return LB_OK;
}

int lindblad_server_stats(lb_server* s, int64_t* completed, size_t* peak_bytes, int64_t* batches,
                          int64_t* batched_requests) {
    if (!s) return lb_fail(LB_ERR_INVALID_ARG, "null server");
    s->core->stats(completed, peak_bytes, batches, batched_requests);
    return LB_OK;
}

int lindblad_server_destroy(lb_server* s) {
    if (!s) return LB_OK;
    s->core->shutdown();
    delete s->core;
    server_free(s);
    return LB_OK;
}

}  // extern "C"
