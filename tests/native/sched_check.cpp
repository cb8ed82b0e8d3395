// CPU check of the serving scheduler core (paper_1912_01491_amd/csrc/serve_sched.h)
// with a stub executor: no device code, built by tests/test_sched_native.py
// with g++ under ThreadSanitizer and under AddressSanitizer + UBSan.
//
// Scenarios (argv[1]):
//   stress     concurrent submitters, registrations and releases; injected
//              allocation failures (LB_ERR_OOM from the executor); checks that
//              the budget is never exceeded, batches are well formed, every
//              accepted request finishes with the expected status and every
//              system is freed once
//   registered a registered system that nearly fills the budget: a plain
//              request is refused at submission, requests on the system run
//   late       a registration racing a queued request: no stall, the request
//              either runs or is failed with LB_ERR_ADMISSION
//   refuse     a registration that would starve a queued request is refused
//   shutdown   shutdown with queued requests cancels them and returns
//   oom        an injected allocation failure is reported on its ticket and
//              its footprint is returned to the budget
//   group      queued requests with the same inputs share their head's
//              preparation (at most 16 states per group, footprint of their
//              states only), other inputs of the same pass shape open further
//              groups, at most max_batch requests per batch, a request of more
//              than 16 states runs alone
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <random>
#include <string>

#include "serve_sched.h"

using lb_sched::Core;
using lb_sched::System;
using lb_sched::Ticket;

#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "CHECK failed: %s (%s:%d)\n", #cond, __FILE__, __LINE__); \
            exit(1);                                                             \
        }                                                                        \
    } while (0)

constexpr int64_t kFailSteps = 13;  // requests with this many steps get LB_ERR_OOM

struct Stub : lb_sched::Executor {
    size_t budget = 0;
    int max_batch = 1;
    std::atomic<int64_t> inflight{0};  // footprints of running batches
    std::atomic<int64_t> resident{0};  // bytes of systems not yet freed
    std::atomic<int> freed{0}, runs{0};
    std::atomic<bool> bad{false};
    std::mutex gate_mu;
    std::condition_variable gate_cv;
    bool gate_closed = false;
    std::atomic<int> at_gate{0};
    unsigned sleep_us = 0;

    std::mutex last_mu;
    std::vector<std::pair<int, int>> last;  // (group, B) of each ticket of the latest batch

    int run(int slot, std::vector<Ticket*>& b) override {
        (void)slot;
        runs++;
        int64_t fp = 0;
        int states = 0;
        const lb_request& h = b[0]->req;
        if (h.kind == LB_REQ_SYSTEM) {
            if ((int)b.size() > max_batch) bad = true;
            for (Ticket* t : b)
                if (t != b[0] && !lb_sched::same_system_pass(h, t->req)) bad = true;
        } else {
            // groups: every member shares its group's first request's inputs, at
            // most 16 states per group (unless the request runs alone), groups of
            // one pass shape, at most max_batch of them
            std::vector<const Ticket*> rep;
            std::vector<int> gs;
            for (Ticket* t : b) {
                if (t->group < 0 || t->group > (int)rep.size()) bad = true;
                if (t->group == (int)rep.size()) {
                    rep.push_back(t);
                    gs.push_back(0);
                    if (t != b[0] && !lb_sched::same_pass(h, t->req)) bad = true;
                } else if (t->group >= 0 && !lb_sched::same_inputs(rep[t->group]->req, t->req)) {
                    bad = true;
                }
                if (t->group >= 0 && t->group < (int)gs.size()) gs[t->group] += t->req.B;
            }
            if ((int)b.size() > max_batch) bad = true;
            for (int x : gs)
                if (x > LB_SYSTEM_BATCH && b.size() > 1) bad = true;
            std::lock_guard<std::mutex> lk(last_mu);
            last.clear();
            for (Ticket* t : b) last.push_back({t->group, t->req.B});
        }
        for (Ticket* t : b) {
            fp += (int64_t)t->footprint;
            states += t->req.B;
        }
        if (h.kind == LB_REQ_SYSTEM && states > LB_SYSTEM_BATCH) bad = true;
        const int64_t now = inflight.fetch_add(fp) + fp;
        if (now > (int64_t)budget) bad = true;
        {
            std::unique_lock<std::mutex> lk(gate_mu);
            at_gate++;
            gate_cv.wait(lk, [&] { return !gate_closed; });
        }
        if (sleep_us) std::this_thread::sleep_for(std::chrono::microseconds(rand() % (sleep_us + 1)));
        inflight.fetch_sub(fp);
        return h.steps == kFailSteps ? LB_ERR_OOM : LB_OK;
    }
    void free_system(System* y) override {
        resident.fetch_sub((int64_t)y->bytes);
        freed++;
        delete y;
    }
    void close_gate() {
        std::lock_guard<std::mutex> lk(gate_mu);
        gate_closed = true;
    }
    void open_gate() {
        {
            std::lock_guard<std::mutex> lk(gate_mu);
            gate_closed = false;
        }
        gate_cv.notify_all();
    }
    void wait_at_gate(int n) {
        while (at_gate.load() < n) std::this_thread::sleep_for(std::chrono::milliseconds(1));
    }
};

// Input arrays are only compared, never read: a request gets addresses of its
// own (plain) or those of a shared key (shared).
static std::atomic<uintptr_t> g_next_input{0x10000};

static lb_request with_inputs(int kind, int N, int B, int64_t steps, uintptr_t base) {
    lb_request r;
    memset(&r, 0, sizeof(r));
    r.kind = kind;
    r.N = N;
    r.B = B;
    r.dt = 1e-3;
    r.steps = steps;
    r.precision = LB_FP64;
    if (kind == LB_REQ_DENSE) {
        r.H = (const double*)base;
        r.gamma = (const double*)(base + 8);
    } else if (kind == LB_REQ_SPARSE) {
        r.Hs.rowptr = (const int64_t*)base;
        r.Hs.col = (const int64_t*)(base + 8);
        r.Hs.val = (const double*)(base + 16);
    }
    return r;
}

static lb_request plain(int kind, int N, int B, int64_t steps) {
    return with_inputs(kind, N, B, steps, g_next_input.fetch_add(64));
}

static lb_request shared(int kind, int N, int B, int64_t steps, int key) {
    return with_inputs(kind, N, B, steps, 0x100 + 64 * (uintptr_t)key);
}

static lb_request on_system(int64_t sid, int B, int64_t steps) {
    lb_request r = plain(LB_REQ_SYSTEM, 0, B, steps);
    r.system = sid;
    return r;
}

// Registers a system of `bytes` through the core as the server does.
static int register_sys(Core& core, Stub& ex, size_t bytes, size_t stage, int64_t* id) {
    const char* why = nullptr;
    int rc = core.reserve_system(bytes, &why);
    if (rc) return rc;
    System* y = new System();
    y->kind = LB_REQ_DENSE;
    y->N = 4;
    y->M = 15;
    y->bytes = bytes;
    y->stage_bytes = stage;
    ex.resident.fetch_add((int64_t)bytes);
    *id = core.commit_system(y);
    return LB_OK;
}

static void scenario_stress() {
    const size_t budget = 1000;
    Stub ex;
    ex.budget = budget;
    ex.max_batch = 4;
    ex.sleep_us = 50;
    int registered = 0;
    {
        Core core(budget, ex.max_batch);
        core.start(4, &ex);
        std::atomic<int64_t> sys_ids[3];
        for (auto& s : sys_ids) s = 0;
        std::vector<std::thread> th;
        std::mutex res_mu;
        std::vector<std::pair<int64_t, int>> accepted;  // ticket, expected status (1: OK or ADMISSION)
        for (int w = 0; w < 4; ++w)
            th.emplace_back([&, w] {
                std::mt19937 g(1234 + w);
                for (int i = 0; i < 400; ++i) {
                    const int k = (int)(g() % 10);
                    const int64_t steps = (g() % 17 == 0) ? kFailSteps : 20 + (int64_t)(g() % 3);
                    int64_t t = 0;
                    const char* why = nullptr;
                    int rc;
                    if (k < 6) {
                        const int N = 4 + (int)(g() % 3);
                        rc = core.submit(plain(LB_REQ_DENSE, N, 1 + (int)(g() % 2), steps), 100 * (size_t)N - 300, 20, &t, &why);
                    } else if (k < 7) {
                        rc = core.submit(plain(LB_REQ_SPARSE, 5, 1, steps), 150, 20, &t, &why);
                    } else if (k < 8) {
                        // shared inputs: grouped with queued requests on the same key
                        const int key = (int)(g() % 3);
                        rc = core.submit(shared(key == 2 ? LB_REQ_SPARSE : LB_REQ_DENSE, 5, 1 + (int)(g() % 6), steps,
                                                key),
                                         200, 30, &t, &why);
                    } else {
                        const int64_t sid = sys_ids[g() % 3].load();
                        if (!sid) continue;
                        rc = core.submit_system(on_system(sid, 1 + (int)(g() % 4), steps), &t, &why);
                        if (rc == LB_ERR_INVALID_ARG) continue;  // released meanwhile
                    }
                    CHECK(rc == LB_OK || rc == LB_ERR_ADMISSION);
                    if (rc == LB_OK) {
                        std::lock_guard<std::mutex> lk(res_mu);
                        accepted.push_back({t, steps == kFailSteps ? LB_ERR_OOM : LB_OK});
                    }
                }
            });
        th.emplace_back([&] {
            for (int round = 0; round < 20; ++round) {
                for (int k = 0; k < 3; ++k) {
                    int64_t id = 0;
                    if (register_sys(core, ex, 120 + 10 * k, 40, &id) == LB_OK) {
                        sys_ids[k] = id;
                        registered++;
                    }
                }
                std::this_thread::sleep_for(std::chrono::milliseconds(2));
                for (int k = 0; k < 3; ++k) {
                    const int64_t id = sys_ids[k].exchange(0);
                    const char* why = nullptr;
                    if (id) CHECK(core.release(id, &why) == LB_OK);
                }
            }
        });
        for (auto& t : th) t.join();
        int ok = 0, oom = 0, adm = 0;
        for (auto& a : accepted) {
            bool known = false;
            const int st = core.wait(a.first, &known);
            CHECK(known);
            if (st == LB_ERR_ADMISSION) {
                adm++;
                continue;
            }
            CHECK(st == a.second);
            (st == LB_OK ? ok : oom)++;
        }
        int64_t completed = 0, batches = 0, batched = 0;
        size_t peak = 0;
        core.stats(&completed, &peak, &batches, &batched);
        CHECK(peak <= budget);
        CHECK(completed == (int64_t)accepted.size());
        CHECK(core.used_bytes() == 0);
        printf("stress: %zu accepted (%d ok, %d injected OOM, %d admission), %lld batches, %lld batched, peak %zu\n",
               accepted.size(), ok, oom, adm, (long long)batches, (long long)batched, peak);
    }
    CHECK(!ex.bad.load());
    CHECK(ex.freed.load() == registered);
    CHECK(ex.resident.load() == 0);
}

static void scenario_registered() {
    Stub ex;
    ex.budget = 1000;
    ex.max_batch = 4;
    Core core(1000, 4);
    core.start(2, &ex);
    int64_t sid = 0, t = 0;
    CHECK(register_sys(core, ex, 900, 50, &sid) == LB_OK);
    const char* why = nullptr;
    CHECK(core.submit(plain(LB_REQ_DENSE, 6, 1, 10), 200, 200, &t, &why) == LB_ERR_ADMISSION);
    std::vector<int64_t> ts;
    for (int i = 0; i < 8; ++i) {
        CHECK(core.submit_system(on_system(sid, 1, 10), &t, &why) == LB_OK);
        ts.push_back(t);
    }
    CHECK(core.submit(plain(LB_REQ_DENSE, 6, 1, 10), 90, 90, &t, &why) == LB_OK);
    ts.push_back(t);
    for (int64_t x : ts) {
        bool known = false;
        CHECK(core.wait(x, &known) == LB_OK);
    }
    CHECK(core.release(sid, &why) == LB_OK);
    CHECK(core.submit(plain(LB_REQ_DENSE, 6, 1, 10), 200, 200, &t, &why) == LB_OK);
    bool known = false;
    CHECK(core.wait(t, &known) == LB_OK);
    printf("registered: plain request refused next to a full system, system requests ran\n");
}

static void scenario_late() {
    for (int rep = 0; rep < 50; ++rep) {
        Stub ex;
        ex.budget = 1000;
        Core core(1000, 1);
        core.start(1, &ex);
        ex.close_gate();
        const char* why = nullptr;
        int64_t a = 0, b = 0, sid = 0;
        CHECK(core.submit(plain(LB_REQ_DENSE, 6, 1, 10), 700, 700, &a, &why) == LB_OK);
        ex.wait_at_gate(1);
        std::thread reg([&] { CHECK(register_sys(core, ex, 400, 10, &sid) == LB_OK); });
        std::this_thread::sleep_for(std::chrono::microseconds(200));
        const int rb = core.submit(plain(LB_REQ_DENSE, 6, 1, 10), 700, 700, &b, &why);
        CHECK(rb == LB_OK || rb == LB_ERR_ADMISSION);  // refused if the reservation already counts
        if (rb != LB_OK) b = 0;
        ex.open_gate();
        reg.join();
        bool known = false;
        CHECK(core.wait(a, &known) == LB_OK);
        if (b) {
            const int st = core.wait(b, &known);
            CHECK(st == LB_OK || st == LB_ERR_ADMISSION);
        }
        CHECK(core.release(sid, &why) == LB_OK);
    }
    printf("late: registration racing a queued request never stalls\n");
}

static void scenario_refuse() {
    Stub ex;
    ex.budget = 1000;
    Core core(1000, 1);
    core.start(1, &ex);
    ex.close_gate();
    const char* why = nullptr;
    int64_t a = 0, b = 0, sid = 0;
    CHECK(core.submit(plain(LB_REQ_DENSE, 6, 1, 10), 500, 500, &a, &why) == LB_OK);
    ex.wait_at_gate(1);
    CHECK(core.submit(plain(LB_REQ_DENSE, 6, 1, 10), 600, 600, &b, &why) == LB_OK);  // queued behind a
    CHECK(register_sys(core, ex, 500, 10, &sid) == LB_ERR_ADMISSION);  // 500 + 600 > 1000
    CHECK(register_sys(core, ex, 300, 10, &sid) == LB_OK);             // 300 + 600 fits
    ex.open_gate();
    bool known = false;
    CHECK(core.wait(a, &known) == LB_OK);
    CHECK(core.wait(b, &known) == LB_OK);
    printf("refuse: a registration that would starve a queued request is refused\n");
}

static void scenario_shutdown() {
    Stub ex;
    ex.budget = 1000;
    int64_t first = 0;
    std::vector<int64_t> queued;
    Core* core = new Core(1000, 1);
    core->start(1, &ex);
    ex.close_gate();
    const char* why = nullptr;
    CHECK(core->submit(plain(LB_REQ_DENSE, 6, 1, 10), 600, 600, &first, &why) == LB_OK);
    ex.wait_at_gate(1);
    for (int i = 0; i < 10; ++i) {
        int64_t t = 0;
        CHECK(core->submit(plain(LB_REQ_DENSE, 7, 1, 10), 600, 600, &t, &why) == LB_OK);
        queued.push_back(t);
    }
    std::atomic<int> cancelled{0};
    std::vector<std::thread> waiters;
    for (int64_t t : queued)
        waiters.emplace_back([&, t] {
            bool known = false;
            if (core->wait(t, &known) == LB_ERR_CANCELLED) cancelled++;
        });
    std::thread stopper([&] { core->shutdown(); });
    for (auto& w : waiters) w.join();
    CHECK(cancelled.load() == (int)queued.size());
    ex.open_gate();
    stopper.join();
    delete core;
    printf("shutdown: %d queued requests cancelled, running batch finished\n", cancelled.load());
}

static void scenario_oom() {
    Stub ex;
    ex.budget = 1000;
    ex.max_batch = 2;
    Core core(1000, 2);
    core.start(2, &ex);
    const char* why = nullptr;
    int64_t bad = 0, good = 0;
    CHECK(core.submit(plain(LB_REQ_SPARSE, 6, 1, kFailSteps), 900, 900, &bad, &why) == LB_OK);
    CHECK(core.submit(plain(LB_REQ_SPARSE, 6, 1, 10), 900, 900, &good, &why) == LB_OK);
    bool known = false;
    CHECK(core.wait(bad, &known) == LB_ERR_OOM);
    CHECK(core.wait(good, &known) == LB_OK);
    CHECK(core.used_bytes() == 0);
    printf("oom: injected allocation failure reported, budget returned\n");
}

static void scenario_group() {
    Stub ex;
    ex.budget = 10000;
    ex.max_batch = 6;
    Core core(10000, 6);
    core.start(1, &ex);
    ex.close_gate();
    const char* why = nullptr;
    int64_t t = 0;
    std::vector<int64_t> all;
    CHECK(core.submit(plain(LB_REQ_DENSE, 6, 1, 10), 500, 50, &t, &why) == LB_OK);  // runs first, holds the slot
    all.push_back(t);
    ex.wait_at_gate(1);
    // head of the next batch and four more on its inputs: 4 + 4 + 4 + 4 states
    // fill group 0, the fifth opens group 1 (same inputs, group full)
    for (int i = 0; i < 5; ++i) {
        CHECK(core.submit(shared(LB_REQ_DENSE, 6, 4, 10, 7), 500, 50, &t, &why) == LB_OK);
        all.push_back(t);
    }
    CHECK(core.submit(plain(LB_REQ_DENSE, 6, 1, 10), 500, 50, &t, &why) == LB_OK);   // group 2: the sixth request
    all.push_back(t);
    CHECK(core.submit(plain(LB_REQ_DENSE, 6, 1, 10), 500, 50, &t, &why) == LB_OK);   // over max_batch: next batch
    all.push_back(t);
    CHECK(core.submit(plain(LB_REQ_DENSE, 6, 20, 10), 500, 50, &t, &why) == LB_OK);  // more than 16 states: alone
    all.push_back(t);
    ex.open_gate();
    bool known = false;
    for (int64_t x : all) CHECK(core.wait(x, &known) == LB_OK);
    CHECK(core.used_bytes() == 0);
    int64_t completed = 0, batches = 0, batched = 0;
    size_t peak = 0;
    core.stats(&completed, &peak, &batches, &batched);
    // batches: the first request, {group 0: 4, group 1: 1, group 2: 1}, the last plain one, the 20-state one
    CHECK(batches == 4);
    CHECK(batched == 6);
    std::lock_guard<std::mutex> lk(ex.last_mu);
    // peak: the second batch, three preparations (500 each) and three joiners (50 each)
    CHECK(peak == 3 * 500 + 3 * 50);
    printf("group: same-input requests shared one preparation, footprints of joiners counted as states only\n");
}

int main(int argc, char** argv) {
    const std::string s = argc > 1 ? argv[1] : "all";
    if (s == "stress" || s == "all") scenario_stress();
    if (s == "registered" || s == "all") scenario_registered();
    if (s == "late" || s == "all") scenario_late();
    if (s == "refuse" || s == "all") scenario_refuse();
    if (s == "shutdown" || s == "all") scenario_shutdown();
    if (s == "oom" || s == "all") scenario_oom();
    if (s == "group" || s == "all") scenario_group();
    printf("OK\n");
    return 0;
}
