// Scheduling core of the serving loop, free of device code: the request
// queue, admission by memory footprint, batch formation, ticket states and the
// worker threads. The device work of a batch (allocations, preparation,
// integration) and of a resident system's memory belongs to an Executor: the
// HIP one is in server.cpp; a stub one drives this header on the CPU under
// the thread and address sanitizers (tests/native/sched_check.cpp).
//
// Admission rules (all byte counts against one budget):
//   * `used` = footprints of running requests + bytes of registered systems;
//     a batch starts only while used + its footprints <= budget, so `used`
//     never exceeds the budget;
//   * a request whose footprint cannot fit next to the registered systems
//     (footprint + registered > budget) is refused at submission, and a
//     queued one that has become impossible (a system registered after it)
//     is failed with LB_ERR_ADMISSION when it reaches the head of the queue,
//     so the queue never stalls behind a request that cannot run;
//   * a registration is refused when the system cannot fit next to the
//     systems already registered together with the largest queued request;
//     otherwise it waits while running requests hold the memory it needs;
//   * submission order is kept: a head that fits later waits, later requests
//     do not overtake it (except those that join the head's batch).
// shutdown() cancels queued requests (LB_ERR_CANCELLED), waits for running
// batches, joins the workers and frees the resident systems.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/lindblad.h"

namespace lb_sched {

inline double now_s() {
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

// A resident (registered) system. Device pointers are the executor's.
struct System {
    int64_t id = 0;
    int kind = LB_REQ_DENSE;
    int N = 0, precision = LB_FP64;
    int64_t M = 0, ldq = 0, nnz = 0;
    void *Q = nullptr, *Q32 = nullptr, *K = nullptr;     // dense
    void *rp = nullptr, *col = nullptr, *val = nullptr;  // sparse (K shared)
    size_t bytes = 0;        // device memory held while registered
    size_t stage_bytes = 0;  // footprint of one pass of requests on it
    int refs = 0;            // queued or running requests
    bool released = false;
};

struct Ticket {
    lb_request req;
    int64_t id = 0;
    size_t footprint = 0;
    size_t join_footprint = 0;  // its footprint when it shares an earlier request's preparation
    int group = 0;              // index of its preparation within the batch
    System* sys = nullptr;
    int status = 1;  // 1 = pending, 0 = ok, < 0 = error
    bool done = false;
    double t_submit = 0, t_start = 0, t_end = 0;
};

class Executor {
   public:
    virtual ~Executor() {}
    // Called once on each worker thread before it takes work.
    virtual void thread_init(int slot) { (void)slot; }
    // Device work of one batch (every ticket has the same shape, or the same
    // system pass); returns the batch's status. Called without any lock held.
    virtual int run(int slot, std::vector<Ticket*>& batch) = 0;
    // Frees a system's device memory and deletes it. Called without the lock.
    virtual void free_system(System* y) = 0;
};

// Dense requests that may be integrated in one pass over several prepared
// systems (one launch per stage for all of them).
inline bool same_pass(const lb_request& a, const lb_request& b) {
    return a.kind == LB_REQ_DENSE && b.kind == LB_REQ_DENSE && a.N == b.N && a.dt == b.dt && a.steps == b.steps &&
           a.precision == b.precision;
}

inline bool same_csr(const lb_csr_c128& a, const lb_csr_c128& b) {
    return a.rowptr == b.rowptr && a.col == b.col && a.val == b.val && a.nnz == b.nnz;
}

// Requests whose preparation is the same: dense or sparse, the same N, the
// same input arrays (device pointers; for sparse requests also the same
// rates), dt, steps and precision. They share one preparation and one pass.
inline bool same_inputs(const lb_request& a, const lb_request& b) {
    if (a.kind != b.kind || a.N != b.N || a.dt != b.dt || a.steps != b.steps || a.precision != b.precision)
        return false;
    if (a.kind == LB_REQ_DENSE) return a.H == b.H && a.gamma == b.gamma;
    if (a.kind != LB_REQ_SPARSE || a.P != b.P || !same_csr(a.Hs, b.Hs)) return false;
    for (int p = 0; p < a.P; ++p)
        if (!(a.rates[p] == b.rates[p]) || !same_csr(a.L[p], b.L[p])) return false;
    return true;
}

inline bool same_system_pass(const lb_request& a, const lb_request& b) {
    return a.kind == LB_REQ_SYSTEM && b.kind == LB_REQ_SYSTEM && a.system == b.system && a.dt == b.dt &&
           a.steps == b.steps && a.precision == b.precision;
}

class Core {
   public:
    Core(size_t budget, int max_batch) : budget_(budget), max_batch_(max_batch) {}
    ~Core() { shutdown(); }
    Core(const Core&) = delete;
    Core& operator=(const Core&) = delete;

    void start(int slots, Executor* ex) {
        ex_ = ex;
        for (int i = 0; i < slots; ++i) workers_.emplace_back(&Core::worker, this, i);
    }

    // Queues a dense or sparse request of footprint fp bytes (join_fp when it
    // shares the preparation of an earlier request in its batch).
    int submit(const lb_request& r, size_t fp, size_t join_fp, int64_t* ticket, const char** why) {
        Ticket* t = new Ticket();
        t->req = r;
        t->footprint = fp;
        t->join_footprint = join_fp < fp ? join_fp : fp;
        t->t_submit = now_s();
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stop_) {
                delete t;
                *why = "the server is shutting down";
                return LB_ERR_CANCELLED;
            }
            if (fp > budget_ || fp + registered_ > budget_) {
                delete t;
                *why = "request footprint does not fit in the budget next to the registered systems";
                return LB_ERR_ADMISSION;
            }
            t->id = next_id_++;
            tickets_[t->id] = t;
            queue_.push_back(t);
            *ticket = t->id;
        }
        cv_work_.notify_all();
        return LB_OK;
    }

    // Queues states to integrate on registered system r.system.
    int submit_system(const lb_request& r, int64_t* ticket, const char** why) {
        Ticket* t = new Ticket();
        t->req = r;
        t->t_submit = now_s();
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = systems_.find(r.system);
            if (stop_) {
                delete t;
                *why = "the server is shutting down";
                return LB_ERR_CANCELLED;
            }
            if (it == systems_.end() || it->second->released) {
                delete t;
                *why = "unknown or released system";
                return LB_ERR_INVALID_ARG;
            }
            System* y = it->second;
            if (r.precision != LB_FP64 && !(r.precision == LB_FP32 && y->Q32)) {
                delete t;
                *why = "the system has no FP32 copy";
                return LB_ERR_INVALID_ARG;
            }
            t->sys = y;
            t->req.N = y->N;
            t->footprint = y->stage_bytes;
            if (t->footprint + registered_ > budget_) {
                delete t;
                *why = "no budget left for the states of a request";
                return LB_ERR_ADMISSION;
            }
            y->refs += 1;
            t->id = next_id_++;
            tickets_[t->id] = t;
            queue_.push_back(t);
            *ticket = t->id;
        }
        cv_work_.notify_all();
        return LB_OK;
    }

    // Reserves `bytes` for a system about to be registered: refused when it
    // cannot fit next to the registered systems and the largest queued
    // request; otherwise waits until running requests leave room.
    int reserve_system(size_t bytes, const char** why) {
        std::unique_lock<std::mutex> lk(mu_);
        if (bytes > budget_ || registered_ + bytes > budget_) {
            *why = "system does not fit next to the registered systems";
            return LB_ERR_ADMISSION;
        }
        if (registered_ + bytes + max_queued_locked() > budget_) {
            *why = "system would leave a queued request no room to run";
            return LB_ERR_ADMISSION;
        }
        cv_done_.wait(lk, [&] { return stop_ || used_ + bytes <= budget_; });
        if (stop_) {
            *why = "the server is shutting down";
            return LB_ERR_CANCELLED;
        }
        used_ += bytes;
        registered_ += bytes;
        if (used_ > peak_) peak_ = used_;
        return LB_OK;
    }

    void cancel_reservation(size_t bytes) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            used_ -= bytes;
            registered_ -= bytes;
        }
        cv_work_.notify_all();
        cv_done_.notify_all();
    }

    // Makes a system (reserved with reserve_system(y->bytes)) usable.
    int64_t commit_system(System* y) {
        std::lock_guard<std::mutex> lk(mu_);
        y->id = next_system_++;
        systems_[y->id] = y;
        return y->id;
    }

    int release(int64_t id, const char** why) {
        System* to_free = nullptr;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = systems_.find(id);
            if (it == systems_.end() || it->second->released) {
                *why = "unknown or released system";
                return LB_ERR_INVALID_ARG;
            }
            System* y = it->second;
            y->released = true;
            if (y->refs == 0) to_free = drop_system_locked(y);
        }
        if (to_free) ex_->free_system(to_free);
        cv_work_.notify_all();
        cv_done_.notify_all();
        return LB_OK;
    }

    int poll(int64_t ticket, int* done) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = tickets_.find(ticket);
        if (it == tickets_.end()) return LB_ERR_INVALID_ARG;
        *done = it->second->done ? 1 : 0;
        return LB_OK;
    }

    // Blocks until the request has finished; its status. LB_ERR_INVALID_ARG
    // (and *known = false) for an unknown ticket.
    int wait(int64_t ticket, bool* known) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = tickets_.find(ticket);
        if (it == tickets_.end()) {
            *known = false;
            return LB_ERR_INVALID_ARG;
        }
        *known = true;
        Ticket* t = it->second;
        cv_done_.wait(lk, [&] { return t->done; });
        return t->status;
    }

    int times(int64_t ticket, double* t_submit, double* t_start, double* t_end) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = tickets_.find(ticket);
        if (it == tickets_.end()) return LB_ERR_INVALID_ARG;
        if (t_submit) *t_submit = it->second->t_submit;
        if (t_start) *t_start = it->second->t_start;
        if (t_end) *t_end = it->second->t_end;
        return LB_OK;
    }

    void stats(int64_t* completed, size_t* peak_bytes, int64_t* batches, int64_t* batched_requests) {
        std::lock_guard<std::mutex> lk(mu_);
        if (completed) *completed = completed_;
        if (peak_bytes) *peak_bytes = peak_;
        if (batches) *batches = batches_;
        if (batched_requests) *batched_requests = batched_requests_;
    }

    size_t used_bytes() {
        std::lock_guard<std::mutex> lk(mu_);
        return used_;
    }

    // Cancels queued requests, waits for running batches, joins the workers
    // and frees every system. Idempotent.
    void shutdown() {
        std::vector<System*> to_free;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (shut_) return;
            shut_ = true;
            stop_ = true;
            const double t = now_s();
            for (Ticket* q : queue_)
                if (System* y = finish_locked(q, LB_ERR_CANCELLED, t)) to_free.push_back(y);
            queue_.clear();
        }
        cv_work_.notify_all();
        cv_done_.notify_all();
        for (auto& w : workers_) w.join();
        workers_.clear();
        std::vector<System*> rest;
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (auto& kv : systems_) rest.push_back(kv.second);
            systems_.clear();
            for (auto& kv : tickets_) delete kv.second;
            tickets_.clear();
        }
        if (ex_) {
            for (System* y : to_free) ex_->free_system(y);
            for (System* y : rest) ex_->free_system(y);
        }
    }

   private:
    size_t max_queued_locked() const {
        size_t m = 0;
        for (const Ticket* t : queue_) m = t->footprint > m ? t->footprint : m;
        return m;
    }

    // Removes a released, unreferenced system from the books; the caller
    // frees it after dropping the lock.
    System* drop_system_locked(System* y) {
        used_ -= y->bytes;
        registered_ -= y->bytes;
        systems_.erase(y->id);
        return y;
    }

    // Marks a ticket finished (not counting its footprint: the caller releases
    // that if it was admitted). Returns a system to free, if any.
    System* finish_locked(Ticket* t, int status, double t_end) {
        t->status = status;
        t->done = true;
        t->t_end = t_end;
        completed_ += 1;
        if (System* y = t->sys)
            if (--y->refs == 0 && y->released) return drop_system_locked(y);
        return nullptr;
    }

    void worker(int slot) {
        ex_->thread_init(slot);
        for (;;) {
            std::vector<Ticket*> batch;
            std::vector<System*> to_free;
            bool refused = false;
            {
                std::unique_lock<std::mutex> lk(mu_);
                for (;;) {
                    // a head that cannot fit next to the registered systems
                    // would never run: fail it instead of stalling the queue
                    while (!queue_.empty() && queue_.front()->footprint + registered_ > budget_) {
                        Ticket* h = queue_.front();
                        queue_.pop_front();
                        if (System* y = finish_locked(h, LB_ERR_ADMISSION, now_s())) to_free.push_back(y);
                        refused = true;
                    }
                    if (!queue_.empty() && used_ + queue_.front()->footprint <= budget_) break;
                    if (refused || !to_free.empty()) break;
                    if (stop_ && queue_.empty()) return;
                    cv_work_.wait(lk);
                }
                if (!queue_.empty() && used_ + queue_.front()->footprint <= budget_) take_batch_locked(batch);
            }
            for (System* y : to_free) ex_->free_system(y);
            if (refused) cv_done_.notify_all();
            if (batch.empty()) continue;
            const int rc = ex_->run(slot, batch);
            {
                std::lock_guard<std::mutex> lk(mu_);
                const double t1 = now_s();
                for (Ticket* t : batch) {
                    used_ -= t->footprint;
                    if (System* y = finish_locked(t, rc, t1)) to_free.push_back(y);
                }
            }
            for (System* y : to_free) ex_->free_system(y);
            cv_done_.notify_all();
            cv_work_.notify_all();
        }
    }

    // Takes the queue head and the queued requests that may share its batch.
    void take_batch_locked(std::vector<Ticket*>& batch) {
        Ticket* h = queue_.front();
        queue_.pop_front();
        used_ += h->footprint;
        batch.push_back(h);
        if (h->req.kind == LB_REQ_SYSTEM) {
            int states = h->req.B;
            for (auto it = queue_.begin(); it != queue_.end() && (int)batch.size() < max_batch_;) {
                Ticket* t = *it;
                if (same_system_pass(h->req, t->req) && states + t->req.B <= LB_SYSTEM_BATCH &&
                    used_ + t->footprint <= budget_) {
                    used_ += t->footprint;
                    states += t->req.B;
                    batch.push_back(t);
                    it = queue_.erase(it);
                } else {
                    ++it;
                }
            }
        } else {
            // at most max_batch_ requests: queued requests with the same inputs as
            // a group of the batch join it (one preparation, at most
            // LB_SYSTEM_BATCH states, footprint of their states only); dense
            // requests of the same pass shape on other inputs open further
            // groups. A request of more than LB_SYSTEM_BATCH states runs alone.
            h->group = 0;
            std::vector<const lb_request*> reps(1, &h->req);
            std::vector<int> states(1, h->req.B);
            const bool solo = h->req.B > LB_SYSTEM_BATCH;
            for (auto it = queue_.begin(); !solo && it != queue_.end() && (int)batch.size() < max_batch_;) {
                Ticket* t = *it;
                int g = -1;
                if (t->req.B <= LB_SYSTEM_BATCH)
                    for (size_t i = 0; i < reps.size() && g < 0; ++i)
                        if (same_inputs(*reps[i], t->req) && states[i] + t->req.B <= LB_SYSTEM_BATCH) g = (int)i;
                if (g >= 0 && used_ + t->join_footprint <= budget_) {
                    t->footprint = t->join_footprint;
                } else if (g < 0 && t->req.B <= LB_SYSTEM_BATCH && same_pass(h->req, t->req) &&
                           used_ + t->footprint <= budget_) {
                    g = (int)reps.size();
                    reps.push_back(&t->req);
                    states.push_back(0);
                } else {
                    ++it;
                    continue;
                }
                used_ += t->footprint;
                states[g] += t->req.B;
                t->group = g;
                batch.push_back(t);
                it = queue_.erase(it);
            }
        }
        if (used_ > peak_) peak_ = used_;
        const double t0 = now_s();
        for (Ticket* t : batch) t->t_start = t0;
        batches_ += 1;
        if (batch.size() > 1) batched_requests_ += (int64_t)batch.size();
    }

    const size_t budget_;
    const int max_batch_;
    Executor* ex_ = nullptr;
    std::mutex mu_;
    std::condition_variable cv_work_;  // workers wait for admissible work
    std::condition_variable cv_done_;  // waiters and registrations wait for completions
    std::deque<Ticket*> queue_;
    std::map<int64_t, Ticket*> tickets_;
    std::map<int64_t, System*> systems_;
    int64_t next_id_ = 1, next_system_ = 1;
    size_t used_ = 0, peak_ = 0, registered_ = 0;
    int64_t completed_ = 0, batches_ = 0, batched_requests_ = 0;
    bool stop_ = false, shut_ = false;
    std::vector<std::thread> workers_;
};

}  // namespace lb_sched
