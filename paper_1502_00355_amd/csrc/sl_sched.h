// Scheduling core of the serving loop, independent of the device.
//
// Requests wait in a FIFO.  The head of the queue is admitted when a slot is
// free and its footprint fits what is left of the budget (it waits
// otherwise, and so does everything behind it); one that can never fit, is
// cancelled or is past its deadline leaves the queue at once.  The loop
// thread launches a step over every admitted request, admits queued
// requests while the step runs (an admitted request joins at the next
// step), then waits for the step and retires the requests that finished,
// were cancelled or passed their deadline.  A failed admission fails only
// that request; a failed step fails the requests in it and stops the
// server, and everything still queued fails with it.
//
// The executor does the device work.  Requirements, all called from the
// loop thread except footprint():
//   using Payload = ...;                                 per-request device state
//   size_t footprint(const sl_mesh_desc&);               budget units of a request
//   sl_status admit(Request&);                           set up (synchronous); on error keeps nothing
//   sl_status launch(const std::vector<Request*>&, bool changed);
//                                                        start one step (asynchronous); requests with
//                                                        !joined join now and must be marked joined;
//                                                        `changed`: the set differs from the last step
//   bool busy();                                         the launched step still runs
//   sl_status wait(const std::vector<Request*>&, std::vector<StepOutcome>&);
//                                                        finish the step: one outcome per request
//   sl_status collect(Request&, const StepOutcome&);     result and report of a finished request
//   void release(Request&);                              free its device state
// Errors are reported through sl::fail / sl_last_error, as everywhere in the
// library.
#ifndef SL_SCHED_H
#define SL_SCHED_H

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/smartlap.h"

namespace sl {

void set_error(const std::string& msg);
sl_status fail(sl_status st, const std::string& msg);

namespace sched {

using Clock = std::chrono::steady_clock;

enum class Phase { QUEUED, ACTIVE, DONE };

// A request's state after a step, as the executor read it back.
struct StepOutcome {
    bool active = false;        // runs the next sweep
    int32_t sweeps = 0;         // sweeps done so far
    int64_t node_updates = 0;   // free nodes x sweeps done so far
};

template <class Payload>
struct Request {
    uint64_t id = 0;
    sl_mesh_desc desc{};
    int32_t iterations = 0;
    double tol = 0.0;
    double deadline_s = 0.0;    // server-clock seconds; <= 0: none
    size_t footprint = 0;
    Phase phase = Phase::QUEUED;
    sl_status status = SL_EBUSY;
    std::string error;
    bool cancel = false;
    int32_t slot = -1;
    bool joined = false;        // stepped by the executor since admission
    std::vector<double> result; // n x 2, filled when done
    sl_report report{};
    sl_request_times times{};
    Payload x;
};

template <class Exec>
class Scheduler {
public:
    using Req = Request<typename Exec::Payload>;

    Scheduler(const sl_server_config& cfg, Exec& ex) : cfg_(cfg), ex_(ex), t0_(Clock::now())
    {
        slots_.assign(static_cast<size_t>(cfg_.max_active), nullptr);
    }
    ~Scheduler() { stop(); }

    void start() { thread_ = std::thread([this] { loop(); }); }

    // Stops the loop thread and releases every admitted request.
    void stop()
    {
        stop_.store(true);
        cv_.notify_all();
        if (thread_.joinable()) thread_.join();
        for (auto& kv : reqs_)
            if (kv.second->slot >= 0) release(kv.second.get());
    }

    double now() const { return std::chrono::duration<double>(Clock::now() - t0_).count(); }

    sl_status submit(const sl_mesh_desc& d, int32_t iterations, double tol, double deadline_s, uint64_t* id)
    {
        auto q = std::make_unique<Req>();
        q->desc = d;
        q->iterations = iterations;
        q->tol = tol;
        q->footprint = ex_.footprint(d);
        std::lock_guard<std::mutex> lk(mu_);
        if (!fatal_.empty()) return fail(SL_EDEVICE, "server stopped: " + fatal_);
        q->id = next_id_++;
        q->times.submitted_s = now();
        q->deadline_s = deadline_s > 0.0 ? q->times.submitted_s + deadline_s : 0.0;
        *id = q->id;
        queue_.push_back(q->id);
        reqs_[q->id] = std::move(q);
        stats_.submitted++;
        cv_.notify_one();
        return SL_OK;
    }

    // SL_EBUSY until done; then the request's status, and it is forgotten.
    sl_status poll(uint64_t id, double* coords_out, sl_report* report, sl_request_times* times)
    {
        std::unique_ptr<Req> q;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = reqs_.find(id);
            if (it == reqs_.end()) return fail(SL_EINVAL, "unknown request id");
            if (it->second->phase != Phase::DONE) return SL_EBUSY;
            q = std::move(it->second);
            reqs_.erase(it);
        }
        if (times) *times = q->times;
        if (q->status != SL_OK) return fail(q->status, q->error);
        if (coords_out && !q->result.empty())
            std::memcpy(coords_out, q->result.data(), q->result.size() * sizeof(double));
        if (report) *report = q->report;
        return SL_OK;
    }

    sl_status cancel(uint64_t id)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(id);
        if (it == reqs_.end()) return fail(SL_EINVAL, "unknown request id");
        it->second->cancel = true;
        cv_.notify_one();
        return SL_OK;
    }

    sl_status stats(sl_server_stats* out)
    {
        std::lock_guard<std::mutex> lk(mu_);
        sl_server_stats s = stats_;
        s.queued = static_cast<int32_t>(queue_.size());
        s.active = 0;
        for (Req* q : slots_) s.active += q != nullptr;
        s.hbm_in_use = in_use_;
        *out = s;
        if (!fatal_.empty()) return fail(SL_EDEVICE, "server stopped: " + fatal_);
        return SL_OK;
    }

private:
    // with mu_ held for a queued request
    void drop(Req* q, sl_status status, const std::string& err)
    {
        queue_.pop_front();
        finish(q, status, err);
        stats_.failed++;
    }

    void finish(Req* q, sl_status status, const std::string& err)
    {
        q->status = status;
        q->error = err;
        q->phase = Phase::DONE;
        q->times.done_s = now();
    }

    // with mu_ held
    void release(Req* q)
    {
        ex_.release(*q);
        in_use_ -= q->footprint;
        if (q->slot >= 0) slots_[q->slot] = nullptr;
        q->slot = -1;
    }

    // With mu_ held: the head of the queue if it can be admitted now (the
    // requests at the head that are cancelled, past their deadline or too
    // large for the budget are finished on the way); nullptr if the queue
    // is empty or the head must wait.
    Req* pop_admissible()
    {
        while (!queue_.empty()) {
            Req* q = reqs_[queue_.front()].get();
            if (q->cancel) {
                drop(q, SL_ECANCELED, "cancelled before admission");
                continue;
            }
            if (q->deadline_s > 0.0 && now() > q->deadline_s) {
                drop(q, SL_ETIMEOUT, "deadline passed before admission");
                continue;
            }
            if (q->footprint > cfg_.hbm_budget_bytes) {
                drop(q, SL_ENOMEM, "request cannot fit the HBM budget");
                continue;
            }
            int32_t slot = -1;
            for (int32_t i = 0; i < cfg_.max_active; ++i)
                if (!slots_[i]) { slot = i; break; }
            if (slot < 0 || in_use_ + q->footprint > cfg_.hbm_budget_bytes) return nullptr;
            queue_.pop_front();
            q->slot = slot;
            slots_[slot] = q;
            in_use_ += q->footprint;
            q->times.admitted_s = now();
            return q;
        }
        return nullptr;
    }

    void loop()
    {
        bool changed = true;
        std::vector<StepOutcome> out;
        while (!stop_.load()) {
            // ---- 1. launch one step over every admitted request
            std::vector<Req*> in_step;
            for (Req* q : slots_)
                if (q && q->phase == Phase::ACTIVE) in_step.push_back(q);
            sl_status r = SL_OK;
            if (!in_step.empty()) {
                r = ex_.launch(in_step, changed);
                changed = false;
            }
            const bool stepping = !in_step.empty();

            // ---- 2. admissions while the step runs; with no step in
            // flight, one admission starts the next step
            for (;;) {
                Req* q = nullptr;
                {
                    std::unique_lock<std::mutex> lk(mu_);
                    if (!stepping && queue_.empty())
                        cv_.wait_for(lk, std::chrono::milliseconds(50),
                                     [&] { return stop_.load() || !queue_.empty(); });
                    q = pop_admissible();
                }
                if (!q) break;
                const sl_status ar = ex_.admit(*q);
                {
                    std::lock_guard<std::mutex> lk(mu_);
                    if (ar) {
                        const std::string msg = sl_last_error();
                        release(q);
                        finish(q, ar, msg);
                        stats_.failed++;
                    } else {
                        q->phase = Phase::ACTIVE;
                        q->joined = false;
                        q->times.started_s = now();
                        changed = true;
                    }
                }
                if (!stepping || !ex_.busy()) break;
            }
            if (!stepping) continue;

            // ---- 3. retire the requests that finished in this step
            out.assign(in_step.size(), StepOutcome{});
            if (!r) r = ex_.wait(in_step, out);
            const std::string step_err = r ? std::string(sl_last_error()) : std::string();
            const double t = now();
            std::lock_guard<std::mutex> lk(mu_);
            stats_.steps++;
            for (size_t k = 0; k < in_step.size(); ++k) {
                Req* q = in_step[k];
                sl_status fs = SL_OK;
                std::string msg;
                bool done = false;
                if (r) {
                    fs = r;
                    msg = step_err;
                    done = true;
                } else if (!out[k].active) {
                    done = true;
                } else if (q->cancel) {
                    fs = SL_ECANCELED;
                    msg = "cancelled";
                    done = true;
                } else if (q->deadline_s > 0.0 && t > q->deadline_s) {
                    fs = SL_ETIMEOUT;
                    msg = "deadline passed";
                    done = true;
                }
                if (!done) continue;
                if (fs == SL_OK) {
                    fs = ex_.collect(*q, out[k]);
                    if (fs) msg = sl_last_error();
                }
                if (fs == SL_OK) {
                    stats_.completed++;
                    stats_.node_updates += out[k].node_updates;
                } else {
                    stats_.failed++;
                }
                release(q);
                finish(q, fs, msg);
                changed = true;
            }
            if (r) {
                fatal_ = step_err.empty() ? "step failed" : step_err;
                while (!queue_.empty()) drop(reqs_[queue_.front()].get(), SL_EDEVICE, "server stopped: " + fatal_);
                break;
            }
        }
    }

    sl_server_config cfg_;
    Exec& ex_;
    Clock::time_point t0_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<uint64_t> queue_;                       // queued request ids, FIFO
    std::map<uint64_t, std::unique_ptr<Req>> reqs_;    // every request not yet polled
    std::vector<Req*> slots_;                          // admitted requests by slot
    size_t in_use_ = 0;
    uint64_t next_id_ = 1;
    std::atomic<bool> stop_{false};
    std::thread thread_;
    sl_server_stats stats_{};
    std::string fatal_;
};

}  // namespace sched

}  // namespace sl

#endif  // SL_SCHED_H
