// Scheduling core of the serving loop, independent of the device.
//
// Requests wait in a queue.  Setup threads admit them: a request is admitted
// when a slot is free and its footprint fits what is left of the budget; a
// queued request that does not fit may be passed by later ones that do, but
// at most kMaxBypass times, after which nothing passes it until it is
// admitted.  One that can never fit, is cancelled or is past its deadline
// leaves the queue at once.  The setup thread then sets the request up
// (upload and device setup) and hands it to the loop thread, which joins it
// at the next step.  The loop thread only steps: it launches a step over
// every set-up request, collects the results of the requests the previous
// step finished while this one runs, waits for the step and retires the
// requests that finished, were cancelled or passed their deadline.  A
// failed admission fails only that request; a failed step fails every
// request the server holds and stops it.
//
// The executor does the device work.  Requirements:
//   using Payload = ...;                                 per-request device state
//   size_t footprint(const sl_mesh_desc&);               budget units of a request (any thread)
//   sl_status admit(Request&);                           set up, synchronously; called by setup
//                                                        threads, several at once; on error keeps nothing
//   sl_status launch(const std::vector<Request*>&, bool changed, int32_t sweeps);
//                                                        start one step of `sweeps` sweeps (asynchronous);
//                                                        requests with !joined join now and must be
//                                                        marked joined; `changed`: the set differs from
//                                                        the last step
//   sl_status wait(const std::vector<Request*>&, std::vector<StepOutcome>&);
//                                                        finish the step: one outcome per request
//   sl_status collect(Request&, const StepOutcome&);     result and report of a finished request, into
//                                                        its `result` (already n_nodes x 2 long); runs
//                                                        while the next step may be in flight (the
//                                                        request is in no step any more)
//   void release(Request&);                              free its device state (any thread)
// launch, wait and collect are called from the loop thread only.  Errors
// are reported through sl::fail / sl_last_error, as everywhere in the
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

// A queued request that does not fit the budget is passed by at most this
// many later ones before the queue waits for it.
constexpr int32_t kMaxBypass = 64;
// A step of a lone request (nothing queued, nothing being set up) runs this
// many times the configured sweeps.
constexpr int32_t kAloneStepFactor = 4;

enum class Phase { QUEUED, ADMITTING, ACTIVE, DONE };

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
    int32_t bypassed = 0;       // later requests admitted while this one waited
    bool joined = false;        // stepped by the executor since admission
    bool finishing = false;     // finished its sweeps; its result is being collected
    StepOutcome outcome{};      // of its last step
    std::vector<double> result; // n x 2, filled when done (sized by the core before collect)
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

    void start()
    {
        thread_ = std::thread([this] { loop(); });
        const int32_t n = std::max<int32_t>(1, cfg_.setup_threads);
        for (int32_t k = 0; k < n; ++k) setup_.emplace_back([this] { setup_loop(); });
    }

    // Stops the threads and releases every request that holds a slot.
    void stop()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        cv_loop_.notify_all();
        if (thread_.joinable()) thread_.join();
        for (auto& t : setup_)
            if (t.joinable()) t.join();
        setup_.clear();
        std::lock_guard<std::mutex> lk(mu_);
        for (auto& kv : reqs_)
            if (kv.second->slot >= 0) release(kv.second.get());
    }

    double now() const { return std::chrono::duration<double>(Clock::now() - t0_).count(); }

    sl_status submit(const sl_mesh_desc& d, int32_t iterations, double tol, double deadline_s, uint64_t* id)
    {
        const double t = now();   // before any wait for the lock
        auto q = std::make_unique<Req>();
        q->desc = d;
        q->iterations = iterations;
        q->tol = tol;
        q->footprint = ex_.footprint(d);
        q->times.submitted_s = t;
        q->deadline_s = deadline_s > 0.0 ? t + deadline_s : 0.0;
        std::lock_guard<std::mutex> lk(mu_);
        if (!fatal_.empty()) return fail(SL_EDEVICE, "server stopped: " + fatal_);
        q->id = next_id_++;
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
        give_result(std::move(q->result));
        return SL_OK;
    }

    sl_status cancel(uint64_t id)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(id);
        if (it == reqs_.end()) return fail(SL_EINVAL, "unknown request id");
        it->second->cancel = true;
        cv_.notify_all();
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
    // ---- with mu_ held

    void finish(Req* q, sl_status status, const std::string& err)
    {
        q->status = status;
        q->error = err;
        q->phase = Phase::DONE;
        q->times.done_s = now();
        if (status == SL_OK) stats_.completed++;
        else stats_.failed++;
    }

    void release(Req* q)
    {
        ex_.release(*q);
        in_use_ -= q->footprint;
        if (q->slot >= 0) slots_[q->slot] = nullptr;
        q->slot = -1;
    }

    // A queued request to admit now, with its slot and budget taken, or
    // nullptr.  Requests that are cancelled, past their deadline or too
    // large for the budget are finished on the way.
    Req* pop_admissible()
    {
        int32_t slot = -1;
        for (int32_t i = 0; i < cfg_.max_active; ++i)
            if (!slots_[i]) { slot = i; break; }
        Req* blocked = nullptr;   // the first queued request that did not fit
        for (auto it = queue_.begin(); it != queue_.end();) {
            Req* q = reqs_[*it].get();
            sl_status drop = SL_OK;
            const char* why = nullptr;
            if (q->cancel) {
                drop = SL_ECANCELED;
                why = "cancelled before admission";
            } else if (q->deadline_s > 0.0 && now() > q->deadline_s) {
                drop = SL_ETIMEOUT;
                why = "deadline passed before admission";
            } else if (q->footprint > cfg_.hbm_budget_bytes) {
                drop = SL_ENOMEM;
                why = "request cannot fit the HBM budget";
            }
            if (drop) {
                it = queue_.erase(it);
                finish(q, drop, why);
                continue;
            }
            if (slot < 0) return nullptr;
            if (in_use_ + q->footprint <= cfg_.hbm_budget_bytes) {
                if (blocked) blocked->bypassed++;
                queue_.erase(it);
                q->slot = slot;
                slots_[slot] = q;
                in_use_ += q->footprint;
                q->phase = Phase::ADMITTING;
                q->times.admitted_s = now();
                return q;
            }
            if (!blocked) {
                blocked = q;
                if (q->bypassed >= kMaxBypass) return nullptr;   // it waits, and so does everything behind it
            }
            ++it;
        }
        return nullptr;
    }

    // Finishes every request the server still holds (the step that failed
    // has been dealt with), and everything queued.
    void fail_all(const std::string& why)
    {
        for (Req* q : slots_) {
            if (!q || q->phase == Phase::ADMITTING) continue;   // its setup thread finishes it
            release(q);
            finish(q, SL_EDEVICE, "server stopped: " + why);
        }
        while (!queue_.empty()) {
            Req* q = reqs_[queue_.front()].get();
            queue_.pop_front();
            finish(q, SL_EDEVICE, "server stopped: " + why);
        }
    }

    // ---- threads

    void setup_loop()
    {
        for (;;) {
            Req* q = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu_);
                for (;;) {
                    if (stop_ || !fatal_.empty()) return;
                    q = pop_admissible();
                    if (q) break;
                    cv_.wait_for(lk, std::chrono::milliseconds(20));
                }
            }
            const sl_status ar = ex_.admit(*q);
            const std::string msg = ar ? std::string(sl_last_error()) : std::string();
            {
                std::lock_guard<std::mutex> lk(mu_);
                if (ar || !fatal_.empty() || stop_) {
                    release(q);
                    if (ar) finish(q, ar, msg);
                    else if (!fatal_.empty()) finish(q, SL_EDEVICE, "server stopped: " + fatal_);
                    else finish(q, SL_ECANCELED, "server stopped");
                } else {
                    q->phase = Phase::ACTIVE;
                    q->joined = false;
                    q->times.started_s = now();
                }
            }
            cv_loop_.notify_one();
            cv_.notify_all();   // a released slot or budget may admit others
        }
    }

    // Collects the results of requests whose sweeps are done, then retires
    // them.  Called from the loop thread, without mu_.
    void collect_all(std::vector<Req*>& done)
    {
        for (Req* q : done) {
            q->result = take_result(2 * static_cast<size_t>(std::max(q->desc.n_nodes, 0)));
            const sl_status cs = ex_.collect(*q, q->outcome);
            const std::string msg = cs ? std::string(sl_last_error()) : std::string();
            std::lock_guard<std::mutex> lk(mu_);
            if (cs == SL_OK) stats_.node_updates += q->outcome.node_updates;
            release(q);
            finish(q, cs, msg);
        }
        if (!done.empty()) cv_.notify_all();
        done.clear();
    }

    void loop()
    {
        std::vector<StepOutcome> out;
        std::vector<Req*> to_collect;
        std::vector<uint64_t> last_ids, ids;   // the requests of the last step and of this one
        for (;;) {
            // ---- 1. the set-up requests that still sweep
            std::vector<Req*> in_step;
            bool alone = false;
            {
                std::unique_lock<std::mutex> lk(mu_);
                auto ready = [&] {
                    for (Req* q : slots_)
                        if (q && q->phase == Phase::ACTIVE && !q->finishing) return true;
                    return false;
                };
                if (to_collect.empty())
                    cv_loop_.wait_for(lk, std::chrono::milliseconds(20), [&] { return stop_ || ready(); });
                if (stop_) break;
                bool admitting = false;
                for (Req* q : slots_) {
                    if (q && q->phase == Phase::ACTIVE && !q->finishing) in_step.push_back(q);
                    if (q && q->phase == Phase::ADMITTING) admitting = true;
                }
                // a lone request with nothing queued or being set up runs
                // longer steps: fewer host round trips, and no one waits to join
                alone = in_step.size() == 1 && queue_.empty() && !admitting;
            }
            if (in_step.empty()) {
                collect_all(to_collect);
                continue;
            }
            // ---- 2. launch; collect the last step's finished requests meanwhile
            ids.clear();
            for (Req* q : in_step) ids.push_back(q->id);
            const int32_t sweeps = cfg_.sweeps_per_step * (alone ? kAloneStepFactor : 1);
            sl_status r = ex_.launch(in_step, ids != last_ids, sweeps);
            last_ids.swap(ids);
            collect_all(to_collect);
            // ---- 3. wait and decide
            out.assign(in_step.size(), StepOutcome{});
            if (!r) r = ex_.wait(in_step, out);
            const std::string step_err = r ? std::string(sl_last_error()) : std::string();
            const double t = now();
            std::lock_guard<std::mutex> lk(mu_);
            stats_.steps++;
            for (size_t k = 0; k < in_step.size(); ++k) {
                Req* q = in_step[k];
                q->outcome = out[k];
                sl_status fs = SL_OK;
                std::string msg;
                if (r) {
                    fs = r;
                    msg = step_err;
                } else if (!out[k].active) {
                    // done: collected while the next step runs
                    q->finishing = true;
                    to_collect.push_back(q);
                    continue;
                } else if (q->cancel) {
                    fs = SL_ECANCELED;
                    msg = "cancelled";
                } else if (q->deadline_s > 0.0 && t > q->deadline_s) {
                    fs = SL_ETIMEOUT;
                    msg = "deadline passed";
                } else {
                    continue;
                }
                release(q);
                finish(q, fs, msg);
            }
            if (r) {
                fatal_ = step_err.empty() ? "step failed" : step_err;
                for (Req* q : to_collect) {   // (none: a failed step finished its requests)
                    release(q);
                    finish(q, SL_EDEVICE, "server stopped: " + fatal_);
                }
                to_collect.clear();
                fail_all(fatal_);
                cv_.notify_all();
                break;
            }
            cv_.notify_all();
        }
        // stopping: results not collected yet are dropped with their requests
        std::lock_guard<std::mutex> lk(mu_);
        for (Req* q : to_collect) {
            release(q);
            finish(q, SL_ECANCELED, "server stopped");
        }
    }

    // Result buffers of polled requests, kept for later results (at most
    // kResultPoolBytes in kResultPoolCount buffers): a fresh buffer costs its
    // zero fill and the first touch of every page again (about 10 ms for a
    // mesh of 4M nodes), a reused one neither.
    static constexpr size_t kResultPoolBytes = size_t(1) << 30;
    static constexpr size_t kResultPoolCount = 256;
    std::mutex pool_mu_;
    std::vector<std::vector<double>> pool_;
    size_t pool_bytes_ = 0;

    // A buffer of n doubles: the smallest pooled one that holds n, else a new one.
    std::vector<double> take_result(size_t n)
    {
        std::vector<double> v;
        {
            std::lock_guard<std::mutex> lk(pool_mu_);
            size_t best = pool_.size();
            for (size_t k = 0; k < pool_.size(); ++k)
                if (pool_[k].capacity() >= n && (best == pool_.size() || pool_[k].capacity() < pool_[best].capacity()))
                    best = k;
            if (best < pool_.size()) {
                v = std::move(pool_[best]);
                if (best + 1 != pool_.size()) pool_[best] = std::move(pool_.back());
                pool_.pop_back();
                pool_bytes_ -= v.capacity() * sizeof(double);
            }
        }
        v.resize(n);
        return v;
    }

    void give_result(std::vector<double>&& v)
    {
        const size_t b = v.capacity() * sizeof(double);
        if (b == 0) return;
        std::lock_guard<std::mutex> lk(pool_mu_);
        if (pool_bytes_ + b > kResultPoolBytes || pool_.size() >= kResultPoolCount)
            return;   // not kept: freed with the request
        pool_bytes_ += b;
        pool_.push_back(std::move(v));
    }

    sl_server_config cfg_;
    Exec& ex_;
    Clock::time_point t0_;
    std::mutex mu_;
    std::condition_variable cv_;        // setup threads: queue, slots or budget changed
    std::condition_variable cv_loop_;   // loop thread: a request is set up
    std::deque<uint64_t> queue_;                       // queued request ids, in arrival order
    std::map<uint64_t, std::unique_ptr<Req>> reqs_;    // every request not yet polled
    std::vector<Req*> slots_;                          // admitted requests by slot
    size_t in_use_ = 0;
    uint64_t next_id_ = 1;
    bool stop_ = false;
    std::thread thread_;
    std::vector<std::thread> setup_;
    sl_server_stats stats_{};
    std::string fatal_;
};

}  // namespace sched

}  // namespace sl

#endif  // SL_SCHED_H
