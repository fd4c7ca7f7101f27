// Host-only tests of the serving scheduler (paper_1502_00355_amd/csrc/sl_sched.h)
// against a mock executor: simulated step durations, a sweep counter per
// request, injected admission and step failures.  Each scenario prints
// "ok <name>" or "FAIL <name>: <why>"; the exit status is the failure count.
#include <chrono>
#include <cstdio>
#include <functional>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../paper_1502_00355_amd/csrc/sl_sched.h"

namespace {
thread_local std::string g_err;
}
namespace sl {
void set_error(const std::string& msg) { g_err = msg; }
sl_status fail(sl_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}
}  // namespace sl
extern "C" const char* sl_last_error(void) { return g_err.c_str(); }

namespace {

using Clock = std::chrono::steady_clock;
using sl::sched::StepOutcome;

struct MockPayload {
    int32_t sweeps = 0;
    bool active = false;
    int32_t converge_at = -1;   // tolerance requests stop after this many sweeps
};

// Budget units are nodes: footprint(d) = d.n_nodes.  A tolerance request
// (tol > 0) "converges" after d.n_tris sweeps.
struct Mock {
    using Payload = MockPayload;
    using Req = sl::sched::Request<Payload>;

    int32_t sweeps_per_step = 4;
    int step_us = 500;
    int admit_us = 200;
    int slow_admit_us = 0;              // admission time of the requests in slow_admit
    std::set<uint64_t> slow_admit;
    std::set<uint64_t> fail_admit;
    int fail_step_at = -1;
    size_t budget = 0;

    // observations (loop thread writes, test thread reads after stop)
    std::mutex mu;
    std::vector<std::vector<uint64_t>> steps;
    std::vector<int32_t> step_sweeps;   // sweeps of each step launched
    std::set<uint64_t> live;
    size_t live_fp = 0, max_live_fp = 0;
    int max_live = 0;
    std::vector<std::string> violations;
    int admitting = 0, max_admitting = 0;
    Clock::time_point step_end;
    std::vector<Req*> pending;

    size_t footprint(const sl_mesh_desc& d) { return static_cast<size_t>(d.n_nodes); }

    // called by several setup threads at once
    sl_status admit(Req& q)
    {
        bool slow, fails;
        {
            std::lock_guard<std::mutex> lk(mu);
            slow = slow_admit.count(q.id) != 0;
            fails = fail_admit.count(q.id) != 0;
            admitting++;
            max_admitting = std::max(max_admitting, admitting);
        }
        std::this_thread::sleep_for(std::chrono::microseconds(slow ? slow_admit_us : admit_us));
        std::lock_guard<std::mutex> lk(mu);
        admitting--;
        if (fails) return sl::fail(SL_ETOPO, "mock: invalid topology");
        if (q.joined) violations.push_back("admitted request already joined");
        live.insert(q.id);
        live_fp += q.footprint;
        max_live_fp = std::max(max_live_fp, live_fp);
        max_live = std::max(max_live, static_cast<int>(live.size()));
        if (budget && live_fp > budget) violations.push_back("budget exceeded");
        q.x.sweeps = 0;
        q.x.active = q.iterations > 0;
        q.x.converge_at = q.tol > 0.0 ? q.desc.n_tris : -1;
        return SL_OK;
    }

    sl_status launch(const std::vector<Req*>& in_step, bool, int32_t sweeps)
    {
        std::lock_guard<std::mutex> lk(mu);
        step_sweeps.push_back(sweeps);
        std::vector<uint64_t> ids;
        for (Req* q : in_step) {
            if (!live.count(q->id)) violations.push_back("stepped a request that is not admitted");
            ids.push_back(q->id);
            q->joined = true;
        }
        steps.push_back(ids);
        pending = in_step;
        step_end = Clock::now() + std::chrono::microseconds(step_us);
        return SL_OK;
    }

    bool busy() { return Clock::now() < step_end; }

    sl_status wait(const std::vector<Req*>& in_step, std::vector<StepOutcome>& out)
    {
        std::this_thread::sleep_until(step_end);
        int idx;
        {
            std::lock_guard<std::mutex> lk(mu);
            idx = static_cast<int>(steps.size()) - 1;
            if (in_step != pending) violations.push_back("wait on a different request set");
        }
        if (idx == fail_step_at) return sl::fail(SL_EDEVICE, "mock: device fault in step");
        for (size_t k = 0; k < in_step.size(); ++k) {
            MockPayload& x = in_step[k]->x;
            for (int32_t j = 0; j < step_sweeps.back() && x.active; ++j) {
                ++x.sweeps;
                x.active = x.sweeps < in_step[k]->iterations && !(x.converge_at >= 0 && x.sweeps >= x.converge_at);
            }
            out[k].active = x.active;
            out[k].sweeps = x.sweeps;
            out[k].node_updates = static_cast<int64_t>(x.sweeps) * in_step[k]->desc.n_nodes;
        }
        return SL_OK;
    }

    sl_status collect(Req& q, const StepOutcome& o)
    {
        q.result.assign(2 * static_cast<size_t>(q.desc.n_nodes), static_cast<double>(q.id));
        q.report = sl_report{};
        q.report.iterations_run = o.sweeps;
        return SL_OK;
    }

    void release(Req& q)
    {
        std::lock_guard<std::mutex> lk(mu);
        if (live.erase(q.id)) live_fp -= q.footprint;
    }
};

struct Server {
    Mock ex;
    sl_server_config cfg{};
    std::unique_ptr<sl::sched::Scheduler<Mock>> core;
    std::vector<int32_t> keep;   // backing for the descriptors (never read by the mock)
    std::mutex nodes_mu;
    std::map<uint64_t, int32_t> nodes_of;   // result buffers are n_nodes x 2
    Server(size_t budget, int32_t max_active, int32_t sweeps_per_step = 4, int32_t setup_threads = 2)
    {
        cfg.hbm_budget_bytes = budget;
        cfg.max_active = max_active;
        cfg.sweeps_per_step = sweeps_per_step;
        cfg.setup_threads = setup_threads;
        ex.sweeps_per_step = sweeps_per_step;
        ex.budget = budget;
        keep.assign(4, 0);
    }
    void start()
    {
        core = std::make_unique<sl::sched::Scheduler<Mock>>(cfg, ex);
        core->start();
    }
    uint64_t submit(int32_t nodes, int32_t iters, double tol = 0.0, int32_t conv = 0, double deadline = 0.0,
                    sl_status want = SL_OK)
    {
        sl_mesh_desc d{};
        d.n_nodes = nodes;
        d.n_tris = conv;
        d.coords = reinterpret_cast<double*>(keep.data());
        uint64_t id = 0;
        const sl_status st = core->submit(d, iters, tol, deadline, &id);
        if (st != want) throw std::runtime_error("submit returned " + std::to_string(st));
        std::lock_guard<std::mutex> lk(nodes_mu);
        nodes_of[id] = nodes;
        return id;
    }
    struct Done {
        sl_status st;
        sl_report rep;
        sl_request_times t;
        std::vector<double> out;
        std::string msg;
    };
    Done wait(uint64_t id, double timeout_s = 20.0)
    {
        Done d{};
        int32_t nodes = 1;
        {
            std::lock_guard<std::mutex> lk(nodes_mu);
            auto it = nodes_of.find(id);
            if (it != nodes_of.end()) nodes = it->second;
        }
        d.out.assign(2 * static_cast<size_t>(nodes), -1.0);
        const auto t0 = Clock::now();
        for (;;) {
            d.st = core->poll(id, d.out.data(), &d.rep, &d.t);
            if (d.st != SL_EBUSY) break;
            if (std::chrono::duration<double>(Clock::now() - t0).count() > timeout_s)
                throw std::runtime_error("request " + std::to_string(id) + " never finished");
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
        d.msg = sl_last_error();
        return d;
    }
    void stop() { core->stop(); }
};

int failures = 0;

void check(bool ok, const std::string& name, const std::string& why)
{
    if (!ok) {
        std::printf("FAIL %s: %s\n", name.c_str(), why.c_str());
        ++failures;
    }
}

void run(const std::string& name, const std::function<void(const std::string&)>& f)
{
    const int before = failures;
    try {
        f(name);
    } catch (const std::exception& e) {
        check(false, name, std::string("exception: ") + e.what());
    }
    if (failures == before) std::printf("ok %s\n", name.c_str());
    std::fflush(stdout);
}

void no_violations(Server& s, const std::string& name)
{
    for (auto& v : s.ex.violations) check(false, name, v);
}

}  // namespace

int main()
{
    run("caps_and_results", [](const std::string& n) {
        Server s(1000, 8);
        s.start();
        const int32_t its[] = {0, 1, 4, 9, 30};
        std::vector<uint64_t> ids;
        for (int32_t it : its) ids.push_back(s.submit(10, it));
        for (size_t k = 0; k < ids.size(); ++k) {
            auto d = s.wait(ids[k]);
            check(d.st == SL_OK, n, "status " + std::to_string(d.st));
            check(d.rep.iterations_run == its[k], n, "iterations_run " + std::to_string(d.rep.iterations_run));
            check(d.out[0] == static_cast<double>(ids[k]), n, "result not copied");
            check(d.t.submitted_s <= d.t.admitted_s && d.t.admitted_s <= d.t.started_s && d.t.started_s <= d.t.done_s,
                  n, "times out of order");
        }
        sl_server_stats st{};
        check(s.core->stats(&st) == SL_OK, n, "stats");
        check(st.submitted == 5 && st.completed == 5 && st.failed == 0, n, "counts");
        check(st.node_updates == 10 * (0 + 1 + 4 + 9 + 30), n, "node updates " + std::to_string(st.node_updates));
        check(st.hbm_in_use == 0 && st.active == 0 && st.queued == 0, n, "budget not returned");
        s.stop();
        no_violations(s, n);
    });

    run("result_buffers_reused_across_sizes", [](const std::string& n) {
        // polled results go back to the core's pool and serve later, smaller
        // or larger, requests: each result must be its own, whole
        Server s(1000, 8);
        s.start();
        const int32_t nodes[] = {50, 10, 200, 30, 200, 1, 120};
        for (int32_t nn : nodes) {
            const uint64_t id = s.submit(nn, 3);
            auto d = s.wait(id);
            check(d.st == SL_OK, n, "status " + std::to_string(d.st));
            bool whole = d.out.size() == 2 * static_cast<size_t>(nn);
            for (double v : d.out) whole = whole && v == static_cast<double>(id);
            check(whole, n, "result of " + std::to_string(nn) + " nodes not its own");
        }
        s.stop();
        no_violations(s, n);
    });

    run("lone_request_takes_longer_steps", [](const std::string& n) {
        // alone, with nothing queued or being set up, a request steps
        // kAloneStepFactor times the configured sweeps; once another is
        // set up next to it, steps go back to the configured length
        Server s(1000, 8, 4, 1);
        s.ex.step_us = 2000;
        s.start();
        const uint64_t a = s.submit(10, 64);
        auto da = s.wait(a);
        check(da.st == SL_OK && da.rep.iterations_run == 64, n, "a");
        const size_t k0 = s.ex.steps.size();
        check(k0 == 4, n, "lone request took " + std::to_string(k0) + " steps, not 4");
        for (size_t k = 0; k < k0; ++k)
            check(s.ex.step_sweeps[k] == 4 * sl::sched::kAloneStepFactor, n, "short lone step");
        const uint64_t b = s.submit(10, 400), c = s.submit(10, 8);
        auto db = s.wait(b), dc = s.wait(c);
        check(db.st == SL_OK && dc.st == SL_OK && db.rep.iterations_run == 400 && dc.rep.iterations_run == 8, n,
              "b and c");
        bool together_short = false;
        for (size_t k = k0; k < s.ex.steps.size(); ++k)
            if (s.ex.steps[k].size() == 2) together_short = together_short || s.ex.step_sweeps[k] == 4;
        check(together_short, n, "no configured-length step with both requests");
        s.stop();
        no_violations(s, n);
    });

    run("budget_bypass", [](const std::string& n) {
        Server s(100, 8, 4, 1);
        s.start();
        const uint64_t a = s.submit(60, 400);
        const uint64_t b = s.submit(50, 4);    // must wait for a (60 + 50 > 100)
        const uint64_t c = s.submit(30, 4);    // fits next to a: passes b
        auto da = s.wait(a), db = s.wait(b), dc = s.wait(c);
        check(da.st == SL_OK && db.st == SL_OK && dc.st == SL_OK, n, "statuses");
        check(db.t.admitted_s >= da.t.done_s - 1e-3, n, "b admitted before a finished");
        check(dc.t.admitted_s < db.t.admitted_s && dc.t.done_s < da.t.done_s, n, "c waited behind b");
        check(s.ex.max_live_fp <= 100, n, "budget exceeded");
        s.stop();
        no_violations(s, n);
    });

    run("bypass_is_bounded", [](const std::string& n) {
        // a holds most of the budget for a while; b does not fit next to it;
        // a stream of small requests fits: at most kMaxBypass of them pass b
        Server s(100, 200, 4, 2);
        s.ex.step_us = 300;
        s.ex.admit_us = 20;
        s.start();
        const uint64_t a = s.submit(60, 600);
        const uint64_t b = s.submit(50, 4);
        std::vector<uint64_t> small;
        for (int k = 0; k < 150; ++k) small.push_back(s.submit(1, 1));
        auto db = s.wait(b);
        int before = 0;
        std::vector<Server::Done> ds;
        for (auto id : small) ds.push_back(s.wait(id));
        for (auto& d : ds) before += d.t.admitted_s < db.t.admitted_s;
        auto da = s.wait(a);
        check(da.st == SL_OK && db.st == SL_OK, n, "statuses");
        check(before >= 1 && before <= sl::sched::kMaxBypass, n, "passed b: " + std::to_string(before));
        check(db.t.admitted_s >= da.t.done_s - 1e-3, n, "b admitted next to a");
        s.stop();
        no_violations(s, n);
    });

    run("setup_does_not_stall_steps", [](const std::string& n) {
        // b's setup takes 40 ms on a setup thread; a keeps stepping meanwhile
        Server s(1000, 4, 4, 2);
        s.ex.step_us = 500;
        s.ex.slow_admit_us = 40000;
        s.ex.slow_admit.insert(2);
        s.start();
        const uint64_t a = s.submit(10, 40);   // 10 steps of 0.5 ms
        const uint64_t b = s.submit(10, 4);
        auto da = s.wait(a), db = s.wait(b);
        check(b == 2 && da.st == SL_OK && db.st == SL_OK, n, "statuses");
        check(da.t.done_s < db.t.started_s, n, "a waited for b's setup");
        s.stop();
        no_violations(s, n);
    });

    run("step_failure_with_admissions_in_flight", [](const std::string& n) {
        // c is being set up while the step that fails runs: it fails too, and
        // the budget comes back
        Server s(1000, 4, 4, 2);
        s.ex.fail_step_at = 3;
        s.ex.step_us = 2000;
        s.ex.slow_admit_us = 20000;
        s.ex.slow_admit.insert(3);
        s.start();
        const uint64_t a = s.submit(60, 100000);
        const uint64_t b = s.submit(60, 100000);
        std::this_thread::sleep_for(std::chrono::milliseconds(3));
        const uint64_t c = s.submit(60, 4);
        auto da = s.wait(a), db = s.wait(b), dc = s.wait(c);
        check(c == 3 && da.st == SL_EDEVICE && db.st == SL_EDEVICE, n, "in-step requests");
        check(dc.st == SL_EDEVICE, n, "request admitted during the failing step: " + std::to_string(dc.st));
        sl_server_stats st{};
        check(s.core->stats(&st) == SL_EDEVICE, n, "stats after the fault");
        check(st.hbm_in_use == 0 && st.active == 0, n, "budget or slots not returned");
        check(st.failed == 3, n, "failed " + std::to_string(st.failed));
        s.stop();
        no_violations(s, n);
    });

    run("slots_limit_concurrency", [](const std::string& n) {
        Server s(1 << 20, 2);
        s.start();
        std::vector<uint64_t> ids;
        for (int k = 0; k < 6; ++k) ids.push_back(s.submit(5, 12));
        for (auto id : ids) check(s.wait(id).st == SL_OK, n, "status");
        check(s.ex.max_live <= 2, n, "more than 2 active: " + std::to_string(s.ex.max_live));
        s.stop();
        no_violations(s, n);
    });

    run("too_large_fails_at_once", [](const std::string& n) {
        Server s(100, 4);
        s.start();
        const uint64_t big = s.submit(150, 4);
        const uint64_t ok = s.submit(20, 4);
        auto d = s.wait(big);
        check(d.st == SL_ENOMEM && d.t.admitted_s == 0.0, n, "oversized request not rejected");
        check(s.wait(ok).st == SL_OK, n, "next request blocked");
        s.stop();
        no_violations(s, n);
    });

    run("cancel_queued_and_active", [](const std::string& n) {
        Server s(100, 4);
        s.ex.step_us = 2000;
        s.start();
        const uint64_t a = s.submit(80, 100000);   // long: blocks the budget
        const uint64_t b = s.submit(50, 4);        // queued behind it
        std::this_thread::sleep_for(std::chrono::milliseconds(5));
        s.core->cancel(b);
        s.core->cancel(a);
        auto db = s.wait(b), da = s.wait(a);
        check(db.st == SL_ECANCELED && db.t.admitted_s == 0.0, n, "queued cancel");
        check(da.st == SL_ECANCELED && da.t.admitted_s > 0.0, n, "active cancel");
        const uint64_t c = s.submit(90, 4);
        check(s.wait(c).st == SL_OK, n, "budget not freed by the cancellations");
        check(s.core->cancel(a) == SL_EINVAL, n, "cancel of a polled request");
        s.stop();
        no_violations(s, n);
    });

    run("deadlines_queued_and_active", [](const std::string& n) {
        Server s(100, 4);
        s.ex.step_us = 2000;
        s.start();
        const uint64_t a = s.submit(80, 100000, 0.0, 0, 0.05);   // active, passes its deadline
        const uint64_t b = s.submit(50, 4, 0.0, 0, 0.01);         // queued, passes its deadline
        auto da = s.wait(a), db = s.wait(b);
        check(da.st == SL_ETIMEOUT && da.t.admitted_s > 0.0, n, "active deadline: " + std::to_string(da.st));
        check(db.st == SL_ETIMEOUT && db.t.admitted_s == 0.0, n, "queued deadline: " + std::to_string(db.st));
        check(da.t.done_s >= 0.05, n, "active request stopped before its deadline");
        s.stop();
        no_violations(s, n);
    });

    run("admission_failure_is_local", [](const std::string& n) {
        Server s(1000, 4);
        s.ex.fail_admit.insert(2);
        s.start();
        const uint64_t a = s.submit(10, 8), b = s.submit(10, 8), c = s.submit(10, 8);
        auto da = s.wait(a), db = s.wait(b), dc = s.wait(c);
        check(b == 2 && db.st == SL_ETOPO && db.msg.find("mock") != std::string::npos, n, "failed admission");
        check(da.st == SL_OK && dc.st == SL_OK, n, "neighbours of the failed request");
        sl_server_stats st{};
        s.core->stats(&st);
        check(st.failed == 1 && st.completed == 2 && st.hbm_in_use == 0, n, "counts after a failed admission");
        s.stop();
        no_violations(s, n);
    });

    run("step_failure_stops_the_server", [](const std::string& n) {
        Server s(100, 4);
        s.ex.fail_step_at = 2;
        s.ex.step_us = 1000;
        s.start();
        const uint64_t a = s.submit(60, 100000);
        const uint64_t b = s.submit(60, 4);   // queued behind a
        auto da = s.wait(a), db = s.wait(b);
        check(da.st == SL_EDEVICE, n, "in-step request: " + std::to_string(da.st));
        check(db.st == SL_EDEVICE, n, "queued request: " + std::to_string(db.st));
        s.submit(10, 4, 0.0, 0, 0.0, SL_EDEVICE);
        sl_server_stats st{};
        check(s.core->stats(&st) == SL_EDEVICE, n, "stats after the fault");
        check(st.hbm_in_use == 0, n, "budget not returned");
        s.stop();
        no_violations(s, n);
    });

    run("continuous_batching_join", [](const std::string& n) {
        Server s(1000, 4);
        s.ex.step_us = 1000;
        s.start();
        const uint64_t a = s.submit(10, 400);
        std::this_thread::sleep_for(std::chrono::milliseconds(10));
        const uint64_t b = s.submit(10, 8);
        auto db = s.wait(b), da = s.wait(a);
        check(da.st == SL_OK && db.st == SL_OK && da.rep.iterations_run == 400 && db.rep.iterations_run == 8, n,
              "results");
        check(db.t.done_s < da.t.done_s, n, "b did not finish while a was running");
        bool shared = false;
        for (auto& ids : s.ex.steps) shared = shared || (std::count(ids.begin(), ids.end(), a) &&
                                                         std::count(ids.begin(), ids.end(), b));
        check(shared, n, "a and b never shared a step");
        s.stop();
        no_violations(s, n);
    });

    run("tolerance_stops_early", [](const std::string& n) {
        Server s(1000, 4);
        s.start();
        const uint64_t a = s.submit(10, 10000, 1e-8, 10);
        auto d = s.wait(a);
        check(d.st == SL_OK && d.rep.iterations_run == 10, n, "iterations_run " + std::to_string(d.rep.iterations_run));
        s.stop();
        no_violations(s, n);
    });

    run("poll_rules", [](const std::string& n) {
        Server s(1000, 4);
        s.start();
        const uint64_t a = s.submit(10, 4);
        check(s.wait(a).st == SL_OK, n, "first poll");
        double buf[20];
        check(s.core->poll(a, buf, nullptr, nullptr) == SL_EINVAL, n, "second poll of one request");
        check(s.core->poll(987654, buf, nullptr, nullptr) == SL_EINVAL, n, "unknown id");
        s.stop();
        no_violations(s, n);
    });

    run("mixed_load_invariants", [](const std::string& n) {
        Server s(400, 6, 2);
        s.ex.step_us = 200;
        s.ex.admit_us = 50;
        s.ex.fail_admit = {7, 77};
        s.start();
        std::mutex mu;
        std::vector<std::pair<uint64_t, int32_t>> ids;
        std::vector<std::thread> th;
        for (int t = 0; t < 4; ++t)
            th.emplace_back([&, t] {
                std::mt19937 rng(1234 + t);
                for (int k = 0; k < 50; ++k) {
                    const int32_t nodes = 1 + static_cast<int32_t>(rng() % 300);
                    const int32_t its = static_cast<int32_t>(rng() % 40);
                    const bool tol = rng() % 2;
                    const uint64_t id = s.submit(nodes, its, tol ? 1e-8 : 0.0, 1 + static_cast<int32_t>(rng() % 20));
                    if (rng() % 10 == 0 && id != 7 && id != 77) s.core->cancel(id);
                    std::lock_guard<std::mutex> lk(mu);
                    ids.emplace_back(id, nodes);
                }
            });
        for (auto& x : th) x.join();
        int ok = 0, canceled = 0, topo = 0;
        for (auto& p : ids) {
            auto d = s.wait(p.first);
            ok += d.st == SL_OK;
            canceled += d.st == SL_ECANCELED;
            topo += d.st == SL_ETOPO;
            check(d.st == SL_OK || d.st == SL_ECANCELED || d.st == SL_ETOPO, n, "status " + std::to_string(d.st));
        }
        sl_server_stats st{};
        s.core->stats(&st);
        check(st.submitted == 200 && st.completed + st.failed == 200, n, "counts");
        check(st.hbm_in_use == 0 && st.queued == 0 && st.active == 0, n, "not drained");
        check(s.ex.max_live_fp <= 400 && s.ex.max_live <= 6, n, "limits exceeded");
        check(s.ex.max_admitting <= 2, n, "more admissions at once than setup threads");
        check(topo == 2, n, "injected admission failures: " + std::to_string(topo));
        s.stop();
        no_violations(s, n);
    });

    std::printf("%d failure(s)\n", failures);
    return failures;
}
