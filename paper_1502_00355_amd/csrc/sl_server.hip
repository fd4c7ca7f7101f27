// Serving: smoothing requests that arrive over time, swept together.
//
// A scheduler thread owns the device.  Submitted requests wait in a FIFO.
// A request is admitted when a slot is free and its estimated device
// footprint fits what is left of the HBM budget; admission uploads the mesh
// and builds its tiles on a setup stream while earlier requests keep
// sweeping on the compute stream.  Every scheduling step runs a few sweeps
// over the tiles of all admitted requests with one launch per sweep
// (continuous batching: a request joins at the next step after its setup and
// leaves as soon as its sweep cap or tolerance is reached, or it is
// cancelled or passes its deadline).  A request's arithmetic is that of a
// single smooth_mesh call: tiles only read their own mesh, so the result does
// not depend on which requests share its launches.
//
// The scheduler launches a step asynchronously and admits queued requests
// while it runs, until the step has finished; admitted requests join at the
// start of the next step, when their sweep state is written on the compute
// stream, so a step never sees a request that is half set up.
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

#include "sl_common.h"

namespace sl {

namespace {

using Clock = std::chrono::steady_clock;

constexpr int32_t kMaxActive = 65536;

double seconds_since(Clock::time_point t0, Clock::time_point t)
{
    return std::chrono::duration<double>(t - t0).count();
}

struct Request {
    uint64_t id = 0;
    sl_mesh_desc desc{};
    int32_t iterations = 0;
    double tol = 0.0;
    double deadline_s = 0.0;          // server-clock seconds; <= 0: none
    size_t footprint = 0;
    // lifecycle
    enum Phase { QUEUED, ACTIVE, DONE } phase = QUEUED;
    sl_status status = SL_EBUSY;
    std::string error;
    bool cancel = false;
    int32_t slot = -1;
    int32_t parity0 = 0;              // launch parity when it joined
    bool joined = false;              // its sweep state is on the device
    MeshState state0{};               // the sweep state it joins with
    DevMesh mesh;
    std::vector<double> result;       // n x 2, filled when done
    sl_report report{};
    sl_request_times times{};
};

size_t estimate_footprint(const sl_mesh_desc& d)
{
    const size_t n = static_cast<size_t>(std::max(d.n_nodes, 0));
    const size_t nnz = d.nbr_ptr ? static_cast<size_t>(std::max(d.nbr_ptr[n], 0)) : 0;
    const size_t ninc = d.tri_ptr ? static_cast<size_t>(std::max(d.tri_ptr[n], 0)) : 0;
    // inputs during setup + resident: coordinates (4 buffers of 16 B), labels,
    // rows, tiles (local rows, triangles, halo), ordering scratch
    return n * (16 * 4 + 8 + 16 + 12) + nnz * (4 + 2 + 4) + ninc * (4 + 2 + 6) + 12 * static_cast<size_t>(d.n_tris) +
           (1u << 20);
}

}  // namespace

}  // namespace sl

struct sl_server {
    sl_server_config cfg{};
    sl_options opts{};
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;                                     // queued request ids, FIFO
    std::map<uint64_t, std::unique_ptr<sl::Request>> reqs;          // every live request
    std::atomic<bool> stop{false};
    std::thread thread;
    uint64_t next_id = 1;
    sl::Clock::time_point t0;
    // scheduler-thread state
    hipStream_t st_compute = nullptr, st_setup = nullptr;
    sl::MeshState* states = nullptr;        // [max_active]
    sl::MeshState* h_states = nullptr;      // [max_active], pinned: read-back after each step
    sl::MeshState* h_join = nullptr;        // [max_active], pinned: the state a joining request starts from
    sl::TileWork* work = nullptr;
    int64_t work_cap = 0;
    double* out = nullptr;
    size_t out_cap = 0;
    std::vector<sl::Request*> slots;        // [max_active]
    size_t hbm_in_use = 0;
    int32_t parity = 0;
    int device = 0;
    // statistics
    sl_server_stats stats{};
    std::string fatal;
};

namespace sl {

namespace {

void finish(sl_server* S, Request* q, sl_status status, const std::string& err)
{
    q->status = status;
    q->error = err;
    q->phase = Request::DONE;
    q->times.done_s = seconds_since(S->t0, Clock::now());
}

// Scheduler-thread side of a failed device call: the request fails, the
// server carries on.
sl_status admit(sl_server* S, Request* q, int32_t slot)
{
    hipStream_t st = S->st_setup;
    const sl_status r = upload_and_prepare(q->desc, S->opts, slot, q->mesh, st);
    if (r) {
        devmesh_free(q->mesh, st);
        return r;
    }
    SL_HIP(hipStreamSynchronize(st));
    MeshState& h = q->state0;
    h = MeshState{};
    h.iters = q->iterations;
    h.active = q->iterations > 0;
    h.tol2 = q->tol > 0.0 ? q->tol * q->tol : 0.0;
    q->joined = false;
    return SL_OK;
}

// Concatenates the tile lists of the admitted tile-path meshes.
sl_status rebuild_work(sl_server* S, int32_t* n_work, int32_t* T, int32_t* hcap, int32_t* rcap)
{
    int64_t total = 0;
    *T = 0;
    *hcap = 0;
    *rcap = 0;
    for (Request* q : S->slots)
        if (q && q->phase == Request::ACTIVE && q->mesh.tile_nodes > 0) total += q->mesh.n_tiles;
    if (total > INT32_MAX) return fail(SL_ENOMEM, "too many tiles in flight");
    if (total > S->work_cap) {
        dfree(S->work, S->st_compute);
        S->work_cap = std::max<int64_t>(total, 2 * S->work_cap);
        sl_status r = dalloc(&S->work, static_cast<size_t>(S->work_cap), S->st_compute);
        if (r) { S->work_cap = 0; return r; }
    }
    int64_t off = 0;
    for (Request* q : S->slots) {
        if (!q || q->phase != Request::ACTIVE || q->mesh.tile_nodes == 0) continue;
        SL_HIP(hipMemcpyAsync(S->work + off, q->mesh.work, sizeof(TileWork) * q->mesh.n_tiles,
                              hipMemcpyDeviceToDevice, S->st_compute));
        off += q->mesh.n_tiles;
        if (*T != 0 && q->mesh.tile_nodes != *T) return fail(SL_EINVAL, "requests with different tile sizes");
        *T = q->mesh.tile_nodes;
        *hcap = std::max(*hcap, q->mesh.halo_max);
        *rcap = std::max(*rcap, q->mesh.rows_max);
    }
    *n_work = static_cast<int32_t>(total);
    return SL_OK;
}

// Copies a finished request's positions back to host memory.
sl_status collect(sl_server* S, Request* q, const MeshState& ms)
{
    const DevMesh& m = q->mesh;
    const size_t n = static_cast<size_t>(m.n);
    if (S->out_cap < 2 * n) {
        dfree(S->out, S->st_compute);
        sl_status r = dalloc(&S->out, 2 * n, S->st_compute);
        if (r) { S->out_cap = 0; return r; }
        S->out_cap = 2 * n;
    }
    const bool jacobi = S->opts.form == SL_JACOBI;
    const int src = jacobi ? ((q->parity0 + ms.s) & 1) : 0;
    sl_status r = unpermute_coords(m, src, S->out, S->st_compute);
    if (r) return r;
    q->result.resize(2 * n);
    SL_HIP(hipMemcpyAsync(q->result.data(), S->out, 2 * n * sizeof(double), hipMemcpyDeviceToHost, S->st_compute));
    SL_HIP(hipStreamSynchronize(S->st_compute));
    sl_report rep{};
    rep.iterations_run = ms.s;
    rep.n_colors = m.n_colors;
    std::memcpy(&rep.max_disp_sq_last, &ms.maxd_last, sizeof(double));
    rep.accepted_last = static_cast<int64_t>(ms.acc_last);
    rep.accepted_total = static_cast<int64_t>(ms.acc_total);
    rep.kernel_used = (jacobi && m.tile_nodes > 0) ? SL_KERNEL_TILE : SL_KERNEL_NODE;
    rep.tile_nodes = m.tile_nodes;
    q->report = rep;
    return SL_OK;
}

void release(sl_server* S, Request* q)
{
    devmesh_free(q->mesh, S->st_compute);
    S->hbm_in_use -= q->footprint;
    if (q->slot >= 0) S->slots[q->slot] = nullptr;
    q->slot = -1;
}

// Takes the head of the queue if it can be admitted now (finishing the
// requests at the head that are cancelled, past their deadline or too large
// for the budget); nullptr if the queue is empty or the head must wait.
Request* pop_admissible(sl_server* S)
{
    const int32_t max_active = S->cfg.max_active;
    while (!S->queue.empty()) {
        Request* q = S->reqs[S->queue.front()].get();
        if (q->cancel) {
            S->queue.pop_front();
            finish(S, q, SL_ECANCELED, "cancelled before admission");
            continue;
        }
        if (q->deadline_s > 0.0 && seconds_since(S->t0, Clock::now()) > q->deadline_s) {
            S->queue.pop_front();
            finish(S, q, SL_ETIMEOUT, "deadline passed before admission");
            continue;
        }
        if (q->footprint > S->cfg.hbm_budget_bytes) {
            S->queue.pop_front();
            finish(S, q, SL_ENOMEM, "request cannot fit the HBM budget");
            continue;
        }
        int32_t slot = -1;
        for (int32_t i = 0; i < max_active; ++i)
            if (!S->slots[i]) { slot = i; break; }
        if (slot < 0 || S->hbm_in_use + q->footprint > S->cfg.hbm_budget_bytes) return nullptr;
        S->queue.pop_front();
        q->slot = slot;
        S->slots[slot] = q;
        S->hbm_in_use += q->footprint;
        q->times.admitted_s = seconds_since(S->t0, Clock::now());
        return q;
    }
    return nullptr;
}

void scheduler(sl_server* S)
{
    (void)hipSetDevice(S->device);
    const int32_t max_active = S->cfg.max_active;
    const MeshState* hstate = S->h_states;
    bool work_dirty = true;
    int32_t n_work = 0, T = 0, hcap = 0, rcap = 0;
    const bool jacobi = S->opts.form == SL_JACOBI;
    const int32_t wg_per_cu = resolve_wg_per_cu(S->opts), block = resolve_block_size(S->opts);
    while (!S->stop.load()) {
        // ---- 1. launch one step (a few sweeps) over every ready request
        std::vector<Request*> in_step;
        for (Request* q : S->slots)
            if (q && q->phase == Request::ACTIVE) in_step.push_back(q);
        sl_status r = SL_OK;
        if (!in_step.empty()) {
            if (work_dirty) {
                r = rebuild_work(S, &n_work, &T, &hcap, &rcap);
                work_dirty = false;
            }
            // joiners start at the current launch parity: both buffers hold
            // their start positions, so either parity reads them
            for (Request* q : in_step) {
                if (r || q->joined) continue;
                // the pinned entry of a slot is rewritten only when a later
                // request takes the slot, after this step has been synchronised
                S->h_join[q->slot] = q->state0;
                if (hipMemcpyAsync(S->states + q->slot, S->h_join + q->slot, sizeof(MeshState), hipMemcpyHostToDevice,
                                   S->st_compute) != hipSuccess)
                    r = fail(SL_EDEVICE, "state upload failed");
                q->parity0 = S->parity;
                q->joined = true;
            }
            const TileLaunch L{S->work, n_work, T, hcap, rcap, S->opts.layout, S->opts.accept, S->states, wg_per_cu, 0};
            for (int32_t k = 0; k < S->cfg.sweeps_per_step && !r; ++k) {
                if (jacobi && n_work > 0) r = launch_sweep_tiles(L, S->parity, nullptr, S->st_compute);
                for (Request* q : in_step) {
                    if (r) break;
                    if (jacobi && q->mesh.tile_nodes > 0) continue;
                    r = launch_sweep_nodes(q->mesh, S->parity, S->opts.form, S->opts.accept, block,
                                           S->states + q->slot, nullptr, S->st_compute);
                }
                if (!r) r = launch_advance(S->states, max_active, S->st_compute);
                S->parity ^= 1;
            }
            if (!r && hipMemcpyAsync(S->h_states, S->states, sizeof(MeshState) * max_active,
                                     hipMemcpyDeviceToHost, S->st_compute) != hipSuccess)
                r = fail(SL_EDEVICE, "state read-back failed");
        }
        const bool stepping = !in_step.empty();

        // ---- 2. admissions while the step runs (FIFO: the head waits until
        // it fits); with no step in flight, one admission starts the next
        for (;;) {
            Request* q = nullptr;
            {
                std::unique_lock<std::mutex> lk(S->mu);
                if (!stepping && S->queue.empty())
                    S->cv.wait_for(lk, std::chrono::milliseconds(50),
                                   [&] { return S->stop.load() || !S->queue.empty(); });
                q = pop_admissible(S);
            }
            if (!q) break;
            const sl_status ar = admit(S, q, q->slot);
            {
                std::lock_guard<std::mutex> lk(S->mu);
                if (ar) {
                    const std::string msg = sl_last_error();
                    release(S, q);
                    finish(S, q, ar, msg);
                    S->stats.failed++;
                } else {
                    q->phase = Request::ACTIVE;
                    q->times.started_s = seconds_since(S->t0, Clock::now());
                    work_dirty = true;
                }
            }
            if (!stepping || hipStreamQuery(S->st_compute) != hipErrorNotReady) break;
        }
        if (!stepping) continue;

        // ---- 3. retire the requests that finished in this step
        if (!r && hipStreamSynchronize(S->st_compute) != hipSuccess) r = fail(SL_EDEVICE, "sweep step failed");
        const double now = seconds_since(S->t0, Clock::now());
        std::lock_guard<std::mutex> lk(S->mu);
        S->stats.steps++;
        for (Request* q : in_step) {
            const MeshState& ms = hstate[q->slot];
            sl_status fs = SL_OK;
            std::string msg;
            bool done = false;
            if (r) {
                fs = r;
                msg = sl_last_error();
                done = true;
            } else if (!ms.active) {
                done = true;
            } else if (q->cancel) {
                fs = SL_ECANCELED;
                msg = "cancelled";
                done = true;
            } else if (q->deadline_s > 0.0 && now > q->deadline_s) {
                fs = SL_ETIMEOUT;
                msg = "deadline passed";
                done = true;
            }
            if (!done) continue;
            if (fs == SL_OK) {
                fs = collect(S, q, ms);
                if (fs) msg = sl_last_error();
            }
            if (fs == SL_OK) {
                S->stats.completed++;
                S->stats.node_updates += static_cast<int64_t>(q->mesh.n_free) * ms.s;
            } else {
                S->stats.failed++;
            }
            // a slot is reused only after its state is rewritten when the
            // next request joins
            release(S, q);
            finish(S, q, fs, msg);
            work_dirty = true;
        }
        if (r) {
            S->fatal = sl_last_error();
            break;
        }
    }
}

// Streams, the per-slot sweep states and their pinned host mirrors.
sl_status init_device(sl_server* S)
{
    sl_status r;
    SL_HIP(hipGetDevice(&S->device));
    SL_HIP(hipStreamCreateWithFlags(&S->st_compute, hipStreamNonBlocking));
    SL_HIP(hipStreamCreateWithFlags(&S->st_setup, hipStreamNonBlocking));
    if ((r = dalloc(&S->states, static_cast<size_t>(S->cfg.max_active), S->st_compute))) return r;
    SL_HIP(hipHostMalloc(reinterpret_cast<void**>(&S->h_states), sizeof(MeshState) * S->cfg.max_active,
                         hipHostMallocDefault));
    SL_HIP(hipHostMalloc(reinterpret_cast<void**>(&S->h_join), sizeof(MeshState) * S->cfg.max_active,
                         hipHostMallocDefault));
    std::vector<MeshState> zero(static_cast<size_t>(S->cfg.max_active));
    SL_HIP(hipMemcpyAsync(S->states, zero.data(), sizeof(MeshState) * zero.size(), hipMemcpyHostToDevice,
                          S->st_compute));
    SL_HIP(hipStreamSynchronize(S->st_compute));
    S->slots.assign(static_cast<size_t>(S->cfg.max_active), nullptr);
    S->t0 = Clock::now();
    return SL_OK;
}

}  // namespace

}  // namespace sl

extern "C" {

void sl_server_config_default(sl_server_config* c)
{
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->hbm_budget_bytes = static_cast<size_t>(200) << 30;
    c->max_active = 256;
    c->sweeps_per_step = 8;
}

sl_status sl_server_create(const sl_server_config* cfg, const sl_options* opts, sl_server** out)
{
    using namespace sl;
    set_error("");
    if (!out) return fail(SL_EINVAL, "null output pointer");
    *out = nullptr;
    auto S = std::make_unique<sl_server>();
    sl_server_config_default(&S->cfg);
    if (cfg) S->cfg = *cfg;
    if (S->cfg.hbm_budget_bytes == 0) S->cfg.hbm_budget_bytes = static_cast<size_t>(200) << 30;
    if (S->cfg.max_active <= 0) S->cfg.max_active = 256;
    if (S->cfg.sweeps_per_step <= 0) S->cfg.sweeps_per_step = 8;
    sl_options_default(&S->opts);
    if (opts) S->opts = *opts;
    S->opts.flags_out = nullptr;
    sl_status r = check_options(S->opts);
    if (r) return r;
    if (S->cfg.max_active > kMaxActive) return fail(SL_EINVAL, "max_active must be <= 65536");
    // automatic launch shapes are fixed when the server starts: every
    // request of one work list has the same tile size
    S->opts.tile_nodes = resolve_tile_nodes(S->opts);
    S->opts.tile_wg_per_cu = resolve_wg_per_cu(S->opts);
    S->opts.block_size = resolve_block_size(S->opts);
    keep_pool_warm();
    if ((r = init_device(S.get()))) {
        const std::string msg = sl_last_error();
        sl_server_destroy(S.release());
        return fail(r, msg);
    }
    sl_server* raw = S.get();
    S->thread = std::thread(scheduler, raw);
    *out = S.release();
    return SL_OK;
}

sl_status sl_server_submit(sl_server* S, const sl_mesh_desc* mesh, int32_t iterations, double tol,
                           double deadline_s, uint64_t* request_id)
{
    using namespace sl;
    set_error("");
    if (!S || !mesh || !request_id) return fail(SL_EINVAL, "null argument");
    if (iterations < 0) return fail(SL_EINVAL, "iterations must be >= 0");
    if (!mesh->coords || !mesh->nbr_ptr || !mesh->tri_ptr || !mesh->boundary || mesh->n_nodes <= 0)
        return fail(SL_EINVAL, "bad mesh arrays");
    auto q = std::make_unique<Request>();
    q->desc = *mesh;
    q->iterations = iterations;
    q->tol = tol;
    q->footprint = estimate_footprint(*mesh);
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->fatal.empty()) return fail(SL_EDEVICE, "server stopped: " + S->fatal);
    q->id = S->next_id++;
    q->times.submitted_s = seconds_since(S->t0, Clock::now());
    q->deadline_s = deadline_s > 0.0 ? q->times.submitted_s + deadline_s : 0.0;
    *request_id = q->id;
    S->queue.push_back(q->id);
    S->reqs[q->id] = std::move(q);
    S->stats.submitted++;
    S->cv.notify_one();
    return SL_OK;
}

sl_status sl_server_poll(sl_server* S, uint64_t id, double* coords_out, sl_report* report, sl_request_times* times)
{
    using namespace sl;
    if (!S) return fail(SL_EINVAL, "null server");
    std::unique_ptr<Request> q;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(id);
        if (it == S->reqs.end()) return fail(SL_EINVAL, "unknown request id");
        if (it->second->phase != Request::DONE) return SL_EBUSY;
        q = std::move(it->second);
        S->reqs.erase(it);
    }
    if (times) *times = q->times;
    if (q->status != SL_OK) return fail(q->status, q->error);
    if (coords_out) std::memcpy(coords_out, q->result.data(), q->result.size() * sizeof(double));
    if (report) *report = q->report;
    return SL_OK;
}

sl_status sl_server_cancel(sl_server* S, uint64_t id)
{
    using namespace sl;
    if (!S) return fail(SL_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return fail(SL_EINVAL, "unknown request id");
    it->second->cancel = true;
    return SL_OK;
}

sl_status sl_server_get_stats(sl_server* S, sl_server_stats* out)
{
    using namespace sl;
    if (!S || !out) return fail(SL_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    sl_server_stats s = S->stats;
    s.queued = static_cast<int32_t>(S->queue.size());
    s.active = 0;
    for (Request* q : S->slots) s.active += q != nullptr;
    s.hbm_in_use = S->hbm_in_use;
    *out = s;
    if (!S->fatal.empty()) return fail(SL_EDEVICE, "server stopped: " + S->fatal);
    return SL_OK;
}

void sl_server_destroy(sl_server* S)
{
    using namespace sl;
    if (!S) return;
    S->stop.store(true);
    S->cv.notify_all();
    if (S->thread.joinable()) S->thread.join();
    for (auto& kv : S->reqs)
        if (kv.second->slot >= 0) release(S, kv.second.get());
    dfree(S->work, S->st_compute);
    dfree(S->states, S->st_compute);
    dfree(S->out, S->st_compute);
    for (hipStream_t st : {S->st_compute, S->st_setup}) {
        if (!st) continue;
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    if (S->h_states) (void)hipHostFree(S->h_states);
    if (S->h_join) (void)hipHostFree(S->h_join);
    delete S;
}

}  // extern "C"
