// Serving: smoothing requests that arrive over time, swept together.
//
// The scheduling (queue, admission by slot and HBM budget, cancellation,
// deadlines, the step loop) is the device-independent core in sl_sched.h;
// this file is its device executor.  Admission uploads a request's mesh and
// builds its tiles on a stream of the setup thread that admits it, while
// the current step keeps sweeping on the compute stream; results are
// un-permuted and copied out on a third stream while the next step runs.
// A step runs a few sweeps over the tiles of all
// joined requests with one launch per sweep (continuous batching): a
// request joins at the first step after its setup, when its sweep state is
// written on the compute stream, so a step never sees a request that is half
// set up; it leaves after the step in which it reaches its cap or tolerance.
// A request's arithmetic is that of a single smooth_mesh call: tiles only
// read their own mesh, so the result does not depend on which requests
// share its launches.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "sl_common.h"
#include "sl_sched.h"

namespace sl {

namespace {

constexpr int32_t kMaxActive = 65536;

size_t estimate_footprint(const sl_mesh_desc& d)
{
    const size_t n = static_cast<size_t>(std::max(d.n_nodes, 0));
    const size_t nnz = d.nbr_ptr ? static_cast<size_t>(std::max(d.nbr_ptr[n], 0)) : 0;
    const size_t ninc = d.tri_ptr ? static_cast<size_t>(std::max(d.tri_ptr[n], 0)) : 0;
    // inputs during setup + resident: coordinates (4 buffers of 16 B), labels,
    // row and incidence offsets, ordering scratch; per neighbour entry the
    // input id, the u16 local row entry and the halo slot; per incidence the
    // input id and the 8-byte triangle word; the input triangles
    return n * (16 * 4 + 8 + 16 + 12) + nnz * (4 + 2 + 4) + ninc * (4 + 8) + 12 * static_cast<size_t>(d.n_tris) +
           (1u << 20);
}

struct HipPayload {
    DevMesh mesh;
    int32_t parity0 = 0;        // launch parity when it joined
    MeshState state0{};         // the sweep state it joins with
    MeshState last{};           // its state after the last step it ran
};

thread_local int t_bound_device = -1;   // the device a setup thread has made current

}  // namespace

// Device side of the server: one compute stream for the steps, one collect
// stream for results, pooled streams for admissions, per-slot sweep states
// with pinned host mirrors.
struct HipExec {
    using Payload = HipPayload;
    using Req = sched::Request<Payload>;

    sl_options opts{};
    int32_t max_active = 0, sweeps_per_step = 0;
    int device = 0;
    hipStream_t st_compute = nullptr, st_collect = nullptr;
    MeshState* states = nullptr;        // [max_active]
    int32_t* sched = nullptr;           // the tile launches' counters
    MeshState* h_states = nullptr;      // [max_active], pinned: read-back after each step
    MeshState* h_join = nullptr;        // [max_active], pinned: the state a joining request starts from
    TileWork* work = nullptr;
    int64_t work_cap = 0;
    double* out = nullptr;
    size_t out_cap = 0;
    int32_t parity = 0;
    int32_t n_work = 0, T = 0, hcap = 0, rcap = 0;
    int32_t wg_per_cu = 0, block = 0;
    int32_t wg_auto = 0;                // wg_per_cu came from the automatic choice

    sl_status init(const sl_server_config& cfg, const sl_options& o)
    {
        opts = o;
        max_active = cfg.max_active;
        sweeps_per_step = cfg.sweeps_per_step;
        wg_per_cu = resolve_wg_per_cu(opts);
        block = resolve_block_size(opts);
        sl_status r;
        SL_HIP(hipGetDevice(&device));
        SL_HIP(hipStreamCreateWithFlags(&st_compute, hipStreamNonBlocking));
        SL_HIP(hipStreamCreateWithFlags(&st_collect, hipStreamNonBlocking));
        if ((r = dalloc(&states, static_cast<size_t>(max_active), st_compute))) return r;
        if ((r = dalloc(&sched, kTileSchedInts, st_compute))) return r;
        SL_HIP(hipMemsetAsync(sched, 0, sizeof(int32_t) * kTileSchedInts, st_compute));
        SL_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_states), sizeof(MeshState) * max_active,
                             hipHostMallocDefault));
        SL_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_join), sizeof(MeshState) * max_active,
                             hipHostMallocDefault));
        std::vector<MeshState> zero(static_cast<size_t>(max_active));
        SL_HIP(hipMemcpyAsync(states, zero.data(), sizeof(MeshState) * zero.size(), hipMemcpyHostToDevice,
                              st_compute));
        SL_HIP(hipStreamSynchronize(st_compute));
        return SL_OK;
    }

    void destroy()
    {
        dfree(work, st_compute);
        dfree(states, st_compute);
        dfree(sched, st_compute);
        dfree(out, st_collect);
        for (hipStream_t st : {st_compute, st_collect}) {
            if (!st) continue;
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
        if (h_states) (void)hipHostFree(h_states);
        if (h_join) (void)hipHostFree(h_join);
        h_states = h_join = nullptr;
        st_compute = st_collect = nullptr;
    }

    size_t footprint(const sl_mesh_desc& d) { return estimate_footprint(d); }

    void bind_thread()
    {
        if (t_bound_device != device) {
            (void)hipSetDevice(device);
            t_bound_device = device;
        }
    }

    // Called by several setup threads at once: each admission runs on a
    // pooled stream of its own.
    sl_status admit(Req& q)
    {
        bind_thread();
        PooledStream ps;
        sl_status r = ps.init();
        if (r) return r;
        q.x.mesh.class_tiles_ok = true;   // Form B: colour-class tiles where the mesh fits them
        r = upload_and_prepare(q.desc, opts, q.slot, q.x.mesh, ps.s);
        if (r) {
            devmesh_free(q.x.mesh, ps.s);
            return r;
        }
        SL_HIP(hipStreamSynchronize(ps.s));
        MeshState& h = q.x.state0;
        h = MeshState{};
        h.iters = q.iterations;
        h.active = q.iterations > 0;
        h.tol2 = q.tol > 0.0 ? q.tol * q.tol : 0.0;
        return SL_OK;
    }

    // Concatenates the tile lists of the requests of the step.
    sl_status rebuild_work(const std::vector<Req*>& in_step)
    {
        // Form A's tiles only: a Form B request on colour-class tiles keeps
        // its own launches, one per class
        const bool jacobi = opts.form == SL_JACOBI;
        int64_t total = 0;
        T = hcap = rcap = 0;
        for (Req* q : in_step)
            if (jacobi && q->x.mesh.tile_nodes > 0) total += q->x.mesh.n_tiles;
        if (total > INT32_MAX) return fail(SL_ENOMEM, "too many tiles in flight");
        if (total > work_cap) {
            dfree(work, st_compute);
            work_cap = std::max<int64_t>(total, 2 * work_cap);
            sl_status r = dalloc(&work, static_cast<size_t>(work_cap), st_compute);
            if (r) {
                work_cap = 0;
                return r;
            }
        }
        int64_t off = 0;
        for (Req* q : in_step) {
            const DevMesh& m = q->x.mesh;
            if (!jacobi || m.tile_nodes == 0) continue;
            if (T != 0 && m.tile_nodes != T) return fail(SL_EINVAL, "requests with different tile sizes");
            SL_HIP(hipMemcpyAsync(work + off, m.work, sizeof(TileWork) * m.n_tiles, hipMemcpyDeviceToDevice,
                                  st_compute));
            off += m.n_tiles;
            T = m.tile_nodes;
            hcap = std::max(hcap, m.halo_max);
            rcap = std::max(rcap, m.rows_max);
        }
        n_work = static_cast<int32_t>(total);
        return SL_OK;
    }

    sl_status launch(const std::vector<Req*>& in_step, bool changed, int32_t sweeps)
    {
        bind_thread();
        sl_status r = SL_OK;
        if (changed && (r = rebuild_work(in_step))) return r;
        // joiners start at the current launch parity: both buffers hold
        // their start positions, so either parity reads them
        for (Req* q : in_step) {
            if (q->joined) continue;
            // the pinned entry of a slot is rewritten only when a later
            // request takes the slot, after this step has been waited for
            h_join[q->slot] = q->x.state0;
            SL_HIP(hipMemcpyAsync(states + q->slot, h_join + q->slot, sizeof(MeshState), hipMemcpyHostToDevice,
                                  st_compute));
            q->x.parity0 = parity;
            q->joined = true;
        }
        const bool jacobi = opts.form == SL_JACOBI;
        // with every request of the step on the tile path, the tile launch
        // closes each sweep itself
        bool all_tiles = jacobi && n_work > 0;
        for (Req* q : in_step) all_tiles = all_tiles && q->x.mesh.tile_nodes > 0;
        const TileLaunch L{work,       n_work, T, hcap, rcap, opts.layout, opts.accept, states, wg_per_cu, 0,
                           opts.precision, sched, all_tiles ? max_active : 0};
        for (int32_t k = 0; k < sweeps && !r; ++k) {
            if (jacobi && n_work > 0) r = launch_sweep_tiles(L, parity, nullptr, st_compute);
            for (Req* q : in_step) {
                if (r) break;
                const DevMesh& m = q->x.mesh;
                if (jacobi && m.tile_nodes > 0) continue;
                if (!jacobi && m.tile_nodes > 0 && m.n_tile_classes > 0) {
                    // Form B on colour-class tiles: its tiles name its slot's
                    // state; the sweep is closed below with the others
                    for (int32_t c = 0; c < m.n_tile_classes && !r; ++c) {
                        TileLaunch Lc{m.work + m.class_tile_h[c], m.class_tile_h[c + 1] - m.class_tile_h[c],
                                      m.tile_nodes, m.halo_max, m.rows_max, opts.layout, opts.accept, states,
                                      wg_auto ? 0 : wg_per_cu, 0, opts.precision, sched, 0};
                        r = launch_sweep_class(Lc, m.fans_max, nullptr, st_compute);
                    }
                    continue;
                }
                r = launch_sweep_nodes(m, parity, opts.form, opts.accept, block, states + q->slot, nullptr,
                                       sched, st_compute);
            }
            if (!r && !all_tiles) r = launch_advance(states, max_active, st_compute);
            parity ^= 1;
        }
        if (r) return r;
        SL_HIP(hipMemcpyAsync(h_states, states, sizeof(MeshState) * max_active, hipMemcpyDeviceToHost, st_compute));
        return SL_OK;
    }

    sl_status wait(const std::vector<Req*>& in_step, std::vector<sched::StepOutcome>& res)
    {
        if (hipStreamSynchronize(st_compute) != hipSuccess) return fail(SL_EDEVICE, "sweep step failed");
        for (size_t k = 0; k < in_step.size(); ++k) {
            const MeshState& ms = h_states[in_step[k]->slot];
            in_step[k]->x.last = ms;
            res[k].active = ms.active != 0;
            res[k].sweeps = ms.s;
            res[k].node_updates = static_cast<int64_t>(in_step[k]->x.mesh.n_free) * ms.s;
        }
        return SL_OK;
    }

    // Copies a finished request's positions back to host memory, on the
    // collect stream: the request is in no step any more, so this overlaps
    // the step that runs meanwhile.
    sl_status collect(Req& q, const sched::StepOutcome&)
    {
        const DevMesh& m = q.x.mesh;
        const MeshState& ms = q.x.last;
        const size_t n = static_cast<size_t>(m.n);
        if (out_cap < 2 * n) {
            dfree(out, st_collect);
            sl_status r = dalloc(&out, 2 * n, st_collect);
            if (r) {
                out_cap = 0;
                return r;
            }
            out_cap = 2 * n;
        }
        const bool jacobi = opts.form == SL_JACOBI;
        const int src = jacobi ? ((q.x.parity0 + ms.s) & 1) : 0;
        sl_status r = unpermute_coords(m, src, out, st_collect);
        if (r) return r;
        q.result.resize(2 * n);
        if ((r = copy_to_host(q.result.data(), out, 2 * n * sizeof(double), st_collect))) return r;
        sl_report rep{};
        rep.iterations_run = ms.s;
        rep.n_colors = m.n_colors;
        std::memcpy(&rep.max_disp_sq_last, &ms.maxd_last, sizeof(double));
        rep.accepted_last = static_cast<int64_t>(ms.acc_last);
        rep.accepted_total = static_cast<int64_t>(ms.acc_total);
        rep.kernel_used = kernel_used(m);
        rep.tile_nodes = m.tile_nodes;
        q.report = rep;
        return SL_OK;
    }

    // After its last step and its collection (stream-ordered on the collect
    // stream, which follows both).
    void release(Req& q) { devmesh_free(q.x.mesh, st_collect); }
};

}  // namespace sl

struct sl_server {
    sl::HipExec exec;
    std::unique_ptr<sl::sched::Scheduler<sl::HipExec>> core;
};

extern "C" {

void sl_server_config_default(sl_server_config* c)
{
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->hbm_budget_bytes = static_cast<size_t>(200) << 30;
    c->max_active = 256;
    c->sweeps_per_step = 8;
    c->setup_threads = 4;
}

sl_status sl_server_create(const sl_server_config* cfg, const sl_options* opts, sl_server** out)
{
    using namespace sl;
    set_error("");
    if (!out) return fail(SL_EINVAL, "null output pointer");
    *out = nullptr;
    sl_server_config c;
    sl_server_config_default(&c);
    if (cfg) c = *cfg;
    if (c.hbm_budget_bytes == 0) c.hbm_budget_bytes = static_cast<size_t>(200) << 30;
    if (c.max_active <= 0) c.max_active = 256;
    if (c.sweeps_per_step <= 0) c.sweeps_per_step = 8;
    if (c.setup_threads <= 0) c.setup_threads = 4;
    if (c.setup_threads > 64) return fail(SL_EINVAL, "setup_threads must be <= 64");
    if (c.max_active > kMaxActive) return fail(SL_EINVAL, "max_active must be <= 65536");
    sl_options o;
    sl_options_default(&o);
    if (opts) o = *opts;
    o.flags_out = nullptr;
    sl_status r = check_options(o);
    if (r) return r;
    // requests join a shared step of a few sweeps; the resident kernel runs
    // a mesh's sweeps all at once, which this schedule has no place for
    if (o.kernel == SL_KERNEL_RESIDENT) return fail(SL_EINVAL, "a server does not run the resident kernel");
    // automatic: Form A's tiles where a request fits them, else (and for
    // Form B) the node kernel
    if (o.kernel == SL_KERNEL_AUTO) o.kernel = o.form == SL_JACOBI ? SL_KERNEL_TILE : SL_KERNEL_NODE;
    // automatic launch shapes are fixed when the server starts: every
    // request of one work list has the same tile size (colour-class tiles
    // size themselves per request)
    const int32_t wg_auto = o.tile_wg_per_cu == 0 ? 1 : 0;
    if (o.form == SL_JACOBI) o.tile_nodes = resolve_tile_nodes(o);
    o.tile_wg_per_cu = resolve_wg_per_cu(o);
    o.block_size = resolve_block_size(o);
    keep_pool_warm();
    auto S = std::make_unique<sl_server>();
    S->exec.wg_auto = wg_auto;
    if ((r = S->exec.init(c, o))) {
        const std::string msg = sl_last_error();
        S->exec.destroy();
        return fail(r, msg);
    }
    S->core = std::make_unique<sched::Scheduler<HipExec>>(c, S->exec);
    S->core->start();
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
    return S->core->submit(*mesh, iterations, tol, deadline_s, request_id);
}

sl_status sl_server_poll(sl_server* S, uint64_t id, double* coords_out, sl_report* report, sl_request_times* times)
{
    using namespace sl;
    if (!S) return fail(SL_EINVAL, "null server");
    return S->core->poll(id, coords_out, report, times);
}

sl_status sl_server_cancel(sl_server* S, uint64_t id)
{
    using namespace sl;
    if (!S) return fail(SL_EINVAL, "null server");
    return S->core->cancel(id);
}

sl_status sl_server_get_stats(sl_server* S, sl_server_stats* out)
{
    using namespace sl;
    if (!S || !out) return fail(SL_EINVAL, "null argument");
    return S->core->stats(out);
}

void sl_server_destroy(sl_server* S)
{
    if (!S) return;
    if (S->core) S->core->stop();
    S->core.reset();
    S->exec.destroy();
    delete S;
}

}  // extern "C"
