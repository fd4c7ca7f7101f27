// Batched Smart Laplacian: many meshes of uneven size swept together.
//
// Every mesh is set up on the device as for a single call (validation,
// Hilbert order, tiles); setups run on a few host threads, each with a
// stream of its own, so the short kernels and host round trips of small
// meshes overlap.  The tile descriptors of all meshes form one work list,
// so one launch of the tile kernel sweeps every mesh once, and the whole
// sweep loop (tile launches plus the per-mesh state update) is captured once
// in a HIP graph and replayed.  Meshes that do not fit the tile path, and
// the coloured form, are swept mesh by mesh on the node path inside the same
// graph.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "sl_common.h"

namespace sl {

namespace {

constexpr int32_t kSetupThreads = 16;   // at most; no more than the host's hardware threads
constexpr size_t kOutGroupValues = size_t(1) << 27;   // un-permute staging: 1 GiB of doubles

struct BatchState {
    hipStream_t st = nullptr;
    std::vector<hipStream_t> setup_st;
    std::vector<DevMesh> meshes;
    unsigned char* block = nullptr;     // every mesh's arrays, when one allocation held them
    TileWork* work = nullptr;
    MeshState* states = nullptr;
    int32_t* sched = nullptr;           // the tile launches' counters
    ResidentArgs* res_list = nullptr;   // the resident meshes' kernel arguments
    double* out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    ~BatchState()
    {
        for (auto& m : meshes) devmesh_free(m, st);
        block_give(block, st);
        dfree(work, st);
        dfree(states, st);
        dfree(sched, st);
        dfree(res_list, st);
        dfree(out, st);
        (void)hipStreamSynchronize(st);
        for (auto s : setup_st)
            if (s) give_stream(s);
        if (st) give_stream(st);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

}  // namespace

sl_status upload_and_prepare(const sl_mesh_desc& d, const sl_options& o, int32_t mesh, DevMesh& m, hipStream_t st)
{
    if (!d.coords || !d.nbr_ptr || !d.tri_ptr || !d.boundary) return fail(SL_EINVAL, "null array argument");
    if (d.n_nodes <= 0) return fail(SL_EINVAL, "n_nodes must be >= 1");
    if (d.n_tris < 0) return fail(SL_EINVAL, "n_tris must be >= 0");
    if (d.n_tris > 0 && !d.tris) return fail(SL_EINVAL, "null tris with n_tris > 0");
    const size_t n = static_cast<size_t>(d.n_nodes);
    const int64_t nnz = d.nbr_ptr[n], ninc = d.tri_ptr[n];
    if (d.nbr_ptr[0] != 0 || d.tri_ptr[0] != 0 || nnz < 0 || ninc < 0) return fail(SL_EINVAL, "bad CSR offsets");
    if ((nnz > 0 && !d.nbr_idx) || (ninc > 0 && !d.tri_idx)) return fail(SL_EINVAL, "null CSR index array");
    DevInputs di;
    sl_status r = upload_inputs(d, nnz, ninc, 0, di, st);
    if (r) {
        di.release(st);
        return r;
    }
    MeshInput in{di.coords, d.n_nodes, di.nbr_ptr, di.nbr_idx, di.tri_ptr, di.tri_idx, di.tris, d.n_tris,
                 di.boundary};
    in.ends_known = true;
    in.ends[0] = d.nbr_ptr[0];
    in.ends[1] = static_cast<int32_t>(nnz);
    in.ends[2] = d.tri_ptr[0];
    in.ends[3] = static_cast<int32_t>(ninc);
    r = prepare_mesh(in, o, mesh, m, st);
    di.release(st);
    return r;
}

}  // namespace sl

extern "C" {

sl_status sl_batch_smooth(const sl_mesh_desc* meshes, int32_t n_meshes, int32_t iterations, double tol,
                          const sl_options* opts, sl_report* reports, sl_batch_report* batch)
{
    using namespace sl;
    const auto t0 = std::chrono::steady_clock::now();
    set_error("");
    if (!meshes || n_meshes <= 0) return fail(SL_EINVAL, "need at least one mesh");
    if (iterations < 0) return fail(SL_EINVAL, "iterations must be >= 0");
    sl_options o;
    sl_options_default(&o);
    if (opts) o = *opts;
    o.flags_out = nullptr;
    sl_status r = check_options(o);
    if (r) return r;
    // automatic launch shapes are fixed once for the whole batch: every
    // mesh of one work list has the same tile size
    const int32_t wg_auto = o.tile_wg_per_cu == 0 ? 1 : 0;
    if (o.form == SL_JACOBI) o.tile_nodes = resolve_tile_nodes(o);   // colour-class tiles size themselves
    o.tile_wg_per_cu = resolve_wg_per_cu(o);
    o.block_size = resolve_block_size(o);
    keep_pool_warm();

    BatchState bs;
    if ((r = take_stream(&bs.st))) return r;
    hipStream_t st = bs.st;
    for (auto& e : bs.ev) SL_HIP(hipEventCreate(&e));

    // ---- setup: meshes taken in index order by a few threads
    bs.meshes.resize(static_cast<size_t>(n_meshes));
    const int32_t hw = static_cast<int32_t>(std::max(1u, std::thread::hardware_concurrency()));
    const int32_t n_threads = std::min({n_meshes, kSetupThreads, std::max(hw, 4)});
    bs.setup_st.assign(static_cast<size_t>(n_threads), nullptr);
    for (auto& s : bs.setup_st)
        if ((r = take_stream(&s))) return r;
    int device = 0;
    SL_HIP(hipGetDevice(&device));
    // Every mesh's own arrays carved from one block, sized from the CSR ends:
    // one allocation and one release for the batch instead of one each per
    // mesh (a release beyond what the block cache keeps costs about 0.2 ms of
    // host time).  Without that block (a bad descriptor, whose setup then
    // reports it, or no room for it) each mesh allocates its own.
    if (n_meshes > 1) {
        std::vector<size_t> sz(static_cast<size_t>(n_meshes), 0);
        size_t total = 0;
        bool ok = true;
        for (int32_t i = 0; i < n_meshes && ok; ++i) {
            const sl_mesh_desc& d = meshes[i];
            ok = d.nbr_ptr && d.tri_ptr && d.n_nodes > 0 && d.nbr_ptr[d.n_nodes] >= 0 && d.tri_ptr[d.n_nodes] >= 0;
            if (ok) sz[i] = mesh_block_bytes(d.n_nodes, d.nbr_ptr[d.n_nodes], d.tri_ptr[d.n_nodes], o, true);
            total += sz[i];
        }
        if (ok && block_take(&bs.block, total, st) == SL_OK) {
            size_t at = 0;
            for (int32_t i = 0; i < n_meshes; ++i) {
                bs.meshes[i].carve = bs.block + at;
                bs.meshes[i].carve_bytes = sz[i];
                at += sz[i];
            }
            SL_HIP(hipStreamSynchronize(st));   // the block is the setup streams' from here
        }
        set_error("");
    }
    std::atomic<int32_t> next{0};
    std::atomic<bool> failed{false};
    std::vector<sl_status> t_status(static_cast<size_t>(n_threads), SL_OK);
    std::vector<std::string> t_msg(static_cast<size_t>(n_threads));
    auto worker = [&](int32_t t) {
        hipStream_t ts = bs.setup_st[t];
        if (hipSetDevice(device) != hipSuccess) {
            t_status[t] = SL_EDEVICE;
            t_msg[t] = "hipSetDevice failed in a setup thread";
            failed.store(true);
            return;
        }
        for (;;) {
            const int32_t i = next.fetch_add(1);
            if (i >= n_meshes || failed.load()) break;
            bs.meshes[i].class_tiles_ok = true;   // Form B: colour-class tiles, when asked for, where a mesh fits them
            const sl_status rr = upload_and_prepare(meshes[i], o, i, bs.meshes[i], ts);
            if (rr) {
                t_status[t] = rr;
                t_msg[t] = "mesh " + std::to_string(i) + ": " + sl_last_error();
                failed.store(true);
                break;
            }
        }
        if (hipStreamSynchronize(ts) != hipSuccess && !t_status[t]) {
            t_status[t] = SL_EDEVICE;
            t_msg[t] = "setup stream failed";
            failed.store(true);
        }
    };
    {
        std::vector<std::thread> pool;
        for (int32_t t = 1; t < n_threads; ++t) pool.emplace_back(worker, t);
        worker(0);
        for (auto& th : pool) th.join();
    }
    for (int32_t t = 0; t < n_threads; ++t)
        if (t_status[t]) return fail(t_status[t], t_msg[t]);

    int64_t total_tiles = 0;
    int32_t T = 0, halo_cap = 0, rows_cap = 0, on_tiles = 0;
    size_t max_nodes = 0, sum_nodes = 0;
    for (int32_t i = 0; i < n_meshes; ++i) {
        const DevMesh& m = bs.meshes[i];
        sum_nodes += static_cast<size_t>(m.n);
        max_nodes = std::max(max_nodes, static_cast<size_t>(m.n));
        if (m.tile_nodes > 0) ++on_tiles;
        // Form A's tiles go into one work list; a Form B mesh on colour-class
        // tiles keeps its own launches, one per class
        if (o.form == SL_JACOBI && m.tile_nodes > 0) {
            if (T != 0 && m.tile_nodes != T) return fail(SL_EINVAL, "meshes of one batch with different tile sizes");
            T = m.tile_nodes;
            total_tiles += m.n_tiles;
            halo_cap = std::max(halo_cap, m.halo_max);
            rows_cap = std::max(rows_cap, m.rows_max);
        }
    }
    if (total_tiles > INT32_MAX) return fail(SL_EINVAL, "batch has more than 2^31 tiles");

    // ---- one work list for all tile-path meshes
    if ((r = dalloc(&bs.work, static_cast<size_t>(std::max<int64_t>(total_tiles, 1)), st))) return r;
    int64_t off = 0;
    for (auto& m : bs.meshes) {
        if (o.form != SL_JACOBI || m.tile_nodes == 0) continue;
        SL_HIP(hipMemcpyAsync(bs.work + off, m.work, sizeof(TileWork) * m.n_tiles, hipMemcpyDeviceToDevice, st));
        off += m.n_tiles;
    }
    // resident meshes run all their sweeps in one launch of their own; their
    // states start inactive, so that the per-sweep closes pass them over
    std::vector<MeshState> h0(static_cast<size_t>(n_meshes));
    const double tol2 = tol > 0.0 ? tol * tol : 0.0;
    for (int32_t i = 0; i < n_meshes; ++i) {
        MeshState& s = h0[i];
        s = MeshState{};
        s.iters = iterations;
        s.active = iterations > 0 && !bs.meshes[i].resident;
        s.tol2 = tol2;
    }
    if ((r = dalloc(&bs.states, static_cast<size_t>(n_meshes), st))) return r;
    SL_HIP(hipMemcpyAsync(bs.states, h0.data(), sizeof(MeshState) * h0.size(), hipMemcpyHostToDevice, st));
    std::vector<ResidentArgs> res;
    size_t res_lds = 0;
    for (int32_t i = 0; i < n_meshes; ++i) {
        const DevMesh& m = bs.meshes[i];
        if (!m.resident) continue;
        const bool in_place = o.form == SL_INPLACE_COLORED;
        ResidentArgs ra{static_cast<double*>(m.X[0]), m.row_ptr, m.nbr, m.fan_ptr, m.fan, m.n, m.n_free,
                        static_cast<int32_t>(m.nnz_free), static_cast<int32_t>(m.ninc_free), iterations,
                        tol2, bs.states + i, nullptr, 0};
        if ((r = resident_classes(m, in_place, ra))) return fail(r, "mesh " + std::to_string(i) + ": " + sl_last_error());
        res.push_back(ra);
        res_lds = std::max(res_lds, resident_lds_bytes(m.n, m.n_free, m.nnz_free, m.ninc_free, in_place));
    }
    if (!res.empty()) {
        if ((r = dalloc(&bs.res_list, res.size(), st))) return r;
        SL_HIP(hipMemcpyAsync(bs.res_list, res.data(), sizeof(ResidentArgs) * res.size(), hipMemcpyHostToDevice, st));
    }
    // with every other mesh on the tile path, the tile launch closes each sweep itself
    const bool jacobi = o.form == SL_JACOBI;
    bool all_tiles = jacobi && total_tiles > 0;
    bool any_node = false;
    for (int32_t i = 0; i < n_meshes; ++i) {
        const DevMesh& m = bs.meshes[i];
        if (m.resident || (jacobi && m.tile_nodes > 0)) continue;
        all_tiles = false;
        any_node = true;
    }
    if ((r = dalloc(&bs.sched, kTileSchedInts, st))) return r;
    SL_HIP(hipMemsetAsync(bs.sched, 0, sizeof(int32_t) * kTileSchedInts, st));
    SL_HIP(hipStreamSynchronize(st));
    const double setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();

    // ---- the sweep loop, captured once and replayed
    const TileLaunch L{bs.work, static_cast<int32_t>(total_tiles), T, halo_cap, rows_cap, o.layout, o.accept,
                       bs.states, resolve_wg_per_cu(o), (n_meshes == 1 && tol2 > 0.0) ? 1 : 0, o.precision,
                       bs.sched, all_tiles ? n_meshes : 0};
    const int32_t block = resolve_block_size(o);
    const int32_t chunk = iterations <= 128 ? iterations + (iterations & 1) : 64;   // even: parity repeats
    auto enqueue_chunk = [&]() -> sl_status {
        for (int32_t s = 0; s < chunk; ++s) {
            sl_status rr = SL_OK;
            if (jacobi && total_tiles > 0) rr = launch_sweep_tiles(L, s & 1, nullptr, st);
            for (int32_t i = 0; i < n_meshes && !rr; ++i) {
                const DevMesh& m = bs.meshes[i];
                if (m.resident || (jacobi && m.tile_nodes > 0)) continue;
                if (!jacobi && m.tile_nodes > 0 && m.n_tile_classes > 0) {
                    // Form B on colour-class tiles: its tiles name its state;
                    // the sweep is closed below with the others
                    for (int32_t c = 0; c < m.n_tile_classes && !rr; ++c) {
                        TileLaunch Lc{m.work + m.class_tile_h[c], m.class_tile_h[c + 1] - m.class_tile_h[c],
                                      m.tile_nodes, m.halo_max, m.rows_max, o.layout, o.accept, bs.states,
                                      wg_auto ? 0 : o.tile_wg_per_cu, 0, o.precision, bs.sched, 0};
                        rr = launch_sweep_class(Lc, m.fans_max, nullptr, st);
                    }
                    continue;
                }
                rr = launch_sweep_nodes(m, s & 1, o.form, o.accept, block, bs.states + i, nullptr, bs.sched, st);
            }
            if (!rr && !all_tiles) rr = launch_advance(bs.states, n_meshes, st);
            if (rr) return rr;
        }
        return SL_OK;
    };
    int32_t graph_used = 0;
    const auto tg0 = std::chrono::steady_clock::now();
    double graph_ms = 0.0;
    if (iterations > 0 && !res.empty()) {
        SL_HIP(hipEventRecord(bs.ev[2], st));
        if ((r = launch_sweep_resident(bs.res_list, static_cast<int32_t>(res.size()), res_lds, o.layout, o.accept,
                                       st)))
            return r;
    }
    if (iterations > 0 && ((jacobi && total_tiles > 0) || any_node)) {
        SL_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        sl_status cr = enqueue_chunk();
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(st, &g);
        bs.graph = g;
        if (cr) return cr;
        if (ce != hipSuccess) return fail(SL_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(ce));
        SL_HIP(hipGraphInstantiate(&bs.exec, bs.graph, nullptr, nullptr, 0));
        graph_used = 1;
        graph_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tg0).count();
        if (res.empty()) SL_HIP(hipEventRecord(bs.ev[2], st));
        const int32_t replays = (iterations + chunk - 1) / chunk;
        for (int32_t k = 0; k < replays; ++k) SL_HIP(hipGraphLaunch(bs.exec, st));
    } else if (iterations <= 0 || res.empty()) {
        SL_HIP(hipEventRecord(bs.ev[2], st));
    }
    SL_HIP(hipEventRecord(bs.ev[3], st));

    // ---- results: un-permuted into a staging buffer a group of meshes at a
    // time, then copied to the callers' arrays
    std::vector<MeshState> hs(static_cast<size_t>(n_meshes));
    SL_HIP(hipMemcpyAsync(hs.data(), bs.states, sizeof(MeshState) * hs.size(), hipMemcpyDeviceToHost, st));
    const size_t group_values = std::max(2 * max_nodes, std::min(2 * sum_nodes, kOutGroupValues));
    if ((r = dalloc(&bs.out, group_values, st))) return r;
    SL_HIP(hipStreamSynchronize(st));
    float sweep_ms = 0.f;
    SL_HIP(hipEventElapsedTime(&sweep_ms, bs.ev[2], bs.ev[3]));
    const auto tr0 = std::chrono::steady_clock::now();
    int64_t updates = 0;
    for (int32_t first = 0; first < n_meshes;) {
        int32_t last = first;
        size_t used = 0;
        for (; last < n_meshes && used + 2 * static_cast<size_t>(bs.meshes[last].n) <= group_values; ++last) {
            const DevMesh& m = bs.meshes[last];
            const int src = jacobi ? (hs[last].s & 1) : 0;
            if ((r = unpermute_coords(m, src, bs.out + used, st))) return r;
            used += 2 * static_cast<size_t>(m.n);
        }
        SL_HIP(hipStreamSynchronize(st));   // the group's positions are in bs.out
        // copied out by the setup threads, each on its own stream with its own
        // staging buffers, so that the host copies run side by side
        std::vector<size_t> off(static_cast<size_t>(last - first) + 1, 0);
        for (int32_t i = first; i < last; ++i) off[i - first + 1] = off[i - first] + 2 * static_cast<size_t>(bs.meshes[i].n);
        std::atomic<int32_t> next_copy{first};
        std::vector<sl_status> c_status(static_cast<size_t>(n_threads), SL_OK);
        std::vector<std::string> c_msg(static_cast<size_t>(n_threads));
        auto copier = [&](int32_t t) {
            if (hipSetDevice(device) != hipSuccess) {
                c_status[t] = SL_EDEVICE;
                c_msg[t] = "hipSetDevice failed in a copy thread";
                return;
            }
            for (;;) {
                const int32_t i = next_copy.fetch_add(1);
                if (i >= last) break;
                const sl_status cr = copy_to_host(meshes[i].coords, bs.out + off[i - first],
                                                  sizeof(double) * (off[i - first + 1] - off[i - first]), bs.setup_st[t]);
                if (cr) {
                    c_status[t] = cr;
                    c_msg[t] = "mesh " + std::to_string(i) + ": " + sl_last_error();
                    break;
                }
            }
        };
        {
            std::vector<std::thread> pool;
            for (int32_t t = 1; t < n_threads; ++t) pool.emplace_back(copier, t);
            copier(0);
            for (auto& th : pool) th.join();
        }
        for (int32_t t = 0; t < n_threads; ++t)
            if (c_status[t]) return fail(c_status[t], c_msg[t]);
        first = last;
    }
    for (int32_t i = 0; i < n_meshes; ++i) {
        const DevMesh& m = bs.meshes[i];
        updates += static_cast<int64_t>(m.n_free) * hs[i].s;
        if (reports) {
            sl_report rep{};
            rep.iterations_run = hs[i].s;
            rep.n_colors = m.n_colors;
            std::memcpy(&rep.max_disp_sq_last, &hs[i].maxd_last, sizeof(double));
            rep.accepted_last = static_cast<int64_t>(hs[i].acc_last);
            rep.accepted_total = static_cast<int64_t>(hs[i].acc_total);
            rep.kernel_used = kernel_used(m);
            rep.tile_nodes = m.tile_nodes;
            reports[i] = rep;
        }
    }
    if (batch) {
        sl_batch_report b{};
        b.setup_ms = setup_ms;
        b.sweep_ms = sweep_ms;
        b.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        b.node_updates = updates;
        b.tiles = total_tiles;
        b.meshes_on_tile_path = on_tiles;
        b.meshes_resident = static_cast<int32_t>(res.size());
        b.graph_used = graph_used;
        b.graph_ms = graph_ms;
        b.results_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tr0).count();
        *batch = b;
    }
    return SL_OK;
}

}  // extern "C"
