// C-ABI entry points of libsmartlap: argument checks, device buffers, the
// sweep loop with its convergence test, and the copy back to the caller.
#include <chrono>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sl_common.h"

namespace sl {

namespace {
thread_local std::string g_last_error;
std::once_flag g_pool_once[64];
std::mutex g_tune_mu;
TunedShape g_tuned[64];

int current_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
    return dev;
}
}  // namespace

TunedShape tuned_shape()
{
    const int dev = current_device();
    if (dev < 0) return TunedShape{0, 0, 0, 0};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tuned[dev];
}

void set_tuned_shape(const TunedShape& t)
{
    const int dev = current_device();
    if (dev < 0) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[dev] = t;
}

void clear_tuned_shape() { set_tuned_shape(TunedShape{0, 0, 0, 0}); }

int32_t resolve_tile_nodes(const sl_options& o)
{
    if (o.tile_nodes) return o.tile_nodes;
    const TunedShape t = tuned_shape();
    return t.tile_nodes ? t.tile_nodes : 512;
}

int32_t resolve_wg_per_cu(const sl_options& o)
{
    if (o.tile_wg_per_cu) return o.tile_wg_per_cu;
    return tuned_shape().wg_per_cu;
}

int32_t resolve_block_size(const sl_options& o)
{
    if (o.block_size) return o.block_size;
    return tuned_shape().block_size;
}

int32_t resolve_lane_width(const sl_options& o)
{
    if (o.lane_width) return o.lane_width;
    const TunedShape t = tuned_shape();
    return t.lane_width ? t.lane_width : 8;
}

// Freed device memory stays in the stream-ordered pool for the next call.
void keep_pool_warm()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    std::call_once(g_pool_once[dev], [dev] {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = ~0ull;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
    });
}

sl_status check_options(const sl_options& o)
{
    if (o.form != SL_JACOBI && o.form != SL_INPLACE_COLORED) return fail(SL_EINVAL, "unknown form");
    if (o.accept != SL_ACCEPT_GE && o.accept != SL_ACCEPT_GT) return fail(SL_EINVAL, "unknown accept rule");
    if (o.layout != SL_AOS && o.layout != SL_SOA) return fail(SL_EINVAL, "unknown layout");
    if (o.reorder != SL_REORDER_NONE && o.reorder != SL_REORDER_HILBERT) return fail(SL_EINVAL, "unknown reorder");
    if (o.block_size != 0 && o.block_size != 64 && o.block_size != 128 && o.block_size != 256)
        return fail(SL_EINVAL, "block_size must be 0, 64, 128 or 256");
    if (o.kernel != SL_KERNEL_AUTO && o.kernel != SL_KERNEL_NODE && o.kernel != SL_KERNEL_TILE &&
        o.kernel != SL_KERNEL_RESIDENT && o.kernel != SL_KERNEL_LANES)
        return fail(SL_EINVAL, "unknown kernel");
    if (o.lane_width != 0 && o.lane_width != 4 && o.lane_width != 8 && o.lane_width != 16)
        return fail(SL_EINVAL, "lane_width must be 0, 4, 8 or 16");
    if (o.kernel == SL_KERNEL_RESIDENT && o.precision != SL_F64)
        return fail(SL_EINVAL, "the resident kernel runs in double precision only");
    if (o.tile_nodes != 0 && o.tile_nodes != 256 && o.tile_nodes != 512 &&
        !(o.tile_nodes == 128 && o.form == SL_INPLACE_COLORED))
        return fail(SL_EINVAL, "tile_nodes must be 0, 256 or 512 (or 128 for the coloured form)");
    if (o.tile_wg_per_cu < 0 || o.tile_wg_per_cu > 8) return fail(SL_EINVAL, "tile_wg_per_cu must be in 0..8");
    if (o.precision != SL_F64 && o.precision != SL_F32) return fail(SL_EINVAL, "unknown precision");
    if (o.precision == SL_F32 && (o.form != SL_JACOBI || o.kernel == SL_KERNEL_NODE || o.kernel == SL_KERNEL_LANES))
        return fail(SL_EINVAL, "single precision runs Form A on the tile kernel only");
    return SL_OK;
}

sl_status prepare_mesh(const MeshInput& in, const sl_options& o, int32_t mesh_index, DevMesh& m, hipStream_t st)
{
    if (!in.coords || !in.nbr_ptr || !in.tri_ptr || !in.boundary) return fail(SL_EINVAL, "null array argument");
    // coordinates are read and written as (x, y) pairs of 16 bytes
    if (reinterpret_cast<uintptr_t>(in.coords) % 16 != 0) return fail(SL_EINVAL, "coords must be 16-byte aligned");
    if (in.n <= 0) return fail(SL_EINVAL, "n_nodes must be >= 1");
    if (in.n_tris < 0) return fail(SL_EINVAL, "n_tris must be >= 0");
    if (in.n_tris > 0 && !in.tris) return fail(SL_EINVAL, "null tris with n_tris > 0");
    if (in.n_tris > (INT32_MAX / 3)) return fail(SL_EINVAL, "n_tris too large");
    int32_t ends[4] = {in.ends[0], in.ends[1], in.ends[2], in.ends[3]};
    if (!in.ends_known) {
        SL_HIP(hipMemcpyAsync(&ends[0], in.nbr_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        SL_HIP(hipMemcpyAsync(&ends[1], in.nbr_ptr + in.n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        SL_HIP(hipMemcpyAsync(&ends[2], in.tri_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        SL_HIP(hipMemcpyAsync(&ends[3], in.tri_ptr + in.n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        SL_HIP(hipStreamSynchronize(st));
    }
    if (ends[0] != 0 || ends[2] != 0) return fail(SL_EINVAL, "nbr_ptr[0] and tri_ptr[0] must be 0");
    if (ends[1] < 0 || ends[3] < 0) return fail(SL_EINVAL, "negative CSR length");
    if (ends[1] > 0 && !in.nbr_idx) return fail(SL_EINVAL, "null nbr_idx with nbr_ptr[n] > 0");
    if (ends[3] > 0 && !in.tri_idx) return fail(SL_EINVAL, "null tri_idx with tri_ptr[n] > 0");
    if (m.region) {
        // everything from the caller's region: the mesh's arrays, then the
        // setup's temporaries, which the caller's region_after bytes reuse
        // once setup is done
        const size_t pb = Arena::piece(mesh_block_bytes(in.n, ends[1], ends[3], o, m.class_tiles_ok));
        const size_t sb = setup_scratch_bytes(in.n);
        const size_t need = pb + std::max(sb, m.region_after);
        if (need > m.region_bytes)
            return fail(SL_ENOMEM, "the mesh needs " + std::to_string(need) + " bytes of device workspace; the "
                                   "static workspace holds " + std::to_string(m.region_bytes));
        m.carve = m.region;
        m.carve_bytes = pb;
        m.scratch_carve = m.region + pb;
        m.scratch_carve_bytes = m.region_bytes - pb;
    }
    SetupArgs sa{in.coords, in.n, in.nbr_ptr, in.nbr_idx, in.tri_ptr, in.tri_idx, in.tris, in.n_tris, in.boundary,
                 ends[1], ends[3]};
    return setup_mesh(sa, o, m, mesh_index, st);
}

namespace {

constexpr int32_t kSweepChunk = 32;   // even

// A device's static workspace, for the entry point that allocates nothing:
// its device address and the call's timing events, both set up once per
// device.
struct StaticWorkspace {
    unsigned char* base = nullptr;
    size_t bytes = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

// Everything a call allocates, released on every exit path.
struct CallState {
    hipStream_t st = nullptr;
    DevMesh m;
    Arena aux;                          // the sweep state, the tile launches' counters, the flag words
    MeshState* state = nullptr;
    int32_t* sched = nullptr;
    uint64_t* bits = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool own_events = true;             // false: a static workspace's events
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture = nullptr;      // where the sweep chunk is captured
    ~CallState()
    {
        if (capture) give_stream(capture);
        devmesh_free(m, st);
        aux.release(st);
        (void)hipStreamSynchronize(st);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (own_events)
            for (auto& e : ev)
                if (e) (void)hipEventDestroy(e);
    }
};

// Bytes of a call's sweep state, tile counters, resident-kernel arguments
// and (with flag output) accept bits, for a mesh of at most n free nodes.
size_t aux_bytes(int64_t n, int32_t iterations, bool want_bits)
{
    const size_t words = static_cast<size_t>((n + 63) / 64);
    return Arena::piece(sizeof(MeshState)) + Arena::piece(sizeof(int32_t) * kTileSchedInts) +
           Arena::piece(sizeof(ResidentArgs)) +
           (want_bits ? Arena::piece(8 * words * static_cast<size_t>(iterations)) : 0);
}

sl_status run_device(double* coords, int32_t n, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                     const int32_t* tri_ptr, const int32_t* tri_idx, const int32_t* tris, int32_t n_tris,
                     const uint8_t* boundary, int32_t iterations, double tol, const sl_options* opts,
                     sl_report* report, hipStream_t stream, const int32_t* known_ends = nullptr,
                     const StaticWorkspace* ws = nullptr)
{
    const auto t0 = std::chrono::steady_clock::now();
    sl_options o;
    sl_options_default(&o);
    if (opts) o = *opts;
    sl_status r = check_options(o);
    if (r) return r;
    if (iterations < 0) return fail(SL_EINVAL, "iterations must be >= 0");
    const bool want_bits = o.flags_out && iterations > 0;
    if (!ws) keep_pool_warm();

    CallState cs;
    cs.st = stream;
    cs.m.class_tiles_ok = true;   // Form B may sweep colour-class tiles
    if (ws) {
        // every device array from the static workspace: the mesh's arrays,
        // the setup's temporaries, then (over those) the sweep state
        for (int k = 0; k < 4; ++k) cs.ev[k] = ws->ev[k];
        cs.own_events = false;
        cs.m.region = ws->base;
        cs.m.region_bytes = ws->bytes;
        cs.m.region_after = aux_bytes(n, iterations, want_bits);
    } else {
        for (auto& e : cs.ev) SL_HIP(hipEventCreate(&e));
    }
    SL_HIP(hipEventRecord(cs.ev[0], stream));
    MeshInput in{coords, n, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, n_tris, boundary};
    if (known_ends) {
        in.ends_known = true;
        for (int k = 0; k < 4; ++k) in.ends[k] = known_ends[k];
    }
    if ((r = prepare_mesh(in, o, 0, cs.m, stream))) return r;
    SL_HIP(hipEventRecord(cs.ev[1], stream));

    const int32_t its = iterations;
    const int64_t words = (static_cast<int64_t>(cs.m.n_free) + 63) / 64;
    const double tol2 = tol > 0.0 ? tol * tol : 0.0;
    MeshState h0{};
    h0.iters = its;
    h0.active = its > 0;
    h0.tol2 = tol2;
    const size_t n_bits = want_bits ? static_cast<size_t>(words) * its : 0;
    if (ws) {
        cs.aux.adopt(ws->base + cs.m.carve_bytes, ws->bytes - cs.m.carve_bytes);
    } else if ((r = cs.aux.reserve(aux_bytes(cs.m.n_free, its, want_bits), stream))) {
        return r;
    }
    if ((r = cs.aux.take(&cs.state, 1)) || (r = cs.aux.take(&cs.sched, kTileSchedInts))) return r;
    SL_HIP(hipMemcpyAsync(cs.state, &h0, sizeof(MeshState), hipMemcpyHostToDevice, stream));
    SL_HIP(hipMemsetAsync(cs.sched, 0, sizeof(int32_t) * kTileSchedInts, stream));
    if (want_bits) {
        if ((r = cs.aux.take(&cs.bits, n_bits))) return r;
        SL_HIP(hipMemsetAsync(cs.bits, 0, sizeof(uint64_t) * n_bits, stream));
    }
    const bool tiles = cs.m.tile_nodes > 0;
    const int32_t block = resolve_block_size(o);
    // with a tolerance, a launch on a converged mesh returns at once; a tile
    // launch closes its own sweep
    const TileLaunch L{cs.m.work, cs.m.n_tiles, cs.m.tile_nodes, cs.m.halo_max, cs.m.rows_max, o.layout, o.accept,
                       cs.state, resolve_wg_per_cu(o), tol2 > 0.0 ? 1 : 0, o.precision, cs.sched, 1, 1};
    auto enqueue = [&](int32_t s, hipStream_t on) -> sl_status {
        uint64_t* bits = cs.bits ? cs.bits + static_cast<int64_t>(s) * words : nullptr;
        if (tiles && cs.m.n_tile_classes > 0) {
            // Form B: one launch per colour class, in place in buffer 0; the
            // last class's launch closes the sweep
            for (int32_t c = 0; c < cs.m.n_tile_classes; ++c) {
                TileLaunch Lc = L;
                Lc.work = cs.m.work + cs.m.class_tile_h[c];
                Lc.n_work = cs.m.class_tile_h[c + 1] - cs.m.class_tile_h[c];
                Lc.n_close = c + 1 == cs.m.n_tile_classes ? 1 : 0;
                Lc.wg_per_cu = o.tile_wg_per_cu;   // a count tuned for Form A's tiles does not apply
                const sl_status rr = launch_sweep_class(Lc, cs.m.fans_max, bits, on);
                if (rr) return rr;
            }
            return SL_OK;
        }
        if (tiles) return launch_sweep_tiles(L, s & 1, bits, on);
        // the sweep's last launch closes it
        return launch_sweep_nodes(cs.m, s & 1, o.form, o.accept, block, cs.state, bits, cs.sched, on, true);
    };

    // The sweep loop runs in chunks of kSweepChunk sweeps; a whole chunk is
    // one replay of a captured HIP graph (the chunk is even, so the buffer
    // parity of sweep s is s & 1 in every replay).  With a tolerance the host
    // reads the sweep state after each chunk and stops launching once the
    // mesh has converged.  Flag output takes per-sweep pointers, so it runs
    // without the graph.  The chunk is captured on a stream of the library's
    // own (the caller's may be the legacy default stream, which cannot be
    // captured) and replayed on the caller's stream.
    SL_HIP(hipEventRecord(cs.ev[2], stream));
    if (cs.m.resident) {
        // every sweep in one launch
        const bool in_place = o.form == SL_INPLACE_COLORED;
        ResidentArgs ra{static_cast<double*>(cs.m.X[0]), cs.m.row_ptr, cs.m.nbr, cs.m.fan_ptr, cs.m.fan,
                        cs.m.n, cs.m.n_free, static_cast<int32_t>(cs.m.nnz_free),
                        static_cast<int32_t>(cs.m.ninc_free), its, tol2, cs.state, cs.bits, words};
        if ((r = resident_classes(cs.m, in_place, ra))) return r;
        ResidentArgs* d_ra = nullptr;
        if ((r = cs.aux.take(&d_ra, 1))) return r;
        SL_HIP(hipMemcpyAsync(d_ra, &ra, sizeof(ra), hipMemcpyHostToDevice, stream));
        const size_t lds = resident_lds_bytes(cs.m.n, cs.m.n_free, cs.m.nnz_free, cs.m.ninc_free, in_place);
        if ((r = launch_sweep_resident(d_ra, 1, lds, o.layout, o.accept, stream))) return r;
    }
    const bool use_graph = !ws && !cs.m.resident && !cs.bits && its >= 2 * kSweepChunk;
    if (use_graph) {
        if ((r = take_stream(&cs.capture))) return r;
        SL_HIP(hipStreamBeginCapture(cs.capture, hipStreamCaptureModeThreadLocal));
        sl_status cr = SL_OK;
        for (int32_t s = 0; s < kSweepChunk && !cr; ++s) cr = enqueue(s, cs.capture);
        const hipError_t ce = hipStreamEndCapture(cs.capture, &cs.graph);
        if (cr) return cr;
        if (ce != hipSuccess) return fail(SL_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(ce));
        SL_HIP(hipGraphInstantiate(&cs.exec, cs.graph, nullptr, nullptr, 0));
    }
    for (int32_t done = cs.m.resident ? its : 0; done < its;) {
        const int32_t c = std::min(kSweepChunk, its - done);
        if (use_graph && c == kSweepChunk) {
            SL_HIP(hipGraphLaunch(cs.exec, stream));
        } else {
            for (int32_t s = done; s < done + c; ++s)
                if ((r = enqueue(s, stream))) return r;
        }
        done += c;
        if (tol2 > 0.0 && done < its) {
            MeshState cur{};
            SL_HIP(hipMemcpyAsync(&cur, cs.state, sizeof(MeshState), hipMemcpyDeviceToHost, stream));
            SL_HIP(hipStreamSynchronize(stream));
            if (!cur.active) break;
        }
    }
    SL_HIP(hipEventRecord(cs.ev[3], stream));

    // the result buffer and the sweeps run are read on the device: one wait
    if ((r = unpermute_coords(cs.m, 0, coords, stream, o.form == SL_JACOBI ? cs.state : nullptr))) return r;
    if (o.flags_out && its > 0)
        if ((r = unpermute_flags(cs.m, cs.bits, its, cs.state, o.flags_out, stream))) return r;
    MeshState hs{};
    SL_HIP(hipMemcpyAsync(&hs, cs.state, sizeof(MeshState), hipMemcpyDeviceToHost, stream));
    SL_HIP(hipStreamSynchronize(stream));
    const int32_t runs = hs.s;

    if (report) {
        sl_report rep{};
        rep.iterations_run = runs;
        rep.n_colors = cs.m.n_colors;
        std::memcpy(&rep.max_disp_sq_last, &hs.maxd_last, sizeof(double));
        rep.accepted_last = static_cast<int64_t>(hs.acc_last);
        rep.accepted_total = static_cast<int64_t>(hs.acc_total);
        float ms = 0.f;
        SL_HIP(hipEventElapsedTime(&ms, cs.ev[0], cs.ev[1]));
        rep.setup_ms = ms;
        SL_HIP(hipEventElapsedTime(&ms, cs.ev[2], cs.ev[3]));
        rep.sweep_ms = ms;
        rep.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        rep.kernel_used = kernel_used(cs.m);
        rep.tile_nodes = cs.m.tile_nodes;
        *report = rep;
    }
    return SL_OK;
}

// Device memory of smooth_mesh_device_noalloc: one file-scope array per
// device, holding a mesh's arrays, the setup's temporaries and the sweep
// state of one call.  It lives as long as the process.  In host code the
// array's name is no device address; the address comes from
// hipGetSymbolAddress, once per device.
constexpr size_t kStaticWorkspaceBytes = size_t(256) << 20;
__device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

struct StaticSlot {
    std::once_flag once;
    sl_status status = SL_OK;
    std::string error;
    StaticWorkspace ws;
    std::mutex mu;   // calls on one device share its workspace: one at a time
};
StaticSlot g_static[64];

// Sets up the current device's workspace: its address and the four timing
// events of a call.
void init_static(StaticSlot& s)
{
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        s.status = SL_EDEVICE;
        s.error = std::string("hipGetSymbolAddress of the static workspace failed: ") + hipGetErrorString(e);
        return;
    }
    for (auto& ev : s.ws.ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            s.status = SL_EDEVICE;
            s.error = std::string("hipEventCreate failed: ") + hipGetErrorString(e);
            return;
        }
    }
    s.ws.base = static_cast<unsigned char*>(p);
    s.ws.bytes = kStaticWorkspaceBytes;
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

sl_status fail(sl_status st, const std::string& msg)
{
    set_error(msg);
    return st;
}

}  // namespace sl

extern "C" {

void sl_options_default(sl_options* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->form = SL_JACOBI;
    o->accept = SL_ACCEPT_GE;
    o->layout = SL_AOS;
    o->reorder = SL_REORDER_HILBERT;
    o->block_size = 0;
    o->kernel = SL_KERNEL_AUTO;
    o->flags_out = nullptr;
}

const char* sl_last_error(void) { return sl::g_last_error.c_str(); }

const char* sl_version(void) { return "smartlap 0.1 (gfx950)"; }

sl_status smooth_mesh_device(double* coords, int32_t n_nodes, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                             const int32_t* tri_ptr, const int32_t* tri_idx, const int32_t* tris, int32_t n_tris,
                             const uint8_t* boundary, int32_t iterations, double tol, const sl_options* opts,
                             sl_report* report, void* stream)
{
    sl::set_error("");
    return sl::run_device(coords, n_nodes, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, n_tris, boundary, iterations,
                          tol, opts, report, static_cast<hipStream_t>(stream));
}

SL_API sl_status smooth_mesh_device_noalloc(double* coords, int32_t n_nodes, const int32_t* nbr_ptr,
                                     const int32_t* nbr_idx, const int32_t* tri_ptr, const int32_t* tri_idx,
                                     const int32_t* tris, int32_t n_tris, const uint8_t* boundary, int32_t iterations,
                                     double tol, const sl_options* opts, sl_report* report, void* stream)
{
    using namespace sl;
    set_error("");
    const int dev = current_device();
    if (dev < 0) return fail(SL_EDEVICE, "no current HIP device (or its ordinal is 64 or more)");
    StaticSlot& s = g_static[dev];
    std::call_once(s.once, [&s] { init_static(s); });
    if (s.status) return fail(s.status, s.error);
    // the call returns only when its work on `stream` is done, so holding
    // the lock for the call keeps calls on this device from overlapping
    std::lock_guard<std::mutex> lk(s.mu);
    return run_device(coords, n_nodes, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, n_tris, boundary, iterations, tol,
                      opts, report, static_cast<hipStream_t>(stream), nullptr, &s.ws);
}

sl_status smooth_mesh(double* coords, int32_t n_nodes, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                      const int32_t* tri_ptr, const int32_t* tri_idx, const int32_t* tris, int32_t n_tris,
                      const uint8_t* boundary, int32_t iterations, double tol, const sl_options* opts,
                      sl_report* report)
{
    using namespace sl;
    set_error("");
    if (!coords || !nbr_ptr || !tri_ptr || !boundary) return fail(SL_EINVAL, "null array argument");
    if (n_nodes <= 0) return fail(SL_EINVAL, "n_nodes must be >= 1");
    if (n_tris < 0) return fail(SL_EINVAL, "n_tris must be >= 0");
    if (iterations < 0) return fail(SL_EINVAL, "iterations must be >= 0");
    if (n_tris > 0 && !tris) return fail(SL_EINVAL, "null tris with n_tris > 0");
    const int64_t nnz = nbr_ptr[n_nodes], ninc = tri_ptr[n_nodes];
    if (nbr_ptr[0] != 0 || tri_ptr[0] != 0 || nnz < 0 || ninc < 0) return fail(SL_EINVAL, "bad CSR offsets");
    if ((nnz > 0 && !nbr_idx) || (ninc > 0 && !tri_idx)) return fail(SL_EINVAL, "null CSR index array");
    sl_options o;
    sl_options_default(&o);
    if (opts) o = *opts;
    sl_status r = check_options(o);
    if (r) return r;
    const auto t_call = std::chrono::steady_clock::now();
    PooledStream ps;
    if ((r = ps.init())) return r;
    hipStream_t st = ps.s;
    const size_t n = static_cast<size_t>(n_nodes);
    uint8_t* host_flags = o.flags_out;
    const size_t flag_bytes = (n + 7) / 8 * static_cast<size_t>(iterations);
    DevInputs di;
    do {
        const sl_mesh_desc d{coords, n_nodes, n_tris, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, boundary};
        const bool want_flags = host_flags && flag_bytes;
        if ((r = upload_inputs(d, nnz, ninc, want_flags ? Arena::piece(flag_bytes) : 0, di, st))) break;
        uint8_t* d_flags = nullptr;
        if (want_flags && (r = di.ar.take(&d_flags, flag_bytes))) break;
        o.flags_out = d_flags;
        const int32_t ends[4] = {0, static_cast<int32_t>(nnz), 0, static_cast<int32_t>(ninc)};
        r = run_device(di.coords, n_nodes, di.nbr_ptr, di.nbr_idx, di.tri_ptr, di.tri_idx, di.tris, n_tris,
                       di.boundary, iterations, tol, &o, report, st, ends);
        if (r) break;
        // the flags first, the positions last and straight into the
        // caller's array (a staging copy of a 4M-node result cost about
        // 10 ms of zero fill and copying): coords is written once every
        // sweep has succeeded, and only a device failure during that last
        // copy leaves it partly written
        if (d_flags && (r = copy_to_host(host_flags, d_flags, flag_bytes, st))) break;
        if ((r = copy_to_host(coords, di.coords, 2 * n * sizeof(double), st))) break;
    } while (false);
    std::string keep = g_last_error;
    di.release(st);
    (void)hipStreamSynchronize(st);
    set_error(keep);
    if (!r && report)
        report->total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_call).count();
    return r;
}

}  // extern "C"
