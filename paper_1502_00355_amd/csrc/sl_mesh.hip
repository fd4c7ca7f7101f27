// Mesh handles: a mesh validated, ordered and tiled once, then kept on the
// device and smoothed any number of times.  This is the mesh object of the
// paper's implementation (Sec. 3.2: vertices with their neighbours and
// incident triangles, triangles with their quality), kept resident so that
// repeated or batched smoothing pays neither the upload nor the setup again.
//
// The host always knows which of the two coordinate buffers holds a handle's
// current positions: a call with no tolerance runs exactly its sweeps, and a
// call with a tolerance reads the sweep state back between chunks of sweeps,
// as smooth_mesh does.  A handle never takes the resident kernel, which
// expects a mesh at its first sweep.  Form B handles sweep colour-class
// tiles where the mesh fits them, else the node kernel.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "sl_common.h"

namespace sl {

namespace {

constexpr int32_t kHandleChunk = 32;   // even: a chunk leaves the buffer parity where it found it

struct EventRef {
    hipEvent_t ev = nullptr;
    ~EventRef()
    {
        if (ev) (void)hipEventDestroy(ev);
    }
};

sl_status new_event(std::shared_ptr<EventRef>* out)
{
    auto e = std::make_shared<EventRef>();
    SL_HIP(hipEventCreateWithFlags(&e->ev, hipEventDisableTiming));
    *out = std::move(e);
    return SL_OK;
}

// Sets up the next call on every state: the cap counts from the sweeps
// already done, the running folds start from zero.
__global__ void k_begin_run(MeshState* __restrict__ s, int32_t n, int32_t iters, double tol2)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    MeshState m = s[i];
    m.iters = m.s + iters;
    m.active = iters > 0;
    m.tol2 = tol2;
    m.maxd_cur = 0;
    m.acc_cur = 0;
    s[i] = m;
}

// One handle of a batch call: where its state and tiles live, where its
// tiles go in the merged list, and the buffer copy that brings its current
// positions to buffer 0 (units == 0: none needed).
struct MergeSrc {
    MeshState* state;
    const TileWork* work;
    int64_t off;          // first merged tile
    int32_t n_tiles;
    int32_t pad;
    const void* from;     // X[1]
    void* to;             // X[0]
    int64_t units;        // units to copy: 16 bytes each when wide, else 4
    int32_t wide;
    int32_t pad2;
};

__global__ void k_gather_states(const MergeSrc* __restrict__ src, int32_t n, MeshState* __restrict__ states,
                                int32_t iters, double tol2)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    MeshState m = *src[i].state;
    m.iters = m.s + iters;
    m.active = iters > 0;
    m.tol2 = tol2;
    m.maxd_cur = 0;
    m.acc_cur = 0;
    states[i] = m;
}

__global__ void k_scatter_states(const MergeSrc* __restrict__ src, int32_t n, const MeshState* __restrict__ states)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    *src[i].state = states[i];
}

// One work-group per handle: its tiles, with their state index set to the
// handle's place in the batch.
__global__ __launch_bounds__(256) void k_merge_work(const MergeSrc* __restrict__ src, TileWork* __restrict__ work)
{
    const MergeSrc s = src[blockIdx.x];
    for (int32_t t = static_cast<int32_t>(threadIdx.x); t < s.n_tiles; t += 256) {
        TileWork w = s.work[t];
        w.mesh = static_cast<int32_t>(blockIdx.x);
        work[s.off + t] = w;
    }
}

// kCopyGroups work-groups per handle copy its X[1] into X[0]: 16-byte units
// where both buffers and the length allow (double precision always), else
// 4-byte units (single precision with an odd node count puts X[1] at an
// 8-byte boundary).
constexpr int kCopyGroups = 8;
__global__ __launch_bounds__(256) void k_copy_buffers(const MergeSrc* __restrict__ src)
{
    const MergeSrc s = src[blockIdx.x / kCopyGroups];
    const int64_t stride = static_cast<int64_t>(kCopyGroups) * 256;
    const int64_t u0 = static_cast<int64_t>(blockIdx.x % kCopyGroups) * 256 + threadIdx.x;
    if (s.wide) {
        const uint4* from = static_cast<const uint4*>(s.from);
        uint4* to = static_cast<uint4*>(s.to);
        for (int64_t u = u0; u < s.units; u += stride) to[u] = from[u];
    } else {
        const uint32_t* from = static_cast<const uint32_t*>(s.from);
        uint32_t* to = static_cast<uint32_t*>(s.to);
        for (int64_t u = u0; u < s.units; u += stride) to[u] = from[u];
    }
}

}  // namespace

}  // namespace sl

struct sl_mesh {
    int device = 0;
    sl_options o{};
    int32_t wg_auto = 0;
    int32_t block = 0;
    sl::DevMesh m;
    sl::Arena aux;                          // the sweep state and the tile launches' counters
    sl::MeshState* state = nullptr;
    int32_t* sched = nullptr;
    int32_t cur = 0;                        // the buffer holding the current positions (Form A)
    int64_t sweeps = 0;                     // sweeps run so far (equal to state->s)
    hipStream_t own = nullptr;              // the library's stream: setup, host downloads, release
    std::shared_ptr<sl::EventRef> last;     // recorded after the last work queued on the mesh
    hipStream_t last_stream = nullptr;      // where that work was queued
    hipEvent_t t0 = nullptr, t1 = nullptr;  // around the sweeps of the last smooth call
    bool timed = false;
    double setup_ms = 0.0;
    hipGraph_t graph[2] = {nullptr, nullptr};   // a chunk of sweeps from buffer 0 / buffer 1
    hipGraphExec_t exec[2] = {nullptr, nullptr};

    ~sl_mesh()
    {
        if (last) (void)hipEventSynchronize(last->ev);
        for (int p = 0; p < 2; ++p) {
            if (exec[p]) (void)hipGraphExecDestroy(exec[p]);
            if (graph[p]) (void)hipGraphDestroy(graph[p]);
        }
        if (own) {
            sl::devmesh_free(m, own);
            aux.release(own);
            (void)hipStreamSynchronize(own);
            sl::give_stream(own);
        }
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
    }

    bool tiles() const { return o.form == SL_JACOBI && m.tile_nodes > 0; }
    bool class_tiles() const { return o.form != SL_JACOBI && m.tile_nodes > 0 && m.n_tile_classes > 0; }

    // Form B on colour-class tiles: one launch per class, in place, with the
    // sweep state at `st_state`; the last class closes the sweep when `close`.
    sl_status sweep_classes(sl::MeshState* st_state, bool close, hipStream_t st) const
    {
        for (int32_t c = 0; c < m.n_tile_classes; ++c) {
            sl::TileLaunch Lc = launch();
            Lc.work = m.work + m.class_tile_h[c];
            Lc.n_work = m.class_tile_h[c + 1] - m.class_tile_h[c];
            Lc.states = st_state;
            Lc.n_close = close && c + 1 == m.n_tile_classes ? 1 : 0;
            Lc.wg_per_cu = wg_auto ? 0 : o.tile_wg_per_cu;   // a count tuned for Form A's tiles does not apply
            const sl_status r = sl::launch_sweep_class(Lc, m.fans_max, nullptr, st);
            if (r) return r;
        }
        return SL_OK;
    }

    sl::TileLaunch launch() const
    {
        // one mesh per launch: a launch on a mesh that has stopped returns at once
        return sl::TileLaunch{m.work, m.n_tiles, m.tile_nodes, m.halo_max, m.rows_max, o.layout, o.accept,
                              state,  sl::resolve_wg_per_cu(o), 1, o.precision, sched, 1, 1};
    }

    // One sweep reading buffer `parity` (Form A) and closing it.
    sl_status sweep(int32_t parity, hipStream_t st) const
    {
        if (tiles()) return sl::launch_sweep_tiles(launch(), parity, nullptr, st);
        if (class_tiles()) return sweep_classes(state, true, st);
        return sl::launch_sweep_nodes(m, parity, o.form, o.accept, block, state, nullptr, sched, st, true);
    }

    // A chunk of kHandleChunk sweeps starting from buffer p, captured once.
    sl_status chunk_graph(int p, hipGraphExec_t* out)
    {
        if (!exec[p]) {
            hipStream_t cap = nullptr;
            sl_status r = sl::take_stream(&cap);
            if (r) return r;
            if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                sl::give_stream(cap);
                return sl::fail(SL_EDEVICE, "graph capture could not start");
            }
            for (int32_t k = 0; k < sl::kHandleChunk && !r; ++k) r = sweep((p + k) & 1, cap);
            const hipError_t ce = hipStreamEndCapture(cap, &graph[p]);
            sl::give_stream(cap);
            if (r) return r;
            if (ce != hipSuccess) return sl::fail(SL_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(ce));
            SL_HIP(hipGraphInstantiate(&exec[p], graph[p], nullptr, nullptr, 0));
        }
        *out = exec[p];
        return SL_OK;
    }

    // Makes `st` wait for the mesh's last queued work.
    sl_status after_last(hipStream_t st)
    {
        if (last && last_stream != st) SL_HIP(hipStreamWaitEvent(st, last->ev, 0));
        return SL_OK;
    }

    sl_status mark(hipStream_t st)
    {
        std::shared_ptr<sl::EventRef> e;
        sl_status r = sl::new_event(&e);
        if (r) return r;
        SL_HIP(hipEventRecord(e->ev, st));
        last = std::move(e);
        last_stream = st;
        return SL_OK;
    }
};

namespace sl {

namespace {

sl_status check_handle(const sl_mesh* h)
{
    if (!h) return fail(SL_EINVAL, "null mesh handle");
    int dev = -1;
    SL_HIP(hipGetDevice(&dev));
    if (dev != h->device) return fail(SL_EINVAL, "the mesh lives on device " + std::to_string(h->device) +
                                                     ", the current device is " + std::to_string(dev));
    return SL_OK;
}

// Options of a handle: automatic values resolved once; no resident kernel.
sl_status handle_options(const sl_options* opts, sl_options* out, int32_t* wg_auto)
{
    sl_options o;
    sl_options_default(&o);
    if (opts) o = *opts;
    o.flags_out = nullptr;
    sl_status r = check_options(o);
    if (r) return r;
    if (o.kernel == SL_KERNEL_RESIDENT) return fail(SL_EINVAL, "mesh handles do not run the resident kernel");
    // automatic Form B: the node kernel (the automatic choice of a one-call
    // smooth would also consider the resident kernel, which handles do not run)
    if (o.kernel == SL_KERNEL_AUTO && o.form == SL_INPLACE_COLORED) o.kernel = SL_KERNEL_NODE;
    *wg_auto = o.tile_wg_per_cu == 0 ? 1 : 0;
    if (o.form == SL_JACOBI) o.tile_nodes = resolve_tile_nodes(o);   // colour-class tiles size themselves
    o.tile_wg_per_cu = resolve_wg_per_cu(o);
    o.block_size = resolve_block_size(o);
    *out = o;
    return SL_OK;
}

// Everything after the mesh's own setup: state, counters, events.
sl_status finish_create(sl_mesh* h, std::chrono::steady_clock::time_point t0)
{
    sl_status r;
    if ((r = h->aux.reserve(Arena::piece(sizeof(MeshState)) + Arena::piece(sizeof(int32_t) * kTileSchedInts),
                            h->own)) ||
        (r = h->aux.take(&h->state, 1)) || (r = h->aux.take(&h->sched, kTileSchedInts)))
        return r;
    SL_HIP(hipMemsetAsync(h->state, 0, sizeof(MeshState), h->own));
    SL_HIP(hipMemsetAsync(h->sched, 0, sizeof(int32_t) * kTileSchedInts, h->own));
    SL_HIP(hipEventCreate(&h->t0));
    SL_HIP(hipEventCreate(&h->t1));
    if ((r = h->mark(h->own))) return r;
    SL_HIP(hipStreamSynchronize(h->own));
    h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return SL_OK;
}

sl_status read_state(sl_mesh* h, MeshState* out, hipStream_t st)
{
    SL_HIP(hipMemcpyAsync(out, h->state, sizeof(MeshState), hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    return SL_OK;
}

sl_status smooth_handle(sl_mesh* h, int32_t iterations, double tol, hipStream_t st)
{
    sl_status r;
    if ((r = check_handle(h))) return r;
    if (iterations < 0) return fail(SL_EINVAL, "iterations must be >= 0");
    if (h->sweeps + iterations > INT32_MAX) return fail(SL_EINVAL, "more than 2^31 sweeps on one mesh");
    const double tol2 = tol > 0.0 ? tol * tol : 0.0;
    if ((r = h->after_last(st))) return r;
    SL_HIP(hipEventRecord(h->t0, st));
    k_begin_run<<<1, 64, 0, st>>>(h->state, 1, iterations, tol2);
    SL_HIP(hipGetLastError());
    const bool jacobi = h->o.form == SL_JACOBI;
    int32_t done = 0;
    while (done < iterations) {
        const int32_t c = std::min(kHandleChunk, iterations - done);
        const int32_t p = jacobi ? ((h->cur + done) & 1) : 0;
        if (c == kHandleChunk) {
            hipGraphExec_t ex = nullptr;
            if ((r = h->chunk_graph(p, &ex))) return r;
            SL_HIP(hipGraphLaunch(ex, st));
        } else {
            for (int32_t k = 0; k < c; ++k)
                if ((r = h->sweep((p + k) & 1, st))) return r;
        }
        done += c;
        if (tol2 > 0.0) {
            // a converged mesh's later launches return at once; the host stops
            // queueing them
            MeshState ms{};
            SL_HIP(hipMemcpyAsync(&ms, h->state, sizeof(MeshState), hipMemcpyDeviceToHost, st));
            SL_HIP(hipStreamSynchronize(st));
            if (!ms.active || done >= iterations) {
                const int32_t ran = static_cast<int32_t>(ms.s - h->sweeps);
                if (jacobi) h->cur = (h->cur + ran) & 1;
                h->sweeps = ms.s;
                break;
            }
        }
    }
    if (tol2 <= 0.0) {
        if (jacobi) h->cur = (h->cur + iterations) & 1;
        h->sweeps += iterations;
    }
    SL_HIP(hipEventRecord(h->t1, st));
    h->timed = true;
    return h->mark(st);
}

void fill_report(const sl_mesh* h, const MeshState& ms, sl_report* rep)
{
    sl_report r{};
    r.iterations_run = ms.s;
    r.n_colors = h->m.n_colors;
    std::memcpy(&r.max_disp_sq_last, &ms.maxd_last, sizeof(double));
    r.accepted_last = static_cast<int64_t>(ms.acc_last);
    r.accepted_total = static_cast<int64_t>(ms.acc_total);
    r.setup_ms = h->setup_ms;
    if (h->timed) {
        float ms_ = 0.f;
        if (hipEventElapsedTime(&ms_, h->t0, h->t1) == hipSuccess) r.sweep_ms = ms_;
        else (void)hipGetLastError();
    }
    r.kernel_used = kernel_used(h->m);
    r.tile_nodes = h->m.tile_nodes;
    *rep = r;
}

}  // namespace

}  // namespace sl

extern "C" {

sl_status sl_mesh_create(const sl_mesh_desc* desc, const sl_options* opts, sl_mesh** out)
{
    using namespace sl;
    const auto t0 = std::chrono::steady_clock::now();
    set_error("");
    if (!out) return fail(SL_EINVAL, "null output pointer");
    *out = nullptr;
    if (!desc) return fail(SL_EINVAL, "null mesh description");
    auto h = std::make_unique<sl_mesh>();
    sl_status r = handle_options(opts, &h->o, &h->wg_auto);
    if (r) return r;
    h->block = h->o.block_size;
    SL_HIP(hipGetDevice(&h->device));
    keep_pool_warm();
    if ((r = take_stream(&h->own))) return r;
    h->m.class_tiles_ok = true;
    if ((r = upload_and_prepare(*desc, h->o, 0, h->m, h->own))) return r;
    if ((r = finish_create(h.get(), t0))) return r;
    *out = h.release();
    return SL_OK;
}

sl_status sl_mesh_create_device(const double* coords, int32_t n_nodes, const int32_t* nbr_ptr,
                                const int32_t* nbr_idx, const int32_t* tri_ptr, const int32_t* tri_idx,
                                const int32_t* tris, int32_t n_tris, const uint8_t* boundary,
                                const sl_options* opts, void* stream, sl_mesh** out)
{
    using namespace sl;
    const auto t0 = std::chrono::steady_clock::now();
    set_error("");
    if (!out) return fail(SL_EINVAL, "null output pointer");
    *out = nullptr;
    auto h = std::make_unique<sl_mesh>();
    sl_status r = handle_options(opts, &h->o, &h->wg_auto);
    if (r) return r;
    h->block = h->o.block_size;
    SL_HIP(hipGetDevice(&h->device));
    keep_pool_warm();
    if ((r = take_stream(&h->own))) return r;
    // the caller's arrays are read on the caller's stream, in its order
    hipStream_t st = static_cast<hipStream_t>(stream);
    MeshInput in{coords, n_nodes, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, n_tris, boundary};
    h->m.class_tiles_ok = true;
    if ((r = prepare_mesh(in, h->o, 0, h->m, st))) return r;
    SL_HIP(hipStreamSynchronize(st));
    if ((r = finish_create(h.get(), t0))) return r;
    *out = h.release();
    return SL_OK;
}

sl_status sl_mesh_smooth_async(sl_mesh* h, int32_t iterations, double tol, void* stream)
{
    sl::set_error("");
    return sl::smooth_handle(h, iterations, tol, static_cast<hipStream_t>(stream));
}

sl_status sl_mesh_download(sl_mesh* h, double* coords, sl_report* report)
{
    using namespace sl;
    set_error("");
    sl_status r;
    if ((r = check_handle(h))) return r;
    if (!coords) return fail(SL_EINVAL, "null coords");
    if ((r = h->after_last(h->own))) return r;
    const size_t n = static_cast<size_t>(h->m.n);
    unsigned char* buf = nullptr;
    if ((r = block_take(&buf, 2 * n * sizeof(double), h->own))) return r;
    double* d = reinterpret_cast<double*>(buf);
    MeshState ms{};
    do {
        if ((r = unpermute_coords(h->m, h->o.form == SL_JACOBI ? h->cur : 0, d, h->own))) break;
        if ((r = read_state(h, &ms, h->own))) break;
        // straight into the caller's array, last
        if ((r = copy_to_host(coords, d, 2 * n * sizeof(double), h->own))) break;
    } while (false);
    block_give(buf, h->own);
    if (r) return r;
    if (report) fill_report(h, ms, report);
    return h->mark(h->own);
}

sl_status sl_mesh_download_device(sl_mesh* h, double* coords, void* stream)
{
    using namespace sl;
    set_error("");
    sl_status r;
    if ((r = check_handle(h))) return r;
    if (!coords) return fail(SL_EINVAL, "null coords");
    if (reinterpret_cast<uintptr_t>(coords) % 16 != 0) return fail(SL_EINVAL, "coords must be 16-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((r = h->after_last(st))) return r;
    if ((r = unpermute_coords(h->m, h->o.form == SL_JACOBI ? h->cur : 0, coords, st))) return r;
    return h->mark(st);
}

sl_status sl_mesh_get_report(sl_mesh* h, sl_report* report)
{
    using namespace sl;
    set_error("");
    sl_status r;
    if ((r = check_handle(h))) return r;
    if (!report) return fail(SL_EINVAL, "null report");
    if ((r = h->after_last(h->own))) return r;
    MeshState ms{};
    if ((r = read_state(h, &ms, h->own))) return r;
    fill_report(h, ms, report);
    return SL_OK;
}

void sl_mesh_destroy(sl_mesh* h)
{
    if (!h) return;
    int prev = -1;
    const bool switched = hipGetDevice(&prev) == hipSuccess && prev != h->device && hipSetDevice(h->device) == hipSuccess;
    delete h;
    if (switched) (void)hipSetDevice(prev);
}

sl_status sl_mesh_smooth_batch_async(sl_mesh* const* meshes, int32_t n_meshes, int32_t iterations, double tol,
                                     void* stream, sl_batch_report* batch)
{
    using namespace sl;
    const auto t0 = std::chrono::steady_clock::now();
    set_error("");
    if (!meshes || n_meshes <= 0) return fail(SL_EINVAL, "need at least one mesh");
    if (iterations < 0) return fail(SL_EINVAL, "iterations must be >= 0");
    sl_status r;
    const sl_mesh* first = meshes[0];
    if ((r = check_handle(first))) return r;
    int32_t T = 0, halo_cap = 0, rows_cap = 0, on_tiles = 0;
    int64_t total_tiles = 0;
    bool any_node = false;
    for (int32_t i = 0; i < n_meshes; ++i) {
        const sl_mesh* h = meshes[i];
        if ((r = check_handle(h))) return fail(r, "mesh " + std::to_string(i) + ": " + sl_last_error());
        if (h->o.form != first->o.form || h->o.accept != first->o.accept || h->o.layout != first->o.layout ||
            h->o.precision != first->o.precision)
            return fail(SL_EINVAL, "mesh " + std::to_string(i) + ": form, accept rule, layout and precision must "
                                   "match the first mesh's");
        if (h->sweeps + iterations > INT32_MAX) return fail(SL_EINVAL, "more than 2^31 sweeps on one mesh");
        if (h->tiles()) {
            if (T != 0 && h->m.tile_nodes != T) return fail(SL_EINVAL, "meshes with different tile sizes");
            T = h->m.tile_nodes;
            halo_cap = std::max(halo_cap, h->m.halo_max);
            rows_cap = std::max(rows_cap, h->m.rows_max);
            total_tiles += h->m.n_tiles;
            ++on_tiles;
        } else {
            any_node = true;
        }
    }
    {
        std::vector<const sl_mesh*> seen(meshes, meshes + n_meshes);
        std::sort(seen.begin(), seen.end());
        if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
            return fail(SL_EINVAL, "a mesh appears twice in one batch");
    }
    if (total_tiles > INT32_MAX) return fail(SL_EINVAL, "batch has more than 2^31 tiles");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool jacobi = first->o.form == SL_JACOBI;
    const double tol2 = tol > 0.0 ? tol * tol : 0.0;

    // per call: the merged states, tiles and counters, and the handles' table
    const size_t un = static_cast<size_t>(n_meshes);
    const size_t bytes = Arena::piece(sizeof(MeshState) * un) + Arena::piece(sizeof(TileWork) * std::max<int64_t>(total_tiles, 1)) +
                         Arena::piece(sizeof(int32_t) * kTileSchedInts) + Arena::piece(sizeof(MergeSrc) * un);
    Arena ar;
    if ((r = ar.reserve(bytes, st))) return r;
    struct GiveBack {
        Arena& a;
        hipStream_t s;
        ~GiveBack() { a.release(s); }
    } give_back{ar, st};
    MeshState* states = nullptr;
    TileWork* work = nullptr;
    int32_t* sched = nullptr;
    MergeSrc* src = nullptr;
    if ((r = ar.take(&states, un)) || (r = ar.take(&work, std::max<int64_t>(total_tiles, 1))) ||
        (r = ar.take(&sched, kTileSchedInts)) || (r = ar.take(&src, un)))
        return r;
    std::vector<MergeSrc> hs(un);
    int64_t off = 0, copies = 0;
    for (int32_t i = 0; i < n_meshes; ++i) {
        sl_mesh* h = meshes[i];
        if ((r = h->after_last(st))) return r;
        MergeSrc s{};
        s.state = h->state;
        s.work = h->m.work;
        s.off = off;
        s.n_tiles = h->tiles() ? h->m.n_tiles : 0;
        off += s.n_tiles;
        // every mesh of one launch reads the same buffer: bring the current
        // positions to buffer 0 where they are in buffer 1
        if (jacobi && h->cur == 1) {
            const size_t bytes = 2 * static_cast<size_t>(h->m.n) * (h->o.precision == SL_F32 ? 4 : 8);
            s.from = h->m.X[1];
            s.to = h->m.X[0];
            s.wide = bytes % 16 == 0 && reinterpret_cast<uintptr_t>(s.from) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(s.to) % 16 == 0;
            s.units = static_cast<int64_t>(s.wide ? bytes / 16 : bytes / 4);
            ++copies;
        }
        hs[i] = s;
    }
    SL_HIP(hipMemcpyAsync(src, hs.data(), sizeof(MergeSrc) * un, hipMemcpyHostToDevice, st));
    SL_HIP(hipMemsetAsync(sched, 0, sizeof(int32_t) * kTileSchedInts, st));
    if (copies) {
        k_copy_buffers<<<n_meshes * kCopyGroups, 256, 0, st>>>(src);
        SL_HIP(hipGetLastError());
    }
    k_gather_states<<<div_up(n_meshes, 256), 256, 0, st>>>(src, n_meshes, states, iterations, tol2);
    SL_HIP(hipGetLastError());
    if (total_tiles > 0) {
        k_merge_work<<<n_meshes, 256, 0, st>>>(src, work);
        SL_HIP(hipGetLastError());
    }
    for (int32_t i = 0; i < n_meshes; ++i)
        if (jacobi) meshes[i]->cur = 0;

    const bool all_tiles = jacobi && total_tiles > 0 && !any_node;
    const sl_options& o = first->o;
    const TileLaunch L{work,  static_cast<int32_t>(total_tiles), T, halo_cap, rows_cap, o.layout, o.accept,
                       states, resolve_wg_per_cu(o), 0, o.precision, sched, all_tiles ? n_meshes : 0};
    int32_t done = 0;
    std::vector<MeshState> back;
    while (done < iterations) {
        const int32_t c = std::min(kHandleChunk, iterations - done);
        for (int32_t k = 0; k < c; ++k) {
            const int32_t parity = (done + k) & 1;
            if (jacobi && total_tiles > 0 && (r = launch_sweep_tiles(L, parity, nullptr, st))) return r;
            for (int32_t i = 0; i < n_meshes; ++i) {
                const sl_mesh* h = meshes[i];
                if (jacobi && h->tiles()) continue;
                // Form B on class tiles: the handle's own launches, closed below with the others
                if (h->class_tiles()) {
                    if ((r = h->sweep_classes(states + i, false, st))) return r;
                    continue;
                }
                if ((r = launch_sweep_nodes(h->m, parity, o.form, o.accept, h->block, states + i, nullptr, sched, st)))
                    return r;
            }
            if (!all_tiles && (r = launch_advance(states, n_meshes, st))) return r;
        }
        done += c;
        if (tol2 > 0.0) {
            back.resize(un);
            SL_HIP(hipMemcpyAsync(back.data(), states, sizeof(MeshState) * un, hipMemcpyDeviceToHost, st));
            SL_HIP(hipStreamSynchronize(st));
            bool any = false;
            for (const MeshState& ms : back) any = any || ms.active;
            if (!any) break;
        }
    }
    k_scatter_states<<<div_up(n_meshes, 256), 256, 0, st>>>(src, n_meshes, states);
    SL_HIP(hipGetLastError());
    int64_t updates = 0;
    if (tol2 > 0.0 && iterations > 0) {
        if (back.size() != un) {
            back.resize(un);
            SL_HIP(hipMemcpyAsync(back.data(), states, sizeof(MeshState) * un, hipMemcpyDeviceToHost, st));
            SL_HIP(hipStreamSynchronize(st));
        }
        for (int32_t i = 0; i < n_meshes; ++i) {
            sl_mesh* h = meshes[i];
            const int64_t ran = back[i].s - h->sweeps;
            if (jacobi) h->cur = static_cast<int32_t>(ran & 1);
            h->sweeps = back[i].s;
            updates += ran * h->m.n_free;
        }
    } else {
        for (int32_t i = 0; i < n_meshes; ++i) {
            sl_mesh* h = meshes[i];
            if (jacobi) h->cur = iterations & 1;
            h->sweeps += iterations;
            updates += static_cast<int64_t>(iterations) * h->m.n_free;
        }
    }
    // one event for the whole call, shared by its meshes
    std::shared_ptr<EventRef> e;
    if ((r = new_event(&e))) return r;
    SL_HIP(hipEventRecord(e->ev, st));
    for (int32_t i = 0; i < n_meshes; ++i) {
        meshes[i]->last = e;
        meshes[i]->last_stream = st;
        meshes[i]->timed = false;
    }
    if (batch) {
        sl_batch_report b{};
        b.node_updates = updates;
        b.tiles = total_tiles;
        b.meshes_on_tile_path = on_tiles;
        b.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *batch = b;
    }
    return SL_OK;
}

sl_status sl_release_cached_memory(void)
{
    sl::set_error("");
    return sl::release_cached_memory();
}

}  // extern "C"
