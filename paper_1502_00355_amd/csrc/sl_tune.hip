// Autotuning of the sweep launch shape.
//
// The tile size (free nodes per tile) and the number of persistent
// work-groups per compute unit change only the speed of a sweep: every tile
// computes the same per-node results whatever the shape.  The tuner sets up
// a sample of the caller's meshes once per tile size, times a few sweeps of
// the batched tile kernel for each work-group count (twice, interleaved,
// keeping the faster time), and keeps the fastest shape as the automatic
// choice of the device, unless the default shape is within 1% of it.  For
// Form B (node kernel) it times the node kernel's work-group sizes instead,
// and for the lane-group kernel the width of a node's lane group.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "sl_common.h"

namespace sl {

namespace {

constexpr size_t kTuneNodes = size_t(8) << 20;   // sampled nodes, about
constexpr int32_t kWarmSweeps = 2;
constexpr int32_t kTimedSweeps = 8;
constexpr int32_t kPasses = 2;          // every shape is timed this often, interleaved; the minimum counts
constexpr double kPreferDefault = 1.01; // the default shape stays unless another is faster by more than this

// Device state of one tuning pass, released on every exit path.
struct TunePass {
    hipStream_t st = nullptr;
    std::vector<DevMesh> meshes;
    TileWork* work = nullptr;
    MeshState* states = nullptr;
    int32_t* sched = nullptr;   // the tile launches' counters; they close their own sweeps
    hipEvent_t ev[2] = {nullptr, nullptr};
    ~TunePass()
    {
        for (auto& m : meshes) devmesh_free(m, st);
        dfree(work, st);
        dfree(states, st);
        dfree(sched, st);
        (void)hipStreamSynchronize(st);
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

struct Candidate {
    int32_t tile_nodes, shape;
    double ns;
};

// Sets up the sampled meshes with options o and fills the sweep states
// (every mesh active, no sweep cap in reach).
sl_status setup_pass(TunePass& p, const sl_mesh_desc* meshes, const std::vector<int32_t>& sample,
                     const sl_options& o)
{
    p.meshes.resize(sample.size());
    for (size_t k = 0; k < sample.size(); ++k) {
        const sl_status r = upload_and_prepare(meshes[sample[k]], o, static_cast<int32_t>(k), p.meshes[k], p.st);
        if (r) return fail(r, "mesh " + std::to_string(sample[k]) + ": " + sl_last_error());
    }
    std::vector<MeshState> h(sample.size());
    for (auto& s : h) {
        s = MeshState{};
        s.iters = INT32_MAX;
        s.active = 1;
    }
    sl_status r = dalloc(&p.states, h.size(), p.st);
    if (r || (r = dalloc(&p.sched, kTileSchedInts, p.st))) return r;
    SL_HIP(hipMemcpyAsync(p.states, h.data(), sizeof(MeshState) * h.size(), hipMemcpyHostToDevice, p.st));
    SL_HIP(hipMemsetAsync(p.sched, 0, sizeof(int32_t) * kTileSchedInts, p.st));
    for (auto& e : p.ev) SL_HIP(hipEventCreate(&e));
    return SL_OK;
}

// Device milliseconds of kTimedSweeps sweeps enqueued by `sweep(parity)`
// (n_states > 0: each followed by a launch_advance over that many states).
template <typename F>
sl_status time_sweeps(TunePass& p, int32_t n_states, F sweep, float* ms)
{
    sl_status r = SL_OK;
    for (int32_t s = 0; s < kWarmSweeps + kTimedSweeps && !r; ++s) {
        if (s == kWarmSweeps) SL_HIP(hipEventRecord(p.ev[0], p.st));
        r = sweep(s & 1);
        if (!r && n_states > 0) r = launch_advance(p.states, n_states, p.st);
    }
    if (r) return r;
    SL_HIP(hipEventRecord(p.ev[1], p.st));
    SL_HIP(hipStreamSynchronize(p.st));
    SL_HIP(hipEventElapsedTime(ms, p.ev[0], p.ev[1]));
    return SL_OK;
}

sl_status tune_tiles(const sl_mesh_desc* meshes, const std::vector<int32_t>& sample, const sl_options& base,
                     hipStream_t st, std::vector<Candidate>& out, int64_t* free_nodes)
{
    for (int32_t T : {512, 256}) {
        sl_options o = base;
        o.tile_nodes = T;
        o.kernel = SL_KERNEL_TILE;
        TunePass p;
        p.st = st;
        sl_status r = setup_pass(p, meshes, sample, o);
        if (r) return r;
        int64_t tiles = 0, on_tiles = 0;
        int32_t hcap = 0, rcap = 0;
        for (const auto& m : p.meshes) {
            if (m.tile_nodes == 0) continue;
            tiles += m.n_tiles;
            on_tiles += m.n_free;
            hcap = std::max(hcap, m.halo_max);
            rcap = std::max(rcap, m.rows_max);
        }
        if (tiles == 0 || on_tiles == 0) continue;
        if (tiles > INT32_MAX) return fail(SL_EINVAL, "sample has more than 2^31 tiles");
        *free_nodes = on_tiles;
        if ((r = dalloc(&p.work, static_cast<size_t>(tiles), st))) return r;
        int64_t off = 0;
        for (const auto& m : p.meshes) {
            if (m.tile_nodes == 0) continue;
            SL_HIP(hipMemcpyAsync(p.work + off, m.work, sizeof(TileWork) * m.n_tiles, hipMemcpyDeviceToDevice, st));
            off += m.n_tiles;
        }
        std::vector<int32_t> shapes;
        int last_grid = -1;
        for (int32_t w = 1; w <= 8; ++w) {
            const int grid = tile_grid(static_cast<int>(tiles), T, hcap, rcap, w, o.precision);
            if (grid == last_grid) continue;   // capped by LDS or by the tile count: same launch
            last_grid = grid;
            shapes.push_back(w);
        }
        const size_t first = out.size();
        for (int32_t pass = 0; pass < kPasses; ++pass) {
            for (size_t k = 0; k < shapes.size(); ++k) {
                const int32_t w = shapes[k];
                const TileLaunch L{p.work, static_cast<int32_t>(tiles), T, hcap, rcap, o.layout, o.accept, p.states,
                                   w, 0, o.precision, p.sched, static_cast<int32_t>(p.meshes.size())};
                float ms = 0.f;
                r = time_sweeps(p, 0, [&](int32_t parity) { return launch_sweep_tiles(L, parity, nullptr, st); },
                                &ms);
                if (r) return r;
                const double ns = 1e6 * ms / (static_cast<double>(kTimedSweeps) * on_tiles);
                if (pass == 0) out.push_back(Candidate{T, w, ns});
                else out[first + k].ns = std::min(out[first + k].ns, ns);
            }
        }
    }
    return SL_OK;
}

sl_status tune_nodes(const sl_mesh_desc* meshes, const std::vector<int32_t>& sample, const sl_options& base,
                     hipStream_t st, std::vector<Candidate>& out, int64_t* free_nodes)
{
    sl_options o = base;
    o.kernel = SL_KERNEL_NODE;
    TunePass p;
    p.st = st;
    sl_status r = setup_pass(p, meshes, sample, o);
    if (r) return r;
    int64_t nfree = 0;
    for (const auto& m : p.meshes) nfree += m.n_free;
    if (nfree == 0) return SL_OK;
    *free_nodes = nfree;
    const size_t first = out.size();
    for (int32_t pass = 0; pass < kPasses; ++pass) {
        for (int32_t bs : {64, 128, 256}) {
            float ms = 0.f;
            r = time_sweeps(p, static_cast<int32_t>(p.meshes.size()),
                            [&](int32_t parity) {
                                for (size_t k = 0; k < p.meshes.size(); ++k) {
                                    const sl_status rr = launch_sweep_nodes(p.meshes[k], parity, o.form, o.accept,
                                                                            bs, p.states + k, nullptr, p.sched, st);
                                    if (rr) return rr;
                                }
                                return SL_OK;
                            },
                            &ms);
            if (r) return r;
            const double ns = 1e6 * ms / (static_cast<double>(kTimedSweeps) * nfree);
            const size_t k = first + static_cast<size_t>(bs == 64 ? 0 : bs == 128 ? 1 : 2);
            if (pass == 0) out.push_back(Candidate{0, bs, ns});
            else out[k].ns = std::min(out[k].ns, ns);
        }
    }
    return SL_OK;
}

sl_status tune_lanes(const sl_mesh_desc* meshes, const std::vector<int32_t>& sample, const sl_options& base,
                     hipStream_t st, std::vector<Candidate>& out, int64_t* free_nodes)
{
    // one setup per width: the width is fixed in each mesh at setup
    const int32_t widths[3] = {4, 8, 16};
    std::vector<TunePass> passes(3);
    int64_t nfree = 0;
    for (int w = 0; w < 3; ++w) {
        sl_options o = base;
        o.kernel = SL_KERNEL_LANES;
        o.lane_width = widths[w];
        passes[w].st = st;
        const sl_status r = setup_pass(passes[w], meshes, sample, o);
        if (r) return r;
        if (w == 0)
            for (const auto& m : passes[w].meshes) nfree += m.n_free;
    }
    if (nfree == 0) return SL_OK;
    *free_nodes = nfree;
    const size_t first = out.size();
    for (int32_t pass = 0; pass < kPasses; ++pass) {
        for (int w = 0; w < 3; ++w) {
            TunePass& p = passes[w];
            float ms = 0.f;
            const sl_status r = time_sweeps(p, static_cast<int32_t>(p.meshes.size()),
                                            [&](int32_t parity) {
                                                for (size_t k = 0; k < p.meshes.size(); ++k) {
                                                    const sl_status rr =
                                                        launch_sweep_nodes(p.meshes[k], parity, base.form, base.accept,
                                                                           0, p.states + k, nullptr, p.sched, st);
                                                    if (rr) return rr;
                                                }
                                                return SL_OK;
                                            },
                                            &ms);
            if (r) return r;
            const double ns = 1e6 * ms / (static_cast<double>(kTimedSweeps) * nfree);
            if (pass == 0) out.push_back(Candidate{0, widths[w], ns});
            else out[first + static_cast<size_t>(w)].ns = std::min(out[first + static_cast<size_t>(w)].ns, ns);
        }
    }
    return SL_OK;
}

}  // namespace

}  // namespace sl

extern "C" {

sl_status sl_autotune(const sl_mesh_desc* meshes, int32_t n_meshes, const sl_options* opts, sl_tuning* out)
{
    using namespace sl;
    const auto t0 = std::chrono::steady_clock::now();
    set_error("");
    if (!meshes || n_meshes <= 0) return fail(SL_EINVAL, "need at least one mesh");
    sl_options o;
    sl_options_default(&o);
    if (opts) o = *opts;
    o.flags_out = nullptr;
    o.tile_nodes = 0;
    o.tile_wg_per_cu = 0;
    o.block_size = 0;
    o.lane_width = 0;
    sl_status r = check_options(o);
    if (r) return r;
    size_t total = 0;
    for (int32_t i = 0; i < n_meshes; ++i) {
        if (meshes[i].n_nodes <= 0) return fail(SL_EINVAL, "mesh " + std::to_string(i) + ": n_nodes must be >= 1");
        total += static_cast<size_t>(meshes[i].n_nodes);
    }
    // every k-th mesh in index order, k chosen so the sample is about kTuneNodes
    const int32_t stride = static_cast<int32_t>(std::max<size_t>(1, (total + kTuneNodes - 1) / kTuneNodes));
    std::vector<int32_t> sample;
    for (int32_t i = 0; i < n_meshes; i += stride) sample.push_back(i);
    keep_pool_warm();

    hipStream_t st = nullptr;
    SL_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    std::vector<Candidate> cands;
    int64_t free_nodes = 0;
    // what is tuned: the lane-group width when the lane-group kernel is asked
    // for, else the tile shape (Form A) or the node kernel's block (Form B)
    const bool lanes = o.kernel == SL_KERNEL_LANES;
    r = lanes ? tune_lanes(meshes, sample, o, st, cands, &free_nodes)
              : o.form == SL_JACOBI ? tune_tiles(meshes, sample, o, st, cands, &free_nodes)
                                    : tune_nodes(meshes, sample, o, st, cands, &free_nodes);
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (r) return r;

    auto shape_of = [&](const Candidate& c) {
        if (lanes) return TunedShape{0, 0, 0, c.shape};
        return c.tile_nodes ? TunedShape{c.tile_nodes, c.shape, 0, 0} : TunedShape{0, 0, c.shape, 0};
    };
    TunedShape best{0, 0, 0, 0};
    double best_ns = 0.0;
    for (const auto& c : cands) {
        if (best_ns == 0.0 || c.ns < best_ns) {
            best_ns = c.ns;
            best = shape_of(c);
        }
    }
    // near-ties go to the default shape (512 nodes and 4 work-groups per CU;
    // block size 256; lane width 8), whose speed holds across meshes and devices
    for (const auto& c : cands) {
        const bool dflt = lanes ? c.shape == 8 : c.tile_nodes ? (c.tile_nodes == 512 && c.shape == 4) : c.shape == 256;
        if (dflt && c.ns <= best_ns * kPreferDefault) best = shape_of(c);
    }
    if (!cands.empty()) {
        // each tuning sets its own fields and leaves the others as they were
        const TunedShape prev = tuned_shape();
        TunedShape next = prev;
        if (lanes) next.lane_width = best.lane_width;
        else if (o.form == SL_JACOBI) {
            next.tile_nodes = best.tile_nodes;
            next.wg_per_cu = best.wg_per_cu;
        } else {
            next.block_size = best.block_size;
        }
        set_tuned_shape(next);
    }
    if (out) {
        sl_tuning t;
        std::memset(&t, 0, sizeof(t));
        t.tile_nodes = !lanes && o.form == SL_JACOBI ? best.tile_nodes : 0;
        t.tile_wg_per_cu = !lanes && o.form == SL_JACOBI ? best.wg_per_cu : 0;
        t.block_size = !lanes && o.form != SL_JACOBI ? best.block_size : 0;
        t.lane_width = lanes ? best.lane_width : 0;
        const int32_t cap = static_cast<int32_t>(sizeof(t.candidates) / sizeof(t.candidates[0]));
        t.n_candidates = std::min(cap, static_cast<int32_t>(cands.size()));
        for (int32_t k = 0; k < t.n_candidates; ++k) {
            t.candidates[k].tile_nodes = cands[k].tile_nodes;
            t.candidates[k].wg_per_cu = cands[k].shape;
            t.candidates[k].ns_per_update = cands[k].ns;
        }
        t.sampled_meshes = static_cast<int32_t>(sample.size());
        t.sampled_free_nodes = free_nodes;
        t.tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *out = t;
    }
    return SL_OK;
}

void sl_autotune_reset(void) { sl::clear_tuned_shape(); }

}  // extern "C"
