// Internal declarations of the smartlap HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "../../include/smartlap.h"

#pragma clang fp contract(off)

namespace sl {

// ---------------------------------------------------------------- errors --

void set_error(const std::string& msg);
sl_status fail(sl_status st, const std::string& msg);

#define SL_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::sl::fail(SL_EDEVICE, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    } while (0)

// Validation error bits written by the device checks.
enum : uint32_t {
    VE_PTR = 1u << 0,       // CSR offsets not monotone / out of range          -> EINVAL
    VE_RANGE = 1u << 1,     // node or triangle id out of range                 -> EINVAL
    VE_COORD = 1u << 2,     // coordinate not finite or |x| >= 2^500 (f32: 2^61) -> EINVAL
    VE_SELF = 1u << 3,      // node lists itself as a neighbour                 -> ETOPO
    VE_TRIREP = 1u << 4,    // triangle with a repeated vertex                  -> ETOPO
    VE_NOTIN = 1u << 5,     // incident triangle does not contain its node      -> ETOPO
    VE_MISSING = 1u << 6,   // triangle vertex missing from the neighbour row   -> ETOPO
    VE_EMPTY = 1u << 7,     // free node without neighbours                     -> ETOPO
    VE_VALENCE = 1u << 8,   // free node valence > 127                          -> ETOPO
    VE_ASYM = 1u << 9,      // neighbour rows not symmetric (coloured form)     -> ETOPO
    // Not an error: a triangle listed in a free node's incidence row is
    // missing from the row of another of its free vertices.  The tile path
    // lists each triangle once per tile and scores it for every own vertex,
    // so it needs consistent rows; such a mesh runs on the node path, which
    // reads each node's own row.
    VI_INCIDENCE = 1u << 16,
};
constexpr uint32_t kValErrors = 0xFFFFu;   // the bits above that reject the input
constexpr int kMaxValence = 127;   // 7-bit neighbour slots in a fan entry
// A node-path fan longer than kGroupFan entries keeps its incidence order:
// its bounds read kFanUngrouped.
constexpr int kGroupFan = 32;
constexpr uint32_t kFanUngrouped = 0xFFFFFFFFu;
// Meshes of at least this many free nodes keep their fans ungrouped (no
// bounds array): there the 4 bytes per node of bounds cost the sweep more
// than the grouping saves (4096^2 grid, Form B: 0.830 against 0.812 ms per
// sweep; 1024^2: 0.097 against 0.101 ms; 100K Delaunay points: 0.081
// against 0.084 ms).
constexpr int32_t kGroupFansBelow = 1 << 22;

// Statistics gathered during validation.
struct ValStats {
    uint32_t err;
    int32_t n_free;
    int32_t max_deg_free;
    int32_t max_inc_free;
};

// ------------------------------------------------------ device memory --

template <typename T>
sl_status dalloc(T** p, size_t count, hipStream_t st)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(p), count * sizeof(T), st);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(SL_ENOMEM, std::string("device allocation of ") + std::to_string(count * sizeof(T)) +
                                   " bytes failed: " + hipGetErrorString(e));
    }
    return SL_OK;
}

template <typename T>
void dfree(T*& p, hipStream_t st)
{
    if (p) (void)hipFreeAsync(p, st);
    p = nullptr;
}

// Large device blocks (the arenas below) come from a per-device cache kept
// for the life of the process.  A stream-ordered allocation and free cost
// 0.1-0.7 ms of host time each, during which a device with nothing queued
// idles; repeated calls on meshes of similar size reuse their blocks
// instead.  A block given back carries an event recorded on the giving
// stream after every use of the block; the next taker's stream waits for
// that event before its first use.  The cache holds a bounded number of
// bytes per device; when an allocation fails, the cached blocks are freed
// and it is tried once more.
sl_status block_take(unsigned char** p, size_t bytes, hipStream_t st);
void block_give(unsigned char*& p, hipStream_t st);
constexpr size_t kBlockCacheBytes = size_t(16) << 30;   // cached bytes kept per device at most
// Frees the current device's cached blocks and trims its stream-ordered pool.
sl_status release_cached_memory();

inline int div_up(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// Device memory carved out of one stream-ordered allocation, so that a
// mesh's setup makes a few allocator calls instead of dozens (each call
// costs tens to hundreds of microseconds of host time).  Pieces are
// 256-byte aligned.  mark()/rewind() give stack-like reuse for temporaries:
// work on the stream that used a rewound piece runs before work that uses
// it again.  A take() past the reservation fails loudly (a sizing error).
struct Arena {
    unsigned char* base = nullptr;
    size_t cap = 0, used = 0;
    bool owned = false;   // base came from block_take (release() gives it back)

    static size_t piece(size_t bytes) { return (std::max<size_t>(bytes, 1) + 255) & ~size_t(255); }

    sl_status reserve(size_t bytes, hipStream_t st)
    {
        used = 0;
        cap = bytes;
        const sl_status r = block_take(&base, std::max<size_t>(bytes, 256), st);
        owned = r == SL_OK;
        return r;
    }
    template <typename T>
    sl_status take(T** p, size_t count)
    {
        const size_t b = piece(count * sizeof(T));
        if (!base || used + b > cap) {
            *p = nullptr;
            return fail(SL_ENOMEM, "arena of " + std::to_string(cap) + " bytes exhausted (" + std::to_string(used) +
                                       " used, " + std::to_string(b) + " asked)");
        }
        *p = reinterpret_cast<T*>(base + used);
        used += b;
        return SL_OK;
    }
    // Carves from `bytes` at p, owned by someone else (release() only forgets it).
    void adopt(unsigned char* p, size_t bytes)
    {
        base = p;
        cap = bytes;
        used = 0;
        owned = false;
    }
    size_t mark() const { return used; }
    void rewind(size_t m) { used = m; }
    void release(hipStream_t st)
    {
        if (owned) block_give(base, st);
        base = nullptr;
        owned = false;
        cap = used = 0;
    }
};

// ------------------------------------------------------- device workspace --

// Sweep state of one mesh on the device.  The sweep kernels read `active`
// and fold into the *_cur fields; close_state (k_advance, or the last
// work-group of a tile launch) closes a sweep.
struct MeshState {
    int32_t s;                      // sweeps completed
    int32_t iters;                  // cap on sweeps
    int32_t active;                 // 1 while the next sweep runs
    int32_t pad;
    double tol2;                    // > 0: stop after a sweep with max |dx|^2 < tol2
    unsigned long long maxd_cur;    // bit pattern of the max squared displacement, sweep in progress
    unsigned long long acc_cur;     // accepted nodes, sweep in progress
    unsigned long long maxd_last;   // last completed sweep
    unsigned long long acc_last;
    unsigned long long acc_total;
};

// Closes one sweep of one mesh: counts it if the mesh ran it, moves the
// sweep's folds to the *_last fields and decides whether the next sweep
// runs.  The *_cur fields are read with atomic loads, since other
// work-groups of the same launch may have folded into them.
__device__ __forceinline__ void close_state(MeshState* p)
{
    MeshState m = *p;
    if (!m.active) return;
    m.maxd_cur = __hip_atomic_load(&p->maxd_cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    m.acc_cur = __hip_atomic_load(&p->acc_cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    m.s += 1;
    m.maxd_last = m.maxd_cur;
    m.acc_last = m.acc_cur;
    m.acc_total += m.acc_cur;
    m.maxd_cur = 0;
    m.acc_cur = 0;
    const double last = __longlong_as_double(static_cast<long long>(m.maxd_last));
    m.active = (m.s < m.iters) && !(m.tol2 > 0.0 && last < m.tol2);
    *p = m;
}

// Counters of a tile launch, one 128-byte line each: [0] XCDs whose groups
// are all done, [1..8] one tile counter per XCD, [9..16] groups done per
// XCD; then (launches over one mesh) one slot per work-group for its
// displacement maximum and accepted count (two u64).
constexpr int kSchedStride = 32;                    // one 128-byte line per counter
constexpr int kSchedCounters = 17;
constexpr int kTileMaxGroups = 8 * 32 * 8;           // 8 XCDs x 32 CUs x at most 8 groups per CU
constexpr int kTileSlotsAt = kSchedCounters * kSchedStride;   // int offset of the slots
constexpr int kTileSchedInts = kTileSlotsAt + 4 * kTileMaxGroups;

// Work-item 0 of a group counts the group done and learns whether it is the
// launch's last: the groups of each XCD count on their own line and the last
// of them counts the XCD on the launch's line, so no line takes more than
// gridDim.x / 8 atomics (atomics on one address are serialised).  The
// launch's grid is a multiple of 8, group g on XCD g % 8.  The group's
// earlier device-scope writes are performed before its count (the
// work-group-scope release waits for them).
// Launches of at most kDirectFoldGroups groups count on the launch's line
// alone and fold straight into the state: so few atomics cost less than
// the longer chain of the two-level count and the slots.
constexpr int kDirectFoldGroups = 64;

__device__ __forceinline__ bool count_group_done(int32_t* sched)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (static_cast<int>(gridDim.x) <= kDirectFoldGroups)
        return __hip_atomic_fetch_add(sched, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
               static_cast<int>(gridDim.x) - 1;
    const int xcd = static_cast<int>(blockIdx.x & 7), per_xcd = static_cast<int>(gridDim.x >> 3);
    const int b = __hip_atomic_fetch_add(sched + kSchedStride * (9 + xcd), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (b != per_xcd - 1) return false;
    return __hip_atomic_fetch_add(sched, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 7;
}

// The launch's last group leaves the counters zeroed for the next launch.
__device__ __forceinline__ void reset_sched(int32_t* sched)
{
    if (threadIdx.x < kSchedCounters)
        __hip_atomic_store(sched + kSchedStride * threadIdx.x, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A launch over one mesh folds its work-groups' displacement maxima and
// accepted counts through per-group slots: each group writes its own slot
// (device-scope stores, performed before its count, as the folds below
// are), and the last group to finish folds every slot into the mesh's state
// with one atomic pair.  Thousands of atomics on the state's one address,
// which the device serialises, become one pair per launch.  (A launch of at
// most kDirectFoldGroups groups folds straight into the state, and counts
// its groups only when the caller needs the last one.)  d2: the
// work-item's maximum; acc: its wave's count (the same on every lane).
// Returns, on every work-item, whether the group was the launch's last
// (always false for a direct fold without NEED_LAST); that group has also
// zeroed the launch's counters.
template <int BS, bool NEED_LAST>
__device__ __forceinline__ bool fold_through_slots(int32_t* sched, MeshState* ms, double d2, unsigned long long acc)
{
    __shared__ double s_d2[BS / 64];
    __shared__ unsigned long long s_acc[BS / 64];
    __shared__ int s_last;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    unsigned long long* const slots = reinterpret_cast<unsigned long long*>(sched + kTileSlotsAt);
    auto block_fold = [&](double& m, unsigned long long& c) {
        for (int off = 32; off > 0; off >>= 1) {
            const double t = __shfl_xor(m, off);
            m = t > m ? t : m;
            c += __shfl_xor(c, off);
        }
        __syncthreads();   // s_d2 / s_acc free
        if (lane == 0) {
            s_d2[wv] = m;
            s_acc[wv] = c;
        }
        __syncthreads();
        m = s_d2[0];
        c = s_acc[0];
        for (int q = 1; q < BS / 64; ++q) {
            m = s_d2[q] > m ? s_d2[q] : m;
            c += s_acc[q];
        }
    };
    unsigned long long c = lane == 0 ? acc : 0ull;   // one lane per wave contributes
    block_fold(d2, c);
    const bool direct = static_cast<int>(gridDim.x) <= kDirectFoldGroups;
    if (direct && !NEED_LAST) {
        if (tid == 0) {
            if (d2 > 0.0) atomicMax(&ms->maxd_cur, static_cast<unsigned long long>(__double_as_longlong(d2)));
            if (c) atomicAdd(&ms->acc_cur, c);
        }
        return false;
    }
    if (tid == 0) {
        if (direct) {
            if (d2 > 0.0) atomicMax(&ms->maxd_cur, static_cast<unsigned long long>(__double_as_longlong(d2)));
            if (c) atomicAdd(&ms->acc_cur, c);
        } else {
            __hip_atomic_store(slots + 2 * blockIdx.x, static_cast<unsigned long long>(__double_as_longlong(d2)),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(slots + 2 * blockIdx.x + 1, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_last = count_group_done(sched);
    }
    __syncthreads();
    if (!s_last) return false;
    if (direct) {
        reset_sched(sched);
        return true;
    }
    double m = 0.0;
    unsigned long long cnt = 0;
    for (int g = tid; g < static_cast<int>(gridDim.x); g += BS) {
        const double mg = __longlong_as_double(static_cast<long long>(
            __hip_atomic_load(slots + 2 * g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
        m = mg > m ? mg : m;
        cnt += __hip_atomic_load(slots + 2 * g + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    block_fold(m, cnt);
    if (tid == 0) {
        if (m > 0.0) atomicMax(&ms->maxd_cur, static_cast<unsigned long long>(__double_as_longlong(m)));
        if (cnt) atomicAdd(&ms->acc_cur, cnt);
    }
    reset_sched(sched);
    return true;
}

// The last work-group of a launch to finish closes the sweep of states[0..n)
// and zeroes the launch's counters for the next launch.  A group's folds into the
// sweep state are device-scope atomics made by its first work-item; the
// work-group-scope release waits until they have completed, so they are
// performed before the group's count.  The closing group reads the folds
// with device-scope atomic loads after it has seen every count.  No
// device-scope release or acquire is needed: those would write back or
// invalidate the XCD's L2, once per work-group.
template <int BS>
__device__ __forceinline__ void close_launch(int32_t* sched, MeshState* states, int32_t n)
{
    __shared__ int s_last;
    __syncthreads();   // every work-item of the group is done with its tiles
    if (threadIdx.x == 0) s_last = count_group_done(sched);
    __syncthreads();
    if (!s_last) return;
    for (int i = threadIdx.x; i < n; i += BS) close_state(states + i);
    reset_sched(sched);
}

// One tile of the tile path: everything a work-group needs to sweep it, with
// absolute pointers so that tiles of many meshes can share one launch.
struct alignas(16) TileWork {
    const void* X;                  // the mesh's buffer pair (double or float): X[0] at X, X[1] at X + 2n
    const int32_t* halo;            // halo node ids (mesh device labels)
    const uint64_t* rows;           // neighbour rows in local indices, 4 x u16 per word
    const uint64_t* tris;           // triangle entries: 3 x u16 local indices, stored order
    const uint16_t* rr;             // T + 1 row starts within `rows`: node i's row is rr[i] .. rr[i+1]
    int32_t own_start, nown;        // own nodes: mesh device labels [own_start, own_start + nown)
    int32_t halo_cnt, tri_cnt;
    int32_t row_words, mesh;        // 64-bit row words; index of the mesh's MeshState
    int64_t n;                      // the mesh's node count (buffer stride)
};
static_assert(sizeof(TileWork) == 80, "TileWork layout");

constexpr int kMaxTileClasses = 32;   // colour classes the Form B tile path takes at most

// One mesh prepared for sweeping: free nodes occupy [0, n_free) in the
// device order, fixed nodes [n_free, n).
struct DevMesh {
    unsigned char* block = nullptr;   // one allocation; every array below is carved from it
    // Set before setup to carve the arrays from a region of a larger block
    // instead (a batch's; not owned, `block` stays null); at least
    // mesh_block_bytes() long.
    unsigned char* carve = nullptr;
    size_t carve_bytes = 0;
    // Set before setup to take the setup's temporaries from a region too
    // (not owned), at least setup_scratch_bytes() long.
    unsigned char* scratch_carve = nullptr;
    size_t scratch_carve_bytes = 0;
    // Set before prepare_mesh to carve everything from one caller-owned
    // region of region_bytes: the mesh's arrays first (carve), then the
    // setup's temporaries (scratch_carve); region_after more bytes must fit
    // after the arrays once setup is done (prepare_mesh fails with
    // SL_ENOMEM before any work otherwise).
    unsigned char* region = nullptr;
    size_t region_bytes = 0;
    size_t region_after = 0;
    int32_t n = 0, n_free = 0, n_tris = 0;
    int64_t nnz_free = 0, ninc_free = 0;
    int32_t max_deg = 0, max_inc = 0;
    int32_t layout = SL_AOS;
    int32_t n_colors = 0;
    int32_t* perm = nullptr;        // [n]  device label -> caller label
    int32_t* new_of_old = nullptr;  // [n]  caller label -> device label
    int32_t* row_ptr = nullptr;     // [n_free+1]
    int32_t* nbr = nullptr;         // [nnz_free] device labels (node path)
    int32_t* fan_ptr = nullptr;     // [n_free+1]
    uint16_t* fan = nullptr;        // [ninc_free] (node path), grouped by stored position where fan_split is set
    uint32_t* fan_split = nullptr;  // [n_free] (node path, below kGroupFansBelow free nodes): the groups' bounds, or kFanUngrouped
    int32_t color_start_h[130] = {0};    // colour class c: device labels [cs[c], cs[c+1])
    int32_t precision = SL_F64;          // element type of X: double, or float for SL_F32
    void* X[2] = {nullptr, nullptr};     // one block of 4n elements: X[1] = X[0] + 2n;
                                         // AoS (x,y pairs) or SoA (x[n] then y[n]) inside each
    bool resident = false;               // Form A on the resident kernel (node-path arrays built)
    int32_t lane_width = 0;              // node path: > 0 sweeps with lane groups of this width
    // Tile path: Form A, or Form B on colour-class tiles (n_tile_classes > 0)
    int32_t tile_nodes = 0;              // 0: tile path not built
    int32_t n_tile_classes = 0;          // Form B: class c sweeps tiles [class_tile_h[c], class_tile_h[c+1])
    int32_t class_tile_h[kMaxTileClasses + 1] = {0};
    bool class_tiles_ok = false;         // set before setup: Form B may take colour-class tiles
    int32_t n_tiles = 0;
    int32_t halo_max = 0;                // largest halo over tiles
    int32_t rows_max = 0;                // largest row segment (u16 entries, padded to 4) over tiles
    int32_t fans_max = 0;                // class tiles: longest fan list over tiles
    TileWork* work = nullptr;            // [n_tiles]
    unsigned char* tile_data = nullptr;  // one contiguous record per tile: row offsets, halo, rows, triangles
};

// Frees every device array of m (stream-ordered).
void devmesh_free(DevMesh& m, hipStream_t st);

// The sweep kernel a set-up mesh runs (sl_report::kernel_used).
inline int32_t kernel_used(const DevMesh& m)
{
    if (m.resident) return SL_KERNEL_RESIDENT;
    if (m.tile_nodes > 0) return SL_KERNEL_TILE;
    return m.lane_width > 0 ? SL_KERNEL_LANES : SL_KERNEL_NODE;
}

struct SetupArgs {
    const double* coords;   // caller layout, n x 2
    int32_t n;
    const int32_t* nbr_ptr;
    const int32_t* nbr_idx;
    const int32_t* tri_ptr;
    const int32_t* tri_idx;
    const int32_t* tris;
    int32_t n_tris;
    const uint8_t* boundary;
    int64_t nnz, ninc;      // nbr_ptr[n], tri_ptr[n] (read by the caller of setup)
};

// Builds the tile path (tile_nodes free nodes per tile) and writes the tile
// list to m.work with MeshState index `mesh`: tiles of consecutive free
// nodes (Form A), or, with `classes`, tiles inside each colour class of
// m.color_start_h (Form B; at most kMaxTileClasses classes).  Leaves
// m.tile_nodes = 0 (node path) when the mesh does not fit it.
sl_status build_tiles(const SetupArgs& a, DevMesh& m, int tile_nodes, int mesh, hipStream_t st, Arena& persist,
                      Arena& scratch, bool classes = false);
// Bytes build_tiles takes from `persist` for a mesh of at most n free nodes
// with at most nnz neighbour entries and ninc incidences, and from `scratch`.
size_t tile_bytes(int64_t n, int64_t nnz, int64_t ninc, int tile_nodes, bool classes = false);
size_t tile_scratch_bytes();
// LDS bytes of one sweep work-group, and the most a work-group may use.
size_t tile_lds_bytes(int tile_nodes, int halo_cap, int rows_cap, int32_t precision);
constexpr size_t kTileLdsLimit = 160 * 1024 - 4096;

// Validates the inputs, orders the nodes, builds rows and fans (node path)
// or tiles (tile path, MeshState index `mesh`) and fills both coordinate
// buffers.  Synchronises `st` (the validation result is needed).
sl_status setup_mesh(const SetupArgs& a, const sl_options& o, DevMesh& m, int32_t mesh, hipStream_t st);
// Bytes of the one allocation setup_mesh makes for a mesh's own arrays,
// from bounds known before validation (n nodes, nnz and ninc CSR entries).
// class_tiles_ok: as DevMesh::class_tiles_ok.
size_t mesh_block_bytes(int32_t n, int64_t nnz, int64_t ninc, const sl_options& o, bool class_tiles_ok = false);
// Bytes of setup_mesh's temporaries for a mesh of n nodes.
size_t setup_scratch_bytes(int32_t n);

// Device arrays of one caller mesh.
struct MeshInput {
    const double* coords;
    int32_t n;
    const int32_t* nbr_ptr;
    const int32_t* nbr_idx;
    const int32_t* tri_ptr;
    const int32_t* tri_idx;
    const int32_t* tris;
    int32_t n_tris;
    const uint8_t* boundary;
    // nbr_ptr[0], nbr_ptr[n], tri_ptr[0], tri_ptr[n] when the caller already
    // read them on the host (the arrays came from host memory)
    bool ends_known = false;
    int32_t ends[4] = {0, 0, 0, 0};
};

// Argument checks, then setup_mesh.
sl_status prepare_mesh(const MeshInput& in, const sl_options& o, int32_t mesh, DevMesh& m, hipStream_t st);
sl_status check_options(const sl_options& o);
void keep_pool_warm();

// Copies between caller host memory and the device through pinned staging
// buffers.  copy_to_device returns once the copy is enqueued on `st` (the
// source may be reused at once); copy_to_host returns when dst holds the
// data (it waits for the work enqueued on `st` before it).
sl_status copy_to_device(void* dst, const void* src, size_t bytes, hipStream_t st);
sl_status copy_to_host(void* dst, const void* src, size_t bytes, hipStream_t st);

// Non-blocking streams of default priority from a per-device pool kept for
// the life of the process (creating a stream costs hundreds of
// microseconds).  A stream may go back with work still queued on it; the
// next user's work then runs after that work.
sl_status take_stream(hipStream_t* st);
void give_stream(hipStream_t st);
struct PooledStream {
    hipStream_t s = nullptr;
    PooledStream() = default;
    PooledStream(const PooledStream&) = delete;
    PooledStream& operator=(const PooledStream&) = delete;
    ~PooledStream()
    {
        if (s) give_stream(s);
    }
    sl_status init() { return take_stream(&s); }
};

// One caller mesh's host arrays copied into a single device allocation
// (nnz = nbr_ptr[n], ninc = tri_ptr[n], already read by the caller), with
// `extra` more bytes left in `ar` for the caller.  release() frees it,
// stream-ordered.
struct DevInputs {
    Arena ar;
    double* coords = nullptr;
    int32_t *nbr_ptr = nullptr, *nbr_idx = nullptr, *tri_ptr = nullptr, *tri_idx = nullptr, *tris = nullptr;
    uint8_t* boundary = nullptr;
    void release(hipStream_t st) { ar.release(st); }
};
sl_status upload_inputs(const sl_mesh_desc& d, int64_t nnz, int64_t ninc, size_t extra, DevInputs& out,
                        hipStream_t st);

// Uploads one caller mesh (host arrays) on `st` and prepares it; the
// uploaded inputs are released once the device copy is built.
sl_status upload_and_prepare(const sl_mesh_desc& d, const sl_options& o, int32_t mesh, DevMesh& m, hipStream_t st);

// Launch shapes that sl_autotune chose for a device (zeros: none chosen).
struct TunedShape {
    int32_t tile_nodes, wg_per_cu, block_size, lane_width;
};
TunedShape tuned_shape();                       // of the current device
void set_tuned_shape(const TunedShape& t);      // for the current device
void clear_tuned_shape();
// Option value if set, else the tuned value, else the built-in default
// (512 nodes per tile; 0 = as many work-groups per CU as fit, at most 4;
// 0 = node-kernel default block).
int32_t resolve_tile_nodes(const sl_options& o);
int32_t resolve_wg_per_cu(const sl_options& o);
int32_t resolve_block_size(const sl_options& o);
int32_t resolve_lane_width(const sl_options& o);   // lane groups: option, else tuned, else 8

// Writes the positions of buffer `src` -- or, when `runs` is given, of
// buffer (runs->s % 2), read on the device -- back to the caller's layout
// and order.
sl_status unpermute_coords(const DevMesh& m, int src, double* coords_out, hipStream_t st,
                           const MeshState* runs = nullptr);

// Unpermutes per-sweep accept bits (device order, 64-bit words) into the
// caller's byte layout; sweeps >= state->s (the sweeps run, read on the
// device) are zeroed.
sl_status unpermute_flags(const DevMesh& m, const uint64_t* bits, int32_t iterations, const MeshState* state,
                          uint8_t* flags_out, hipStream_t st);

// Queues one Jacobi or coloured sweep of a single mesh on the node path
// (Form A reads X[parity], writes X[parity^1]; Form B works in place in
// X[0]).  Skipped on the device when the mesh's state is inactive.  bits:
// nullable accept bits of this sweep (device labels, 64-bit words).  close:
// the sweep's last launch also closes it (no k_advance after it); else the
// caller closes it.
sl_status launch_sweep_nodes(const DevMesh& m, int32_t parity, int32_t form, int32_t accept, int32_t block,
                             MeshState* state, uint64_t* bits, int32_t* sched, hipStream_t st, bool close = false);

// Queues one sweep of every tile in work[0..n_work) (any number of meshes,
// all reading X[parity]).  bits: nullable, single-mesh runs only.
struct TileLaunch {
    const TileWork* work;
    int32_t n_work;
    int32_t tile_nodes;
    int32_t halo_cap, rows_cap;
    int32_t layout, accept;
    MeshState* states;
    int32_t wg_per_cu;          // 0: as many as fit, at most 4
    int32_t exit_if_inactive;   // 1: every tile is of one mesh; a launch on it returns at once once it stops
    int32_t precision;          // SL_F64 or SL_F32: every mesh of the list has it
    // kTileSchedInts counters, zeroed before the first launch on them; each
    // launch leaves them zeroed (launches sharing them must not overlap)
    int32_t* sched;
    // > 0: the launch's last work-group closes the sweep of
    // states[0..n_close), in place of a launch_advance after it
    int32_t n_close;
    // 1: every tile is of one mesh; its work-groups hand their folds to the
    // closing group through per-group slots instead of atomics on the one
    // state (atomics on one address are serialised)
    int32_t one_mesh = 0;
};
sl_status launch_sweep_tiles(const TileLaunch& L, int32_t parity, uint64_t* bits, hipStream_t st);
// Queues one class launch of Form B on colour-class tiles (L.work: the
// class's tiles, whose `tris` are u16 fan entries; fans_cap: the longest fan
// list of a tile), in place in buffer 0.  L.n_close > 0 on the last class.
sl_status launch_sweep_class(const TileLaunch& L, int32_t fans_cap, uint64_t* bits, hipStream_t st);
// LDS bytes of one class-tile work-group.
size_t class_lds_bytes(int tile_nodes, int halo_cap, int rows_cap, int fans_cap);

// Resident meshes (Form A, double precision): one work-group runs all the
// sweeps of one mesh with its coordinates, rows and fans in LDS.  One entry
// per mesh, in device memory; the launch's dynamic LDS is the largest
// resident_lds_bytes of the list.  The mesh's state must start at s = 0;
// the kernel leaves it as the sweep-by-sweep closes would, inactive.
constexpr int kResidentClasses = 32;
struct ResidentArgs {
    double* X;                  // X[0] at X, X[1] at X + 2n (the mesh's layout)
    const int32_t* row_ptr;     // [n_free + 1]
    const int32_t* nbr;         // [nnz] device labels
    const int32_t* fan_ptr;     // [n_free + 1]
    const uint16_t* fan;        // [ninc]
    int32_t n, n_free, nnz, ninc;
    int32_t iters;              // sweeps to run at most
    double tol2;                // > 0: stop after a sweep with max |dx|^2 < tol2
    MeshState* state;
    uint64_t* bits;             // nullable: sweep s's accept bits at bits + s * words
    int64_t words;
    int32_t in_place;           // 1: Form B, one buffer, the colour classes below in order
    int32_t n_classes;
    int32_t class_start[kResidentClasses + 1];   // class c: device labels [class_start[c], class_start[c+1])
};
constexpr size_t kResidentLdsLimit = 160 * 1024 - 1024;
size_t resident_lds_bytes(int64_t n, int64_t n_free, int64_t nnz, int64_t ninc, bool in_place);
// Whether a mesh of n nodes and nnz, ninc CSR entries in all (bounds of its
// free rows and fans) fits the resident kernel (Form B keeps one buffer).
bool resident_fits(int64_t n, int64_t nnz, int64_t ninc, bool in_place);
// Fills the Form B part of a (the colour classes of m); SL_EINVAL when m
// has more than kResidentClasses classes.
sl_status resident_classes(const DevMesh& m, bool in_place, ResidentArgs& a);
sl_status launch_sweep_resident(const ResidentArgs* list, int32_t count, size_t lds, int32_t layout,
                                int32_t accept, hipStream_t st);

// Closes a sweep for states[0..n): counts it for the active meshes and
// decides whether each runs the next one.
sl_status launch_advance(MeshState* states, int32_t n, hipStream_t st);

// Work-group count of a tile launch (persistent work-groups, XCD-aware).
int tile_grid(int n_work, int tile_nodes, int halo_cap, int rows_cap, int wg_per_cu, int32_t precision);

// Exclusive scan of n int32 values; out[n] receives the total (out has n+1).
// Temporaries come from `scratch` when given (and are given back before
// the call returns), else from the allocator.
sl_status scan_exclusive(const int32_t* in, int32_t* out, int64_t n, hipStream_t st, Arena* scratch = nullptr);

}  // namespace sl
