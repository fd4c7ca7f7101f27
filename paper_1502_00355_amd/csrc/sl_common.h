// Internal declarations of the smartlap HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

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
    VE_COORD = 1u << 2,     // non-finite coordinate                            -> EINVAL
    VE_SELF = 1u << 3,      // node lists itself as a neighbour                 -> ETOPO
    VE_TRIREP = 1u << 4,    // triangle with a repeated vertex                  -> ETOPO
    VE_NOTIN = 1u << 5,     // incident triangle does not contain its node      -> ETOPO
    VE_MISSING = 1u << 6,   // triangle vertex missing from the neighbour row   -> ETOPO
    VE_EMPTY = 1u << 7,     // free node without neighbours                     -> ETOPO
    VE_VALENCE = 1u << 8,   // free node valence > 127                          -> ETOPO
    VE_ASYM = 1u << 9,      // neighbour rows not symmetric (coloured form)     -> ETOPO
};
constexpr int kMaxValence = 127;   // 7-bit neighbour slots in a fan entry

// Statistics gathered during validation.
struct ValStats {
    uint32_t err;
    int32_t n_free;
    int32_t max_deg_free;
    int32_t max_inc_free;
};

// ------------------------------------------------------- device workspace --

// One mesh prepared for sweeping: free nodes occupy [0, n_free) in the
// device order, fixed nodes [n_free, n).  Neighbour rows and fans exist for
// free nodes only and are in device labels.
struct DevMesh {
    int32_t n = 0, n_free = 0, n_tris = 0;
    int64_t nnz_free = 0, ninc_free = 0;
    int32_t max_deg = 0, max_inc = 0;
    int32_t layout = SL_AOS;
    int32_t n_colors = 0;
    int32_t* perm = nullptr;        // [n]  device label -> caller label
    int32_t* new_of_old = nullptr;  // [n]  caller label -> device label
    int32_t* row_ptr = nullptr;     // [n_free+1]
    int32_t* nbr = nullptr;         // [nnz_free] device labels
    int32_t* fan_ptr = nullptr;     // [n_free+1]
    uint16_t* fan = nullptr;        // [ninc_free]
    int32_t color_start_h[130] = {0};    // colour class c: device labels [cs[c], cs[c+1])
    double* X[2] = {nullptr, nullptr};   // AoS: 2n doubles; SoA: x[n] then y[n]
    // Tile path (Form A): free nodes in tiles of tile_nodes consecutive device
    // labels; per tile a halo list, local neighbour rows and a local triangle list.
    int32_t tile_nodes = 0;              // 0: tile path not built
    int32_t n_tiles = 0;
    int32_t halo_max = 0;                // largest halo over tiles
    int32_t rows_max = 0;                // largest row segment (u16 entries, padded to 4) over tiles
    int4* tile_meta = nullptr;           // [n_tiles] {halo_off, halo_cnt, tri_off, tri_cnt}
    int2* tile_rows = nullptr;           // [n_tiles] {row segment offset (multiple of 4), padded length}
    int32_t* halo = nullptr;             // [sum halo] device labels
    uint16_t* nbr_loc = nullptr;         // tile row segments: local index of each neighbour, row order
    uint16_t* row_rel = nullptr;         // [n_tiles * (tile_nodes+1)] row start inside the tile's segment
    uint64_t* tri_loc = nullptr;         // [sum tri] 3 x 16-bit local vertex indices, stored order
};

// Frees every device array of m (stream-ordered).
void devmesh_free(DevMesh& m, hipStream_t st);

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

// Builds the tile path for Form A (tile_nodes free nodes per tile).  Leaves
// m.tile_nodes = 0 (node path) when the mesh does not fit it.
sl_status build_tiles(const SetupArgs& a, DevMesh& m, int tile_nodes, hipStream_t st);

// Validates the inputs, orders the nodes, builds rows and fans and fills both
// coordinate buffers.  Synchronises `st` (the validation result is needed).
sl_status setup_mesh(const SetupArgs& a, const sl_options& o, DevMesh& m, hipStream_t st);

// Writes the positions of buffer `src` back to the caller's layout and order.
sl_status unpermute_coords(const DevMesh& m, int src, double* coords_out, hipStream_t st);

// Unpermutes per-sweep accept bits (device order, 64-bit words) into the
// caller's byte layout; sweeps >= iterations_run are zeroed.
sl_status unpermute_flags(const DevMesh& m, const uint64_t* bits, int32_t iterations, int32_t iterations_run,
                          uint8_t* flags_out, hipStream_t st);

// Per-sweep outputs of the sweep kernels.
struct SweepOut {
    uint64_t* maxd;            // [iterations] bit pattern of the largest squared displacement
    unsigned long long* acc;   // [iterations] accepted count
    uint64_t* bits;            // nullable: [iterations][words] accept bits, device order
    int64_t words;             // 64-bit words per sweep
};

// Queues sweep `s` of the Jacobi form (reads X[s%2], writes X[(s+1)%2]) or
// of the coloured form (in place in X[0]); skipped on the device when the
// previous sweep's displacement is below tol2 (tol2 > 0).
sl_status launch_sweep(const DevMesh& m, int32_t s, int32_t form, int32_t accept, int32_t block, double tol2,
                       const SweepOut& out, hipStream_t st);

// Queues sweep `s` on the tile path (Form A).
sl_status launch_sweep_tiles(const DevMesh& m, int32_t s, int32_t accept, double tol2, const SweepOut& out,
                             hipStream_t st);

// Exclusive scan of n int32 values; out[n] receives the total (out has n+1).
sl_status scan_exclusive(const int32_t* in, int32_t* out, int64_t n, hipStream_t st);

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

inline int div_up(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

}  // namespace sl
