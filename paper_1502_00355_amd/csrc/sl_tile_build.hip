// Tile build of the Form A (Jacobi) sweep.
//
// The free nodes (device order: Hilbert cells) are cut into tiles of T
// consecutive labels; the sweep runs one work-group per tile.  The tiles are
// built on the device: one work-group per tile collects the halo (every
// node an own node reads) and the incident triangles in LDS, sorts and
// deduplicates them, and rewrites rows and triangles in tile-local indices
// (own nodes 0..T-1, halo nodes T..T+H-1).
#include <algorithm>
#include <climits>
#include <cstdlib>

#include "sl_common.h"

namespace sl {

namespace {

constexpr int kTileMaxDeg = 16;                       // neighbour entries per own node, on average over a tile
constexpr int kBuildBS = 256;

// ------------------------------------------------------ block primitives --

template <int BS>
__device__ int block_excl_scan(int v, int* total, int* s_warp)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(x, off);
        if (lane >= off) x += t;
    }
    if (lane == 63) s_warp[w] = x;
    __syncthreads();
    int base = 0, tot = 0;
    for (int q = 0; q < BS / 64; ++q) {
        const int c = s_warp[q];
        if (q < w) base += c;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

__device__ __forceinline__ int pow2ceil(int n)
{
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Bitonic sort of a[0..n) (padded to P, a power of two, with INT_MAX).
template <int BS>
__device__ void block_sort(int32_t* a, int n, int P)
{
    for (int i = n + threadIdx.x; i < P; i += BS) a[i] = INT_MAX;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += BS) {
                const int l = i ^ j;
                if (l > i) {
                    const int32_t x = a[i], y = a[l];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) { a[i] = y; a[l] = x; }
                }
            }
            __syncthreads();
        }
    }
}

// In-place removal of duplicates from the sorted a[0..n); returns the count.
template <int BS>
__device__ int block_unique(int32_t* a, int n, int* s_warp)
{
    int out = 0;
    for (int base = 0; base < n; base += BS) {
        const int i = base + threadIdx.x;
        int32_t v = 0;
        int f = 0;
        if (i < n) {
            v = a[i];
            f = (i == 0) || (v != a[i - 1]);
        }
        int tot;
        const int pos = block_excl_scan<BS>(f, &tot, s_warp);
        if (f) a[out + pos] = v;
        out += tot;
        __syncthreads();
    }
    return out;
}

__device__ __forceinline__ int lower_bound_lds(const int32_t* a, int n, int32_t v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------ tile build --

struct TileBuildArgs {
    const int32_t* perm;
    const int32_t* new_of_old;
    const int32_t* nbr_ptr;
    const int32_t* nbr_idx;
    const int32_t* tri_ptr;
    const int32_t* tri_idx;
    const int32_t* tris;
    const int32_t* row_ptr;    // device-order rows of the free nodes
    const int32_t* fan_ptr;    // device-order incidence offsets of the free nodes
    int32_t n_free;
    int32_t mesh;              // MeshState index written into the descriptors
    int64_t n;
    const void* X;
    int32_t* halo;             // [nnz_free]: tile k writes at row_ptr[k0] (halo <= row entries)
    uint16_t* nbr_loc;         // tile k writes at align4(row_ptr[k0]) + 8k (segments never overlap)
    uint32_t* row_rel;         // [n_tiles * T]
    uint64_t* tri_loc;         // [ninc_free]: tile k writes at fan_ptr[k0] (kept <= incidences)
    TileWork* work;            // [n_tiles]
    int32_t* mx;               // {largest halo, largest padded row segment}
    int32_t* err;
};

__host__ __device__ __forceinline__ int64_t row_seg_off(int32_t row_start, int32_t tile)
{
    return ((static_cast<int64_t>(row_start) + 3) & ~int64_t(3)) + 8 * static_cast<int64_t>(tile);
}

// One work-group per tile, in one pass: every output of tile k goes to a
// place fixed by the row and incidence offsets of its first node, so no
// tile needs another's counts.  Halo: every neighbour of an own node that
// is not own, sorted and deduplicated.  Triangles: each triangle incident to
// an own node, listed once per tile by its own vertex of smallest label.
// Rows: the tile's neighbour rows in local indices, one segment padded to 4
// entries.
template <int T>
__global__ __launch_bounds__(kBuildBS) void k_tile_build(TileBuildArgs a)
{
    constexpr int BS = kBuildBS, CAP = T * kTileMaxDeg, NPT = T / BS;
    __shared__ int32_t hb[CAP];
    __shared__ int32_t s_cnt;
    __shared__ int32_t s_warp[BS / 64];
    const int tile = blockIdx.x;
    const int32_t k0 = tile * T;
    const int nown = min(T, a.n_free - k0);
    const int32_t rb = a.row_ptr[k0];
    const int32_t len = a.row_ptr[k0 + nown] - rb;
    if (len > CAP) {   // more neighbour entries than the halo staging holds: the mesh takes the node path
        if (threadIdx.x == 0) atomicOr(a.err, 2);
        return;
    }
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < nown; i += BS) {
        const int32_t o = a.perm[k0 + i];
        for (int32_t q = a.nbr_ptr[o]; q < a.nbr_ptr[o + 1]; ++q) {
            const int32_t jd = a.new_of_old[a.nbr_idx[q]];
            if (jd < k0 || jd >= k0 + nown) hb[atomicAdd(&s_cnt, 1)] = jd;
        }
    }
    __syncthreads();
    const int nh0 = s_cnt;
    block_sort<BS>(hb, nh0, pow2ceil(nh0));
    const int H = block_unique<BS>(hb, nh0, s_warp);

    // triangles kept by this tile: the listing node is the smallest own vertex
    auto kept = [&](int32_t o, int32_t kd, int64_t t) -> bool {
        for (int s = 0; s < 3; ++s) {
            const int32_t v = a.tris[3 * t + s];
            if (v == o) continue;
            const int32_t vd = a.new_of_old[v];
            if (vd >= k0 && vd < k0 + nown && vd < kd) return false;
        }
        return true;
    };
    auto local = [&](int32_t jd) -> int {
        if (jd >= k0 && jd < k0 + nown) return jd - k0;
        const int h = lower_bound_lds(hb, H, jd);
        if (h >= H || hb[h] != jd) { atomicOr(a.err, 1); return T; }
        return T + h;
    };
    const int32_t len4 = (len + 3) & ~3;
    int32_t* halo = a.halo + rb;
    uint16_t* seg = a.nbr_loc + row_seg_off(rb, tile);
    uint64_t* tri = a.tri_loc + a.fan_ptr[k0];
    for (int h = threadIdx.x; h < H; h += BS) halo[h] = hb[h];
    uint32_t* rr = a.row_rel + static_cast<int64_t>(tile) * T;
    for (int i = threadIdx.x; i < T; i += BS)
        rr[i] = static_cast<uint32_t>(a.row_ptr[k0 + min(i, nown)] - rb) |
                (static_cast<uint32_t>(a.row_ptr[k0 + min(i + 1, nown)] - rb) << 16);
    for (int j = len + threadIdx.x; j < len4; j += BS) seg[j] = 0;
    for (int m = 0; m < NPT; ++m) {
        const int i = m * BS + threadIdx.x;
        if (i >= nown) continue;
        const int32_t o = a.perm[k0 + i];
        const int32_t b = a.nbr_ptr[o], d = a.nbr_ptr[o + 1] - b, out = a.row_ptr[k0 + i] - rb;
        for (int j = 0; j < d; ++j) seg[out + j] = static_cast<uint16_t>(local(a.new_of_old[a.nbr_idx[b + j]]));
    }
    // triangles are listed in node order (work-item t lists nodes NPT*t ..
    // NPT*t+NPT-1), so that the lanes of a wave walking the list touch one
    // compact patch of nodes in LDS
    int c = 0;
    for (int m = 0; m < NPT; ++m) {
        const int i = NPT * threadIdx.x + m;
        if (i < nown) {
            const int32_t o = a.perm[k0 + i];
            for (int32_t q = a.tri_ptr[o]; q < a.tri_ptr[o + 1]; ++q) c += kept(o, k0 + i, a.tri_idx[q]);
        }
    }
    int R;
    int tpos = block_excl_scan<BS>(c, &R, s_warp);
    for (int m = 0; m < NPT; ++m) {
        const int i = NPT * threadIdx.x + m;
        if (i >= nown) continue;
        const int32_t o = a.perm[k0 + i];
        for (int32_t q = a.tri_ptr[o]; q < a.tri_ptr[o + 1]; ++q) {
            const int64_t t = a.tri_idx[q];
            if (!kept(o, k0 + i, t)) continue;
            uint64_t w = 0;
            for (int s = 0; s < 3; ++s)
                w |= static_cast<uint64_t>(local(a.new_of_old[a.tris[3 * t + s]])) << (16 * s);
            tri[tpos++] = w;
        }
    }
    if (threadIdx.x == 0) {
        TileWork w;
        w.X = a.X;
        w.halo = halo;
        w.rows = reinterpret_cast<const uint64_t*>(seg);
        w.tris = tri;
        w.rr = rr;
        w.own_start = k0;
        w.nown = nown;
        w.halo_cnt = H;
        w.tri_cnt = R;
        w.row_words = len4 >> 2;
        w.mesh = a.mesh;
        w.n = a.n;
        a.work[tile] = w;
        atomicMax(a.mx, H);
        atomicMax(a.mx + 1, len4);
    }
}

}  // namespace

size_t tile_bytes(int64_t n, int64_t nnz, int64_t ninc, int tile_nodes)
{
    if (tile_nodes != 256 && tile_nodes != 512) return 0;   // build_tiles takes nothing then
    const size_t nt = static_cast<size_t>(div_up(std::max<int64_t>(n, 1), tile_nodes));
    const size_t z = static_cast<size_t>(std::max<int64_t>(nnz, 1)), c = static_cast<size_t>(std::max<int64_t>(ninc, 1));
    return Arena::piece(sizeof(TileWork) * nt) + Arena::piece(4 * z) + Arena::piece(2 * (z + 8 * nt + 8)) +
           Arena::piece(4 * nt * tile_nodes) + Arena::piece(8 * c);
}

size_t tile_scratch_bytes() { return Arena::piece(3 * sizeof(int32_t)); }

sl_status build_tiles(const SetupArgs& a, DevMesh& m, int tile_nodes, int mesh, hipStream_t st, Arena& persist,
                      Arena& scratch)
{
    m.tile_nodes = 0;
    if ((tile_nodes != 256 && tile_nodes != 512) || m.n_free == 0) return SL_OK;
    const int T = tile_nodes;
    const int nt = div_up(m.n_free, T);
    const size_t pmark = persist.mark(), smark = scratch.mark();
    sl_status r = SL_OK;
    int32_t* flags = nullptr;   // {err, largest halo, largest row segment}
    if ((r = scratch.take(&flags, 3))) return r;
    SL_HIP(hipMemsetAsync(flags, 0, 3 * sizeof(int32_t), st));
    if ((r = persist.take(&m.work, nt)) || (r = persist.take(&m.halo, std::max<int64_t>(m.nnz_free, 1))) ||
        (r = persist.take(&m.nbr_loc, static_cast<size_t>(m.nnz_free) + 8 * static_cast<size_t>(nt) + 8)) ||
        (r = persist.take(&m.row_rel, static_cast<size_t>(nt) * T)) ||
        (r = persist.take(&m.tri_loc, std::max<int64_t>(m.ninc_free, 1))))
        return r;
    TileBuildArgs b{};
    b.perm = m.perm;
    b.new_of_old = m.new_of_old;
    b.nbr_ptr = a.nbr_ptr;
    b.nbr_idx = a.nbr_idx;
    b.tri_ptr = a.tri_ptr;
    b.tri_idx = a.tri_idx;
    b.tris = a.tris;
    b.row_ptr = m.row_ptr;
    b.fan_ptr = m.fan_ptr;
    b.n_free = m.n_free;
    b.mesh = mesh;
    b.n = m.n;
    b.X = m.X[0];
    b.halo = m.halo;
    b.nbr_loc = m.nbr_loc;
    b.row_rel = m.row_rel;
    b.tri_loc = m.tri_loc;
    b.work = m.work;
    b.err = flags;
    b.mx = flags + 1;
    if (T == 256) k_tile_build<256><<<nt, kBuildBS, 0, st>>>(b);
    else k_tile_build<512><<<nt, kBuildBS, 0, st>>>(b);
    SL_HIP(hipGetLastError());
    int32_t h[3] = {0, 0, 0};
    SL_HIP(hipMemcpyAsync(h, flags, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    scratch.rewind(smark);
    if (h[0] & 1) return fail(SL_ETOPO, "triangle vertex outside its tile's neighbourhood");
    // a tile denser than the staging holds, or a halo or row segment too big
    // for LDS: the node path, whose arrays reuse the tile arrays' room
    if ((h[0] & 2) || tile_lds_bytes(T, h[1], h[2], m.precision) > kTileLdsLimit) {
        m.work = nullptr;
        m.halo = nullptr;
        m.nbr_loc = nullptr;
        m.row_rel = nullptr;
        m.tri_loc = nullptr;
        persist.rewind(pmark);
        return SL_OK;
    }
    m.halo_max = h[1];
    m.rows_max = h[2];
    m.n_tiles = nt;
    m.tile_nodes = T;
    return SL_OK;
}

}  // namespace sl
