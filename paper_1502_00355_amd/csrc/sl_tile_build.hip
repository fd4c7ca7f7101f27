// Tile build of the tile sweeps.
//
// Form A (Jacobi): the free nodes (device order: Hilbert cells) are cut into
// tiles of T consecutive labels.  Form B (coloured, in place): each colour
// class (contiguous in device order, Hilbert cells inside) is cut into tiles
// of T consecutive labels.  The sweeps run one work-group per tile.  The
// tiles are built on the device: one work-group per tile collects the halo
// (every node an own node reads) in an LDS hash set and rewrites the rows in
// tile-local indices (own nodes 0..T-1, halo nodes T..T+H-1); a Form A tile
// lists its incident triangles in local indices, a colour-class tile gets
// one fan entry per incidence instead.
#include <algorithm>
#include <climits>
#include <cstdlib>

#include "sl_common.h"

namespace sl {

namespace {

constexpr int kTileMaxDeg = 16;   // row entries, and incidences, per own node on average over a tile
constexpr int kBuildBS = 256;
constexpr int kBuildU = 4;        // entries a work-item takes per chunk: their gathers are in flight together

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

// Open-addressing set of node labels in LDS (-1 = empty slot), linear
// probing from the label's low bits: halo labels come in runs of nearby
// labels, which then land in nearby slots with few collisions.  A
// colour-class tile's halo is a run in each of the other classes' label
// ranges, runs whose low bits overlap: MIX starts the probe at a
// multiplicative hash of the label instead.  Probing stops after HS slots,
// so a full table reports failure instead of looping.
template <int HS, bool MIX>
__device__ __forceinline__ int set_home(int32_t key)
{
    if (!MIX) return key & (HS - 1);
    return static_cast<int>((static_cast<uint32_t>(key) * 2654435761u) >> (32 - __builtin_ctz(HS)));
}

template <int HS, bool MIX>
__device__ bool set_insert(int32_t* tab, int32_t key)
{
    int s = set_home<HS, MIX>(key);
    for (int p = 0; p < HS; ++p) {
        const int32_t cur = tab[s];
        if (cur == key) return true;
        if (cur == -1) {
            const int32_t prev = atomicCAS(&tab[s], -1, key);
            if (prev == -1 || prev == key) return true;
        }
        s = (s + 1) & (HS - 1);
    }
    return false;
}

template <int HS, bool MIX>
__device__ int set_find(const int32_t* tab, int32_t key)
{
    int s = set_home<HS, MIX>(key);
    for (int p = 0; p < HS; ++p) {
        const int32_t cur = tab[s];
        if (cur == key) return s;
        if (cur == -1) return -1;
        s = (s + 1) & (HS - 1);
    }
    return -1;
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
    unsigned char* data;       // tile k's record at tile_record(k): row offsets, halo, rows, triangles
    TileWork* work;            // [n_tiles]
    int32_t* err;
    // 0: tile k holds free nodes [k T, k T + T).  Else colour-class tiles:
    // class c (device labels [cls_start[c], cls_start[c+1])) is cut into
    // tiles [cls_tile[c], cls_tile[c+1]) of T consecutive labels, the last
    // one of a class possibly shorter
    int32_t n_class;
    int32_t cls_start[kMaxTileClasses + 1];
    int32_t cls_tile[kMaxTileClasses + 1];
};

__host__ __device__ __forceinline__ int64_t align16(int64_t b) { return (b + 15) & ~int64_t(15); }

// Byte offset of tile k's record, from the row and incidence offsets of its
// first node.  A record holds T + 1 u16 row starts (node i's row is entries
// start[i] .. start[i+1] of the rows), then room for len halo ids (len = the
// tile's row entries; the halo is never longer), the rows (len rounded up to
// 4 u16), and flen triangle words (flen = its incidences, an upper bound of
// its triangles), each part 16-byte aligned: at most 2T + 6 len + 8 flen +
// 48 bytes, which the next record's offset leaves.  One record per tile
// keeps the static data a tile reads in one stream.
__host__ __device__ __forceinline__ int64_t tile_record(int32_t row_start, int32_t fan_start, int32_t tile, int T)
{
    return static_cast<int64_t>(tile) * (2 * T + 64) +
           align16(6 * static_cast<int64_t>(row_start) + 8 * static_cast<int64_t>(fan_start));
}
__host__ __device__ __forceinline__ int64_t halo_at(int T) { return align16(2 * static_cast<int64_t>(T) + 2); }

// A colour-class tile's record holds T + 1 u16 row starts, T + 1 u16 fan
// starts (node i's fan entries are start[i] .. start[i+1]), T u32 splits of
// each fan by stored position (low half: entries with p = 0, high half:
// those with p <= 1), room for len halo ids, the rows (len rounded up to 4
// u16) and flen u16 fan entries, each part 16-byte aligned: at most 8T +
// 6 len + 2 flen + 100 bytes.
__host__ __device__ __forceinline__ int64_t class_record(int32_t row_start, int32_t fan_start, int32_t tile, int T)
{
    return static_cast<int64_t>(tile) * (8 * T + 128) +
           align16(6 * static_cast<int64_t>(row_start) + 2 * static_cast<int64_t>(fan_start));
}
__host__ __device__ __forceinline__ int64_t class_halo_at(int T) { return 2 * halo_at(T) + align16(4 * static_cast<int64_t>(T)); }

// One work-group per tile, in one pass: every output of tile k goes to a
// place fixed by the row and incidence offsets of its first node, so no
// tile needs another's counts.
//   Halo: every neighbour of an own node that is not own, once, in the
//   order of an LDS hash set (local index T + position).
//   Rows: the tile's neighbour rows in local indices, one segment padded to
//   4 entries.
//   Triangles: each triangle incident to an own node, listed once per tile,
//   by its own vertex of smallest label, in incidence order.
// The tile's row entries and incidences are walked as flat ranges, a few
// per work-item at a time, so the dependent gathers (entry -> neighbour or
// triangle -> device label) of different entries overlap.  An entry's own
// node is found from the owner of its 16-entry block, stepping forward over
// the node offsets (a node has at least one row entry); the small LDS
// footprint lets more tiles build at once.  Neither the halo order nor the triangle order
// changes a result: sums run over rows, minima are exact.
// CLS: a colour-class tile (Form B).  Its nodes are spread out (no two
// adjacent), so its halo is several times longer and the halo set has 8 T
// slots instead of 4 T; and instead of triangle words it gets one fan entry
// per incidence, in incidence order: the node's position p in the
// triangle's stored order and the row slots of the vertices at p+1 and
// p+2 (mod 3), p | slot << 2 | slot << 9, with the fan starts.
template <int T, bool CLS>
__global__ __launch_bounds__(kBuildBS) void k_tile_build(TileBuildArgs a)
{
    constexpr int HS = CLS ? 8 * T : 4 * T;
    constexpr int BS = kBuildBS, U = kBuildU, CAP = T * kTileMaxDeg, SPT = HS / BS;
    __shared__ int32_t htab[HS];
    __shared__ uint16_t hidx[HS];
    __shared__ uint16_t own[CAP / 16];   // owner of entries 16b, 16b+1, ... starts the search
    __shared__ int32_t s_nb[T], s_tb[T], s_rs[T + 1], s_fs[T + 1];
    __shared__ uint16_t s_seg[CLS ? CAP : 1];   // class tiles: the rows in local indices, for the slot search
    __shared__ int32_t s_warp[BS / 64];
    __shared__ int32_t s_full;
    const int tid = threadIdx.x;
    const int tile = blockIdx.x;
    int32_t k0 = tile * T, kend = a.n_free;
    if (a.n_class > 0) {
        int c = 0;
        while (c + 1 < a.n_class && tile >= a.cls_tile[c + 1]) ++c;
        k0 = a.cls_start[c] + (tile - a.cls_tile[c]) * T;
        kend = a.cls_start[c + 1];
    }
    const int nown = min(T, kend - k0);
    const int32_t rb = a.row_ptr[k0], fb = a.fan_ptr[k0];
    const int32_t len = a.row_ptr[k0 + nown] - rb, flen = a.fan_ptr[k0 + nown] - fb;
    if (len > CAP || flen > CAP) {   // denser than the LDS maps hold: the mesh takes the node path
        if (tid == 0) atomicOr(a.err, 2);
        return;
    }
    for (int s = tid; s < HS; s += BS) htab[s] = -1;
    if (tid == 0) {
        s_full = 0;
        s_rs[nown] = len;
        s_fs[nown] = flen;
    }
    for (int i = tid; i < nown; i += BS) {
        const int32_t o = a.perm[k0 + i];
        s_nb[i] = a.nbr_ptr[o];
        s_tb[i] = a.tri_ptr[o];
        s_rs[i] = a.row_ptr[k0 + i] - rb;
        s_fs[i] = a.fan_ptr[k0 + i] - fb;
    }
    __syncthreads();
    for (int i = tid; i < nown; i += BS)
        for (int b = (s_rs[i] + 15) >> 4; (b << 4) < s_rs[i + 1]; ++b) own[b] = static_cast<uint16_t>(i);
    __syncthreads();

    auto in_tile = [&](int32_t jd) { return jd >= k0 && jd < k0 + nown; };
    auto row_label = [&](int j) -> int32_t {
        int i = own[j >> 4];
        while (s_rs[i + 1] <= j) ++i;
        return a.new_of_old[a.nbr_idx[s_nb[i] + (j - s_rs[i])]];
    };

    // ---- halo set; the row entries' device labels are parked in the halo
    // part of the record (room for len entries) until the rows are
    // rewritten below
    unsigned char* rec = a.data + (CLS ? class_record(rb, fb, tile, T) : tile_record(rb, fb, tile, T));
    uint16_t* rr = reinterpret_cast<uint16_t*>(rec);
    const int64_t hat = CLS ? class_halo_at(T) : halo_at(T);
    int32_t* halo = reinterpret_cast<int32_t*>(rec + hat);
    bool full = false;
    for (int base = 0; base < len; base += BS * U) {
        int32_t jd[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * BS + tid;
            jd[u] = j < len ? row_label(j) : k0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * BS + tid;
            if (j < len) halo[j] = jd[u];
            if (!in_tile(jd[u]) && !set_insert<HS, CLS>(htab, jd[u])) full = true;
        }
    }
    if (full) s_full = 1;
    __syncthreads();
    if (s_full) {   // more distinct halo nodes than the set holds: the node path
        if (tid == 0) atomicOr(a.err, 2);
        return;
    }
    int c = 0;
#pragma unroll
    for (int q = 0; q < SPT; ++q) c += htab[tid * SPT + q] != -1;
    int H;
    const int h0 = block_excl_scan<BS>(c, &H, s_warp);
    {
        int h = h0;
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int s = tid * SPT + q;
            if (htab[s] != -1) hidx[s] = static_cast<uint16_t>(h++);
        }
    }
    __syncthreads();
    auto local = [&](int32_t jd) -> int {
        if (in_tile(jd)) return jd - k0;
        const int s = set_find<HS, CLS>(htab, jd);
        if (s < 0) {
            atomicOr(a.err, 1);
            return T;
        }
        return T + hidx[s];
    };

    // ---- rows in local indices, and their offsets
    const int32_t len4 = (len + 3) & ~3;
    const int64_t seg_at = align16(hat + 4 * static_cast<int64_t>(len));
    uint16_t* seg = reinterpret_cast<uint16_t*>(rec + seg_at);
    for (int j = tid; j < len; j += BS) {
        const uint16_t l = static_cast<uint16_t>(local(halo[j]));
        seg[j] = l;
        if (CLS) s_seg[j] = l;
    }
    for (int j = len + tid; j < len4; j += BS) seg[j] = 0;
    __syncthreads();   // every parked label is read: the halo list takes their place
    {
        int h = h0;
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int32_t key = htab[tid * SPT + q];
            if (key != -1) halo[h++] = key;
        }
    }
    for (int i = tid; i <= T; i += BS) rr[i] = static_cast<uint16_t>(s_rs[min(i, nown)]);
    __syncthreads();   // the entry map is rebuilt for the incidences
    for (int i = tid; i < nown; i += BS)
        for (int b = (s_fs[i] + 15) >> 4; (b << 4) < s_fs[i + 1]; ++b) own[b] = static_cast<uint16_t>(i);
    __syncthreads();

    uint64_t* tri = reinterpret_cast<uint64_t*>(rec + align16(seg_at + 2 * static_cast<int64_t>(len4)));
    int R = 0;
    if (CLS) {
        // ---- fan entries, one per incidence, and the fan starts
        uint16_t* fans = reinterpret_cast<uint16_t*>(tri);
        uint16_t* fr = rr + halo_at(T) / 2;
        for (int i = tid; i <= T; i += BS) fr[i] = static_cast<uint16_t>(s_fs[min(i, nown)]);
        for (int base = 0; base < flen; base += BS * U) {
            int32_t v[U][3], kd[U], i_of[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int f = base + u * BS + tid;
                int64_t t = 0;
                kd[u] = k0;
                i_of[u] = 0;
                if (f < flen) {
                    int i = own[f >> 4];
                    while (s_fs[i + 1] <= f) ++i;
                    kd[u] = k0 + i;
                    i_of[u] = i;
                    t = a.tri_idx[s_tb[i] + (f - s_fs[i])];
                }
#pragma unroll
                for (int q = 0; q < 3; ++q) v[u][q] = f < flen ? a.new_of_old[a.tris[3 * t + q]] : kd[u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int f = base + u * BS + tid;
                if (f >= flen) continue;
                const int p = v[u][0] == kd[u] ? 0 : (v[u][1] == kd[u] ? 1 : 2);
                const int la = local(v[u][(p + 1) % 3]), lb = local(v[u][(p + 2) % 3]);
                const int r0 = s_rs[i_of[u]], r1 = s_rs[i_of[u] + 1];
                int sa = -1, sb = -1;
                for (int j = r0; j < r1; ++j) {
                    const int l = s_seg[j];
                    if (l == la) sa = j - r0;
                    if (l == lb) sb = j - r0;
                }
                if (sa < 0 || sb < 0) atomicOr(a.err, 1);   // validation rules this out
                fans[f] = static_cast<uint16_t>(p | (max(sa, 0) << 2) | (max(sb, 0) << 9));
            }
        }
        R = flen;
    }
    // ---- triangles: work-item t takes incidences U*t .. U*t+U-1 of each
    // chunk, so that a scan of the per-item counts keeps incidence order
    for (int base = 0; !CLS && base < flen; base += BS * U) {
        int32_t v[U][3], kd[U];
        bool keep[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int f = base + tid * U + u;
            keep[u] = f < flen;
            int64_t t = 0;
            kd[u] = k0;
            if (keep[u]) {
                int i = own[f >> 4];
                while (s_fs[i + 1] <= f) ++i;
                kd[u] = k0 + i;
                t = a.tri_idx[s_tb[i] + (f - s_fs[i])];
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) v[u][q] = keep[u] ? a.new_of_old[a.tris[3 * t + q]] : kd[u];
        }
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // listed by this incidence iff no other own vertex has a smaller label
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (v[u][q] != kd[u] && in_tile(v[u][q]) && v[u][q] < kd[u]) keep[u] = false;
            cnt += keep[u];
        }
        int tot;
        int pos = R + block_excl_scan<BS>(cnt, &tot, s_warp);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!keep[u]) continue;
            uint64_t w = 0;
#pragma unroll
            for (int q = 0; q < 3; ++q) w |= static_cast<uint64_t>(local(v[u][q])) << (16 * q);
            tri[pos++] = w;
        }
        R += tot;
    }
    if (tid == 0) {
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
    }
}

// Groups each tile's triangle list by which of its vertices are own nodes
// (all three first, then the patterns with two, then with one), keeping
// incidence order inside a group.  The sweep evaluates a vertex's candidate
// quality only for own vertices; with the list grouped, the lanes of a wave
// mostly agree on which of the three evaluations to skip.  Lists longer than
// the LDS staging keep their order (any order gives the same results).
constexpr int kOrderWords = 4096;

template <int T>
// LDS: room for `cap` triangle words (the longest list, at most kOrderWords).
__global__ __launch_bounds__(256) void k_tile_order(const TileWork* __restrict__ work, int cap)
{
    constexpr int BS = 256;
    extern __shared__ uint64_t s_w[];
    __shared__ int32_t s_warp[BS / 64];
    const TileWork d = work[blockIdx.x];
    const int R = d.tri_cnt;
    if (R > cap || R == 0) return;
    uint64_t* tris = const_cast<uint64_t*>(d.tris);
    for (int j = threadIdx.x; j < R; j += BS) s_w[j] = tris[j];
    __syncthreads();
    // rank of each own-vertex pattern (bit r: vertex r is own) in the output
    constexpr uint32_t kRank = (0u << 28) | (1u << 12) | (2u << 20) | (3u << 24) | (4u << 4) | (5u << 8) |
                               (6u << 16) | (7u << 0);
    auto rank = [&](uint64_t w) -> int {
        const int p = (static_cast<int>(w & 0xFFFF) < T) | ((static_cast<int>((w >> 16) & 0xFFFF) < T) << 1) |
                      ((static_cast<int>((w >> 32) & 0xFFFF) < T) << 2);
        return static_cast<int>((kRank >> (4 * p)) & 7u);
    };
    // each work-item takes a contiguous segment; counts per rank packed two to an int
    const int per = (R + BS - 1) / BS, b = min(R, static_cast<int>(threadIdx.x) * per), e = min(R, b + per);
    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int j = b; j < e; ++j) ++cnt[rank(s_w[j])];
    int pre[8], tot[8];
    for (int k = 0; k < 4; ++k) {
        int t;
        const int x = block_excl_scan<BS>(cnt[2 * k] | (cnt[2 * k + 1] << 16), &t, s_warp);
        pre[2 * k] = x & 0xFFFF;
        pre[2 * k + 1] = x >> 16;
        tot[2 * k] = t & 0xFFFF;
        tot[2 * k + 1] = t >> 16;
    }
    int base = 0;
    for (int k = 0; k < 8; ++k) {
        const int c = tot[k];
        pre[k] += base;
        base += c;
    }
    for (int j = b; j < e; ++j) {
        const uint64_t w = s_w[j];
        tris[pre[rank(w)]++] = w;
    }
}

// Colour-class tiles: each node's fan entries grouped by the node's stored
// position p (0, then 1, then 2), in incidence order inside a group, and the
// group bounds written beside the fan starts, so that the sweep evaluates
// each group with the stored order fixed at compile time.  The minima over a
// fan are exact, so the order of its entries changes no result.  One
// work-group per tile; the tile's entries (at most T * kTileMaxDeg, the
// build's limit) are read into LDS first and written back grouped.
template <int T>
__global__ __launch_bounds__(256) void k_class_fan_sort(const TileWork* __restrict__ work)
{
    __shared__ uint16_t s_f[T * kTileMaxDeg];
    const TileWork d = work[blockIdx.x];
    uint16_t* const rr = const_cast<uint16_t*>(d.rr);
    const uint16_t* const fr = rr + halo_at(T) / 2;
    uint32_t* const pc = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(rr) + 2 * halo_at(T));
    uint16_t* const fans = reinterpret_cast<uint16_t*>(const_cast<uint64_t*>(d.tris));
    const int flen = d.tri_cnt;
    for (int j = threadIdx.x; j < flen; j += 256) s_f[j] = fans[j];
    __syncthreads();
    for (int i = threadIdx.x; i < d.nown; i += 256) {
        const int b = fr[i], e = fr[i + 1];
        int c[4] = {0, 0, 0, 0};
        for (int j = b; j < e; ++j) ++c[s_f[j] & 3u];
        int pos[4] = {b, b + c[0], b + c[0] + c[1], e};
        for (int j = b; j < e; ++j) {
            const uint16_t v = s_f[j];
            fans[pos[v & 3u]++] = v;
        }
        pc[i] = static_cast<uint32_t>(c[0]) | (static_cast<uint32_t>(c[0] + c[1]) << 16);
    }
}

// Largest halo, padded row segment and triangle list over the tiles (one
// work-group).
__global__ __launch_bounds__(1024) void k_tile_caps(const TileWork* __restrict__ work, int32_t nt,
                                                    int32_t* __restrict__ mx)
{
    __shared__ int32_t s_h[16], s_r[16], s_t[16];
    int32_t h = 0, r = 0, c = 0;
    for (int32_t t = threadIdx.x; t < nt; t += 1024) {
        h = max(h, work[t].halo_cnt);
        r = max(r, 4 * work[t].row_words);
        c = max(c, work[t].tri_cnt);
    }
    for (int off = 32; off > 0; off >>= 1) {
        h = max(h, __shfl_xor(h, off));
        r = max(r, __shfl_xor(r, off));
        c = max(c, __shfl_xor(c, off));
    }
    if ((threadIdx.x & 63) == 0) {
        s_h[threadIdx.x >> 6] = h;
        s_r[threadIdx.x >> 6] = r;
        s_t[threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 16; ++q) {
            h = max(h, s_h[q]);
            r = max(r, s_r[q]);
            c = max(c, s_t[q]);
        }
        mx[0] = h;
        mx[1] = r;
        mx[2] = c;
    }
}

}  // namespace

size_t tile_bytes(int64_t n, int64_t nnz, int64_t ninc, int tile_nodes, bool classes)
{
    // build_tiles takes nothing for other sizes
    if (tile_nodes != 256 && tile_nodes != 512 && !(classes && tile_nodes == 128)) return 0;
    // colour-class tiles: at most one short tile per class more
    const size_t nt = static_cast<size_t>(div_up(std::max<int64_t>(n, 1), tile_nodes)) +
                      (classes ? static_cast<size_t>(kMaxTileClasses) : 0);
    const size_t z = static_cast<size_t>(std::max<int64_t>(nnz, 1)), c = static_cast<size_t>(std::max<int64_t>(ninc, 1));
    const size_t rec = classes ? nt * (8 * tile_nodes + 128) + 6 * z + 2 * c + 16
                               : nt * (2 * tile_nodes + 64) + 6 * z + 8 * c + 16;
    return Arena::piece(sizeof(TileWork) * nt) + Arena::piece(rec);
}

size_t tile_scratch_bytes() { return Arena::piece(4 * sizeof(int32_t)); }

sl_status build_tiles(const SetupArgs& a, DevMesh& m, int tile_nodes, int mesh, hipStream_t st, Arena& persist,
                      Arena& scratch, bool classes)
{
    m.tile_nodes = 0;
    m.n_tile_classes = 0;
    if ((tile_nodes != 256 && tile_nodes != 512 && !(classes && tile_nodes == 128)) || m.n_free == 0) return SL_OK;
    if (classes && (m.n_colors < 1 || m.n_colors > kMaxTileClasses)) return SL_OK;
    const int T = tile_nodes;
    int nt = div_up(m.n_free, T);
    if (classes) {
        nt = 0;
        for (int c = 0; c < m.n_colors; ++c) {
            m.class_tile_h[c] = nt;
            nt += div_up(m.color_start_h[c + 1] - m.color_start_h[c], T);
        }
        m.class_tile_h[m.n_colors] = nt;
    }
    const size_t pmark = persist.mark(), smark = scratch.mark();
    sl_status r = SL_OK;
    int32_t* flags = nullptr;   // {err, largest halo, largest row segment, largest triangle list}
    if ((r = scratch.take(&flags, 4))) return r;
    SL_HIP(hipMemsetAsync(flags, 0, 4 * sizeof(int32_t), st));
    const size_t data_bytes =
        static_cast<size_t>(classes ? class_record(static_cast<int32_t>(m.nnz_free), static_cast<int32_t>(m.ninc_free), nt, T)
                                    : tile_record(static_cast<int32_t>(m.nnz_free), static_cast<int32_t>(m.ninc_free), nt, T));
    if ((r = persist.take(&m.work, nt)) || (r = persist.take(&m.tile_data, data_bytes))) return r;
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
    b.data = m.tile_data;
    b.work = m.work;
    b.err = flags;
    b.n_class = classes ? m.n_colors : 0;
    for (int c = 0; classes && c <= m.n_colors; ++c) {
        b.cls_start[c] = m.color_start_h[c];
        b.cls_tile[c] = m.class_tile_h[c];
    }
    if (classes) {
        if (T == 128) k_tile_build<128, true><<<nt, kBuildBS, 0, st>>>(b);
        else if (T == 256) k_tile_build<256, true><<<nt, kBuildBS, 0, st>>>(b);
        else k_tile_build<512, true><<<nt, kBuildBS, 0, st>>>(b);
    } else {
        if (T == 256) k_tile_build<256, false><<<nt, kBuildBS, 0, st>>>(b);
        else k_tile_build<512, false><<<nt, kBuildBS, 0, st>>>(b);
    }
    k_tile_caps<<<1, 1024, 0, st>>>(m.work, nt, flags + 1);
    SL_HIP(hipGetLastError());
    int32_t h[4] = {0, 0, 0, 0};
    SL_HIP(hipMemcpyAsync(h, flags, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    scratch.rewind(smark);
    if (h[0] & 1) return fail(SL_ETOPO, "triangle vertex outside its tile's neighbourhood");
    // a tile denser than the staging holds, or a halo or row segment too big
    // for LDS: the node path, whose arrays reuse the tile arrays' room
    const size_t lds = classes ? class_lds_bytes(T, h[1], h[2], h[3]) : tile_lds_bytes(T, h[1], h[2], m.precision);
    if ((h[0] & 2) || lds > kTileLdsLimit) {
        m.work = nullptr;
        m.tile_data = nullptr;
        persist.rewind(pmark);
        return SL_OK;
    }
    if (classes) {
        if (T == 128) k_class_fan_sort<128><<<nt, 256, 0, st>>>(m.work);
        else if (T == 256) k_class_fan_sort<256><<<nt, 256, 0, st>>>(m.work);
        else k_class_fan_sort<512><<<nt, 256, 0, st>>>(m.work);
    }
    // (class tiles have fan entries, not triangle words: nothing to group)
    const int cap = classes ? 0 : std::min(h[3], kOrderWords);
    if (cap > 0) {
        const size_t lds = sizeof(uint64_t) * static_cast<size_t>(cap);
        if (T == 256) k_tile_order<256><<<nt, 256, lds, st>>>(m.work, cap);
        else k_tile_order<512><<<nt, 256, lds, st>>>(m.work, cap);
    }
    SL_HIP(hipGetLastError());
    m.halo_max = h[1];
    m.rows_max = h[2];
    m.fans_max = h[3];
    m.n_tiles = nt;
    m.tile_nodes = T;
    m.n_tile_classes = classes ? m.n_colors : 0;
    return SL_OK;
}

}  // namespace sl
