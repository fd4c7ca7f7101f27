// Mesh setup on the device: validation, node ordering, relabelling, fan
// build, coordinate buffers, and the inverse steps on the way out.
//
// The paper prepares a mesh in three procedures before iterating (Sec. 3.3.1
// initiating, Sec. 3.3.2 finding neighbours, Sec. 3.3.3 determining
// constraints).  Here the caller hands in the neighbour rows, incident
// triangles and the boundary mask; setup checks them and turns them into the
// layout the sweep kernels read:
//   - free nodes first, in Hilbert order of their position (or in the
//     caller's order), fixed nodes after them;
//   - neighbour rows relabelled, order inside a row kept (it is the
//     centroid's summation order);
//   - a 16-bit "fan" entry per (free node, incident triangle): the node's
//     position p in the triangle's stored order (bits 0-1) and the row slots
//     of the vertices at stored positions p+1 and p+2 mod 3 (bits 2-8, 9-15).
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "sl_common.h"

namespace sl {

namespace {

constexpr int kBS = 256;

// Order-preserving map of a double to uint64 (for atomic min/max).
__device__ __forceinline__ uint64_t ord_bits(double v)
{
    uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__host__ __device__ __forceinline__ double from_ord_bits(uint64_t u)
{
    u = (u & 0x8000000000000000ull) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u;
    double d;
    memcpy(&d, &u, sizeof(d));
    return d;
}

// SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014), applied to
// the caller's node id: the colouring priority.
__device__ __forceinline__ uint64_t splitmix64(uint64_t v)
{
    uint64_t z = v + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------- scan ----
//
// Reduce, then scan: one pass sums each tile of kScanTile values, one
// work-group scans the tile sums, and a second pass scans each tile from its
// offset.  Each work-item holds 16 consecutive values, loaded and stored as
// four 16-byte vectors when the arrays allow it.

constexpr int kScanPer = 16;
constexpr int kScanTile = kBS * kScanPer;
constexpr int kSumsBS = 1024;

// This work-item's values of tile `b` (zeros past n).
__device__ __forceinline__ void scan_load(const int32_t* __restrict__ in, int64_t n, int64_t base, bool vec,
                                          int32_t (&v)[kScanPer])
{
    if (vec && base + kScanPer <= n) {
        const int4* p = reinterpret_cast<const int4*>(in + base);
#pragma unroll
        for (int q = 0; q < kScanPer / 4; ++q) {
            const int4 w = p[q];
            v[4 * q] = w.x;
            v[4 * q + 1] = w.y;
            v[4 * q + 2] = w.z;
            v[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) v[j] = base + j < n ? in[base + j] : 0;
    }
}

// Exclusive scan of one value per work-item over a work-group of BS
// work-items (wave scans, then the wave totals); *total = the group's sum.
template <int BS>
__device__ __forceinline__ int32_t group_excl_scan(int32_t x, int32_t* s_wave, int32_t* total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t t = __shfl_up(inc, off, 64);
        if (lane >= off) inc += t;
    }
    if (lane == 63) s_wave[wv] = inc;
    __syncthreads();
    int32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) {
        const int32_t t = s_wave[w];
        before += w < wv ? t : 0;
        all += t;
    }
    __syncthreads();   // s_wave may be reused at once
    *total = all;
    return before + inc - x;
}

__global__ __launch_bounds__(kBS) void k_scan_sums(const int32_t* __restrict__ in, int64_t n, bool vec,
                                                   int32_t* __restrict__ sums)
{
    __shared__ int32_t s_wave[kBS / 64];
    int32_t v[kScanPer];
    scan_load(in, n, (static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x) * kScanPer, vec, v);
    int32_t x = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) x += v[j];
    int32_t total;
    (void)group_excl_scan<kBS>(x, s_wave, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the nb tile sums in place, by one work-group; *total =
// their sum.
__global__ __launch_bounds__(kSumsBS) void k_scan_offsets(int32_t* __restrict__ sums, int32_t nb,
                                                          int32_t* __restrict__ total)
{
    __shared__ int32_t s_wave[kSumsBS / 64];
    const int per = (nb + kSumsBS - 1) / kSumsBS;
    const int b0 = min(static_cast<int>(threadIdx.x) * per, nb), b1 = min(b0 + per, nb);
    int32_t x = 0;
    for (int b = b0; b < b1; ++b) x += sums[b];
    int32_t all;
    int32_t run = group_excl_scan<kSumsBS>(x, s_wave, &all);
    for (int b = b0; b < b1; ++b) {
        const int32_t t = sums[b];
        sums[b] = run;
        run += t;
    }
    if (threadIdx.x == 0) *total = all;
}

__global__ __launch_bounds__(kBS) void k_scan_tiles(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                    int64_t n, bool vec, const int32_t* __restrict__ offs)
{
    __shared__ int32_t s_wave[kBS / 64];
    const int64_t base = (static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x) * kScanPer;
    int32_t v[kScanPer];
    scan_load(in, n, base, vec, v);
    int32_t x = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) x += v[j];
    int32_t total;
    int32_t run = offs[blockIdx.x] + group_excl_scan<kBS>(x, s_wave, &total);
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int32_t t = v[j];
        v[j] = run;
        run += t;
    }
    if (vec && base + kScanPer <= n) {
        int4* p = reinterpret_cast<int4*>(out + base);
#pragma unroll
        for (int q = 0; q < kScanPer / 4; ++q) p[q] = make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < kScanPer; ++j)
            if (base + j < n) out[base + j] = v[j];
    }
}

// Exclusive scan of a short in[0..n) by one work-group, kSumsBS*kScanPer
// values at a time with a running carry: one launch in place of three, for
// setups whose time goes into launches (a batch of small meshes).  In place
// (in == out) is allowed: every value is read and written by one work-item.
__global__ __launch_bounds__(kSumsBS) void k_scan_one(const int32_t* in, int32_t* out, int64_t n, bool vec,
                                                      int32_t* total)
{
    __shared__ int32_t s_wave[kSumsBS / 64];
    int32_t carry = 0;
    for (int64_t c0 = 0; c0 < n; c0 += static_cast<int64_t>(kSumsBS) * kScanPer) {
        const int64_t base = c0 + static_cast<int64_t>(threadIdx.x) * kScanPer;
        int32_t v[kScanPer];
        scan_load(in, n, base, vec, v);
        int32_t x = 0;
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) x += v[j];
        int32_t all;
        int32_t run = carry + group_excl_scan<kSumsBS>(x, s_wave, &all);
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) {
            const int32_t t = v[j];
            v[j] = run;
            run += t;
        }
        if (vec && base + kScanPer <= n) {
            int4* p = reinterpret_cast<int4*>(out + base);
#pragma unroll
            for (int q = 0; q < kScanPer / 4; ++q) p[q] = make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        } else {
#pragma unroll
            for (int j = 0; j < kScanPer; ++j)
                if (base + j < n) out[base + j] = v[j];
        }
        carry += all;
    }
    if (threadIdx.x == 0) *total = carry;
}

// Scans this long or shorter take the one-launch path (at most 16 passes of
// its loop).
constexpr int64_t kScanOneMax = int64_t(16) * kSumsBS * kScanPer;

// Exclusive scan of in[0..n) into out[0..n); *total = sum.  The tile sums
// come from `ar` when given, else from the allocator.
sl_status scan_rec(const int32_t* in, int32_t* out, int64_t n, int32_t* total, hipStream_t st, Arena* ar)
{
    if (n <= kScanOneMax) {
        const bool vec1 = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
        k_scan_one<<<1, kSumsBS, 0, st>>>(in, out, n, vec1, total);
        SL_HIP(hipGetLastError());
        return SL_OK;
    }
    const int nb = div_up(n > 0 ? n : 1, kScanTile);
    int32_t* sums = nullptr;
    sl_status r = ar ? ar->take(&sums, static_cast<size_t>(nb)) : dalloc(&sums, static_cast<size_t>(nb), st);
    if (r) return r;
    const bool vec = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    k_scan_sums<<<nb, kBS, 0, st>>>(in, n, vec, sums);
    k_scan_offsets<<<1, kSumsBS, 0, st>>>(sums, nb, total);
    k_scan_tiles<<<nb, kBS, 0, st>>>(in, out, n, vec, sums);
    if (!ar) dfree(sums, st);
    SL_HIP(hipGetLastError());
    return SL_OK;
}

// Arena bytes the temporaries of a scan of n values take.
size_t scan_bytes(int64_t n) { return Arena::piece(4 * static_cast<size_t>(div_up(n > 0 ? n : 1, kScanTile))); }

// ----------------------------------------------------------- validation ---

struct ValArgs {
    const double* coords;
    int32_t n;
    const int32_t* nbr_ptr;
    const int32_t* nbr_idx;
    const int32_t* tri_ptr;
    const int32_t* tri_idx;
    const int32_t* tris;
    int32_t n_tris;
    const uint8_t* boundary;
    int64_t nnz, ninc;
    int check_symmetry;
    double coord_limit;    // coordinates must be below this in magnitude
};

constexpr int kRowRegs = 16;

__device__ __forceinline__ bool row_has(const int32_t* __restrict__ idx, int32_t b, int32_t e, int32_t v)
{
    for (int32_t k = b; k < e; ++k)
        if (idx[k] == v) return true;
    return false;
}

__global__ __launch_bounds__(kBS) void k_validate_tris(const int32_t* __restrict__ tris, int32_t n_tris, int32_t n,
                                                       ValStats* __restrict__ vs)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
    uint32_t e = 0;
    if (t < n_tris) {
        const int32_t a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
        if (a < 0 || b < 0 || c < 0 || a >= n || b >= n || c >= n) e |= VE_RANGE;
        if (a == b || b == c || a == c) e |= VE_TRIREP;
    }
    if (e) atomicOr(&vs->err, e);
}

// Incidence rows that disagree (for the Form A tile path, which lists a
// triangle once per tile and scores it for every own vertex): a triangle
// listed by some of its free vertices but not by all of them.  One
// work-item per triangle looks for it in its free vertices' rows, the three
// rows' offsets and first kIncRegs entries loaded together.  Vertices out of
// range and offsets out of order are left to the other checks.
constexpr int kIncRegs = 8;
__global__ __launch_bounds__(kBS) void k_validate_incidence(const int32_t* __restrict__ tris, int32_t n_tris, int32_t n,
                                                            const uint8_t* __restrict__ bnd,
                                                            const int32_t* __restrict__ tri_ptr,
                                                            const int32_t* __restrict__ tri_idx, int64_t ninc,
                                                            ValStats* __restrict__ vs)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
    if (t >= n_tris) return;
    int32_t v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = tris[3 * t + k];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (v[k] < 0 || v[k] >= n) return;
    int32_t ob[3], oe[3];
    uint8_t fl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        fl[k] = bnd[v[k]];
        ob[k] = tri_ptr[v[k]];
        oe[k] = tri_ptr[v[k] + 1];
    }
    bool use[3];
    int32_t len[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        use[k] = fl[k] == 0 && 0 <= ob[k] && ob[k] <= oe[k] && oe[k] <= ninc;
        len[k] = use[k] ? oe[k] - ob[k] : 0;
    }
    int32_t x[3][kIncRegs];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int q = 0; q < kIncRegs; ++q) x[k][q] = tri_idx[len[k] > 0 ? ob[k] + min(q, len[k] - 1) : 0];
    int lists = 0, free_v = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (!use[k]) continue;
        ++free_v;
        bool found = false;
#pragma unroll
        for (int q = 0; q < kIncRegs; ++q) found |= q < len[k] && x[k][q] == static_cast<int32_t>(t);
        if (!found && len[k] > kIncRegs) found = row_has(tri_idx, ob[k] + kIncRegs, oe[k], static_cast<int32_t>(t));
        lists += found;
    }
    if (lists > 0 && lists < free_v) atomicOr(&vs->err, static_cast<uint32_t>(VI_INCIDENCE));
}

__global__ __launch_bounds__(kBS) void k_validate_nodes(ValArgs a, ValStats* __restrict__ part)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x * kBS + threadIdx.x);
    uint32_t e = 0;
    int is_free = 0, deg = 0, inc = 0;
    if (i < a.n) {
        const double x = a.coords[2 * static_cast<int64_t>(i)], y = a.coords[2 * static_cast<int64_t>(i) + 1];
        // finite and below the limit in magnitude (2^500 in double, 2^61 in
        // single precision): squared edge lengths, their sums and cross
        // products cannot overflow, so every quality is a finite number
        if (!(fabs(x) < a.coord_limit) || !(fabs(y) < a.coord_limit)) e |= VE_COORD;
        const int32_t b = a.nbr_ptr[i], en = a.nbr_ptr[i + 1];
        const bool row_ok = 0 <= b && b <= en && en <= a.nnz;
        const int32_t tb = a.tri_ptr[i], te = a.tri_ptr[i + 1];
        const bool trow_ok = 0 <= tb && tb <= te && te <= a.ninc;
        if (!row_ok || !trow_ok) e |= VE_PTR;
        is_free = a.boundary[i] == 0;
        // rows of up to kRowRegs entries are held in registers for the
        // membership tests below; longer rows are searched in memory
        int32_t rowv[kRowRegs];
        const bool in_regs = row_ok && en - b <= kRowRegs;
        if (row_ok) {
            deg = en - b;
#pragma unroll
            for (int k = 0; k < kRowRegs; ++k) rowv[k] = (in_regs && k < deg) ? a.nbr_idx[b + k] : -1;
            auto check = [&](int32_t j) {
                if (j < 0 || j >= a.n) {
                    e |= VE_RANGE;
                    return;
                }
                if (j == i) e |= VE_SELF;
                if (is_free && a.check_symmetry && a.boundary[j] == 0) {
                    const int32_t jb = a.nbr_ptr[j], je = a.nbr_ptr[j + 1];
                    if (!(0 <= jb && jb <= je && je <= a.nnz) || !row_has(a.nbr_idx, jb, je, i)) e |= VE_ASYM;
                }
            };
            if (in_regs) {
#pragma unroll
                for (int k = 0; k < kRowRegs; ++k)
                    if (k < deg) check(rowv[k]);
            } else {
                for (int32_t k = b; k < en; ++k) check(a.nbr_idx[k]);
            }
            if (is_free && deg == 0) e |= VE_EMPTY;
            if (is_free && deg > kMaxValence) e |= VE_VALENCE;
        }
        auto in_row = [&](int32_t v) -> bool {
            if (!in_regs) return row_has(a.nbr_idx, b, en, v);
            bool f = false;
#pragma unroll
            for (int k = 0; k < kRowRegs; ++k) f |= rowv[k] == v;
            return f;
        };
        if (trow_ok) {
            inc = te - tb;
            // incident triangles four at a time: their loads are in flight together
            for (int32_t k0 = tb; k0 < te; k0 += 4) {
                int32_t t[4], v[4][3];
#pragma unroll
                for (int u = 0; u < 4; ++u) t[u] = k0 + u < te ? a.tri_idx[k0 + u] : -1;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool ok = t[u] >= 0 && t[u] < a.n_tris;
                    if (k0 + u < te && !ok) e |= VE_RANGE;
#pragma unroll
                    for (int s3 = 0; s3 < 3; ++s3) v[u][s3] = ok ? a.tris[3 * static_cast<int64_t>(t[u]) + s3] : -1;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (!(t[u] >= 0 && t[u] < a.n_tris)) continue;
                    const int32_t v0 = v[u][0], v1 = v[u][1], v2 = v[u][2];
                    if (v0 != i && v1 != i && v2 != i) { e |= VE_NOTIN; continue; }
                    // the other two vertices, in stored cyclic order after i
                    const int32_t o1 = v0 == i ? v1 : (v1 == i ? v2 : v0);
                    const int32_t o2 = v0 == i ? v2 : (v1 == i ? v0 : v1);
                    if (is_free && row_ok && (!in_row(o1) || !in_row(o2))) e |= VE_MISSING;
                }
            }
        }
    }
    // block reductions: free count, max degree, max incidence, error bits
    __shared__ int32_t s_cnt[kBS / 64], s_deg[kBS / 64], s_inc[kBS / 64];
    __shared__ uint32_t s_err[kBS / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int df = is_free ? deg : 0, inf = is_free ? inc : 0;
    int32_t c = __popcll(__ballot(is_free != 0));
    int32_t md = df, mi = inf;
    uint32_t me = e;
    for (int off = 32; off > 0; off >>= 1) {
        md = max(md, __shfl_xor(md, off));
        mi = max(mi, __shfl_xor(mi, off));
        me |= __shfl_xor(me, off);
    }
    if (lane == 0) { s_cnt[w] = c; s_deg[w] = md; s_inc[w] = mi; s_err[w] = me; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t C = 0, D = 0, I = 0;
        uint32_t E = 0;
        for (int q = 0; q < kBS / 64; ++q) { C += s_cnt[q]; D = max(D, s_deg[q]); I = max(I, s_inc[q]); E |= s_err[q]; }
        part[blockIdx.x] = ValStats{E, C, D, I};
    }
}

// Folds the per-block statistics into *vs (whose error bits the triangle
// check may already have set); one work-group, no atomics.
__global__ __launch_bounds__(1024) void k_validate_fold(const ValStats* __restrict__ part, int32_t nb,
                                                        ValStats* __restrict__ vs)
{
    __shared__ ValStats s_part[16];
    uint32_t e = 0;
    int32_t c = 0, d = 0, in = 0;
    for (int32_t b = threadIdx.x; b < nb; b += 1024) {
        const ValStats p = part[b];
        e |= p.err;
        c += p.n_free;
        d = max(d, p.max_deg_free);
        in = max(in, p.max_inc_free);
    }
    for (int off = 32; off > 0; off >>= 1) {
        e |= __shfl_xor(e, off);
        c += __shfl_xor(c, off);
        d = max(d, __shfl_xor(d, off));
        in = max(in, __shfl_xor(in, off));
    }
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = ValStats{e, c, d, in};
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 16; ++q) {
            e |= s_part[q].err;
            c += s_part[q].n_free;
            d = max(d, s_part[q].max_deg_free);
            in = max(in, s_part[q].max_inc_free);
        }
        vs->err |= e;
        vs->n_free = c;
        vs->max_deg_free = d;
        vs->max_inc_free = in;
    }
}

// ------------------------------------------------------------- ordering ---

constexpr int kBboxBlocks = 1024;

// Per-block bounding box of the coordinates, as order-preserving bit
// patterns {min x, min y, max x, max y}; k_bbox_fold folds the blocks.
__global__ __launch_bounds__(kBS) void k_bbox(const double* __restrict__ coords, int32_t n, uint64_t* __restrict__ part)
{
    uint64_t mnx = ~0ull, mny = ~0ull, mxx = 0, mxy = 0;
    const double2* c2 = reinterpret_cast<const double2*>(coords);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBS) {
        const double2 p = c2[i];
        const uint64_t ox = ord_bits(p.x), oy = ord_bits(p.y);
        mnx = min(mnx, ox); mxx = max(mxx, ox);
        mny = min(mny, oy); mxy = max(mxy, oy);
    }
    __shared__ uint64_t s_bb[kBS / 64][4];
    for (int off = 32; off > 0; off >>= 1) {
        mnx = min(mnx, static_cast<uint64_t>(__shfl_xor(static_cast<unsigned long long>(mnx), off)));
        mny = min(mny, static_cast<uint64_t>(__shfl_xor(static_cast<unsigned long long>(mny), off)));
        mxx = max(mxx, static_cast<uint64_t>(__shfl_xor(static_cast<unsigned long long>(mxx), off)));
        mxy = max(mxy, static_cast<uint64_t>(__shfl_xor(static_cast<unsigned long long>(mxy), off)));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_bb[w][0] = mnx; s_bb[w][1] = mny; s_bb[w][2] = mxx; s_bb[w][3] = mxy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kBS / 64; ++q) {
            mnx = min(mnx, s_bb[q][0]); mny = min(mny, s_bb[q][1]);
            mxx = max(mxx, s_bb[q][2]); mxy = max(mxy, s_bb[q][3]);
        }
        uint64_t* o = part + 4 * static_cast<int64_t>(blockIdx.x);
        o[0] = mnx; o[1] = mny; o[2] = mxx; o[3] = mxy;
    }
}

__global__ __launch_bounds__(kBS) void k_bbox_fold(const uint64_t* __restrict__ part, int nb, uint64_t* __restrict__ bb)
{
    uint64_t mnx = ~0ull, mny = ~0ull, mxx = 0, mxy = 0;
    for (int b = threadIdx.x; b < nb; b += kBS) {
        mnx = min(mnx, part[4 * b]); mny = min(mny, part[4 * b + 1]);
        mxx = max(mxx, part[4 * b + 2]); mxy = max(mxy, part[4 * b + 3]);
    }
    __shared__ uint64_t s_bb[kBS][4];
    s_bb[threadIdx.x][0] = mnx; s_bb[threadIdx.x][1] = mny; s_bb[threadIdx.x][2] = mxx; s_bb[threadIdx.x][3] = mxy;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kBS; ++q) {
            mnx = min(mnx, s_bb[q][0]); mny = min(mny, s_bb[q][1]);
            mxx = max(mxx, s_bb[q][2]); mxy = max(mxy, s_bb[q][3]);
        }
        bb[0] = mnx; bb[1] = mny; bb[2] = mxx; bb[3] = mxy;
    }
}

// Hilbert index of cell (x, y) on a 2^bits x 2^bits grid.
__device__ __forceinline__ uint32_t hilbert_index(int bits, uint32_t x, uint32_t y)
{
    uint32_t d = 0;
    for (uint32_t s = 1u << (bits - 1); s > 0; s >>= 1) {
        const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += s * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) { x = (s - 1) ^ x; y = (s - 1) ^ y; }
            const uint32_t t = x; x = y; y = t;
        }
    }
    return d;
}

// Bucket of each free node: colour * 4^bits + Hilbert cell (bits may be 0).
__global__ __launch_bounds__(kBS) void k_bucket(const double* __restrict__ coords, const uint8_t* __restrict__ bnd,
                                                const int32_t* __restrict__ color, int32_t n, int bits,
                                                const uint64_t* __restrict__ bb, int32_t* __restrict__ key,
                                                int32_t* __restrict__ count, int32_t* __restrict__ rank)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
    if (i >= n || bnd[i]) return;
    uint32_t cell = 0;
    if (bits > 0) {
        const double x0 = from_ord_bits(bb[0]), y0 = from_ord_bits(bb[1]);
        const double ext = fmax(from_ord_bits(bb[2]) - x0, from_ord_bits(bb[3]) - y0);
        const double side = static_cast<double>(1u << bits);
        const double sc = ext > 0.0 ? side / ext : 0.0;
        const uint32_t lim = (1u << bits) - 1u;
        const double fx = (coords[2 * i] - x0) * sc, fy = (coords[2 * i + 1] - y0) * sc;
        const uint32_t cx = fx <= 0.0 ? 0u : (fx >= lim ? lim : static_cast<uint32_t>(fx));
        const uint32_t cy = fy <= 0.0 ? 0u : (fy >= lim ? lim : static_cast<uint32_t>(fy));
        cell = hilbert_index(bits, cx, cy);
    }
    const int32_t k = (color ? color[i] : 0) * (1 << (2 * bits)) + static_cast<int32_t>(cell);
    key[i] = k;
    rank[i] = atomicAdd(count + k, 1);   // place inside the bucket (in no particular order)
}

__global__ __launch_bounds__(kBS) void k_bucket_scatter(const uint8_t* __restrict__ bnd, int32_t n,
                                                        const int32_t* __restrict__ key,
                                                        const int32_t* __restrict__ rank,
                                                        const int32_t* __restrict__ start,
                                                        int32_t* __restrict__ new_of_old, int32_t* __restrict__ perm)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
    if (i >= n || bnd[i]) return;
    const int32_t pos = start[key[i]] + rank[i];
    new_of_old[i] = pos;
    perm[pos] = static_cast<int32_t>(i);
}

// flag[i] = (bnd[i] != 0) == want_fixed  (and, if color given, color[i] == c)
__global__ __launch_bounds__(kBS) void k_select(const uint8_t* __restrict__ bnd, const int32_t* __restrict__ color,
                                                int32_t c, int want_fixed, int32_t n, int32_t* __restrict__ flag)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
    if (i >= n) return;
    int f = (bnd[i] != 0) == (want_fixed != 0);
    if (f && color) f = color[i] == c;
    flag[i] = f;
}

__global__ __launch_bounds__(kBS) void k_place(const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                                               int32_t base, int32_t n, int32_t* __restrict__ new_of_old,
                                               int32_t* __restrict__ perm)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const int32_t p = base + pos[i];
    new_of_old[i] = p;
    perm[p] = static_cast<int32_t>(i);
}

// ------------------------------------------------------------ colouring ---

// One round of greedy colouring in decreasing priority: a free node takes
// the smallest colour unused by its free neighbours once every free
// neighbour of higher priority has a colour.
// Appends v to list[] for every work-item of the group whose `keep` is set:
// one atomic per work-group reserves the group's places (one per wave, or
// per work-item, on a single counter would queue behind each other).  Every
// work-item of the group must call it.
constexpr int kColorBS = 1024;
__device__ __forceinline__ void append_group(bool keep, int32_t v, int32_t* __restrict__ list,
                                             int32_t* __restrict__ count, int32_t* s_tmp /* [kColorBS/64 + 1] */)
{
    const int lane = static_cast<int>(threadIdx.x & 63), wv = static_cast<int>(threadIdx.x >> 6);
    const unsigned long long mask = __ballot(keep);
    if (lane == 0) s_tmp[wv] = __popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t tot = 0;
        for (int w = 0; w < kColorBS / 64; ++w) {
            const int32_t c = s_tmp[w];
            s_tmp[w] = tot;
            tot += c;
        }
        s_tmp[kColorBS / 64] = tot ? atomicAdd(count, tot) : 0;
    }
    __syncthreads();
    if (keep) list[s_tmp[kColorBS / 64] + s_tmp[wv] + __popcll(mask & ((1ull << lane) - 1ull))] = v;
}

constexpr int kColorRounds = 8;

// One Jones-Plassmann round over the listed (uncoloured) free nodes: a node
// whose neighbours of higher priority are all coloured takes the smallest
// colour none of them has; the others go to the next list.  The colour a
// node gets depends only on those neighbours' colours, so neither the
// round nor the list order changes the result.
__global__ __launch_bounds__(kColorBS) void k_color_round(const int32_t* __restrict__ nbr_ptr,
                                                     const int32_t* __restrict__ nbr_idx,
                                                     const uint8_t* __restrict__ bnd, int32_t* color,
                                                     const int32_t* __restrict__ list, const int32_t* cnt_in,
                                                     int32_t* __restrict__ next, int32_t* __restrict__ next_cnt)
{
    __shared__ int32_t s_tmp[kColorBS / 64 + 1];
    const int32_t cnt = *cnt_in;   // the list's length, left by the previous round
    const int32_t t = static_cast<int32_t>(blockIdx.x * kColorBS + threadIdx.x);
    bool left = false;
    int32_t i = -1;
    if (t < cnt) {
        i = list[t];
        const uint64_t pi = splitmix64(static_cast<uint64_t>(i));
        uint64_t used0 = 0, used1 = 0;
        bool ready = true;
        for (int32_t k = nbr_ptr[i]; k < nbr_ptr[i + 1]; ++k) {
            const int32_t j = nbr_idx[k];
            if (bnd[j] || splitmix64(static_cast<uint64_t>(j)) < pi) continue;
            const int32_t cj = __atomic_load_n(color + j, __ATOMIC_RELAXED);
            if (cj < 0) { ready = false; break; }
            if (cj < 64) used0 |= 1ull << cj; else used1 |= 1ull << (cj - 64);
        }
        if (ready) {
            const int32_t c = (~used0) ? __builtin_ctzll(~used0) : 64 + __builtin_ctzll(~used1);
            __atomic_store_n(color + i, c, __ATOMIC_RELAXED);
        } else {
            left = true;
        }
    }
    append_group(left, i, next, next_cnt, s_tmp);
}

// Every node uncoloured; the free ones listed (in no particular order).
__global__ __launch_bounds__(kColorBS) void k_color_init(int32_t n, const uint8_t* __restrict__ bnd, int32_t* color,
                                                         int32_t* __restrict__ list, int32_t* __restrict__ count)
{
    __shared__ int32_t s_tmp[kColorBS / 64 + 1];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kColorBS + threadIdx.x;
    if (i < n) color[i] = -1;
    append_group(i < n && !bnd[i], static_cast<int32_t>(i), list, count, s_tmp);
}

__global__ __launch_bounds__(kBS) void k_max_i32(const int32_t* __restrict__ v, int32_t n, int32_t* __restrict__ out)
{
    int32_t m = -1;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBS)
        m = max(m, v[i]);
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------ relabel -----

__global__ __launch_bounds__(kBS) void k_degrees(const int32_t* __restrict__ perm, int32_t n_free,
                                                 const int32_t* __restrict__ nbr_ptr,
                                                 const int32_t* __restrict__ tri_ptr, int32_t* __restrict__ deg,
                                                 int32_t* __restrict__ inc)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
    if (k >= n_free) return;
    const int32_t o = perm[k];
    deg[k] = nbr_ptr[o + 1] - nbr_ptr[o];
    inc[k] = tri_ptr[o + 1] - tri_ptr[o];
}

__global__ __launch_bounds__(kBS) void k_rows_fans(const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ new_of_old, int32_t n_free,
                                                   const int32_t* __restrict__ nbr_ptr,
                                                   const int32_t* __restrict__ nbr_idx,
                                                   const int32_t* __restrict__ tri_ptr,
                                                   const int32_t* __restrict__ tri_idx,
                                                   const int32_t* __restrict__ tris,
                                                   const int32_t* __restrict__ row_ptr, int32_t* __restrict__ nbr,
                                                   const int32_t* __restrict__ fan_ptr, uint16_t* __restrict__ fan)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
    if (k >= n_free) return;
    const int32_t o = perm[k];
    const int32_t b = nbr_ptr[o], d = nbr_ptr[o + 1] - b;
    const int32_t out = row_ptr[k];
    // rows of up to kRowRegs entries are held in registers (their loads in
    // flight together) for the slot searches below; longer rows are
    // searched in memory
    const bool in_regs = d <= kRowRegs;
    int32_t rowv[kRowRegs];
#pragma unroll
    for (int j = 0; j < kRowRegs; ++j) rowv[j] = (in_regs && j < d) ? nbr_idx[b + j] : -1;
    if (in_regs) {
#pragma unroll
        for (int j = 0; j < kRowRegs; ++j)
            if (j < d) nbr[out + j] = new_of_old[rowv[j]];
    } else {
        for (int32_t j = 0; j < d; ++j) nbr[out + j] = new_of_old[nbr_idx[b + j]];
    }
    // the row position of u (the last one, should u repeat)
    auto slot = [&](int32_t u) -> int {
        int sj = 0;
        if (in_regs) {
#pragma unroll
            for (int j = 0; j < kRowRegs; ++j)
                if (j < d && rowv[j] == u) sj = j;
        } else {
            for (int32_t j = 0; j < d; ++j)
                if (nbr_idx[b + j] == u) sj = j;
        }
        return sj;
    };
    const int32_t tb = tri_ptr[o], nt = tri_ptr[o + 1] - tb;
    const int32_t fo = fan_ptr[k];
    // incidences four at a time: their loads are in flight together
    for (int32_t q0 = 0; q0 < nt; q0 += 4) {
        int64_t t[4];
        int32_t v[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] = q0 + u < nt ? tri_idx[tb + q0 + u] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) v[u][c] = t[u] >= 0 ? tris[3 * t[u] + c] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (q0 + u >= nt) break;
            const int p = v[u][0] == o ? 0 : (v[u][1] == o ? 1 : 2);
            const int32_t va = v[u][(p + 1) % 3], vc = v[u][(p + 2) % 3];
            fan[fo + q0 + u] = static_cast<uint16_t>(p | (slot(va) << 2) | (slot(vc) << 9));
        }
    }
}

// Groups each free node's fan entries by the node's position p in the
// triangle's stored order (0, then 1, then 2; incidence order inside a
// group) and stores the groups' bounds, c0 | (c0 + c1) << 16 for c_p entries
// of position p, so that the node kernel evaluates each group with the
// position fixed at compile time.  A minimum over a fan is exact, so the
// order of its entries changes no result.  Fans longer than kGroupFan keep
// their order and get kFanUngrouped.  The entries are held in registers.
__global__ __launch_bounds__(kBS) void k_fan_group(const int32_t* __restrict__ fan_ptr, uint16_t* __restrict__ fan,
                                                   uint32_t* __restrict__ split, int32_t n_free)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
    if (k >= n_free) return;
    const int32_t f0 = fan_ptr[k], n = fan_ptr[k + 1] - f0;
    if (n > kGroupFan) {
        split[k] = kFanUngrouped;
        return;
    }
    uint32_t e[kGroupFan];
    int c0 = 0, c1 = 0;
#pragma unroll
    for (int j = 0; j < kGroupFan; ++j) {
        e[j] = j < n ? fan[f0 + j] : 3u;   // 3: no entry
        c0 += (e[j] & 3u) == 0u;
        c1 += (e[j] & 3u) == 1u;
    }
    int q0 = f0, q1 = f0 + c0, q2 = f0 + c0 + c1;
#pragma unroll
    for (int j = 0; j < kGroupFan; ++j) {
        const uint32_t p = e[j] & 3u;
        if (p == 3u) continue;
        const int at = p == 0u ? q0++ : (p == 1u ? q1++ : q2++);
        fan[at] = static_cast<uint16_t>(e[j]);
    }
    split[k] = static_cast<uint32_t>(c0) | (static_cast<uint32_t>(c0 + c1) << 16);
}

// Both buffers of the ping-pong pair start at the caller's positions,
// rounded to R (float for the single-precision form).
template <typename R>
__global__ __launch_bounds__(kBS) void k_init_coords(const double* __restrict__ coords,
                                                     const int32_t* __restrict__ perm, int32_t n, int soa,
                                                     R* __restrict__ X0, R* __restrict__ X1)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
    if (k >= n) return;
    const int64_t o = perm[k];
    const double2 p = *reinterpret_cast<const double2*>(coords + 2 * o);
    const R x = static_cast<R>(p.x), y = static_cast<R>(p.y);
    if (soa) {
        X0[k] = x; X0[n + k] = y;
        X1[k] = x; X1[n + k] = y;
    } else {
        X0[2 * k] = x; X0[2 * k + 1] = y;
        X1[2 * k] = x; X1[2 * k + 1] = y;
    }
}

// Buffer src = X[src], or X[sweeps run % 2] when `runs` is given (Form A,
// read on the device so that the host need not wait for the sweep loop).
template <typename R>
__global__ __launch_bounds__(kBS) void k_unpermute(const R* __restrict__ X0, int src, const MeshState* __restrict__ runs,
                                                   const int32_t* __restrict__ perm, int32_t n, int soa,
                                                   double* __restrict__ out)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
    if (k >= n) return;
    const R* X = X0 + 2 * static_cast<int64_t>(n) * (runs ? (runs->s & 1) : src);
    const int64_t o = perm[k];
    const R x = soa ? X[k] : X[2 * k], y = soa ? X[n + k] : X[2 * k + 1];
    *reinterpret_cast<double2*>(out + 2 * o) = make_double2(static_cast<double>(x), static_cast<double>(y));
}

__global__ __launch_bounds__(kBS) void k_unpermute_flags(const uint64_t* __restrict__ bits, int64_t words,
                                                         const int32_t* __restrict__ new_of_old, int32_t n,
                                                         int32_t n_free, int32_t iterations,
                                                         const MeshState* __restrict__ state, uint8_t* __restrict__ out)
{
    const int64_t nbytes = (static_cast<int64_t>(n) + 7) / 8;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
    if (g >= nbytes * iterations) return;
    const int32_t runs = state->s;
    const int64_t s = g / nbytes, B = g % nbytes;
    uint32_t byte = 0;
    if (s < runs) {
        for (int q = 0; q < 8; ++q) {
            const int64_t i = 8 * B + q;
            if (i >= n) break;
            const int32_t k = new_of_old[i];
            if (k < n_free && ((bits[s * words + k / 64] >> (k % 64)) & 1ull)) byte |= 1u << q;
        }
    }
    out[g] = static_cast<uint8_t>(byte);
}

// Bits per axis of the Hilbert cells of the counting sort for n_free free
// nodes in nc colour classes: grown while a class still has about two nodes
// per cell or more, at most 2^25 buckets.  The bucket count stays below
// max(4 nc, 2 n_free).
int hilbert_bits(int64_t n_free, int nc)
{
    int bits = 1;
    while (bits < 12 && (static_cast<int64_t>(nc) << (2 * bits)) < n_free / 2 &&
           (static_cast<int64_t>(nc) << (2 * (bits + 1))) <= (int64_t(1) << 25))
        ++bits;
    return bits;
}

// Scratch bytes make_order takes for n nodes (at most 128 colour classes).
size_t order_bytes(int64_t n)
{
    const int64_t nbk = std::max<int64_t>(4 * 128, 2 * n);
    return 3 * Arena::piece(4 * static_cast<size_t>(n + 1)) + Arena::piece(4 * sizeof(uint64_t)) +
           Arena::piece(4 * sizeof(uint64_t) * kBboxBlocks) +
           2 * Arena::piece(4 * static_cast<size_t>(nbk + 1)) + scan_bytes(std::max<int64_t>(n, nbk));
}

sl_status make_order(const SetupArgs& a, const sl_options& o, const uint8_t* bnd, int32_t n_free,
                     const int32_t* color, int32_t n_colors, DevMesh& m, hipStream_t st, Arena& scratch)
{
    const int32_t n = a.n;
    const int gb = div_up(n, kBS);
    const size_t mk = scratch.mark();
    int32_t *flag = nullptr, *pos = nullptr;
    sl_status r;
    if ((r = scratch.take(&flag, n)) || (r = scratch.take(&pos, static_cast<size_t>(n) + 1))) return r;
    int32_t* cs = m.color_start_h;
    cs[0] = 0;
    if (o.reorder == SL_REORDER_HILBERT && n_free > 0) {
        // bucket counting sort: (colour, Hilbert cell); order inside a bucket is arbitrary,
        // which no result depends on (rows and triangles keep their order).
        const int nc = color ? n_colors : 1;
        const int bits = hilbert_bits(n_free, nc);
        const int64_t nbk = static_cast<int64_t>(nc) << (2 * bits);
        const int nbb = std::min(gb, kBboxBlocks);
        uint64_t *bb = nullptr, *bbp = nullptr;
        int32_t *count = nullptr, *start = nullptr, *key = nullptr;
        if ((r = scratch.take(&bb, 4)) || (r = scratch.take(&bbp, 4 * static_cast<size_t>(nbb))) ||
            (r = scratch.take(&count, nbk)) || (r = scratch.take(&start, nbk + 1)) || (r = scratch.take(&key, n)))
            return r;
        k_bbox<<<nbb, kBS, 0, st>>>(a.coords, n, bbp);
        k_bbox_fold<<<1, kBS, 0, st>>>(bbp, nbb, bb);
        k_fill_i32<<<div_up(nbk, 256), 256, 0, st>>>(count, nbk, 0);
        k_bucket<<<gb, kBS, 0, st>>>(a.coords, bnd, color, n, bits, bb, key, count, flag);
        if ((r = scan_exclusive(count, start, nbk, st, &scratch))) return r;
        if (color) {
            // nc <= 128: the class starts fit the mesh's table
            for (int c = 0; c <= nc; ++c) {
                SL_HIP(hipMemcpyAsync(&cs[c], start + (static_cast<int64_t>(c) << (2 * bits)), sizeof(int32_t),
                                      hipMemcpyDeviceToHost, st));
            }
            SL_HIP(hipStreamSynchronize(st));
        } else {
            cs[1] = n_free;
        }
        k_bucket_scatter<<<gb, kBS, 0, st>>>(bnd, n, key, flag, start, m.new_of_old, m.perm);
    } else if (n_free > 0) {
        // stable: free nodes (by colour class when coloured) in caller order
        const int nc = color ? n_colors : 1;
        int32_t base = 0;
        for (int c = 0; c < nc; ++c) {
            k_select<<<gb, kBS, 0, st>>>(bnd, color, c, 0, n, flag);
            if ((r = scan_exclusive(flag, pos, n, st, &scratch))) return r;
            k_place<<<gb, kBS, 0, st>>>(flag, pos, base, n, m.new_of_old, m.perm);
            int32_t cnt = 0;
            SL_HIP(hipMemcpyAsync(&cnt, pos + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            SL_HIP(hipStreamSynchronize(st));
            base += cnt;
            cs[c + 1] = base;
        }
    }
    if (n_free < n) {
        k_select<<<gb, kBS, 0, st>>>(bnd, nullptr, 0, 1, n, flag);
        if ((r = scan_exclusive(flag, pos, n, st, &scratch))) return r;
        k_place<<<gb, kBS, 0, st>>>(flag, pos, n_free, n, m.new_of_old, m.perm);
    }
    scratch.rewind(mk);
    SL_HIP(hipGetLastError());
    return SL_OK;
}

}  // namespace

sl_status scan_exclusive(const int32_t* in, int32_t* out, int64_t n, hipStream_t st, Arena* scratch)
{
    const size_t mk = scratch ? scratch->mark() : 0;
    const sl_status r = scan_rec(in, out, n, out + n, st, scratch);
    if (scratch) scratch->rewind(mk);
    return r;
}

void devmesh_free(DevMesh& m, hipStream_t st)
{
    block_give(m.block, st);
    m.perm = m.new_of_old = m.row_ptr = m.nbr = m.fan_ptr = nullptr;
    m.fan = nullptr;
    m.X[0] = m.X[1] = nullptr;
    m.work = nullptr;
    m.tile_data = nullptr;
}

// Nodes per tile: Form A's tuned or default size; a colour-class tile
// (Form B) holds 256 unless asked otherwise (its halo is several times
// longer than a Form A tile's, and 512-node class tiles leave room for only
// two work-groups per CU).
// Colour-class tiles of 512 nodes from this many mesh nodes up, else 256.
// A larger class tile re-reads fewer halo positions per own node, but gives
// fewer tiles: on the 4096^2 grid 512 took 1.04 ms per sweep against 1.11
// (256) and 1.36 (128), on the 1024^2 grid 0.118 against 0.130 ms; on
// Delaunay meshes of 30K and 100K points 256 was faster (0.078 and 0.080
// against 0.096 and 0.100 ms).
constexpr int32_t kLargeClassMesh = 1 << 20;

// Form A tiles of 512 nodes from this many mesh nodes up, else 256, when
// neither the options nor sl_autotune fix the size (batches, servers and
// handles fix it before setup, so that one work list has one size).  A
// small mesh's sweep is one round of tiles, so smaller tiles finish sooner:
// Delaunay meshes of 10K, 30K and 100K points took 8.3, 9.4 and 11.2 us per
// sweep with 256 against 10.4, 10.8 and 12.1 with 512; the 1024^2 grid
// 0.033 ms with either.
constexpr int32_t kLargeTileMesh = 1 << 19;

static int32_t tile_size_for(const sl_options& o, int32_t n)
{
    if (o.form == SL_JACOBI) {
        if (o.tile_nodes || tuned_shape().tile_nodes) return resolve_tile_nodes(o);
        return n >= kLargeTileMesh ? 512 : 256;
    }
    if (o.tile_nodes) return o.tile_nodes;
    return n >= kLargeClassMesh ? 512 : 256;
}

// Whether setup aims for the tile path, decided before validation as
// setup_mesh decides it.
static bool wants_tiles(const sl_options& o, bool resident, bool class_tiles_ok)
{
    if (o.kernel == SL_KERNEL_NODE || o.kernel == SL_KERNEL_LANES || resident) return false;
    // Form B takes its colour-class tiles on request only: the node kernel
    // sweeps it faster (each class phase gathers its neighbours through L2
    // instead of staging halos several times longer than the class tile)
    return o.form == SL_JACOBI || (o.kernel == SL_KERNEL_TILE && class_tiles_ok && o.precision == SL_F64);
}

size_t mesh_block_bytes(int32_t n, int64_t nnz, int64_t ninc, const sl_options& o, bool class_tiles_ok)
{
    // the same kernel choice as setup_mesh makes before validation
    const bool resident = o.kernel == SL_KERNEL_RESIDENT ||
                          (o.kernel == SL_KERNEL_AUTO && o.form == SL_INPLACE_COLORED &&
                           resident_fits(n, nnz, ninc, o.form == SL_INPLACE_COLORED));
    const bool want_tiles = wants_tiles(o, resident, class_tiles_ok);
    const size_t rb = o.precision == SL_F32 ? 4 : 8;
    const size_t un = static_cast<size_t>(n);
    size_t pb = 2 * Arena::piece(4 * un) + 2 * Arena::piece(4 * (un + 1)) + Arena::piece(4 * un * rb);
    pb += want_tiles ? tile_bytes(n, nnz, ninc, tile_size_for(o, n), o.form != SL_JACOBI)
                     : Arena::piece(4 * static_cast<size_t>(nnz)) + Arena::piece(2 * static_cast<size_t>(ninc)) +
                           Arena::piece(4 * un);
    return pb;
}

size_t setup_scratch_bytes(int32_t n)
{
    const size_t un = static_cast<size_t>(n);
    const size_t rows_bytes = 2 * Arena::piece(4 * un) + scan_bytes(n);
    const int gb = div_up(n, kBS);
    return Arena::piece(sizeof(ValStats)) + Arena::piece(sizeof(ValStats) * static_cast<size_t>(gb)) +
           Arena::piece(4 * un) + Arena::piece(4) +
           std::max({order_bytes(n), rows_bytes, tile_scratch_bytes(),
                     2 * Arena::piece(4 * un) + Arena::piece(8)});   // the colouring's lists
}

sl_status setup_mesh(const SetupArgs& a, const sl_options& o, DevMesh& m, int32_t mesh, hipStream_t st)
{
    const int32_t n = a.n;
    m.n = n;
    m.n_tris = a.n_tris;
    m.layout = o.layout;
    m.precision = o.precision;
    sl_status r;
    // the resident kernel when asked for, and automatically for Form B
    // (faster there than the node kernel's launch per colour class),
    // checked against bounds known before validation (check_options has
    // restricted it to f64; Form B is f64 only)
    const bool res_fit = resident_fits(n, a.nnz, a.ninc, o.form == SL_INPLACE_COLORED);
    if (o.kernel == SL_KERNEL_RESIDENT && !res_fit) return fail(SL_EINVAL, "mesh too large for the resident kernel");
    m.resident = o.kernel == SL_KERNEL_RESIDENT ||
                 (o.kernel == SL_KERNEL_AUTO && o.form == SL_INPLACE_COLORED && res_fit);
    m.lane_width = o.kernel == SL_KERNEL_LANES ? resolve_lane_width(o) : 0;
    const bool want_tiles = wants_tiles(o, m.resident, m.class_tiles_ok);
    const size_t un = static_cast<size_t>(n);
    // Two reservations: the mesh's own arrays, sized from bounds known before
    // validation (n >= free nodes, a.nnz and a.ninc >= their rows and fans),
    // and the setup's temporaries, given back when setup ends.
    Arena persist, scratch;
    const size_t pb = mesh_block_bytes(n, a.nnz, a.ninc, o, m.class_tiles_ok);
    const size_t sb = setup_scratch_bytes(n);
    const int gb = div_up(n, kBS);
    if (m.carve) {
        if (m.carve_bytes < pb) return fail(SL_EINVAL, "internal: mesh region smaller than its arrays");
        persist.adopt(m.carve, pb);
    } else {
        if ((r = persist.reserve(pb, st))) return r;
        m.block = persist.base;
    }
    if (m.scratch_carve) {
        if (m.scratch_carve_bytes < sb) return fail(SL_EINVAL, "internal: setup region smaller than its temporaries");
        scratch.adopt(m.scratch_carve, sb);
    } else if ((r = scratch.reserve(sb, st))) {
        return r;
    }
    struct GiveBack {
        Arena& ar;
        hipStream_t st;
        ~GiveBack() { ar.release(st); }
    } give_back{scratch, st};

    // ---- validation
    ValStats *vs = nullptr, *vpart = nullptr;
    if ((r = scratch.take(&vs, 1)) || (r = scratch.take(&vpart, gb))) return r;
    SL_HIP(hipMemsetAsync(vs, 0, sizeof(ValStats), st));
    ValArgs va{a.coords, n, a.nbr_ptr, a.nbr_idx, a.tri_ptr, a.tri_idx, a.tris, a.n_tris, a.boundary,
               a.nnz, a.ninc, o.form == SL_INPLACE_COLORED, o.precision == SL_F32 ? 0x1p61 : 0x1p500};
    if (a.n_tris > 0) k_validate_tris<<<div_up(a.n_tris, kBS), kBS, 0, st>>>(a.tris, a.n_tris, n, vs);
    if (want_tiles && o.form == SL_JACOBI && a.n_tris > 0 && a.ninc > 0)
        k_validate_incidence<<<div_up(a.n_tris, kBS), kBS, 0, st>>>(a.tris, a.n_tris, n, a.boundary, a.tri_ptr,
                                                                  a.tri_idx, a.ninc, vs);
    k_validate_nodes<<<gb, kBS, 0, st>>>(va, vpart);
    k_validate_fold<<<1, 1024, 0, st>>>(vpart, gb, vs);
    SL_HIP(hipGetLastError());
    ValStats h{};
    SL_HIP(hipMemcpyAsync(&h, vs, sizeof(ValStats), hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    if (h.err & (VE_PTR | VE_RANGE | VE_COORD)) {
        std::string msg = "invalid input:";
        if (h.err & VE_PTR) msg += " CSR offsets not monotone or out of range;";
        if (h.err & VE_RANGE) msg += " node or triangle id out of range;";
        if (h.err & VE_COORD)
            msg += o.precision == SL_F32 ? " coordinate not finite or of magnitude >= 2^61 (single precision);"
                                         : " coordinate not finite or of magnitude >= 2^500;";
        return fail(SL_EINVAL, msg);
    }
    if (h.err & kValErrors) {
        std::string msg = "invalid topology:";
        if (h.err & VE_SELF) msg += " node lists itself as a neighbour;";
        if (h.err & VE_TRIREP) msg += " triangle with a repeated vertex;";
        if (h.err & VE_NOTIN) msg += " incident triangle does not contain its node;";
        if (h.err & VE_MISSING) msg += " triangle vertex missing from the node's neighbour row;";
        if (h.err & VE_EMPTY) msg += " free node without neighbours;";
        if (h.err & VE_VALENCE) msg += " free node with more than 127 neighbours;";
        if (h.err & VE_ASYM) msg += " neighbour rows are not symmetric (needed by the coloured form);";
        return fail(SL_ETOPO, msg);
    }
    m.n_free = h.n_free;
    m.max_deg = h.max_deg_free;
    m.max_inc = h.max_inc_free;

    if ((r = persist.take(&m.perm, n)) || (r = persist.take(&m.new_of_old, n))) return r;

    // ---- colouring (coloured form)
    int32_t* color = nullptr;
    m.n_colors = 0;
    if (o.form == SL_INPLACE_COLORED && m.n_free > 0) {
        int32_t* remaining = nullptr;
        if ((r = scratch.take(&color, n)) || (r = scratch.take(&remaining, 1))) return r;
        // rounds over a shrinking list of the uncoloured free nodes
        const size_t cmark = scratch.mark();
        int32_t *list = nullptr, *next = nullptr, *cnt2 = nullptr;
        if ((r = scratch.take(&list, m.n_free)) || (r = scratch.take(&next, m.n_free)) ||
            (r = scratch.take(&cnt2, 2)))
            return r;
        k_fill_i32<<<1, 2, 0, st>>>(cnt2, 2, 0);
        k_color_init<<<div_up(n, kColorBS), kColorBS, 0, st>>>(n, a.boundary, color, list, cnt2);
        // rounds read their list's length on the device; the host looks at
        // it every kColorRounds rounds (rounds past the last are empty), and
        // sizes the launches by the last length it saw
        int32_t left = m.n_free, cur = 0;
        for (int round = 0; left > 0; round += kColorRounds) {
            if (round > m.n_free) return fail(SL_EDEVICE, "colouring made no progress");
            for (int k = 0; k < kColorRounds; ++k) {
                k_fill_i32<<<1, 1, 0, st>>>(cnt2 + (cur ^ 1), 1, 0);
                k_color_round<<<div_up(left, kColorBS), kColorBS, 0, st>>>(a.nbr_ptr, a.nbr_idx, a.boundary, color,
                                                                          list, cnt2 + cur, next, cnt2 + (cur ^ 1));
                std::swap(list, next);
                cur ^= 1;
            }
            SL_HIP(hipMemcpyAsync(&left, cnt2 + cur, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            SL_HIP(hipStreamSynchronize(st));
        }
        scratch.rewind(cmark);
        k_fill_i32<<<1, 1, 0, st>>>(remaining, 1, -1);
        k_max_i32<<<std::min(gb, 1024), kBS, 0, st>>>(color, n, remaining);
        int32_t mx = -1;
        SL_HIP(hipMemcpyAsync(&mx, remaining, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        SL_HIP(hipStreamSynchronize(st));
        m.n_colors = mx + 1;
        if (m.n_colors > 128) return fail(SL_ETOPO, "more than 128 colour classes");
        // the resident kernel holds a bounded number of classes: an automatic
        // choice falls back to the node kernel, an explicit one fails
        if (m.resident && m.n_colors > kResidentClasses) {
            if (o.kernel == SL_KERNEL_RESIDENT)
                return fail(SL_EINVAL, "the resident kernel holds at most " + std::to_string(kResidentClasses) +
                                           " colour classes");
            m.resident = false;
        }
    }

    // ---- node order
    if ((r = make_order(a, o, a.boundary, m.n_free, color, m.n_colors, m, st, scratch))) return r;

    // ---- rows and fans of free nodes
    if ((r = persist.take(&m.row_ptr, static_cast<size_t>(m.n_free) + 1)) ||
        (r = persist.take(&m.fan_ptr, static_cast<size_t>(m.n_free) + 1)))
        return r;
    const size_t mk = scratch.mark();
    int32_t *deg = nullptr, *inc = nullptr;
    if ((r = scratch.take(&deg, m.n_free)) || (r = scratch.take(&inc, m.n_free))) return r;
    const int gf = div_up(m.n_free > 0 ? m.n_free : 1, kBS);
    if (m.n_free > 0) k_degrees<<<gf, kBS, 0, st>>>(m.perm, m.n_free, a.nbr_ptr, a.tri_ptr, deg, inc);
    if ((r = scan_exclusive(deg, m.row_ptr, m.n_free, st, &scratch)) ||
        (r = scan_exclusive(inc, m.fan_ptr, m.n_free, st, &scratch)))
        return r;
    int32_t tot[2] = {0, 0};
    SL_HIP(hipMemcpyAsync(&tot[0], m.row_ptr + m.n_free, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SL_HIP(hipMemcpyAsync(&tot[1], m.fan_ptr + m.n_free, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    scratch.rewind(mk);
    m.nnz_free = tot[0];
    m.ninc_free = tot[1];
    // coordinate buffers: one block, X[1] right after X[0], in the sweep's precision
    const size_t n2 = 2 * un;
    if (m.precision == SL_F32) {
        float* xf = nullptr;
        if ((r = persist.take(&xf, 2 * n2))) return r;
        m.X[0] = xf;
        m.X[1] = xf + n2;
        k_init_coords<float><<<gb, kBS, 0, st>>>(a.coords, m.perm, n, o.layout == SL_SOA, xf, xf + n2);
    } else {
        double* xd = nullptr;
        if ((r = persist.take(&xd, 2 * n2))) return r;
        m.X[0] = xd;
        m.X[1] = xd + n2;
        k_init_coords<double><<<gb, kBS, 0, st>>>(a.coords, m.perm, n, o.layout == SL_SOA, xd, xd + n2);
    }
    // tile path for Form A (which needs consistent incidence rows: a tile
    // lists a triangle once and scores it for every own vertex) and, on
    // colour-class tiles, for Form B (each listed triangle has one own
    // vertex, whose row listed it); the node path's rows and fans otherwise
    const bool jacobi = o.form == SL_JACOBI;
    const bool tiles_ok = !jacobi || (h.err & VI_INCIDENCE) == 0;
    if (want_tiles && tiles_ok &&
        (r = build_tiles(a, m, tile_size_for(o, n), mesh, st, persist, scratch, !jacobi)))
        return r;
    if (m.tile_nodes == 0 && m.precision == SL_F32 && m.n_free > 0)
        return fail(SL_EINVAL, tiles_ok ? "single precision needs the tile path, and this mesh does not fit it"
                                        : "single precision needs the tile path, which needs every free vertex of "
                                          "a listed triangle to list it too");
    if (m.tile_nodes == 0) {
        // (a mesh that did not fit the tile path gave the tile arrays' room back,
        // which bounds this)
        const bool group = m.n_free > 0 && m.n_free < kGroupFansBelow;
        if ((r = persist.take(&m.nbr, m.nnz_free)) || (r = persist.take(&m.fan, m.ninc_free)) ||
            (group && (r = persist.take(&m.fan_split, m.n_free))))
            return r;
        if (m.n_free > 0)
            k_rows_fans<<<gf, kBS, 0, st>>>(m.perm, m.new_of_old, m.n_free, a.nbr_ptr, a.nbr_idx, a.tri_ptr,
                                            a.tri_idx, a.tris, m.row_ptr, m.nbr, m.fan_ptr, m.fan);
        if (group) k_fan_group<<<gf, kBS, 0, st>>>(m.fan_ptr, m.fan, m.fan_split, m.n_free);
    }
    SL_HIP(hipGetLastError());
    return SL_OK;
}

sl_status unpermute_coords(const DevMesh& m, int src, double* coords_out, hipStream_t st, const MeshState* runs)
{
    if (m.precision == SL_F32)
        k_unpermute<float><<<div_up(m.n, kBS), kBS, 0, st>>>(static_cast<const float*>(m.X[0]), src, runs, m.perm,
                                                              m.n, m.layout == SL_SOA, coords_out);
    else
        k_unpermute<double><<<div_up(m.n, kBS), kBS, 0, st>>>(static_cast<const double*>(m.X[0]), src, runs, m.perm,
                                                               m.n, m.layout == SL_SOA, coords_out);
    SL_HIP(hipGetLastError());
    return SL_OK;
}

sl_status unpermute_flags(const DevMesh& m, const uint64_t* bits, int32_t iterations, const MeshState* state,
                          uint8_t* out, hipStream_t st)
{
    const int64_t words = (static_cast<int64_t>(m.n_free) + 63) / 64;
    const int64_t total = (static_cast<int64_t>(m.n) + 7) / 8 * iterations;
    if (total == 0) return SL_OK;
    k_unpermute_flags<<<div_up(total, kBS), kBS, 0, st>>>(bits, words, m.new_of_old, m.n, m.n_free, iterations, state,
                                                          out);
    SL_HIP(hipGetLastError());
    return SL_OK;
}

}  // namespace sl
