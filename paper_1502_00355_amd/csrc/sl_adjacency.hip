// Adjacency from a bare triangle list, on the device.
//
// What the smoothing pass takes as input -- the node->triangle and
// node->neighbour CSR and the boundary mask -- built the way the paper
// describes it (Sec. 3.3.2 finding of neighbours, Sec. 3.3.3 determining of
// constraints):
//   * a node's incident triangles are listed in index order;
//   * its neighbours are the other two vertices of those triangles, taken
//     triangle by triangle in index order and, inside a triangle, in stored
//     order (a triangle (v1,v2,v3) gives v1 the pair v2,v3; v2 the pair
//     v1,v3; v3 the pair v1,v2), each kept once where it first appears;
//   * a node is interior iff every neighbour was seen exactly twice (each
//     edge at the node lies in two triangles).
// Steps: incidence counts, scan, unordered fill, per-row sort; then one
// work-item per node walks its sorted incidence row, deduplicates into a
// scratch row of capacity 2 x incidences, counts, scan, compaction.
#include <algorithm>
#include <string>

#include "sl_common.h"

namespace sl {

namespace {

constexpr int kAB = 256;

__global__ __launch_bounds__(kAB) void k_adj_validate(const int32_t* __restrict__ tris, int32_t n_tris, int32_t n,
                                                      uint32_t* __restrict__ err)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kAB + threadIdx.x;
    if (t >= n_tris) return;
    const int32_t a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    uint32_t e = 0;
    if (a < 0 || b < 0 || c < 0 || a >= n || b >= n || c >= n) e |= 1u;
    else if (a == b || b == c || a == c) e |= 2u;
    if (e) atomicOr(err, e);
}

__global__ __launch_bounds__(kAB) void k_adj_count(const int32_t* __restrict__ tris, int64_t m3,
                                                   int32_t* __restrict__ cnt)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kAB + threadIdx.x;
    if (k < m3) atomicAdd(cnt + tris[k], 1);
}

__global__ __launch_bounds__(kAB) void k_adj_fill(const int32_t* __restrict__ tris, int64_t m3,
                                                  const int32_t* __restrict__ tri_ptr, int32_t* __restrict__ cursor,
                                                  int32_t* __restrict__ tri_idx)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kAB + threadIdx.x;
    if (k >= m3) return;
    const int32_t v = tris[k];
    tri_idx[tri_ptr[v] + atomicAdd(cursor + v, 1)] = static_cast<int32_t>(k / 3);
}

// Insertion sort of each incidence row (rows are short: a node is in few
// triangles on the meshes this serves).
__global__ __launch_bounds__(kAB) void k_adj_sort_rows(int32_t n, const int32_t* __restrict__ tri_ptr,
                                                       int32_t* __restrict__ tri_idx)
{
    const int32_t v = static_cast<int32_t>(blockIdx.x) * kAB + threadIdx.x;
    if (v >= n) return;
    const int32_t b = tri_ptr[v], e = tri_ptr[v + 1];
    for (int32_t i = b + 1; i < e; ++i) {
        const int32_t x = tri_idx[i];
        int32_t j = i - 1;
        while (j >= b && tri_idx[j] > x) {
            tri_idx[j + 1] = tri_idx[j];
            --j;
        }
        tri_idx[j + 1] = x;
    }
}

// One node: its distinct neighbours in order of first appearance (into the
// scratch row at 2*tri_ptr[v]), their count and the boundary flag.
__global__ __launch_bounds__(kAB) void k_adj_rows(int32_t n, const int32_t* __restrict__ tris,
                                                  const int32_t* __restrict__ tri_ptr,
                                                  const int32_t* __restrict__ tri_idx, int32_t* __restrict__ row,
                                                  uint8_t* __restrict__ seen, int32_t* __restrict__ deg,
                                                  uint8_t* __restrict__ boundary)
{
    const int32_t v = static_cast<int32_t>(blockIdx.x) * kAB + threadIdx.x;
    if (v >= n) return;
    const int32_t b = tri_ptr[v], e = tri_ptr[v + 1];
    int32_t* r = row + 2 * static_cast<int64_t>(b);
    uint8_t* c = seen + 2 * static_cast<int64_t>(b);
    int32_t L = 0;
    for (int32_t q = b; q < e; ++q) {
        const int64_t t = tri_idx[q];
        const int32_t a0 = tris[3 * t], a1 = tris[3 * t + 1], a2 = tris[3 * t + 2];
        const int32_t u0 = a0 == v ? a1 : a0;
        const int32_t u1 = a2 == v ? a1 : a2;
        for (int s = 0; s < 2; ++s) {
            const int32_t u = s == 0 ? u0 : u1;
            int32_t k = 0;
            while (k < L && r[k] != u) ++k;
            if (k == L) {
                r[L] = u;
                c[L] = 1;
                ++L;
            } else if (c[k] < 255) {
                c[k] = static_cast<uint8_t>(c[k] + 1);
            }
        }
    }
    bool interior = L > 0;
    for (int32_t k = 0; k < L; ++k) interior = interior && c[k] == 2;
    deg[v] = L;
    boundary[v] = interior ? 0 : 1;
}

__global__ __launch_bounds__(kAB) void k_adj_copy(int32_t n, const int32_t* __restrict__ tri_ptr,
                                                  const int32_t* __restrict__ row,
                                                  const int32_t* __restrict__ nbr_ptr, int32_t* __restrict__ nbr_idx)
{
    const int32_t v = static_cast<int32_t>(blockIdx.x) * kAB + threadIdx.x;
    if (v >= n) return;
    const int32_t* r = row + 2 * static_cast<int64_t>(tri_ptr[v]);
    const int32_t b = nbr_ptr[v], L = nbr_ptr[v + 1] - b;
    for (int32_t k = 0; k < L; ++k) nbr_idx[b + k] = r[k];
}

// Device buffers of one build, released on every exit path.
struct AdjState {
    hipStream_t st;
    uint32_t* err = nullptr;
    int32_t *cnt = nullptr, *tri_ptr = nullptr, *tri_idx = nullptr, *row = nullptr, *deg = nullptr;
    int32_t *nbr_ptr = nullptr, *nbr_idx = nullptr;
    uint8_t *seen = nullptr, *bnd = nullptr;
    explicit AdjState(hipStream_t s) : st(s) {}
    ~AdjState()
    {
        dfree(err, st); dfree(cnt, st); dfree(tri_ptr, st); dfree(tri_idx, st); dfree(row, st); dfree(deg, st);
        dfree(nbr_ptr, st); dfree(nbr_idx, st); dfree(seen, st); dfree(bnd, st);
        (void)hipStreamSynchronize(st);
    }
};

}  // namespace

// Builds the adjacency of a device triangle list on `st` into device
// buffers of the library and copies it to the caller's arrays with `kind`
// (device-to-device or device-to-host).  The caller's arrays are written
// only when everything succeeded; a null nbr_idx asks for *nnz only.
sl_status build_adjacency(const int32_t* d_tris, int32_t n_tris, int32_t n, int32_t* nbr_ptr, int32_t* nbr_idx,
                          int64_t nbr_capacity, int32_t* tri_ptr, int32_t* tri_idx, uint8_t* boundary, int64_t* nnz,
                          hipMemcpyKind kind, hipStream_t st)
{
    AdjState s(st);
    const int64_t m3 = 3 * static_cast<int64_t>(n_tris);
    sl_status r;
    if ((r = dalloc(&s.err, 1, st)) || (r = dalloc(&s.cnt, static_cast<size_t>(n) + 1, st)) ||
        (r = dalloc(&s.tri_ptr, static_cast<size_t>(n) + 1, st)) ||
        (r = dalloc(&s.tri_idx, static_cast<size_t>(std::max<int64_t>(m3, 1)), st)) ||
        (r = dalloc(&s.row, static_cast<size_t>(std::max<int64_t>(2 * m3, 1)), st)) ||
        (r = dalloc(&s.seen, static_cast<size_t>(std::max<int64_t>(2 * m3, 1)), st)) ||
        (r = dalloc(&s.deg, static_cast<size_t>(n) + 1, st)) ||
        (r = dalloc(&s.nbr_ptr, static_cast<size_t>(n) + 1, st)) || (r = dalloc(&s.bnd, n, st)))
        return r;
    SL_HIP(hipMemsetAsync(s.err, 0, sizeof(uint32_t), st));
    SL_HIP(hipMemsetAsync(s.cnt, 0, sizeof(int32_t) * (static_cast<size_t>(n) + 1), st));
    if (n_tris > 0) {
        k_adj_validate<<<div_up(n_tris, kAB), kAB, 0, st>>>(d_tris, n_tris, n, s.err);
        SL_HIP(hipGetLastError());
    }
    uint32_t herr = 0;
    SL_HIP(hipMemcpyAsync(&herr, s.err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    if (herr & 1u) return fail(SL_EINVAL, "triangle vertex id out of range");
    if (herr & 2u) return fail(SL_ETOPO, "triangle with a repeated vertex");

    const int gn = div_up(std::max(n, 1), kAB);
    if (m3 > 0) k_adj_count<<<div_up(m3, kAB), kAB, 0, st>>>(d_tris, m3, s.cnt);
    if ((r = scan_exclusive(s.cnt, s.tri_ptr, n, st))) return r;
    SL_HIP(hipMemsetAsync(s.cnt, 0, sizeof(int32_t) * (static_cast<size_t>(n) + 1), st));
    if (m3 > 0) k_adj_fill<<<div_up(m3, kAB), kAB, 0, st>>>(d_tris, m3, s.tri_ptr, s.cnt, s.tri_idx);
    k_adj_sort_rows<<<gn, kAB, 0, st>>>(n, s.tri_ptr, s.tri_idx);
    k_adj_rows<<<gn, kAB, 0, st>>>(n, d_tris, s.tri_ptr, s.tri_idx, s.row, s.seen, s.deg, s.bnd);
    if ((r = scan_exclusive(s.deg, s.nbr_ptr, n, st))) return r;
    SL_HIP(hipGetLastError());
    int32_t total = 0;
    SL_HIP(hipMemcpyAsync(&total, s.nbr_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    *nnz = total;
    if (!nbr_idx) return SL_OK;
    if (total > nbr_capacity)
        return fail(SL_EINVAL, "nbr_idx holds " + std::to_string(nbr_capacity) + " entries, " +
                                   std::to_string(total) + " are needed");
    if ((r = dalloc(&s.nbr_idx, static_cast<size_t>(std::max(total, 1)), st))) return r;
    k_adj_copy<<<gn, kAB, 0, st>>>(n, s.tri_ptr, s.row, s.nbr_ptr, s.nbr_idx);
    SL_HIP(hipGetLastError());
    const size_t n1 = static_cast<size_t>(n) + 1;
    if (kind == hipMemcpyDeviceToHost) {
        if ((r = copy_to_host(nbr_ptr, s.nbr_ptr, sizeof(int32_t) * n1, st)) ||
            (r = copy_to_host(nbr_idx, s.nbr_idx, sizeof(int32_t) * total, st)) ||
            (r = copy_to_host(tri_ptr, s.tri_ptr, sizeof(int32_t) * n1, st)) ||
            (r = copy_to_host(tri_idx, s.tri_idx, sizeof(int32_t) * m3, st)) ||
            (r = copy_to_host(boundary, s.bnd, static_cast<size_t>(n), st)))
            return r;
        return SL_OK;
    }
    SL_HIP(hipMemcpyAsync(nbr_ptr, s.nbr_ptr, sizeof(int32_t) * n1, kind, st));
    if (total) SL_HIP(hipMemcpyAsync(nbr_idx, s.nbr_idx, sizeof(int32_t) * total, kind, st));
    SL_HIP(hipMemcpyAsync(tri_ptr, s.tri_ptr, sizeof(int32_t) * n1, kind, st));
    if (m3) SL_HIP(hipMemcpyAsync(tri_idx, s.tri_idx, sizeof(int32_t) * m3, kind, st));
    SL_HIP(hipMemcpyAsync(boundary, s.bnd, n, kind, st));
    SL_HIP(hipStreamSynchronize(st));
    return SL_OK;
}

namespace {

sl_status check_adj_args(const int32_t* tris, int32_t n_tris, int32_t n_nodes, const int32_t* nbr_ptr,
                         const int32_t* nbr_idx, int64_t nbr_capacity, const int32_t* tri_ptr,
                         const int32_t* tri_idx, const uint8_t* boundary, const int64_t* nnz)
{
    if (!nnz) return fail(SL_EINVAL, "null nnz");
    if (n_nodes <= 0) return fail(SL_EINVAL, "n_nodes must be >= 1");
    if (n_tris < 0) return fail(SL_EINVAL, "n_tris must be >= 0");
    if (n_tris > INT32_MAX / 6) return fail(SL_EINVAL, "n_tris too large");
    if (n_tris > 0 && !tris) return fail(SL_EINVAL, "null tris with n_tris > 0");
    if (nbr_idx && (!nbr_ptr || !tri_ptr || (n_tris > 0 && !tri_idx) || !boundary))
        return fail(SL_EINVAL, "null output array");
    if (nbr_capacity < 0) return fail(SL_EINVAL, "nbr_capacity must be >= 0");
    return SL_OK;
}

}  // namespace

}  // namespace sl

extern "C" {

sl_status sl_build_adjacency_device(const int32_t* tris, int32_t n_tris, int32_t n_nodes, int32_t* nbr_ptr,
                                    int32_t* nbr_idx, int64_t nbr_capacity, int32_t* tri_ptr, int32_t* tri_idx,
                                    uint8_t* boundary, int64_t* nnz, void* stream)
{
    using namespace sl;
    set_error("");
    sl_status r = check_adj_args(tris, n_tris, n_nodes, nbr_ptr, nbr_idx, nbr_capacity, tri_ptr, tri_idx, boundary,
                                 nnz);
    if (r) return r;
    keep_pool_warm();
    return build_adjacency(tris, n_tris, n_nodes, nbr_ptr, nbr_idx, nbr_capacity, tri_ptr, tri_idx, boundary, nnz,
                           hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
}

sl_status sl_build_adjacency(const int32_t* tris, int32_t n_tris, int32_t n_nodes, int32_t* nbr_ptr,
                             int32_t* nbr_idx, int64_t nbr_capacity, int32_t* tri_ptr, int32_t* tri_idx,
                             uint8_t* boundary, int64_t* nnz)
{
    using namespace sl;
    set_error("");
    sl_status r = check_adj_args(tris, n_tris, n_nodes, nbr_ptr, nbr_idx, nbr_capacity, tri_ptr, tri_idx, boundary,
                                 nnz);
    if (r) return r;
    keep_pool_warm();
    hipStream_t st = nullptr;
    SL_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    int32_t* d_tris = nullptr;
    const size_t m3 = 3 * static_cast<size_t>(n_tris);
    r = dalloc(&d_tris, std::max<size_t>(m3, 1), st);
    if (!r) r = copy_to_device(d_tris, tris, sizeof(int32_t) * m3, st);
    if (!r)
        r = build_adjacency(d_tris, n_tris, n_nodes, nbr_ptr, nbr_idx, nbr_capacity, tri_ptr, tri_idx, boundary, nnz,
                            hipMemcpyDeviceToHost, st);
    dfree(d_tris, st);
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    return r;
}

}  // extern "C"
