// The Smart Laplacian sweep on gfx950.
//
// One work-item per free node (paper Sec. 3.3.4, "The Iterating Procedure"):
//   1. gather the neighbours' positions in row order, summing them, and
//      divide once by the neighbour count: the Laplacian candidate (eq. (2));
//   2. for every incident triangle evaluate the quality in the triangle's
//      stored vertex order twice -- with the node at its current position
//      and at the candidate -- keeping the two minima (Sec. 2.1);
//   3. keep the candidate iff the new minimum is >= the old one (or >, for
//      the strict rule), write the node's position to the output buffer;
//   4. fold the squared displacement into the sweep's maximum and count the
//      accepted nodes.
// The gathered neighbour positions are parked in LDS, one column per
// work-item, so that the triangle loop can address them by the row slots
// stored in the fan entries.  The paper re-evaluates every triangle from
// each of its three vertices (Sec. 5.3); so does this kernel -- each
// evaluation reads only data the node already holds, which costs less than
// a per-triangle pass that would have to write and re-read qualities.
//
// Form A (eq. (2)): reads buffer s%2, writes buffer (s+1)%2.
// Form B (eq. (3)): one launch per colour class, in place; no two nodes of a
// class are adjacent, so no work-item reads a position another writes.
#include <cmath>
#include <type_traits>

#include "sl_common.h"

namespace sl {

namespace {

// 2*sqrt(3) rounded to double: q = 4*sqrt(3)*A / sum(l^2) = (2*sqrt(3)*cr) / S.
constexpr double kTwoSqrt3 = 0x1.bb67ae8584caap+1;

// Old and new quality of the triangle whose stored order puts the node at
// position p, the vertex `a` at p+1 and `b` at p+2 (mod 3): the node at o,
// then at its candidate c.  With u = a - node, v = b - node and w = b - a,
// the stored order's edge vectors p1 - p0, p2 - p0, p2 - p1 are (u, v, w)
// for p = 0, (-v, -w, u) for p = 1 and (w, -u, -v) for p = 2.  A negation
// is exact and fl(y - x) = -fl(x - y), so the cross product is
// P.x Q.y - Q.x P.y with (P, Q) = (u, v), (v, w) or (u, w), and the sum of
// squared lengths (|p1-p0|^2 + |p2-p1|^2) + |p2-p0|^2 is (Lu + Lw) + Lv,
// (Lv + Lu) + Lw or (Lw + Lv) + Lu: the same roundings as evaluating the
// stored order directly, every operation one rounded double operation
// without contraction.  w and its length are shared by the
// two evaluations, and selects pick operands instead of rebuilding the
// order (the lanes of a wave hold different p: a branch per p made a wave
// run all three orders one after the other).
__device__ __forceinline__ void fan_qualities(int p, const double2 o, const double2 c, const double2 a,
                                              const double2 b, double& qold, double& qnew)
{
    const double wx = b.x - a.x, wy = b.y - a.y;
    const double Lw = wx * wx + wy * wy;
    auto one = [&](double px, double py) {
        const double ux = a.x - px, uy = a.y - py, vx = b.x - px, vy = b.y - py;
        const double Lu = ux * ux + uy * uy, Lv = vx * vx + vy * vy;
        const double Px = p == 1 ? vx : ux, Py = p == 1 ? vy : uy;
        const double Qx = p == 0 ? vx : wx, Qy = p == 0 ? vy : wy;
        const double X = p == 2 ? Lv : Lu, Y = p == 1 ? Lv : Lw, Z = p == 0 ? Lv : (p == 1 ? Lw : Lu);
        const double cr = Px * Qy - Qx * Py;
        const double S = (X + Y) + Z;
        const double q = (kTwoSqrt3 * cr) / S;
        return S == 0.0 ? 0.0 : q;
    };
    qold = one(o.x, o.y);
    qnew = one(c.x, c.y);
}

// The same for a stored position P known at compile time (the colour-class
// tiles list each node's fan entries grouped by position): no selects.
template <int P>
__device__ __forceinline__ void fan_qualities_p(const double2 o, const double2 c, const double2 a, const double2 b,
                                                double& qold, double& qnew)
{
    const double wx = b.x - a.x, wy = b.y - a.y;
    const double Lw = wx * wx + wy * wy;
    auto one = [&](double px, double py) {
        const double ux = a.x - px, uy = a.y - py, vx = b.x - px, vy = b.y - py;
        const double Lu = ux * ux + uy * uy, Lv = vx * vx + vy * vy;
        double cr, S;
        if (P == 0) {
            cr = ux * vy - vx * uy;
            S = (Lu + Lw) + Lv;
        } else if (P == 1) {
            cr = vx * wy - wx * vy;
            S = (Lu + Lv) + Lw;
        } else {
            cr = ux * wy - wx * uy;
            S = (Lv + Lw) + Lu;
        }
        const double q = (kTwoSqrt3 * cr) / S;
        return S == 0.0 ? 0.0 : q;
    };
    qold = one(o.x, o.y);
    qnew = one(c.x, c.y);
}

template <bool SOA>
__device__ __forceinline__ double2 ld(const double* X, int64_t n, int64_t i)
{
    if (SOA) return make_double2(X[i], X[n + i]);
    return reinterpret_cast<const double2*>(X)[i];
}

template <bool SOA>
__device__ __forceinline__ void st(double* X, int64_t n, int64_t i, double x, double y)
{
    if (SOA) { X[i] = x; X[n + i] = y; }
    else reinterpret_cast<double2*>(X)[i] = make_double2(x, y);
}

struct SweepArgs {
    const double* Xin;
    double* Xout;
    int64_t n;                      // total nodes (SoA stride)
    const int32_t* row_ptr;
    const int32_t* nbr;
    const int32_t* fan_ptr;
    const uint16_t* fan;            // each node's entries grouped by stored position
    const uint32_t* fan_split;      // nullable: the groups' bounds per node, or kFanUngrouped
    int32_t k_begin, k_end;         // device labels handled by this launch
    int32_t n_tiles, tiles_per_xcd; // work-group tiles; XCD-contiguous mapping
    MeshState* state;               // skip unless active; max displacement and count fold here
    uint64_t* bits;                 // nullable: this sweep's accept bits (device labels)
    int32_t* sched;                 // [kTileSchedInts]: the launch's counters and per-group slots
    int32_t close;                  // 1: the launch's last group closes the sweep of *state
};

// The end of a node-path launch: the groups' folds, and, when the launch
// closes the sweep, the close by its last group (in place of a k_advance).
template <int BS>
__device__ __forceinline__ void finish_node_launch(const SweepArgs& a, double d2, unsigned long long acc)
{
    if (a.close) {
        if (fold_through_slots<BS, true>(a.sched, a.state, d2, acc) && threadIdx.x == 0) close_state(a.state);
    } else {
        fold_through_slots<BS, false>(a.sched, a.state, d2, acc);
    }
}

// a / d correctly rounded for an integer count d in [1, 127] with y = 1/d
// correctly rounded, while the quotient is a normal number (Markstein's
// correction step: q = a*y is within an ulp, the remainder a - q*d is
// exact, and a normal quotient by an integer below 2^7 lies at least
// ulp/254 from a rounding midpoint).  Callers divide instead when |a| is
// below 128 x the smallest normal.
__device__ __forceinline__ double div_small(double a, double d, double y)
{
    const double q = a * y;
    const double r = fma(-q, d, a);
    return fma(r, y, q);
}
constexpr double kStepMin = 0x1p-1015;   // 128 x the smallest normal double

constexpr int kNodeRow = 8;   // neighbour entries whose loads are in flight together
constexpr int kNodeFan = 4;   // fan entries read together

// The fan entries [g_begin, g_end) of one node, all of stored position P,
// a few at a time with clamped indices so that their loads overlap; the
// vertices come from the work-item's LDS column.
template <int P, int MAXV, int BLOCK>
__device__ __forceinline__ void node_fan_range(int g_begin, int g_end, const uint16_t* fan,
                                               const double2 (*nb)[BLOCK], int tid, const double2 o, const double2 c,
                                               double& qo, double& qn)
{
    for (int g0 = g_begin; g0 < g_end; g0 += kNodeFan) {
        uint32_t e[kNodeFan];
#pragma unroll
        for (int u = 0; u < kNodeFan; ++u) e[u] = fan[min(g0 + u, g_end - 1)];
#pragma unroll
        for (int u = 0; u < kNodeFan; ++u) {
            if (g0 + u < g_end) {
                const double2 va = nb[(e[u] >> 2) & 127u][tid];
                const double2 vb = nb[(e[u] >> 9) & 127u][tid];
                double v, w;
                fan_qualities_p<P>(o, c, va, vb, v, w);
                if (v < qo) qo = v;
                if (w < qn) qn = w;
            }
        }
    }
}

// Persistent work-groups over the launch's tiles (BLOCK consecutive nodes
// each): the tiles are cut into 8 contiguous runs, one per XCD (work-groups
// are dealt to the XCDs round-robin), so that neighbouring tiles share an L2.
template <int BLOCK, int MAXV, bool SOA, bool GT>
__global__ __launch_bounds__(BLOCK) void k_sweep(SweepArgs a)
{
    if (!a.state->active) return;   // the whole launch returns: no group counts
    const int xcd = static_cast<int>(blockIdx.x & 7), nw = static_cast<int>(gridDim.x >> 3);
    const int t_begin = xcd * a.tiles_per_xcd, t_end = min(t_begin + a.tiles_per_xcd, a.n_tiles);

    __shared__ double2 nb[MAXV][BLOCK];   // column tid: this work-item's neighbours
    __shared__ double s_recip[kMaxValence + 1];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int i = tid; i <= kMaxValence; i += BLOCK) s_recip[i] = i ? 1.0 / static_cast<double>(i) : 0.0;
    __syncthreads();   // the reciprocal table
    double run_d2 = 0.0;
    unsigned long long run_acc = 0;
    for (int tile = t_begin + static_cast<int>(blockIdx.x >> 3); tile < t_end; tile += nw) {
        const int k = a.k_begin + tile * BLOCK + tid;
        const bool live = k < a.k_end;
        // a lane past the range repeats the last node's loads and stores nothing
        const int kk = live ? k : a.k_end - 1;
        const int32_t r0 = a.row_ptr[kk], d = a.row_ptr[kk + 1] - r0;   // d >= 1 for a free node
        const int32_t f0 = a.fan_ptr[kk], f1 = a.fan_ptr[kk + 1];
        const double2 o = ld<SOA>(a.Xin, a.n, kk);
        // the row's ids, then its positions, each group's loads in flight
        // together; the sums run in stored order
        double sx = 0.0, sy = 0.0;
        for (int j0 = 0; j0 < d; j0 += kNodeRow) {
            int32_t id[kNodeRow];
#pragma unroll
            for (int u = 0; u < kNodeRow; ++u) id[u] = a.nbr[r0 + min(j0 + u, d - 1)];
            double2 p[kNodeRow];
#pragma unroll
            for (int u = 0; u < kNodeRow; ++u) p[u] = ld<SOA>(a.Xin, a.n, id[u]);
#pragma unroll
            for (int u = 0; u < kNodeRow; ++u)
                if (j0 + u < d) {
                    sx += p[u].x;
                    sy += p[u].y;
                    nb[j0 + u][tid] = p[u];
                }
        }
        const double dn = static_cast<double>(d), y = s_recip[d];
        double cx = div_small(sx, dn, y), cy = div_small(sy, dn, y);
        const bool tiny = !(fabs(sx) >= kStepMin) || !(fabs(sy) >= kStepMin);
        // a wave-uniform branch: the full division only when some lane needs it
        if (__builtin_amdgcn_ballot_w64(tiny) != 0ull) {
            if (tiny) {
                cx = sx / dn;
                cy = sy / dn;
            }
        }
        double qo = INFINITY, qn = INFINITY;
        const double2 c = make_double2(cx, cy);
        const uint32_t sp = a.fan_split ? a.fan_split[kk] : kFanUngrouped;   // a uniform test
        if (sp != kFanUngrouped) {
            // entries with p = 0 in [f0, b1), p = 1 in [b1, b2), p = 2 in [b2, f1)
            const int b1 = f0 + static_cast<int>(sp & 0xFFFFu), b2 = f0 + static_cast<int>(sp >> 16);
            node_fan_range<0, MAXV, BLOCK>(f0, b1, a.fan, nb, tid, o, c, qo, qn);
            node_fan_range<1, MAXV, BLOCK>(b1, b2, a.fan, nb, tid, o, c, qo, qn);
            node_fan_range<2, MAXV, BLOCK>(b2, f1, a.fan, nb, tid, o, c, qo, qn);
        } else {
            for (int g0 = f0; g0 < f1; g0 += kNodeFan) {
                uint32_t e[kNodeFan];
#pragma unroll
                for (int u = 0; u < kNodeFan; ++u) e[u] = a.fan[min(g0 + u, f1 - 1)];
#pragma unroll
                for (int u = 0; u < kNodeFan; ++u) {
                    if (g0 + u < f1) {
                        const int p = static_cast<int>(e[u] & 3u);
                        const double2 va = nb[(e[u] >> 2) & 127u][tid];
                        const double2 vb = nb[(e[u] >> 9) & 127u][tid];
                        double v, wq;
                        fan_qualities(p, o, c, va, vb, v, wq);
                        if (v < qo) qo = v;
                        if (wq < qn) qn = wq;
                    }
                }
            }
        }
        bool accepted = false;
        if (live) {
            accepted = GT ? (qn > qo) : (qn >= qo);
            const double nx = accepted ? cx : o.x, ny = accepted ? cy : o.y;
            st<SOA>(a.Xout, a.n, k, nx, ny);
            const double dx = nx - o.x, dy = ny - o.y;
            const double d2 = dx * dx + dy * dy;
            run_d2 = d2 > run_d2 ? d2 : run_d2;
        }
        const unsigned long long ball = __ballot(accepted);
        run_acc += __popcll(ball);
        if (a.bits != nullptr && lane == 0 && ball != 0ull) {
            const int kw = a.k_begin + tile * BLOCK + w * 64;
            const int sh = kw & 63;
            unsigned long long* word = reinterpret_cast<unsigned long long*>(a.bits) + (kw >> 6);
            atomicOr(word, ball << sh);
            if (sh != 0 && (ball >> (64 - sh)) != 0ull) atomicOr(word + 1, ball >> (64 - sh));
        }
    }
    // every group folds, those without a tile too: the last one counts them all
    finish_node_launch<BLOCK>(a, run_d2, run_acc);
}

// Persistent grid: 8 XCDs x 32 CUs x the work-groups a CU holds (by the
// group's static LDS; at most 32 waves per CU), never more work-groups on
// an XCD than it has tiles.  Every group takes an equal share of tiles, so
// an estimate that is too high only runs the shares in two rounds.
int persistent_grid(int tiles_per_xcd, int block, size_t lds_bytes)
{
    const int by_lds = static_cast<int>((160 * 1024) / std::max<size_t>(lds_bytes, 1));
    const int per_cu = std::max(1, std::min({by_lds, 2048 / block, kTileMaxGroups / 256}));
    return 8 * std::min(tiles_per_xcd, 32 * per_cu);
}

// Static LDS of a node-kernel work-group.
constexpr size_t node_lds(int block, int maxv)
{
    return static_cast<size_t>(maxv) * block * 16 + (block / 64) * 16 + (kMaxValence + 1) * 8;
}

template <int BLOCK, int MAXV>
void launch_variant(const SweepArgs& a, bool soa, bool gt, hipStream_t st)
{
    const int grid = persistent_grid(a.tiles_per_xcd, BLOCK, node_lds(BLOCK, MAXV));
    if (soa) {
        if (gt) k_sweep<BLOCK, MAXV, true, true><<<grid, BLOCK, 0, st>>>(a);
        else k_sweep<BLOCK, MAXV, true, false><<<grid, BLOCK, 0, st>>>(a);
    } else {
        if (gt) k_sweep<BLOCK, MAXV, false, true><<<grid, BLOCK, 0, st>>>(a);
        else k_sweep<BLOCK, MAXV, false, false><<<grid, BLOCK, 0, st>>>(a);
    }
}

// Work-group size of the variant used for a given largest valence.
int block_for(int max_deg, int requested)
{
    if (max_deg <= 8) return (requested == 64 || requested == 128) ? requested : 256;
    if (max_deg <= 16) return 256;
    if (max_deg <= 32) return 128;
    return 64;
}

void launch_range(SweepArgs a, int max_deg, int requested_block, bool soa, bool gt, hipStream_t st)
{
    const int64_t cnt = static_cast<int64_t>(a.k_end) - a.k_begin;
    if (cnt <= 0) return;
    const int block = block_for(max_deg, requested_block);
    a.n_tiles = div_up(cnt, block);
    a.tiles_per_xcd = div_up(a.n_tiles, 8);
    if (max_deg <= 8) {
        if (block == 64) launch_variant<64, 8>(a, soa, gt, st);
        else if (block == 128) launch_variant<128, 8>(a, soa, gt, st);
        else launch_variant<256, 8>(a, soa, gt, st);
    } else if (max_deg <= 16) {
        launch_variant<256, 16>(a, soa, gt, st);
    } else if (max_deg <= 32) {
        launch_variant<128, 32>(a, soa, gt, st);
    } else {
        launch_variant<64, 128>(a, soa, gt, st);
    }
}

// ----------------------------------------------------------- lane groups --
//
// A lane group of W consecutive work-items of one wave (W = 4, 8 or 16)
// takes one free node.  Lane j gathers the node's neighbour slots j, j + W,
// ... from L2/HBM and parks them in the group's LDS row; every lane of the
// group then forms the row-order sum from that row and divides once by the
// count (eq. (2)); lane j evaluates fan entries j, j + W, ... with the node
// at its position and at the candidate (Sec. 2.1); DPP moves inside the
// group fold the lanes' minima (a minimum is exact, so the fold order
// changes nothing), and the group's first lane takes the accept test and the
// write.  The arithmetic is the node kernel's, operation for operation.
// Several lanes share one node's latency chains, at the price of issuing a
// wave instruction for 64 / W nodes instead of 64.

// Work-group size of the lane-group variant for W and the largest valence
// MAXV: 256, or 16 groups when one group's LDS row is 129 positions long.
template <int W, int MAXV>
constexpr int lane_block() { return MAXV <= 32 ? 256 : 16 * W; }

// The minimum over the W lanes of each group (every lane of the wave
// active): swaps of neighbouring lanes and of lane pairs inside each quad,
// then the mirror inside each half row (8 lanes) and each row (16 lanes).
template <int W>
__device__ __forceinline__ double group_min(double v)
{
    auto fold = [&v](auto ctrl) {
        constexpr int c = decltype(ctrl)::value;
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), c, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), c, 0xF, 0xF, false);
        const double t = __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<uint32_t>(lo));
        v = t < v ? t : v;
    };
    fold(std::integral_constant<int, 0xB1>{});                   // quad_perm [1,0,3,2]
    fold(std::integral_constant<int, 0x4E>{});                   // quad_perm [2,3,0,1]
    if (W >= 8) fold(std::integral_constant<int, 0x141>{});      // row_half_mirror
    if (W >= 16) fold(std::integral_constant<int, 0x140>{});     // row_mirror
    return v;
}

template <int W, int MAXV, bool SOA, bool GT>
__global__ __launch_bounds__((lane_block<W, MAXV>())) void k_sweep_lanes(SweepArgs a)
{
    constexpr int BS = lane_block<W, MAXV>(), G = BS / W, NPW = 64 / W;   // groups per work-group, per wave
    if (!a.state->active) return;   // the whole launch returns: no group counts
    // persistent work-groups over tiles of G nodes, a contiguous run of
    // tiles per XCD, as in the node kernel
    const int xcd = static_cast<int>(blockIdx.x & 7), nw = static_cast<int>(gridDim.x >> 3);
    const int t_begin = xcd * a.tiles_per_xcd, t_end = min(t_begin + a.tiles_per_xcd, a.n_tiles);

    __shared__ double2 nb[G][MAXV + 1];   // one row per group; the pad spreads the rows over the banks
    __shared__ double s_recip[kMaxValence + 1];

    const int tid = threadIdx.x, g = tid / W, j = tid % W, lane = tid & 63, wv = tid >> 6;
    for (int i = tid; i <= kMaxValence; i += BS) s_recip[i] = i ? 1.0 / static_cast<double>(i) : 0.0;
    double run_d2 = 0.0;
    unsigned long long run_acc = 0;
    for (int tile = t_begin + static_cast<int>(blockIdx.x >> 3); tile < t_end; tile += nw) {
        const int k = a.k_begin + tile * G + g;
        const bool live = k < a.k_end;
        // a group past the range repeats the last node's loads and stores nothing
        const int kk = live ? k : a.k_end - 1;
        const int32_t r0 = a.row_ptr[kk], d = a.row_ptr[kk + 1] - r0;   // d >= 1 for a free node
        const int32_t f0 = a.fan_ptr[kk], f1 = a.fan_ptr[kk + 1];
        const double2 o = ld<SOA>(a.Xin, a.n, kk);
        __syncthreads();   // the previous tile's rows are read (and, first, the reciprocal table written)
        // lane j: slots j, j + W, ..., two per step with their loads in flight together
        for (int s0 = j; s0 < d; s0 += 2 * W) {
            const int32_t id0 = a.nbr[r0 + s0], id1 = a.nbr[r0 + min(s0 + W, d - 1)];
            const double2 p0 = ld<SOA>(a.Xin, a.n, id0), p1 = ld<SOA>(a.Xin, a.n, id1);
            nb[g][s0] = p0;
            if (s0 + W < d) nb[g][s0 + W] = p1;
        }
        __syncthreads();   // the group's row

        // the row-order sum, on every lane of the group (the same LDS reads)
        double sx = 0.0, sy = 0.0;
        for (int s = 0; s < d; ++s) {
            const double2 p = nb[g][s];
            sx += p.x;
            sy += p.y;
        }
        const double dn = static_cast<double>(d), y = s_recip[d];
        double cx = div_small(sx, dn, y), cy = div_small(sy, dn, y);
        const bool tiny = !(fabs(sx) >= kStepMin) || !(fabs(sy) >= kStepMin);
        if (__builtin_amdgcn_ballot_w64(tiny) != 0ull) {
            if (tiny) {
                cx = sx / dn;
                cy = sy / dn;
            }
        }
        const double2 c = make_double2(cx, cy);
        double qo = INFINITY, qn = INFINITY;
        for (int f = f0 + j; f < f1; f += W) {
            const uint32_t e = a.fan[f];
            const double2 va = nb[g][(e >> 2) & 127u], vb = nb[g][(e >> 9) & 127u];
            double v, w;
            fan_qualities(static_cast<int>(e & 3u), o, c, va, vb, v, w);
            if (v < qo) qo = v;
            if (w < qn) qn = w;
        }
        qo = group_min<W>(qo);
        qn = group_min<W>(qn);

        bool accepted = false;
        if (live && j == 0) {
            accepted = GT ? (qn > qo) : (qn >= qo);
            const double nx = accepted ? cx : o.x, ny = accepted ? cy : o.y;
            st<SOA>(a.Xout, a.n, k, nx, ny);
            const double dx = nx - o.x, dy = ny - o.y;
            const double d2 = dx * dx + dy * dy;
            run_d2 = d2 > run_d2 ? d2 : run_d2;
        }
        // accept bits: one per group, gathered from the wave's ballot
        const unsigned long long ball = __ballot(accepted);
        run_acc += __popcll(ball);
        if (a.bits != nullptr && lane == 0 && ball != 0ull) {
            unsigned long long nodes = 0;   // bit q: the wave's group q accepted
#pragma unroll
            for (int q = 0; q < NPW; ++q) nodes |= ((ball >> (q * W)) & 1ull) << q;
            const int kw = a.k_begin + tile * G + wv * NPW, sh = kw & 63;
            unsigned long long* word = reinterpret_cast<unsigned long long*>(a.bits) + (kw >> 6);
            atomicOr(word, nodes << sh);
            if (sh != 0 && (nodes >> (64 - sh)) != 0ull) atomicOr(word + 1, nodes >> (64 - sh));
        }
    }
    finish_node_launch<BS>(a, run_d2, run_acc);
}

template <int W, int MAXV>
void launch_lanes_v(SweepArgs a, int64_t cnt, bool soa, bool gt, hipStream_t st)
{
    constexpr int BS = lane_block<W, MAXV>(), G = BS / W;
    a.n_tiles = static_cast<int32_t>(div_up(cnt, G));
    a.tiles_per_xcd = div_up(a.n_tiles, 8);
    const size_t lds = static_cast<size_t>(G) * (MAXV + 1) * 16 + (BS / 64) * 16 + (kMaxValence + 1) * 8;
    const int grid = persistent_grid(a.tiles_per_xcd, BS, lds);
    if (soa) {
        if (gt) k_sweep_lanes<W, MAXV, true, true><<<grid, BS, 0, st>>>(a);
        else k_sweep_lanes<W, MAXV, true, false><<<grid, BS, 0, st>>>(a);
    } else {
        if (gt) k_sweep_lanes<W, MAXV, false, true><<<grid, BS, 0, st>>>(a);
        else k_sweep_lanes<W, MAXV, false, false><<<grid, BS, 0, st>>>(a);
    }
}

template <int W>
void launch_lanes_w(const SweepArgs& a, int64_t cnt, int max_deg, bool soa, bool gt, hipStream_t st)
{
    if (max_deg <= 8) launch_lanes_v<W, 8>(a, cnt, soa, gt, st);
    else if (max_deg <= 16) launch_lanes_v<W, 16>(a, cnt, soa, gt, st);
    else if (max_deg <= 32) launch_lanes_v<W, 32>(a, cnt, soa, gt, st);
    else launch_lanes_v<W, 128>(a, cnt, soa, gt, st);
}

void launch_lanes(const SweepArgs& a, int max_deg, int width, bool soa, bool gt, hipStream_t st)
{
    const int64_t cnt = static_cast<int64_t>(a.k_end) - a.k_begin;
    if (cnt <= 0) return;
    if (width == 4) launch_lanes_w<4>(a, cnt, max_deg, soa, gt, st);
    else if (width == 16) launch_lanes_w<16>(a, cnt, max_deg, soa, gt, st);
    else launch_lanes_w<8>(a, cnt, max_deg, soa, gt, st);
}

// ------------------------------------------------------- resident meshes --
//
// One work-group runs every sweep of one small mesh without leaving the
// launch: the coordinates and the mesh's rows and fans (u16) sit in LDS and
// the group's barriers separate the steps.  Form A reads one buffer and
// writes the other; Form B updates one buffer in place, colour class by
// colour class (no two nodes of a class are adjacent), a barrier after each
// class.  The per-node arithmetic is that of k_sweep, operation for
// operation; the fan's row slots index the node's row in LDS instead of a
// column of gathered positions.  The sweep state is written once, at the
// end, as the per-sweep closes would have left it; the final positions go to
// buffer (sweeps run) % 2 (Form A) or buffer 0 (Form B) in global memory.

constexpr int kResBS = 1024;
constexpr int kResRow = 8;   // row entries read together
constexpr int kResFan = 4;   // fan entries read together

// Node i's candidate, qualities and decision from positions `cur`; the new
// position goes to nxt[i].  Returns whether it accepted; *d2 takes the
// squared displacement.
template <bool GT>
__device__ __forceinline__ bool resident_node(int i, const double2* cur, double2* nxt, const uint16_t* rp,
                                              const uint16_t* fp, const uint16_t* nb, const uint16_t* fn, double* d2)
{
    // the row and the fan are read a few entries at a time, with clamped
    // indices, so that their dependent LDS loads overlap; sums and minima
    // still run in stored order
    const int r0 = rp[i], d = rp[i + 1] - r0;   // d >= 1: a free node has neighbours
    double sx = 0.0, sy = 0.0;
    for (int j0 = 0; j0 < d; j0 += kResRow) {
        int lab[kResRow];
#pragma unroll
        for (int u = 0; u < kResRow; ++u) lab[u] = nb[r0 + min(j0 + u, d - 1)];
        double2 p[kResRow];
#pragma unroll
        for (int u = 0; u < kResRow; ++u) p[u] = cur[lab[u]];
#pragma unroll
        for (int u = 0; u < kResRow; ++u)
            if (j0 + u < d) {
                sx += p[u].x;
                sy += p[u].y;
            }
    }
    const double dn = static_cast<double>(d);
    const double cx = sx / dn, cy = sy / dn;
    const double2 o = cur[i];
    double qo = INFINITY, qn = INFINITY;
    const int f1 = fp[i + 1];
    for (int f0 = fp[i]; f0 < f1; f0 += kResFan) {
        uint32_t e[kResFan];
#pragma unroll
        for (int u = 0; u < kResFan; ++u) e[u] = fn[min(f0 + u, f1 - 1)];
        int la[kResFan], lb[kResFan];
#pragma unroll
        for (int u = 0; u < kResFan; ++u) {
            la[u] = nb[r0 + ((e[u] >> 2) & 127u)];
            lb[u] = nb[r0 + ((e[u] >> 9) & 127u)];
        }
        double2 va[kResFan], vb[kResFan];
#pragma unroll
        for (int u = 0; u < kResFan; ++u) {
            va[u] = cur[la[u]];
            vb[u] = cur[lb[u]];
        }
#pragma unroll
        for (int u = 0; u < kResFan; ++u) {
            if (f0 + u >= f1) break;
            const int p = static_cast<int>(e[u] & 3u);
            double v, w;
            fan_qualities(p, o, make_double2(cx, cy), va[u], vb[u], v, w);
            if (v < qo) qo = v;
            if (w < qn) qn = w;
        }
    }
    const bool accepted = GT ? (qn > qo) : (qn >= qo);
    const double nx = accepted ? cx : o.x, ny = accepted ? cy : o.y;
    nxt[i] = make_double2(nx, ny);
    const double dx = nx - o.x, dy = ny - o.y;
    const double t = dx * dx + dy * dy;
    *d2 = t > *d2 ? t : *d2;
    return accepted;
}

template <bool SOA, bool GT>
__global__ __launch_bounds__(kResBS) void k_sweep_resident(const ResidentArgs* __restrict__ list)
{
    const ResidentArgs a = list[blockIdx.x];
    extern __shared__ double2 res_lds[];
    __shared__ double s_d2[kResBS / 64];
    __shared__ unsigned long long s_acc[kResBS / 64];
    const int n = a.n, nf = a.n_free;
    const bool in_place = a.in_place != 0;
    const int nbuf = in_place ? 1 : 2;
    double2* buf0 = res_lds;
    double2* buf1 = in_place ? res_lds : res_lds + n;
    uint16_t* rp = reinterpret_cast<uint16_t*>(res_lds + nbuf * n);   // [nf + 1] row starts
    uint16_t* fp = rp + (nf + 1);                                       // [nf + 1] fan starts
    uint16_t* nb = fp + (nf + 1);                                       // [nnz] neighbours (device labels)
    uint16_t* fn = nb + a.nnz;                                          // [ninc] fan entries
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    for (int i = tid; i < n; i += kResBS) {
        const double2 p = ld<SOA>(a.X, n, i);
        buf0[i] = p;
        if (!in_place) buf1[i] = p;
    }
    for (int i = tid; i <= nf; i += kResBS) {
        rp[i] = static_cast<uint16_t>(a.row_ptr[i]);
        fp[i] = static_cast<uint16_t>(a.fan_ptr[i]);
    }
    for (int k = tid; k < a.nnz; k += kResBS) nb[k] = static_cast<uint16_t>(a.nbr[k]);
    for (int k = tid; k < a.ninc; k += kResBS) fn[k] = a.fan[k];
    __syncthreads();

    // one range of device labels: Form A all free nodes, Form B one class
    auto sweep_range = [&](int lo, int hi, const double2* cur, double2* nxt, int s, double* d2,
                           unsigned long long* cnt) {
        for (int i0 = lo; i0 < hi; i0 += kResBS) {
            const int i = i0 + tid;
            const bool accepted = i < hi && resident_node<GT>(i, cur, nxt, rp, fp, nb, fn, d2);
            const unsigned long long ball = __ballot(accepted);
            *cnt += __popcll(ball);
            if (a.bits != nullptr && lane == 0 && ball != 0ull) {
                // the wave's labels start at kw, which need not be a multiple of 64
                const int kw = i0 + wv * 64, sh = kw & 63;
                unsigned long long* word = reinterpret_cast<unsigned long long*>(a.bits) + s * a.words + (kw >> 6);
                atomicOr(word, ball << sh);
                if (sh != 0 && (ball >> (64 - sh)) != 0ull) atomicOr(word + 1, ball >> (64 - sh));
            }
        }
    };

    int s = 0;
    double maxd = 0.0;
    unsigned long long acc = 0, acc_total = 0;
    while (s < a.iters) {
        double d2 = 0.0;
        unsigned long long cnt = 0;
        if (in_place) {
            for (int c = 0; c < a.n_classes; ++c) {
                sweep_range(a.class_start[c], a.class_start[c + 1], buf0, buf0, s, &d2, &cnt);
                __syncthreads();   // the next class reads this one's positions
            }
        } else {
            sweep_range(0, nf, (s & 1) ? buf1 : buf0, (s & 1) ? buf0 : buf1, s, &d2, &cnt);
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double t = __shfl_xor(d2, off);
            d2 = t > d2 ? t : d2;
        }
        if (lane == 0) {
            s_d2[wv] = d2;
            s_acc[wv] = cnt;
        }
        __syncthreads();   // also: every read and write of this sweep is done
        double m = s_d2[0];
        unsigned long long c = s_acc[0];
        for (int q = 1; q < kResBS / 64; ++q) {
            m = s_d2[q] > m ? s_d2[q] : m;
            c += s_acc[q];
        }
        __syncthreads();   // s_d2 and s_acc are rewritten by the next sweep
        ++s;
        maxd = m;
        acc = c;
        acc_total += c;
        if (a.tol2 > 0.0 && m < a.tol2) break;
    }

    const int fb = in_place ? 0 : (s & 1);
    const double2* fin = fb ? buf1 : buf0;
    double* out = a.X + fb * 2 * static_cast<int64_t>(n);
    for (int i = tid; i < nf; i += kResBS) st<SOA>(out, n, i, fin[i].x, fin[i].y);
    if (tid == 0) {
        MeshState ms = *a.state;
        ms.s += s;
        ms.maxd_last = s > 0 ? static_cast<unsigned long long>(__double_as_longlong(maxd)) : ms.maxd_last;
        ms.acc_last = s > 0 ? acc : ms.acc_last;
        ms.acc_total += acc_total;
        ms.maxd_cur = 0;
        ms.acc_cur = 0;
        ms.active = 0;
        *a.state = ms;
    }
}

// Closes a sweep (one work-item per mesh).
__global__ void k_advance(MeshState* __restrict__ st, int32_t n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) close_state(st + i);
}

}  // namespace

size_t resident_lds_bytes(int64_t n, int64_t n_free, int64_t nnz, int64_t ninc, bool in_place)
{
    return static_cast<size_t>((in_place ? 16 : 32) * n + 2 * (2 * (n_free + 1) + nnz + ninc));
}

bool resident_fits(int64_t n, int64_t nnz, int64_t ninc, bool in_place)
{
    // u16 labels and offsets; the free-node counts are bounded by n
    return n >= 1 && n <= 65535 && nnz <= 65535 && ninc <= 65535 &&
           resident_lds_bytes(n, n, nnz, ninc, in_place) <= kResidentLdsLimit;
}

sl_status resident_classes(const DevMesh& m, bool in_place, ResidentArgs& a)
{
    a.in_place = in_place ? 1 : 0;
    a.n_classes = 0;
    if (!in_place) return SL_OK;
    if (m.n_colors > kResidentClasses)
        return fail(SL_EINVAL, "the resident kernel holds at most " + std::to_string(kResidentClasses) +
                                   " colour classes, this mesh has " + std::to_string(m.n_colors));
    a.n_classes = m.n_colors;
    for (int c = 0; c <= m.n_colors; ++c) a.class_start[c] = m.color_start_h[c];
    return SL_OK;
}

sl_status launch_sweep_resident(const ResidentArgs* list, int32_t count, size_t lds, int32_t layout,
                                int32_t accept, hipStream_t st)
{
    if (count <= 0) return SL_OK;
    if (lds > kResidentLdsLimit) return fail(SL_EINVAL, "resident mesh does not fit in LDS");
    const bool soa = layout == SL_SOA, gt = accept == SL_ACCEPT_GT;
    const void* fn = soa ? (gt ? reinterpret_cast<const void*>(&k_sweep_resident<true, true>)
                               : reinterpret_cast<const void*>(&k_sweep_resident<true, false>))
                         : (gt ? reinterpret_cast<const void*>(&k_sweep_resident<false, true>)
                               : reinterpret_cast<const void*>(&k_sweep_resident<false, false>));
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        (void)hipGetLastError();
    }
    if (soa) {
        if (gt) k_sweep_resident<true, true><<<count, kResBS, lds, st>>>(list);
        else k_sweep_resident<true, false><<<count, kResBS, lds, st>>>(list);
    } else {
        if (gt) k_sweep_resident<false, true><<<count, kResBS, lds, st>>>(list);
        else k_sweep_resident<false, false><<<count, kResBS, lds, st>>>(list);
    }
    SL_HIP(hipGetLastError());
    return SL_OK;
}

namespace {

// ---------------------------------------------------- colour-class tiles --
//
// Form B (eq. (3)) on colour-class tiles: the free nodes of one colour class
// are cut into tiles of T consecutive labels, one work-group per tile and
// one launch per class, in place (no two nodes of a class are adjacent, so
// no tile reads a position another tile writes).  A work-group stages its
// nodes' positions, its halo (every neighbour, all of other classes), its
// rows in tile-local indices and its nodes' fan entries in LDS, with every
// global load of the tile in flight together; then each work-item takes one
// node: the row-order sum and one division by the count (eq. (2)), every
// incident triangle evaluated twice through the fan slots (Sec. 2.1), the
// accept test and the write.  The arithmetic is the node kernel's,
// operation for operation, so results are bit-identical to it and to the
// oracle's coloured sweep.

constexpr int kClassHalo = 8;    // halo positions per work-item at most (the build's set holds 8 T)
constexpr int kClassWords = 4;   // row words, and fan words, per work-item at most

struct ClassSweepArgs {
    const TileWork* work;   // the tiles of one class of one mesh (TileWork::tris holds the fan entries)
    int32_t n_work, tiles_per_xcd;
    int32_t halo_cap, rows_cap, fans_cap;   // LDS: largest halo, padded row segment and fan list
    MeshState* states;      // the mesh's state is states[work[0].mesh]
    uint64_t* bits;         // nullable: accept bits of this sweep (device labels)
    int32_t* sched;         // [kTileSchedInts]: the launch's counters and per-group slots
};

// Persistent work-groups: the class's tile list is cut into 8 contiguous
// ranges, one per XCD (work-groups are dealt to the XCDs round-robin), so
// that neighbouring tiles share an L2; the work-groups of an XCD take its
// tiles round-robin.  The displacement maximum and accepted count run per
// work-item over the group's tiles and are folded once per launch through
// the per-group slots (with a group per tile, tens of thousands of atomics
// on the same two words per launch queued behind each other).
// Old and new quality over the fan entries [g_begin, g_end) of one node,
// all with stored position P, folded into the running minima.  Entries are
// read a group at a time with clamped indices so that their dependent LDS
// loads overlap; minima are exact, so the order of the entries does not
// matter.
template <int P>
__device__ __forceinline__ void class_fan_range(int g_begin, int g_end, const uint16_t* fans, const uint16_t* rows,
                                                int r0, const double2* Xl, const double2 o, const double2 c,
                                                double& qo, double& qn)
{
    for (int g0 = g_begin; g0 < g_end; g0 += kResFan) {
        uint32_t e[kResFan];
#pragma unroll
        for (int u = 0; u < kResFan; ++u) e[u] = fans[min(g0 + u, g_end - 1)];
        int la[kResFan], lb[kResFan];
#pragma unroll
        for (int u = 0; u < kResFan; ++u) {
            la[u] = rows[r0 + ((e[u] >> 2) & 127u)];
            lb[u] = rows[r0 + ((e[u] >> 9) & 127u)];
        }
        double2 va[kResFan], vb[kResFan];
#pragma unroll
        for (int u = 0; u < kResFan; ++u) {
            va[u] = Xl[la[u]];
            vb[u] = Xl[lb[u]];
        }
#pragma unroll
        for (int u = 0; u < kResFan; ++u) {
            if (g0 + u >= g_end) break;
            double v, w;
            fan_qualities_p<P>(o, c, va[u], vb[u], v, w);
            if (v < qo) qo = v;
            if (w < qn) qn = w;
        }
    }
}

template <int T, bool SOA, bool GT>
__global__ __launch_bounds__(T) void k_sweep_class(ClassSweepArgs a)
{
    extern __shared__ double2 cls_lds[];
    __shared__ double s_recip[kMaxValence + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int i = tid; i <= kMaxValence; i += T) s_recip[i] = i ? 1.0 / static_cast<double>(i) : 0.0;
    const int xcd = static_cast<int>(blockIdx.x & 7), nw = static_cast<int>(gridDim.x >> 3);
    const int t_begin = xcd * a.tiles_per_xcd;
    const int t_end = min(t_begin + a.tiles_per_xcd, a.n_work);
    double2* Xl = cls_lds;                                               // [T + halo_cap]
    uint16_t* rows = reinterpret_cast<uint16_t*>(Xl + T + a.halo_cap);   // [rows_cap]
    uint16_t* fans = rows + a.rows_cap;                                  // [fans_cap]
    uint64_t* rows64 = reinterpret_cast<uint64_t*>(rows);
    uint64_t* fans64 = reinterpret_cast<uint64_t*>(fans);
    double run_d2 = 0.0;
    unsigned long long run_acc = 0;
    for (int tile = t_begin + static_cast<int>(blockIdx.x >> 3); tile < t_end; tile += nw) {
        const TileWork d = a.work[tile];
        if (!a.states[d.mesh].active) continue;   // uniform: the whole group skips the tile
        double* X = static_cast<double*>(const_cast<void*>(d.X));   // buffer 0, in place
        const int nown = d.nown;
        const int ic = min(tid, nown - 1);   // a work-item past the tile repeats the last node's loads
        const uint16_t* fr = d.rr + ((2 * T + 2 + 15) & ~15) / 2;   // fan starts follow the row starts
        const uint32_t* pc = reinterpret_cast<const uint32_t*>(fr + ((2 * T + 2 + 15) & ~15) / 2);   // then the splits
        // every global load of the tile, then the LDS stores.  The loads
        // are unconditional, with indices clamped into the tile's lists
        // (a work-item past a list's end re-loads its last entry and
        // stores nothing), so that none waits behind a branch: a tile's
        // halo is at most 8 T long (the build's halo set), its row and
        // fan words at most 4 T each (16 entries per node on average).
        const int hc = d.halo_cnt, row_words = d.row_words, fan_words = (d.tri_cnt + 3) >> 2;
        const int r0 = d.rr[ic], r1 = d.rr[ic + 1], f0 = fr[ic], f1 = fr[ic + 1];
        // the node's fan entries come grouped by stored position: p = 0 in
        // [f0, f0 + lo16), p = 1 up to f0 + hi16, p = 2 up to f1
        const uint32_t pcv = pc[ic];
        const double2 o = ld<SOA>(X, d.n, d.own_start + ic);
        int32_t hid[kClassHalo];
#pragma unroll
        for (int q = 0; q < kClassHalo; ++q) hid[q] = d.halo[min(q * T + tid, max(hc - 1, 0))];
        uint64_t rwv[kClassWords], fwv[kClassWords];
#pragma unroll
        for (int q = 0; q < kClassWords; ++q) {
            rwv[q] = d.rows[min(q * T + tid, max(row_words - 1, 0))];
            fwv[q] = d.tris[min(q * T + tid, max(fan_words - 1, 0))];
        }
        double2 hp[kClassHalo];
#pragma unroll
        for (int q = 0; q < kClassHalo; ++q) hp[q] = ld<SOA>(X, d.n, hid[q]);
        __syncthreads();   // the previous tile is done with the LDS
        Xl[tid] = o;
#pragma unroll
        for (int q = 0; q < kClassWords; ++q) {
            if (q * T + tid < row_words) rows64[q * T + tid] = rwv[q];
            if (q * T + tid < fan_words) fans64[q * T + tid] = fwv[q];
        }
#pragma unroll
        for (int q = 0; q < kClassHalo; ++q)
            if (q * T + tid < hc) Xl[T + q * T + tid] = hp[q];
        __syncthreads();

        bool accepted = false;
        if (tid < nown) {
            // the row and the fan are read a group of entries at a time,
            // with clamped indices, so that their dependent LDS loads
            // overlap; sums and minima still run in stored order
            const int dg = r1 - r0;   // >= 1 for a free node
            double sx = 0.0, sy = 0.0;
            for (int j0 = 0; j0 < dg; j0 += kResRow) {
                int lab[kResRow];
#pragma unroll
                for (int u = 0; u < kResRow; ++u) lab[u] = rows[r0 + min(j0 + u, dg - 1)];
                double2 p[kResRow];
#pragma unroll
                for (int u = 0; u < kResRow; ++u) p[u] = Xl[lab[u]];
#pragma unroll
                for (int u = 0; u < kResRow; ++u)
                    if (j0 + u < dg) {
                        sx += p[u].x;
                        sy += p[u].y;
                    }
            }
            const double dn = static_cast<double>(dg), y = s_recip[dg];
            double cx = div_small(sx, dn, y), cy = div_small(sy, dn, y);
            const bool tiny = !(fabs(sx) >= kStepMin) || !(fabs(sy) >= kStepMin);
            if (tiny) {
                cx = sx / dn;
                cy = sy / dn;
            }
            double qo = INFINITY, qn = INFINITY;
            const double2 cc = make_double2(cx, cy);
            const int b1 = f0 + static_cast<int>(pcv & 0xFFFFu), b2 = f0 + static_cast<int>(pcv >> 16);
            class_fan_range<0>(f0, b1, fans, rows, r0, Xl, o, cc, qo, qn);
            class_fan_range<1>(b1, b2, fans, rows, r0, Xl, o, cc, qo, qn);
            class_fan_range<2>(b2, f1, fans, rows, r0, Xl, o, cc, qo, qn);
            accepted = GT ? (qn > qo) : (qn >= qo);
            const double nx = accepted ? cx : o.x, ny = accepted ? cy : o.y;
            st<SOA>(X, d.n, d.own_start + tid, nx, ny);
            const double dx = nx - o.x, dy = ny - o.y;
            const double t2 = dx * dx + dy * dy;
            run_d2 = t2 > run_d2 ? t2 : run_d2;
        }
        const unsigned long long ball = __ballot(accepted);
        run_acc += __popcll(ball);
        if (a.bits != nullptr && lane == 0 && ball != 0ull) {
            // a class tile starts at any label: the wave's bits may straddle two words
            const int kw = d.own_start + wv * 64, sh = kw & 63;
            unsigned long long* word = reinterpret_cast<unsigned long long*>(a.bits) + (kw >> 6);
            atomicOr(word, ball << sh);
            if (sh != 0 && (ball >> (64 - sh)) != 0ull) atomicOr(word + 1, ball >> (64 - sh));
        }
    }
    fold_through_slots<T, false>(a.sched, a.states + a.work[0].mesh, run_d2, run_acc);
}

template <int T>
void launch_class_t(const ClassSweepArgs& a, bool soa, bool gt, int grid, size_t lds, hipStream_t st)
{
    const void* fn = soa ? (gt ? reinterpret_cast<const void*>(&k_sweep_class<T, true, true>)
                               : reinterpret_cast<const void*>(&k_sweep_class<T, true, false>))
                         : (gt ? reinterpret_cast<const void*>(&k_sweep_class<T, false, true>)
                               : reinterpret_cast<const void*>(&k_sweep_class<T, false, false>));
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        (void)hipGetLastError();
    }
    if (soa) {
        if (gt) k_sweep_class<T, true, true><<<grid, T, lds, st>>>(a);
        else k_sweep_class<T, true, false><<<grid, T, lds, st>>>(a);
    } else {
        if (gt) k_sweep_class<T, false, true><<<grid, T, lds, st>>>(a);
        else k_sweep_class<T, false, false><<<grid, T, lds, st>>>(a);
    }
}

}  // namespace

size_t class_lds_bytes(int tile_nodes, int halo_cap, int rows_cap, int fans_cap)
{
    return static_cast<size_t>(tile_nodes + halo_cap) * 16 + static_cast<size_t>(rows_cap) * 2 +
           static_cast<size_t>((fans_cap + 3) & ~3) * 2;
}

sl_status launch_sweep_class(const TileLaunch& L, int32_t fans_cap, uint64_t* bits, hipStream_t st)
{
    if (L.halo_cap > kClassHalo * L.tile_nodes) return fail(SL_EINVAL, "internal: class tile halo too long");
    if (L.n_work > 0) {
        ClassSweepArgs a{};
        a.work = L.work;
        a.n_work = L.n_work;
        a.tiles_per_xcd = div_up(L.n_work, 8);
        a.halo_cap = L.halo_cap;
        a.rows_cap = L.rows_cap;
        a.fans_cap = (fans_cap + 3) & ~3;
        a.states = L.states;
        a.bits = bits;
        a.sched = L.sched;
        if (!a.sched) return fail(SL_EINVAL, "internal: class tile launch without its counters");
        const size_t lds = class_lds_bytes(L.tile_nodes, L.halo_cap, L.rows_cap, fans_cap);
        // persistent: as many groups per CU as the LDS holds (at most
        // 2048 / T, at most the 8 a launch has slots for, or the option's
        // count), 32 CUs per XCD, never more groups on an XCD than it has tiles
        const int fit = std::max(1, static_cast<int>(kTileLdsLimit / std::max<size_t>(lds, 1)));
        int per_cu = std::min({fit, 2048 / L.tile_nodes, kTileMaxGroups / 256});
        if (L.wg_per_cu > 0) per_cu = std::min(per_cu, static_cast<int>(L.wg_per_cu));
        const int grid = 8 * std::min(a.tiles_per_xcd, 32 * per_cu);
        if (grid > kTileMaxGroups) return fail(SL_EINVAL, "internal: class launch of more groups than slots");
        const bool soa = L.layout == SL_SOA, gt = L.accept == SL_ACCEPT_GT;
        if (L.tile_nodes == 128) launch_class_t<128>(a, soa, gt, grid, lds, st);
        else if (L.tile_nodes == 256) launch_class_t<256>(a, soa, gt, grid, lds, st);
        else launch_class_t<512>(a, soa, gt, grid, lds, st);
        SL_HIP(hipGetLastError());
    }
    return L.n_close > 0 ? launch_advance(L.states, L.n_close, st) : SL_OK;
}

sl_status launch_advance(MeshState* states, int32_t n, hipStream_t st)
{
    if (n <= 0) return SL_OK;
    k_advance<<<div_up(n, 256), 256, 0, st>>>(states, n);
    SL_HIP(hipGetLastError());
    return SL_OK;
}

sl_status launch_sweep_nodes(const DevMesh& m, int32_t parity, int32_t form, int32_t accept, int32_t block,
                             MeshState* state, uint64_t* bits, int32_t* sched, hipStream_t st, bool close)
{
    if (!sched) return fail(SL_EINVAL, "internal: node launch without its counters");
    // the launch that closes the sweep: Form A's one, or Form B's last
    // non-empty class; with no free node, a k_advance
    int last = -1;
    if (form == SL_JACOBI) last = m.n_free > 0 ? 0 : -1;
    else
        for (int c = 0; c < m.n_colors; ++c)
            if (m.color_start_h[c + 1] > m.color_start_h[c]) last = c;
    SweepArgs a{};
    a.sched = sched;
    a.n = m.n;
    a.row_ptr = m.row_ptr;
    a.nbr = m.nbr;
    a.fan_ptr = m.fan_ptr;
    a.fan = m.fan;
    a.fan_split = m.fan_split;
    a.state = state;
    a.bits = bits;
    const bool soa = m.layout == SL_SOA, gt = accept == SL_ACCEPT_GT;
    if (form == SL_JACOBI) {
        a.Xin = static_cast<const double*>(m.X[parity & 1]);
        a.Xout = static_cast<double*>(m.X[(parity + 1) & 1]);
        a.k_begin = 0;
        a.k_end = m.n_free;
        a.close = close && last == 0 ? 1 : 0;
        if (m.lane_width > 0) launch_lanes(a, m.max_deg, m.lane_width, soa, gt, st);
        else launch_range(a, m.max_deg, block, soa, gt, st);
    } else {
        a.Xin = static_cast<const double*>(m.X[0]);
        a.Xout = static_cast<double*>(m.X[0]);
        for (int c = 0; c < m.n_colors; ++c) {
            a.k_begin = m.color_start_h[c];
            a.k_end = m.color_start_h[c + 1];
            a.close = close && c == last ? 1 : 0;
            if (m.lane_width > 0) launch_lanes(a, m.max_deg, m.lane_width, soa, gt, st);
            else launch_range(a, m.max_deg, block, soa, gt, st);
        }
    }
    SL_HIP(hipGetLastError());
    if (close && last < 0) return launch_advance(state, 1, st);
    return SL_OK;
}

}  // namespace sl
