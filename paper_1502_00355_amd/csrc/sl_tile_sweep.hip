// Tile sweep of the Form A (Jacobi) form.
//
// The free nodes (device order: Hilbert cells) are cut into tiles of T
// consecutive labels, one work-group per tile.  Per sweep a work-group
//   1. stages the positions of its own nodes and of its halo (every node an
//      own node reads) in LDS,
//   2. computes each own node's Laplacian candidate: the row-order sum of its
//      neighbours divided by their count (eq. (2)),
//   3. walks the triangles incident to its own nodes, each once: the quality
//      in stored order with all vertices at pass-q positions (the "old"
//      quality, Sec. 2.1), then for every own vertex the quality with that
//      vertex at its candidate -- the vertex role is fixed in the code, so
//      no lane selects between stored positions -- folding both into the
//      vertices' minima with LDS atomics,
//   4. keeps each own node's candidate iff its new minimum is >= (or >) its
//      old one and writes the node to the other buffer.
// A triangle's old quality is evaluated by every tile that owns one of its
// vertices (the paper evaluates it once per vertex, Sec. 5.3); each
// (triangle, moved vertex) pair is evaluated exactly once.
#include <algorithm>
#include <climits>
#include <cstdlib>

#include "sl_common.h"

namespace sl {

namespace {

constexpr double kTwoSqrt3 = 0x1.bb67ae8584caap+1;   // 2*sqrt(3) rounded to double

// ------------------------------------------------------------ tile sweep --

// The sweep runs in the precision of its real type R: double, or float for
// the single-precision form (every operation then one float operation, the
// constant the float nearest 2*sqrt(3)).
template <typename R>
struct Real;
template <>
struct Real<double> {
    using V2 = double2;
    static constexpr double k_two_sqrt3 = kTwoSqrt3;
    static constexpr double k_smallest = 0x1p-1074;            // smallest subnormal
    static constexpr double k_step_min = 0x1p-1015;            // 128 x smallest normal
    __device__ static V2 make(double x, double y) { return make_double2(x, y); }
};
template <>
struct Real<float> {
    using V2 = float2;
    static constexpr float k_two_sqrt3 = 0x1.bb67aep+1f;   // 2*sqrt(3) rounded to float
    static constexpr float k_smallest = 0x1p-149f;          // smallest subnormal
    static constexpr float k_step_min = 0x1p-119f;          // 128 x smallest normal
    __device__ static V2 make(float x, float y) { return make_float2(x, y); }
};

// Minimum into an LDS value (one ds_min_f64 / ds_min_f32).  Qualities are
// finite -- coordinates are validated below 2^500 (single precision: 2^61)
// in magnitude and S == 0 gives 0 -- so no NaN reaches it; which zero a min
// keeps when +0 meets -0 does not matter, the accept test compares them
// equal.
template <typename R>
__device__ __forceinline__ void lds_min(R* p, R v)
{
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// (2*sqrt(3)*cr)/S, or 0 when S == 0.  S is zero only when the three
// vertices coincide, and then cr is a zero too: dividing it by the smallest
// subnormal instead gives the zero quality (its sign never matters, the
// minima and the accept test compare zeros equal) with one max instead of a
// compare and two selects.
template <typename R>
__device__ __forceinline__ R finish_q(R cr, R S)
{
    return (Real<R>::k_two_sqrt3 * cr) / fmax(S, Real<R>::k_smallest);
}

// a / d correctly rounded, for an integer count d in [1, 127] and y = 1/d
// correctly rounded, while the quotient is a normal number: q = a*y is
// within one ulp of a/d, so the remainder a - q*d is exact (a multiple of
// ulp(q) below 127 ulp(q)), and q + r*y differs from a/d by less than
// ulp(q)*2^-p (p = 53 or 24).  A normal quotient by an integer below 2^7 is
// never a rounding midpoint and lies at least ulp/254 from one, so that sum
// rounds to the correctly rounded a/d (Markstein's correction step): three
// operations instead of a full division.  Below 128 x the smallest normal
// number (zero included) the caller divides instead: a subnormal quotient
// can be an exact midpoint.
template <typename R>
__device__ __forceinline__ R div_step(R a, R d, R y)
{
    const R q = a * y;
    const R r = fma(-q, d, a);
    return fma(r, y, q);
}

struct TileSweepArgs {
    const TileWork* work;
    int32_t n_work, tiles_per_xcd, halo_cap, rows_cap;
    int32_t parity;            // every mesh of the launch reads buffer `parity`, writes parity ^ 1
    int32_t exit_if_inactive;  // all tiles are of one mesh: return at once if it has stopped
    MeshState* states;
    uint64_t* bits;            // nullable: accept bits of this sweep (single mesh)
    int32_t* sched;            // [kTileSchedInts]: the launch's counters and slots (sl_common.h)
    int32_t n_close;           // the last work-group closes the sweep of states[0..n_close)
    int32_t one_mesh;          // every tile is of one mesh: groups fold through their slots
};

// Old quality of one triangle and the new quality for each own vertex,
// folded into the per-node minima.  Local indices below T are own nodes.
template <int T, typename R>
__device__ __forceinline__ void tile_triangle(uint64_t w, const typename Real<R>::V2* Xl,
                                              const typename Real<R>::V2* cand, R* qo, R* qn)
{
    using V2 = typename Real<R>::V2;
    const int l0 = static_cast<int>(w & 0xFFFF), l1 = static_cast<int>((w >> 16) & 0xFFFF),
              l2 = static_cast<int>((w >> 32) & 0xFFFF);
    // every read up front, so that one wait covers them all (a halo vertex
    // reads some own candidate that it then ignores); a candidate quality is
    // evaluated for own vertices only -- the tile's triangle list is grouped
    // by which vertices are own, so a wave mostly takes one branch
    const V2 p0 = Xl[l0], p1 = Xl[l1], p2 = Xl[l2];
    const V2 c0 = cand[l0 & (T - 1)], c1 = cand[l1 & (T - 1)], c2 = cand[l2 & (T - 1)];
    const R ax = p1.x - p0.x, ay = p1.y - p0.y;
    const R bx = p2.x - p0.x, by = p2.y - p0.y;
    const R cx = p2.x - p1.x, cy = p2.y - p1.y;
    const R La = ax * ax + ay * ay, Lb = bx * bx + by * by, Lc = cx * cx + cy * cy;
    const R qold = finish_q(ax * by - bx * ay, (La + Lc) + Lb);
    // each own vertex at its candidate, the other two where they are; the
    // squared length of the opposite edge is shared with the old quality
    if (l0 < T) {
        const R ax2 = p1.x - c0.x, ay2 = p1.y - c0.y, bx2 = p2.x - c0.x, by2 = p2.y - c0.y;
        const R q0 = finish_q(ax2 * by2 - bx2 * ay2, ((ax2 * ax2 + ay2 * ay2) + Lc) + (bx2 * bx2 + by2 * by2));
        lds_min(qo + l0, qold);
        lds_min(qn + l0, q0);
    }
    if (l1 < T) {
        const R ax2 = c1.x - p0.x, ay2 = c1.y - p0.y, cx2 = p2.x - c1.x, cy2 = p2.y - c1.y;
        const R q1 = finish_q(ax2 * by - bx * ay2, ((ax2 * ax2 + ay2 * ay2) + (cx2 * cx2 + cy2 * cy2)) + Lb);
        lds_min(qo + l1, qold);
        lds_min(qn + l1, q1);
    }
    if (l2 < T) {
        const R bx2 = c2.x - p0.x, by2 = c2.y - p0.y, cx2 = c2.x - p1.x, cy2 = c2.y - p1.y;
        const R q2 = finish_q(ax * by2 - bx2 * ay, (La + (cx2 * cx2 + cy2 * cy2)) + (bx2 * bx2 + by2 * by2));
        lds_min(qo + l2, qold);
        lds_min(qn + l2, q2);
    }
}

// Registers holding the global data of the next tile while the current one
// is computed.  Loaded in two steps, the second a phase after the first:
// (A) halo ids, own positions, row offsets; (B) halo positions, the row
// segment, triangle entries.  Tile descriptors are loaded a tile earlier.
template <typename R, int NPT, int RPRE, int KPRE>
struct TileStage {
    typename Real<R>::V2 own[NPT];
    uint16_t rs[NPT], re[NPT];   // row start and end of each own node
    uint64_t rw[RPRE];
    uint64_t tw[KPRE];
    int hidx;
    typename Real<R>::V2 hx;
};

// The descriptor is loaded through an index the compiler treats as per-lane,
// so the loads stay vector loads (counted with the other global loads)
// instead of scalar loads that the next LDS barrier would wait for.
__device__ __forceinline__ TileWork load_work(const TileWork* work, int i)
{
    int t = i;
    asm volatile("" : "+v"(t));
    const __attribute__((address_space(1))) uint64_t* p =
        reinterpret_cast<const __attribute__((address_space(1))) uint64_t*>(reinterpret_cast<uint64_t>(work)) +
        static_cast<int64_t>(t) * (sizeof(TileWork) / 8);
    uint64_t raw[sizeof(TileWork) / 8];
#pragma unroll
    for (int q = 0; q < static_cast<int>(sizeof(TileWork) / 8); ++q) raw[q] = p[q];
    TileWork w;
    __builtin_memcpy(&w, raw, sizeof(TileWork));
    return w;
}

// Global-address-space pointers: loads through them are global loads,
// counted only by vmcnt (flat loads would also hold lgkmcnt, which every LDS
// barrier waits for).
template <typename V>
using gptr = const __attribute__((address_space(1))) V*;

template <typename V>
__device__ __forceinline__ gptr<V> to_global(const V* p)
{
    return reinterpret_cast<gptr<V>>(reinterpret_cast<uint64_t>(p));
}

__device__ __forceinline__ TileWork uniform_work(const TileWork& w)
{
    auto uv = [](uint64_t v) {
        const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
        const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
        return (static_cast<uint64_t>(hi) << 32) | lo;
    };
    auto u64 = [&](const void* p) { return uv(reinterpret_cast<uint64_t>(p)); };
    TileWork u;
    u.X = reinterpret_cast<const void*>(u64(w.X));
    u.halo = reinterpret_cast<const int32_t*>(u64(w.halo));
    u.rows = reinterpret_cast<const uint64_t*>(u64(w.rows));
    u.tris = reinterpret_cast<const uint64_t*>(u64(w.tris));
    u.rr = reinterpret_cast<const uint16_t*>(u64(w.rr));
    u.own_start = __builtin_amdgcn_readfirstlane(w.own_start);
    u.nown = __builtin_amdgcn_readfirstlane(w.nown);
    u.halo_cnt = __builtin_amdgcn_readfirstlane(w.halo_cnt);
    u.tri_cnt = __builtin_amdgcn_readfirstlane(w.tri_cnt);
    u.row_words = __builtin_amdgcn_readfirstlane(w.row_words);
    u.mesh = __builtin_amdgcn_readfirstlane(w.mesh);
    u.n = static_cast<int64_t>(uv(static_cast<uint64_t>(w.n)));
    return u;
}

template <bool SOA, typename R>
__device__ __forceinline__ typename Real<R>::V2 ldxg(gptr<R> X, int64_t n, int64_t i)
{
    if (SOA) return Real<R>::make(X[i], X[n + i]);
    return Real<R>::make(X[2 * i], X[2 * i + 1]);
}

// The buffer `parity` of a tile's mesh.
template <typename R>
__device__ __forceinline__ gptr<R> xin(const TileWork& d, int parity)
{
    return to_global(static_cast<const R*>(d.X)) + parity * 2 * d.n;
}

// The prefetch loads are unconditional, with indices clamped into the tile
// (a lane past the end re-loads the last element and its value is not
// used): straight-line loads let the compiler wait for exactly the ones the
// next step needs, where loads under per-lane branches made it wait for all.
template <int T, int BS, bool SOA, typename R, int NPT, int RPRE, int KPRE>
__device__ __forceinline__ void stage_a(TileStage<R, NPT, RPRE, KPRE>& s, const TileWork& d, int parity)
{
    const int tid = threadIdx.x;
    const gptr<R> Xin = xin<R>(d, parity);
    const gptr<int32_t> halo = to_global(d.halo);
    const gptr<uint16_t> rr = to_global(d.rr);
    s.hidx = halo[min(tid, max(d.halo_cnt - 1, 0))];   // meaningful for tid < halo_cnt only
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
        const int i = m * BS + tid;
        s.rs[m] = rr[i];
        s.re[m] = rr[i + 1];
        s.own[m] = ldxg<SOA>(Xin, d.n, d.own_start + min(i, d.nown - 1));
    }
}

template <int T, int BS, bool SOA, typename R, int NPT, int RPRE, int KPRE>
__device__ __forceinline__ void stage_b(TileStage<R, NPT, RPRE, KPRE>& s, const TileWork& d, int parity)
{
    const int tid = threadIdx.x;
    const gptr<R> Xin = xin<R>(d, parity);
    const gptr<uint64_t> rows = to_global(d.rows);
    const gptr<uint64_t> tris = to_global(d.tris);
    s.hx = ldxg<SOA>(Xin, d.n, tid < d.halo_cnt ? s.hidx : d.own_start);
#pragma unroll
    for (int q = 0; q < RPRE; ++q) s.rw[q] = rows[min(q * BS + tid, d.row_words - 1)];
#pragma unroll
    for (int q = 0; q < KPRE; ++q) s.tw[q] = tris[min(q * BS + tid, max(d.tri_cnt - 1, 0))];
}

// Persistent work-groups: the work list is cut into 8 contiguous ranges, one
// per XCD (work-groups are dealt to the XCDs round-robin), shared round-robin
// by the work-groups that XCD runs; each work-group computes one tile while
// the next one's data is on its way.
// (one_mesh: the group's displacement maximum and accepted count are left
// in out_d2 / out_acc, per work-item as the fold below takes them, for
// close_one_mesh; otherwise they are folded into the states here.)
template <int T, int BS, bool SOA, bool GT, typename R>
__device__ __forceinline__ void sweep_tiles(const TileSweepArgs& a, double& out_d2, unsigned long long& out_acc)
{
    out_d2 = 0.0;
    out_acc = 0;
    using V2 = typename Real<R>::V2;
    constexpr int NPT = T / BS;   // own nodes per work-item
    // per work-item register budget for the next tile: about 2.4 triangles
    // and 1.5 row words per free node on meshes of valence 6
    constexpr int KPRE = T == 256 ? 3 : 5;   // triangle entries
    constexpr int RPRE = T == 256 ? 2 : 4;   // 64-bit row words
    const int xcd = static_cast<int>(blockIdx.x & 7), nw = static_cast<int>(gridDim.x >> 3);
    const int t_begin = xcd * a.tiles_per_xcd;
    const int t_end = min(t_begin + a.tiles_per_xcd, a.n_work);
    int it = t_begin + static_cast<int>(blockIdx.x >> 3);
    if (it >= t_end) return;
    // A group's first two tiles are fixed (its slot, then one slot-row
    // further); the rest of the XCD's range is dealt one tile at a time from
    // the XCD's counter.  The SIMDs issue the oldest waves first, so the
    // groups dispatched first on a CU run faster; with fixed shares they
    // finished up to 1.6x earlier than the last, leaving the CU part-idle.
    // Each counter has a 128-byte line of its own: on one shared line the
    // device-scope atomics of all XCDs queued behind each other.
    int32_t* const deal = a.sched + kSchedStride * (1 + xcd);
    const int t_dealt = t_begin + 2 * nw;
    __shared__ int s_deal;
    int nxt = it + nw < t_end ? it + nw : -1;

    extern __shared__ double2 lds[];
    V2* Xl = reinterpret_cast<V2*>(lds);                    // [T + halo_cap]
    V2* cand = Xl + T + a.halo_cap;                         // [T]
    R* qo = reinterpret_cast<R*>(cand + T);                 // [T] worst old quality per own node
    R* qn = qo + T;                                         // [T] worst candidate quality
    uint16_t* rows = reinterpret_cast<uint16_t*>(qn + T);   // [rows_cap]
    uint64_t* rows64 = reinterpret_cast<uint64_t*>(rows);
    __shared__ double s_d2[BS / 64];
    __shared__ unsigned long long s_acc[BS / 64];
    __shared__ R s_recip[kMaxValence + 1];
    const int tid = threadIdx.x;
    // 1/d for every possible row length d, correctly rounded (read after the first barrier)
    if (tid <= kMaxValence) s_recip[tid] = tid ? R(1) / static_cast<R>(tid) : R(0);
    const int lane = tid & 63, wv = tid >> 6;
    const int parity = a.parity;

    // descriptors run two tiles ahead of the data, data one tile ahead; the
    // prefetches are unconditional (past the last tile they re-load it) so
    // that no branch forces them to complete early
    TileWork dcur = uniform_work(load_work(a.work, it));
    TileWork dnext = load_work(a.work, nxt >= 0 ? nxt : it);
    int act_cur = a.states[dcur.mesh].active;
    if (a.exit_if_inactive && act_cur == 0) return;
    TileStage<R, NPT, RPRE, KPRE> sg;
    stage_a<T, BS, SOA>(sg, dcur, parity);
    stage_b<T, BS, SOA>(sg, dcur, parity);
    double run_d2 = 0.0;
    unsigned long long run_acc = 0;

    for (;;) {
        const int nown = dcur.nown;
        int r0[NPT], r1[NPT];
        uint64_t tw[KPRE];
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            r0[m] = sg.rs[m];
            r1[m] = sg.re[m];
            if (m * BS + tid < nown) Xl[m * BS + tid] = sg.own[m];
        }
#pragma unroll
        for (int q = 0; q < RPRE; ++q)
            if (q * BS + tid < dcur.row_words) rows64[q * BS + tid] = sg.rw[q];
#pragma unroll
        for (int q = 0; q < KPRE; ++q) tw[q] = sg.tw[q];
        if (tid < dcur.halo_cnt) Xl[T + tid] = sg.hx;
        {
            // rare overflow beyond what the registers hold
            const gptr<R> Xin = xin<R>(dcur, parity);
            const gptr<int32_t> halo = to_global(dcur.halo);
            const gptr<uint64_t> rws = to_global(dcur.rows);
            for (int h = BS + tid; h < dcur.halo_cnt; h += BS) Xl[T + h] = ldxg<SOA>(Xin, dcur.n, halo[h]);
            for (int j = RPRE * BS + tid; j < dcur.row_words; j += BS) rows64[j] = rws[j];
        }
        __syncthreads();
        const bool has_next = nxt >= 0;
        // the tile after next, read after two more barriers
        if (tid == 0 && has_next) s_deal = t_dealt + atomicAdd(deal, 1);
        dnext = uniform_work(dnext);
        const int act_next = a.states[dnext.mesh].active;
        stage_a<T, BS, SOA>(sg, dnext, parity);
        const bool run = act_cur != 0;

        // candidates: row-order sum of the neighbours, one division by the count
        if (run) {
#pragma unroll
            for (int m = 0; m < NPT; ++m) {
                const int i = m * BS + tid;
                if (i < nown) {
                    R sx = R(0), sy = R(0);
                    for (int j = r0[m]; j < r1[m]; ++j) {
                        const V2 p = Xl[rows[j]];
                        sx += p.x;
                        sy += p.y;
                    }
                    const R dn = static_cast<R>(r1[m] - r0[m]), y = s_recip[r1[m] - r0[m]];
                    R cx = div_step(sx, dn, y), cy = div_step(sy, dn, y);
                    const bool tiny = !(fabs(sx) >= Real<R>::k_step_min) || !(fabs(sy) >= Real<R>::k_step_min);
                    // a wave-uniform branch, so that the division is skipped, not
                    // computed and discarded, when no lane needs it
                    if (__builtin_amdgcn_ballot_w64(tiny) != 0ull) {
                        if (tiny) {
                            cx = sx / dn;
                            cy = sy / dn;
                        }
                    }
                    cand[i] = Real<R>::make(cx, cy);
                    qo[i] = static_cast<R>(__builtin_inf());
                    qn[i] = static_cast<R>(__builtin_inf());
                }
            }
        }
        __syncthreads();
        stage_b<T, BS, SOA>(sg, dnext, parity);

        // triangles
        if (run) {
#pragma unroll
            for (int q = 0; q < KPRE; ++q)
                if (q * BS + tid < dcur.tri_cnt) tile_triangle<T, R>(tw[q], Xl, cand, qo, qn);
            const gptr<uint64_t> tris = to_global(dcur.tris);
            for (int r = KPRE * BS + tid; r < dcur.tri_cnt; r += BS) tile_triangle<T, R>(tris[r], Xl, cand, qo, qn);
        }
        __syncthreads();
        int nxt2 = -1;
        if (has_next) {
            const int g = s_deal;
            nxt2 = g < t_end ? g : -1;
        }
        const TileWork dnext2 = load_work(a.work, nxt2 >= 0 ? nxt2 : (has_next ? nxt : it));

        // accept and write; the displacement maximum and the accepted count
        // accumulate per work-item over consecutive tiles of one mesh and are
        // folded into its MeshState when the mesh changes (one pair of
        // atomics per work-group and mesh)
        if (run) {
            __attribute__((address_space(1))) R* Xout =
                reinterpret_cast<__attribute__((address_space(1))) R*>(reinterpret_cast<uint64_t>(dcur.X)) +
                (parity ^ 1) * 2 * dcur.n;
            const int k0 = dcur.own_start;
#pragma unroll
            for (int m = 0; m < NPT; ++m) {
                const int i = m * BS + tid;
                bool accepted = false;
                if (i < nown) {
                    const R vo = qo[i], vn = qn[i];
                    accepted = GT ? (vn > vo) : (vn >= vo);
                    const V2 o = Xl[i];
                    const V2 c = cand[i];
                    const R nx = accepted ? c.x : o.x, ny = accepted ? c.y : o.y;
                    if (SOA) {
                        Xout[k0 + i] = nx;
                        Xout[dcur.n + k0 + i] = ny;
                    } else {
                        Xout[2 * (k0 + i)] = nx;
                        Xout[2 * (k0 + i) + 1] = ny;
                    }
                    const R dx = nx - o.x, dy = ny - o.y;
                    const double d2 = static_cast<double>(dx * dx + dy * dy);   // exact widening
                    run_d2 = d2 > run_d2 ? d2 : run_d2;
                }
                const unsigned long long ball = __ballot(accepted);
                run_acc += __popcll(ball);
                if (a.bits != nullptr && lane == 0 && ball != 0ull)
                    atomicOr(reinterpret_cast<unsigned long long*>(a.bits) + ((k0 + m * BS + wv * 64) >> 6), ball);
            }
        }
        if (a.one_mesh && !has_next) {
            out_d2 = run_d2;
            out_acc = run_acc;
        } else if (!has_next || dnext.mesh != dcur.mesh) {
            double d2 = run_d2;
            for (int off = 32; off > 0; off >>= 1) {
                const double t = __shfl_xor(d2, off);
                d2 = t > d2 ? t : d2;
            }
            if (lane == 0) {
                s_d2[wv] = d2;
                s_acc[wv] = run_acc;
            }
            __syncthreads();
            if (tid == 0) {
                double mx = s_d2[0];
                unsigned long long c = s_acc[0];
                for (int q = 1; q < BS / 64; ++q) {
                    mx = s_d2[q] > mx ? s_d2[q] : mx;
                    c += s_acc[q];
                }
                MeshState* ms = a.states + dcur.mesh;
                if (mx > 0.0) atomicMax(&ms->maxd_cur, static_cast<unsigned long long>(__double_as_longlong(mx)));
                if (c) atomicAdd(&ms->acc_cur, c);
            }
            run_d2 = 0.0;
            run_acc = 0;
        }
        if (!has_next) break;
        it = nxt;
        nxt = nxt2;
        dcur = dnext;
        dnext = dnext2;
        act_cur = act_next;
        __syncthreads();
    }
}

template <int T, int BS, bool SOA, bool GT, typename R>
__global__ __launch_bounds__(BS) void k_sweep_tile(TileSweepArgs a)
{
    double d2;
    unsigned long long acc;
    sweep_tiles<T, BS, SOA, GT, R>(a, d2, acc);
    if (!a.one_mesh) {
        close_launch<BS>(a.sched, a.states, a.n_close);
    } else if (fold_through_slots<BS, true>(a.sched, a.states + a.work[0].mesh, d2, acc) && threadIdx.x == 0) {
        // the last group (its fold into the state came from work-item 0)
        for (int i = 0; i < a.n_close; ++i) close_state(a.states + i);
    }
}

constexpr int kTileBS = 256;

template <int T, int BS, bool SOA, bool GT, typename R>
void launch_tile_variant(const TileSweepArgs& a, int grid, size_t lds, hipStream_t st)
{
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_tile<T, BS, SOA, GT, R>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        (void)hipGetLastError();
    }
    k_sweep_tile<T, BS, SOA, GT, R><<<grid, BS, lds, st>>>(a);
}

template <int T, typename R>
void launch_tile_t(const TileSweepArgs& a, bool soa, bool gt, int grid, size_t lds, hipStream_t st)
{
    if (soa) {
        if (gt) launch_tile_variant<T, kTileBS, true, true, R>(a, grid, lds, st);
        else launch_tile_variant<T, kTileBS, true, false, R>(a, grid, lds, st);
    } else {
        if (gt) launch_tile_variant<T, kTileBS, false, true, R>(a, grid, lds, st);
        else launch_tile_variant<T, kTileBS, false, false, R>(a, grid, lds, st);
    }
}

}  // namespace

// LDS of one work-group: own and halo positions, candidates and the two
// per-node minima in the sweep's precision, u16 rows.
size_t tile_lds_bytes(int tile_nodes, int halo_cap, int rows_cap, int32_t precision)
{
    const size_t rb = precision == SL_F32 ? 4 : 8;
    return static_cast<size_t>(tile_nodes + halo_cap) * 2 * rb + static_cast<size_t>(tile_nodes) * 4 * rb +
           static_cast<size_t>(rows_cap) * 2;
}

int tile_grid(int n_work, int tile_nodes, int halo_cap, int rows_cap, int wg_per_cu, int32_t precision)
{
    const size_t lds = tile_lds_bytes(tile_nodes, halo_cap, rows_cap, precision);
    // work-groups per CU: as requested (else 4), no more than fit the LDS;
    // 32 CUs per XCD; never more work-groups than tiles on an XCD.  (Small
    // launches were capped at 3 per CU while every group ended with atomics
    // on the mesh's state; with the folds through slots 4 is faster there
    // too: 1024^2 grid 0.0305 against 0.0325 ms, 2048^2 0.0842 against
    // 0.0889 ms.)
    const int fit = std::max(1, static_cast<int>(kTileLdsLimit / std::max<size_t>(lds, 1)));
    const int want = wg_per_cu > 0 ? wg_per_cu : 4;
    const int per_cu = std::min(want, fit);
    const int tpx = div_up(std::max(n_work, 1), 8);
    const int nw = std::min(tpx, 32 * per_cu);
    return 8 * nw;
}

sl_status launch_sweep_tiles(const TileLaunch& L, int32_t parity, uint64_t* bits, hipStream_t st)
{
    if (L.n_work <= 0) return L.n_close > 0 ? launch_advance(L.states, L.n_close, st) : SL_OK;
    if (!L.sched) return fail(SL_EINVAL, "tile launch without its counters");
    TileSweepArgs a{};
    a.work = L.work;
    a.n_work = L.n_work;
    a.tiles_per_xcd = div_up(L.n_work, 8);
    a.halo_cap = L.halo_cap;
    a.rows_cap = L.rows_cap;
    a.parity = parity;
    a.exit_if_inactive = L.exit_if_inactive;
    a.states = L.states;
    a.bits = bits;
    a.sched = L.sched;
    a.n_close = L.n_close;
    a.one_mesh = L.one_mesh;
    const size_t lds = tile_lds_bytes(L.tile_nodes, L.halo_cap, L.rows_cap, L.precision);
    const int grid = tile_grid(L.n_work, L.tile_nodes, L.halo_cap, L.rows_cap, L.wg_per_cu, L.precision);
    if (grid > kTileMaxGroups) return fail(SL_EINVAL, "internal: tile launch of more groups than slots");
    const bool soa = L.layout == SL_SOA, gt = L.accept == SL_ACCEPT_GT;
    if (L.precision == SL_F32) {
        if (L.tile_nodes == 256) launch_tile_t<256, float>(a, soa, gt, grid, lds, st);
        else launch_tile_t<512, float>(a, soa, gt, grid, lds, st);
    } else {
        if (L.tile_nodes == 256) launch_tile_t<256, double>(a, soa, gt, grid, lds, st);
        else launch_tile_t<512, double>(a, soa, gt, grid, lds, st);
    }
    SL_HIP(hipGetLastError());
    return SL_OK;
}

}  // namespace sl
