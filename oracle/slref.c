/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, FP64 CPU implementation of two-dimensional Smart Laplacian
 * smoothing (Zhao, Mei, Xu, Zhang, "On the Accelerating of Two-dimensional
 * Smart Laplacian Smoothing on the GPU", ICCS 2015).  Only the tests, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header or constant with the GPU library and must never be
 * used as a fallback for it.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math), on
 * x86-64 SSE2, so every operation below is one IEEE-754 double operation,
 * rounded to nearest, in the order written.
 *
 * What is computed (paper Sec. 2.1 "Laplacian Smoothing", eq. (2) "Form A",
 * eq. (3) "Form B", Sec. 3.3.4 "The Iterating Procedure"):
 *   - every free node is moved to the geometric centre of its neighbours;
 *   - the move is kept only if the worst quality among the node's incident
 *     triangles does not drop (quality compared before/after);
 *   - Form A: all neighbour positions come from the previous pass (Jacobi);
 *   - Form B: positions already updated in the current pass are used; here
 *     the split is fixed by a node colouring (one colour class at a time).
 * The paper names the Lee-Lo quality alpha without printing it; the quality
 * used is 4*sqrt(3)*A / (l0^2 + l1^2 + l2^2) with A the signed area.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* 4*sqrt(3)*A = 2*sqrt(3) * (twice the signed area).  sqrt is correctly
 * rounded and the doubling is exact, so this is the double nearest 2*sqrt(3). */
static double two_sqrt3(void) { return 2.0 * sqrt(3.0); }

/* Quality of the triangle (p0, p1, p2) taken in its stored vertex order.
 * Edges a = p1-p0, b = p2-p0, c = p2-p1; cr = a x b (twice the signed area,
 * positive for CCW); S = (|a|^2 + |c|^2) + |b|^2; q = (2*sqrt(3)*cr) / S.
 * An equilateral CCW triangle has q = 1, a CW one q < 0; S == 0 gives 0. */
double slref_quality(double x0, double y0, double x1, double y1, double x2, double y2)
{
    double ax = x1 - x0, ay = y1 - y0;
    double bx = x2 - x0, by = y2 - y0;
    double cx = x2 - x1, cy = y2 - y1;
    double cr = ax * by - bx * ay;
    double la = ax * ax + ay * ay;
    double lb = bx * bx + by * by;
    double lc = cx * cx + cy * cy;
    double S = (la + lc) + lb;
    if (S == 0.0) return 0.0;
    return (two_sqrt3() * cr) / S;
}

/* Quality of triangle t with node `who` (one of its vertices) placed at
 * (wx, wy); every other vertex read from X.  who < 0: no substitution. */
static double tri_q(const double* X, const int32_t* tris, int32_t t, int32_t who, double wx, double wy)
{
    double px[3], py[3];
    for (int s = 0; s < 3; ++s) {
        int32_t v = tris[3 * (int64_t)t + s];
        if (v == who) { px[s] = wx; py[s] = wy; }
        else { px[s] = X[2 * (int64_t)v]; py[s] = X[2 * (int64_t)v + 1]; }
    }
    return slref_quality(px[0], py[0], px[1], py[1], px[2], py[2]);
}

/* One Smart Laplacian update of free node i, reading positions from X.
 * Centroid (eq. (2)): neighbours summed in row order, then one division by
 * the neighbour count.  Accept test (Sec. 2.1, Sec. 3.3.4): min quality of
 * the incident triangles with the node at the candidate vs at its current
 * position.  accept_gt = 0: accept iff new_min >= old_min; 1: strictly >.
 * Returns 1 if accepted; writes the node's resulting position to (*ox,*oy). */
static int update_node(const double* X, int32_t i, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                       const int32_t* tri_ptr, const int32_t* tri_idx, const int32_t* tris,
                       int accept_gt, double* ox, double* oy)
{
    int32_t b = nbr_ptr[i], e = nbr_ptr[i + 1];
    double sx = 0.0, sy = 0.0;
    for (int32_t k = b; k < e; ++k) {
        sx += X[2 * (int64_t)nbr_idx[k]];
        sy += X[2 * (int64_t)nbr_idx[k] + 1];
    }
    double dn = (double)(e - b);
    double cx = sx / dn, cy = sy / dn;
    double xi = X[2 * (int64_t)i], yi = X[2 * (int64_t)i + 1];
    double qo = INFINITY, qn = INFINITY;
    for (int32_t k = tri_ptr[i]; k < tri_ptr[i + 1]; ++k) {
        int32_t t = tri_idx[k];
        double v = tri_q(X, tris, t, -1, 0.0, 0.0);
        if (v < qo) qo = v;
        double w = tri_q(X, tris, t, i, cx, cy);
        if (w < qn) qn = w;
    }
    int acc = accept_gt ? (qn > qo) : (qn >= qo);
    *ox = acc ? cx : xi;
    *oy = acc ? cy : yi;
    return acc;
}

/* Checks the oracle needs to run at all: ranges, ptr monotone, free nodes
 * with at least one neighbour, each incident triangle contains its node.
 * Returns 0 if usable, -1 otherwise. */
static int check_inputs(int32_t n, const int32_t* nbr_ptr, const int32_t* nbr_idx, const int32_t* tri_ptr,
                        const int32_t* tri_idx, const int32_t* tris, int32_t n_tris, const uint8_t* boundary)
{
    if (n < 0 || n_tris < 0 || nbr_ptr[0] != 0 || tri_ptr[0] != 0) return -1;
    for (int32_t i = 0; i < n; ++i) {
        if (nbr_ptr[i + 1] < nbr_ptr[i] || tri_ptr[i + 1] < tri_ptr[i]) return -1;
        for (int32_t k = nbr_ptr[i]; k < nbr_ptr[i + 1]; ++k)
            if (nbr_idx[k] < 0 || nbr_idx[k] >= n) return -1;
        for (int32_t k = tri_ptr[i]; k < tri_ptr[i + 1]; ++k) {
            int32_t t = tri_idx[k];
            if (t < 0 || t >= n_tris) return -1;
            if (tris[3 * (int64_t)t] != i && tris[3 * (int64_t)t + 1] != i && tris[3 * (int64_t)t + 2] != i)
                return -1;
        }
        if (!boundary[i] && nbr_ptr[i + 1] == nbr_ptr[i]) return -1;
    }
    for (int64_t k = 0; k < 3 * (int64_t)n_tris; ++k)
        if (tris[k] < 0 || tris[k] >= n) return -1;
    return 0;
}

/* One Jacobi (Form A, eq. (2)) sweep: Xout = sweep(Xin).  Free nodes read
 * only Xin; fixed (boundary) nodes are copied.  flags (nullable, n bytes):
 * 1 accepted, 0 rejected, 2 fixed.  Returns the number of accepted nodes and
 * the largest squared displacement dx*dx + dy*dy in *max_disp_sq. */
int64_t slref_sweep_jacobi(const double* Xin, double* Xout, int32_t n, const int32_t* nbr_ptr,
                           const int32_t* nbr_idx, const int32_t* tri_ptr, const int32_t* tri_idx,
                           const int32_t* tris, const uint8_t* boundary, int accept_gt, int n_threads,
                           uint8_t* flags, double* max_disp_sq)
{
    int64_t acc_count = 0;
    double dmax = 0.0;
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for num_threads(n_threads) schedule(static) reduction(+ : acc_count) reduction(max : dmax)
#endif
    for (int32_t i = 0; i < n; ++i) {
        double x = Xin[2 * (int64_t)i], y = Xin[2 * (int64_t)i + 1];
        if (boundary[i]) {
            Xout[2 * (int64_t)i] = x;
            Xout[2 * (int64_t)i + 1] = y;
            if (flags) flags[i] = 2;
            continue;
        }
        double nx, ny;
        int acc = update_node(Xin, i, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, accept_gt, &nx, &ny);
        Xout[2 * (int64_t)i] = nx;
        Xout[2 * (int64_t)i + 1] = ny;
        if (flags) flags[i] = (uint8_t)acc;
        acc_count += acc;
        double dx = nx - x, dy = ny - y;
        double d2 = dx * dx + dy * dy;
        if (d2 > dmax) dmax = d2;
    }
    *max_disp_sq = dmax;
    return acc_count;
}

/* Smart Laplacian, Form A, iterated (Sec. 3.3.4): sweeps k = 0, 1, ... while
 * k < iterations; if tol > 0 the loop also ends after the first sweep whose
 * largest squared displacement is below tol*tol.  coords (n x 2, in/out).
 * Optional per-sweep outputs: flags (iterations * n bytes), disp (iterations
 * doubles), accepted (iterations counts).  Returns sweeps run, or -1 on
 * unusable input (coords untouched). */
int32_t slref_smooth(double* coords, int32_t n, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                     const int32_t* tri_ptr, const int32_t* tri_idx, const int32_t* tris, int32_t n_tris,
                     const uint8_t* boundary, int32_t iterations, double tol, int accept_gt, int n_threads,
                     uint8_t* flags, double* disp, int64_t* accepted)
{
    if (iterations < 0) return -1;
    if (check_inputs(n, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, n_tris, boundary)) return -1;
    double* A = (double*)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
    double* B = (double*)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
    if (!A || !B) { free(A); free(B); return -1; }
    memcpy(A, coords, sizeof(double) * 2 * (size_t)n);
    double tol2 = tol * tol;
    int32_t k = 0;
    while (k < iterations) {
        double d2;
        int64_t a = slref_sweep_jacobi(A, B, n, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, boundary, accept_gt,
                                       n_threads, flags ? flags + (size_t)k * n : NULL, &d2);
        if (disp) disp[k] = d2;
        if (accepted) accepted[k] = a;
        double* t = A; A = B; B = t;
        ++k;
        if (tol > 0.0 && d2 < tol2) break;
    }
    memcpy(coords, A, sizeof(double) * 2 * (size_t)n);
    free(A);
    free(B);
    return k;
}

/* ---- Form B (eq. (3)) with a node colouring --------------------------- */

/* Priority of node v for the colouring order: the SplitMix64 output
 * function (Steele, Lea, Flood, OOPSLA 2014) applied to v. */
uint64_t slref_priority(uint64_t v)
{
    uint64_t z = v + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static const uint64_t* g_prio_sort_key;
static int cmp_prio_desc(const void* a, const void* b)
{
    uint64_t pa = g_prio_sort_key[*(const int32_t*)a], pb = g_prio_sort_key[*(const int32_t*)b];
    return pa < pb ? 1 : (pa > pb ? -1 : 0);
}

/* Greedy colouring of the free nodes: visit them in decreasing priority and
 * give each the smallest colour not already held by one of its free
 * neighbours.  Fixed nodes get colour -1.  Returns the number of colours. */
int32_t slref_color(int32_t n, const int32_t* nbr_ptr, const int32_t* nbr_idx, const uint8_t* boundary,
                    int32_t* color)
{
    uint64_t* pr = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t m = 0, ncol = 0;
    for (int32_t v = 0; v < n; ++v) {
        pr[v] = slref_priority((uint64_t)v);
        color[v] = -1;
        if (!boundary[v]) order[m++] = v;
    }
    g_prio_sort_key = pr;
    qsort(order, (size_t)m, sizeof(int32_t), cmp_prio_desc);
    for (int32_t q = 0; q < m; ++q) {
        int32_t v = order[q];
        for (int32_t c = 0;; ++c) {
            int used = 0;
            for (int32_t k = nbr_ptr[v]; k < nbr_ptr[v + 1]; ++k)
                if (color[nbr_idx[k]] == c) { used = 1; break; }
            if (!used) { color[v] = c; if (c + 1 > ncol) ncol = c + 1; break; }
        }
    }
    free(pr);
    free(order);
    return ncol;
}

/* Smart Laplacian, Form B, iterated: each sweep runs the colour classes in
 * increasing colour; inside a class every free node is updated in place
 * (reads the current positions, so neighbours of earlier classes are already
 * at pass q+1 and the others at pass q).  Nodes of one class are never
 * adjacent, so the order inside a class does not matter.  Outputs as
 * slref_smooth; colors_out (nullable, n) receives the colouring. */
int32_t slref_smooth_colored(double* coords, int32_t n, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                             const int32_t* tri_ptr, const int32_t* tri_idx, const int32_t* tris, int32_t n_tris,
                             const uint8_t* boundary, int32_t iterations, double tol, int accept_gt,
                             uint8_t* flags, double* disp, int64_t* accepted, int32_t* colors_out)
{
    if (iterations < 0) return -1;
    if (check_inputs(n, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, n_tris, boundary)) return -1;
    int32_t* color = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t ncol = slref_color(n, nbr_ptr, nbr_idx, boundary, color);
    if (colors_out) memcpy(colors_out, color, sizeof(int32_t) * (size_t)n);
    double tol2 = tol * tol;
    int32_t k = 0;
    while (k < iterations) {
        double dmax = 0.0;
        int64_t acc_count = 0;
        uint8_t* fl = flags ? flags + (size_t)k * n : NULL;
        for (int32_t c = 0; c < ncol; ++c) {
            for (int32_t i = 0; i < n; ++i) {
                if (color[i] != c) continue;
                double x = coords[2 * (int64_t)i], y = coords[2 * (int64_t)i + 1];
                double nx, ny;
                int acc = update_node(coords, i, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, accept_gt, &nx, &ny);
                coords[2 * (int64_t)i] = nx;
                coords[2 * (int64_t)i + 1] = ny;
                if (fl) fl[i] = (uint8_t)acc;
                acc_count += acc;
                double dx = nx - x, dy = ny - y;
                double d2 = dx * dx + dy * dy;
                if (d2 > dmax) dmax = d2;
            }
        }
        if (fl)
            for (int32_t i = 0; i < n; ++i)
                if (boundary[i]) fl[i] = 2;
        if (disp) disp[k] = dmax;
        if (accepted) accepted[k] = acc_count;
        ++k;
        if (tol > 0.0 && dmax < tol2) break;
    }
    free(color);
    return k;
}

/* ---- single precision (the paper's precision, Sec. 4) ------------------ */

/* The same Form A computation carried out in IEEE single precision: the
 * caller's coordinates are rounded to float once, every operation below is
 * one float operation in the order written, and the constant is the float
 * nearest 2*sqrt(3) (sqrtf is correctly rounded, the doubling exact).  The
 * convergence test widens the float squared displacement to double. */
static float two_sqrt3f(void) { return 2.0f * sqrtf(3.0f); }

float slref32_quality(float x0, float y0, float x1, float y1, float x2, float y2)
{
    float ax = x1 - x0, ay = y1 - y0;
    float bx = x2 - x0, by = y2 - y0;
    float cx = x2 - x1, cy = y2 - y1;
    float cr = ax * by - bx * ay;
    float la = ax * ax + ay * ay;
    float lb = bx * bx + by * by;
    float lc = cx * cx + cy * cy;
    float S = (la + lc) + lb;
    if (S == 0.0f) return 0.0f;
    return (two_sqrt3f() * cr) / S;
}

static float tri_q32(const float* X, const int32_t* tris, int32_t t, int32_t who, float wx, float wy)
{
    float px[3], py[3];
    for (int s = 0; s < 3; ++s) {
        int32_t v = tris[3 * (int64_t)t + s];
        if (v == who) { px[s] = wx; py[s] = wy; }
        else { px[s] = X[2 * (int64_t)v]; py[s] = X[2 * (int64_t)v + 1]; }
    }
    return slref32_quality(px[0], py[0], px[1], py[1], px[2], py[2]);
}

static int update_node32(const float* X, int32_t i, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                         const int32_t* tri_ptr, const int32_t* tri_idx, const int32_t* tris, int accept_gt,
                         float* ox, float* oy)
{
    int32_t b = nbr_ptr[i], e = nbr_ptr[i + 1];
    float sx = 0.0f, sy = 0.0f;
    for (int32_t k = b; k < e; ++k) {
        sx += X[2 * (int64_t)nbr_idx[k]];
        sy += X[2 * (int64_t)nbr_idx[k] + 1];
    }
    float dn = (float)(e - b);
    float cx = sx / dn, cy = sy / dn;
    float xi = X[2 * (int64_t)i], yi = X[2 * (int64_t)i + 1];
    float qo = INFINITY, qn = INFINITY;
    for (int32_t k = tri_ptr[i]; k < tri_ptr[i + 1]; ++k) {
        int32_t t = tri_idx[k];
        float v = tri_q32(X, tris, t, -1, 0.0f, 0.0f);
        if (v < qo) qo = v;
        float w = tri_q32(X, tris, t, i, cx, cy);
        if (w < qn) qn = w;
    }
    int acc = accept_gt ? (qn > qo) : (qn >= qo);
    *ox = acc ? cx : xi;
    *oy = acc ? cy : yi;
    return acc;
}

/* Form A in single precision, iterated; arguments and outputs as
 * slref_smooth.  coords (double, n x 2) are rounded to float on entry and
 * receive the float results on exit (exactly representable). */
int32_t slref32_smooth(double* coords, int32_t n, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                       const int32_t* tri_ptr, const int32_t* tri_idx, const int32_t* tris, int32_t n_tris,
                       const uint8_t* boundary, int32_t iterations, double tol, int accept_gt, int n_threads,
                       uint8_t* flags, double* disp, int64_t* accepted)
{
    if (iterations < 0) return -1;
    if (check_inputs(n, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, n_tris, boundary)) return -1;
    float* A = (float*)malloc(sizeof(float) * 2 * (size_t)(n > 0 ? n : 1));
    float* B = (float*)malloc(sizeof(float) * 2 * (size_t)(n > 0 ? n : 1));
    if (!A || !B) { free(A); free(B); return -1; }
    for (int64_t k = 0; k < 2 * (int64_t)n; ++k) A[k] = (float)coords[k];
    double tol2 = tol * tol;
    int32_t k = 0;
    if (n_threads < 1) n_threads = 1;
    while (k < iterations) {
        int64_t acc_count = 0;
        float dmax = 0.0f;
        uint8_t* fl = flags ? flags + (size_t)k * n : NULL;
#ifdef _OPENMP
#pragma omp parallel for num_threads(n_threads) schedule(static) reduction(+ : acc_count) reduction(max : dmax)
#endif
        for (int32_t i = 0; i < n; ++i) {
            float x = A[2 * (int64_t)i], y = A[2 * (int64_t)i + 1];
            if (boundary[i]) {
                B[2 * (int64_t)i] = x;
                B[2 * (int64_t)i + 1] = y;
                if (fl) fl[i] = 2;
                continue;
            }
            float nx, ny;
            int acc = update_node32(A, i, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, accept_gt, &nx, &ny);
            B[2 * (int64_t)i] = nx;
            B[2 * (int64_t)i + 1] = ny;
            if (fl) fl[i] = (uint8_t)acc;
            acc_count += acc;
            float dx = nx - x, dy = ny - y;
            float d2 = dx * dx + dy * dy;
            if (d2 > dmax) dmax = d2;
        }
        if (disp) disp[k] = (double)dmax;
        if (accepted) accepted[k] = acc_count;
        float* t = A; A = B; B = t;
        ++k;
        if (tol > 0.0 && (double)dmax < tol2) break;
    }
    for (int64_t q = 0; q < 2 * (int64_t)n; ++q) coords[q] = (double)A[q];
    free(A);
    free(B);
    return k;
}

/* Largest number of threads OpenMP would use (1 without OpenMP). */
int slref_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
