/*
 * Input-side mesh bookkeeping for the synthetic workloads.
 *
 * This file builds the adjacency arrays that a caller of the smoothing
 * library hands in (node->neighbour CSR, node->triangle CSR) and the
 * boundary mask.  It holds none of the smoothing arithmetic: no quality,
 * no centroid, no accept test.  Both the oracle and the GPU library
 * receive what it produces as plain inputs.
 *
 * Neighbour order (paper, Sec. 3.3.2 "The Finding of Neighbors"): the
 * triangles are scanned in index order; for a triangle (v1,v2,v3) the second
 * and third vertices are recorded as neighbours of the first, the first and
 * third as neighbours of the second, the first and second as neighbours of
 * the third.  A neighbour already recorded for a node is not recorded again,
 * so each row lists the distinct neighbours in order of first appearance.
 * Each triangle is incident to its three vertices; incident-triangle rows
 * list triangle ids ascending.
 *
 * Boundary (paper, Sec. 3.3.3 "The Determining of Constraints"): a node is
 * interior iff every one of its neighbours was recorded twice during the
 * scan above (each edge lies in exactly two triangles); otherwise it is a
 * boundary node.  A node that belongs to no triangle is marked boundary.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Returns 0 on success, -1 on bad input (vertex id out of range or a
 * triangle with a repeated vertex), -2 on allocation failure.
 * Outputs: nbr_ptr[n+1], nbr_idx[<= 6*n_tris] (caller allocates 6*n_tris),
 * tri_ptr[n+1], tri_idx[3*n_tris], boundary[n], *nnz_out. */
int mg_build_adjacency(int32_t n_nodes, int32_t n_tris, const int32_t* tris,
                       int32_t* nbr_ptr, int32_t* nbr_idx, int32_t* tri_ptr,
                       int32_t* tri_idx, uint8_t* boundary, int64_t* nnz_out)
{
    if (n_nodes < 0 || n_tris < 0) return -1;
    for (int64_t t = 0; t < n_tris; ++t) {
        int32_t a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
        if (a < 0 || b < 0 || c < 0 || a >= n_nodes || b >= n_nodes || c >= n_nodes) return -1;
        if (a == b || b == c || a == c) return -1;
    }
    /* incident-triangle counts -> tri_ptr */
    int32_t* tcount = (int32_t*)calloc((size_t)n_nodes + 1, sizeof(int32_t));
    if (!tcount) return -2;
    for (int64_t k = 0; k < 3 * (int64_t)n_tris; ++k) tcount[tris[k]]++;
    tri_ptr[0] = 0;
    for (int32_t v = 0; v < n_nodes; ++v) tri_ptr[v + 1] = tri_ptr[v] + tcount[v];
    /* fill incident triangles ascending (triangles visited in order) */
    int32_t* fill = (int32_t*)malloc(((size_t)n_nodes + 1) * sizeof(int32_t));
    if (!fill) { free(tcount); return -2; }
    memcpy(fill, tri_ptr, (size_t)n_nodes * sizeof(int32_t));
    for (int32_t t = 0; t < n_tris; ++t)
        for (int s = 0; s < 3; ++s) {
            int32_t v = tris[3 * (int64_t)t + s];
            tri_idx[fill[v]++] = t;
        }
    /* neighbour rows: each node has at most 2*t_v distinct neighbours; use a
     * scratch area of that capacity, deduplicate by linear scan, record the
     * number of times each neighbour was seen. */
    int64_t* cap_ptr = (int64_t*)malloc(((size_t)n_nodes + 1) * sizeof(int64_t));
    int32_t* len = (int32_t*)calloc((size_t)n_nodes + 1, sizeof(int32_t));
    if (!cap_ptr || !len) { free(tcount); free(fill); free(cap_ptr); free(len); return -2; }
    cap_ptr[0] = 0;
    for (int32_t v = 0; v < n_nodes; ++v) cap_ptr[v + 1] = cap_ptr[v] + 2 * (int64_t)tcount[v];
    int32_t* scratch = (int32_t*)malloc((size_t)(cap_ptr[n_nodes] > 0 ? cap_ptr[n_nodes] : 1) * sizeof(int32_t));
    uint8_t* seen = (uint8_t*)calloc((size_t)(cap_ptr[n_nodes] > 0 ? cap_ptr[n_nodes] : 1), 1);
    if (!scratch || !seen) {
        free(tcount); free(fill); free(cap_ptr); free(len); free(scratch); free(seen);
        return -2;
    }
    for (int32_t t = 0; t < n_tris; ++t) {
        const int32_t* tv = tris + 3 * (int64_t)t;
        /* (owner slot, first recorded, second recorded) */
        static const int order[3][3] = {{0, 1, 2}, {1, 0, 2}, {2, 0, 1}};
        for (int r = 0; r < 3; ++r) {
            int32_t v = tv[order[r][0]];
            for (int q = 1; q < 3; ++q) {
                int32_t u = tv[order[r][q]];
                int32_t* row = scratch + cap_ptr[v];
                uint8_t* rs = seen + cap_ptr[v];
                int32_t L = len[v], k;
                for (k = 0; k < L; ++k)
                    if (row[k] == u) break;
                if (k == L) { row[L] = u; rs[L] = 1; len[v] = L + 1; }
                else if (rs[k] < 255) rs[k]++;
            }
        }
    }
    nbr_ptr[0] = 0;
    for (int32_t v = 0; v < n_nodes; ++v) {
        int32_t L = len[v];
        const int32_t* row = scratch + cap_ptr[v];
        const uint8_t* rs = seen + cap_ptr[v];
        memcpy(nbr_idx + nbr_ptr[v], row, (size_t)L * sizeof(int32_t));
        nbr_ptr[v + 1] = nbr_ptr[v] + L;
        int interior = (L > 0);
        for (int32_t k = 0; k < L; ++k)
            if (rs[k] != 2) { interior = 0; break; }
        boundary[v] = interior ? 0 : 1;
    }
    *nnz_out = nbr_ptr[n_nodes];
    free(tcount); free(fill); free(cap_ptr); free(len); free(scratch); free(seen);
    return 0;
}

/*
 * Delaunay triangulation of distinct points on an integer lattice, for the
 * random-point workloads (the paper's test meshes are Delaunay meshes of
 * uniformly distributed points, Sec. 4).  Coordinates are integers below
 * 2^21 in magnitude, so the orientation and in-circle determinants are exact
 * in 128-bit integers and the result is a true Delaunay triangulation.
 *
 * Method: the points are swept in (x, y) order, each new point joined to
 * the hull edges it sees (a triangulation of the convex hull), then edges
 * are flipped until every interior edge is locally Delaunay (Lawson).
 * Output triangles are counter-clockwise; their count is 2n - h - 2 for h
 * points on the hull.
 */
typedef __int128 i128;

typedef struct {
    int32_t v[3];
    int32_t nb[3];   /* nb[i]: triangle across the edge opposite v[i], -1 on the hull */
} DTri;

static i128 orient(const int64_t* x, const int64_t* y, int32_t a, int32_t b, int32_t c)
{
    return (i128)(x[b] - x[a]) * (y[c] - y[a]) - (i128)(y[b] - y[a]) * (x[c] - x[a]);
}

/* > 0 iff d lies strictly inside the circumcircle of the CCW triangle abc */
static i128 incircle(const int64_t* x, const int64_t* y, int32_t a, int32_t b, int32_t c, int32_t d)
{
    const i128 adx = x[a] - x[d], ady = y[a] - y[d];
    const i128 bdx = x[b] - x[d], bdy = y[b] - y[d];
    const i128 cdx = x[c] - x[d], cdy = y[c] - y[d];
    const i128 al = adx * adx + ady * ady, bl = bdx * bdx + bdy * bdy, cl = cdx * cdx + cdy * cdy;
    return adx * (bdy * cl - bl * cdy) - ady * (bdx * cl - bl * cdx) + al * (bdx * cdy - bdy * cdx);
}

static const int64_t* g_sx;
static const int64_t* g_sy;
static int cmp_xy(const void* pa, const void* pb)
{
    const int32_t a = *(const int32_t*)pa, b = *(const int32_t*)pb;
    if (g_sx[a] != g_sx[b]) return g_sx[a] < g_sx[b] ? -1 : 1;
    if (g_sy[a] != g_sy[b]) return g_sy[a] < g_sy[b] ? -1 : 1;
    return 0;
}

static int32_t slot_of(const DTri* t, int32_t v)
{
    return t->v[0] == v ? 0 : (t->v[1] == v ? 1 : 2);
}

/* links the edge (u, v) of triangle `tri` to triangle `to` */
static void link_edge(DTri* T, int32_t tri, int32_t u, int32_t v, int32_t to)
{
    for (int k = 0; k < 3; ++k)
        if (T[tri].v[k] != u && T[tri].v[k] != v) { T[tri].nb[k] = to; return; }
}

/* points the neighbour link of triangle `tri` that referred to `from` at `to` */
static void relink(DTri* T, int32_t tri, int32_t from, int32_t to)
{
    if (tri < 0) return;
    for (int k = 0; k < 3; ++k)
        if (T[tri].nb[k] == from) { T[tri].nb[k] = to; return; }
}

/* Returns 0 on success, -1 for fewer than 3 points or all points collinear,
 * -2 on allocation failure, -3 for a duplicate point.  tris_out holds at
 * least 3*(2n-5) entries. */
int mg_delaunay(int32_t n, const int64_t* x, const int64_t* y, int32_t* tris_out, int32_t* n_tris_out)
{
    if (n < 3) return -1;
    const int64_t cap = 2 * (int64_t)n;
    int32_t* order = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    DTri* T = (DTri*)malloc((size_t)cap * sizeof(DTri));
    int32_t* hnext = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* hprev = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* htri = (int32_t*)malloc((size_t)n * sizeof(int32_t));   /* triangle holding hull edge v -> hnext[v] */
    int64_t stack_cap = 4 * cap;
    int64_t* stack = (int64_t*)malloc((size_t)stack_cap * sizeof(int64_t));
    if (!order || !T || !hnext || !hprev || !htri || !stack) {
        free(order); free(T); free(hnext); free(hprev); free(htri); free(stack);
        return -2;
    }
    int rc = 0;
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    g_sx = x;
    g_sy = y;
    qsort(order, (size_t)n, sizeof(int32_t), cmp_xy);
    for (int32_t i = 1; i < n && !rc; ++i)
        if (x[order[i]] == x[order[i - 1]] && y[order[i]] == y[order[i - 1]]) rc = -3;
    int32_t k = 2;
    while (!rc && k < n && orient(x, y, order[0], order[1], order[k]) == 0) ++k;
    if (!rc && k == n) rc = -1;
    int32_t nt = 0;
    if (!rc) {
        /* the collinear chain order[0..k-1] fanned to order[k] */
        const int32_t p = order[k];
        const int left = orient(x, y, order[0], order[1], p) > 0;
        for (int32_t i = 0; i + 1 < k; ++i) {
            DTri* t = &T[nt];
            const int32_t a = order[i], b = order[i + 1];
            if (left) { t->v[0] = a; t->v[1] = b; t->v[2] = p; }
            else { t->v[0] = b; t->v[1] = a; t->v[2] = p; }
            t->nb[0] = t->nb[1] = t->nb[2] = -1;
            if (i > 0) {
                /* shares the edge (order[i], p) with the previous triangle */
                const int32_t s_prev = slot_of(&T[nt - 1], order[i - 1]);
                const int32_t s_cur = slot_of(t, order[i + 1]);
                T[nt - 1].nb[s_prev] = nt;
                t->nb[s_cur] = nt - 1;
            }
            ++nt;
        }
        /* CCW hull */
        if (left) {
            for (int32_t i = 0; i + 1 < k; ++i) { hnext[order[i]] = order[i + 1]; htri[order[i]] = i; }
            hnext[order[k - 1]] = p; htri[order[k - 1]] = k - 2;
            hnext[p] = order[0]; htri[p] = 0;
        } else {
            hnext[order[0]] = p; htri[order[0]] = 0;
            hnext[p] = order[k - 1]; htri[p] = k - 2;
            for (int32_t i = k - 1; i > 0; --i) { hnext[order[i]] = order[i - 1]; htri[order[i]] = i - 1; }
        }
        for (int32_t i = 0; i <= k; ++i) hprev[hnext[order[i]]] = order[i];
    }
    /* sweep: each point sees a contiguous run of hull edges */
    for (int32_t i = k + 1; i < n && !rc; ++i) {
        const int32_t p = order[i], q = order[i - 1];   /* q: the previous point, a hull vertex */
        /* the visible run: edges u -> hnext[u] with p strictly to their right */
        int32_t s = q, e = q;
        while (orient(x, y, hprev[s], s, p) < 0) s = hprev[s];
        while (orient(x, y, e, hnext[e], p) < 0) e = hnext[e];
        if (s == e) { rc = -1; break; }
        int32_t prev_new = -1, first_new = -1;
        for (int32_t u = s; u != e; u = hnext[u]) {
            const int32_t v = hnext[u];
            if (nt >= cap) { rc = -2; break; }
            DTri* t = &T[nt];
            t->v[0] = v; t->v[1] = u; t->v[2] = p;   /* CCW: p is right of u -> v */
            t->nb[2] = htri[u];                        /* across (v, u): the old hull triangle */
            link_edge(T, htri[u], u, v, nt);
            t->nb[0] = -1;                             /* across (u, p) */
            t->nb[1] = -1;                             /* across (p, v) */
            if (prev_new >= 0) {
                /* previous new triangle (u, w, p) shares the edge (u, p) */
                t->nb[0] = prev_new;
                T[prev_new].nb[1] = nt;
            } else {
                first_new = nt;
            }
            prev_new = nt;
            ++nt;
        }
        if (rc) break;
        /* hull: s -> p -> e */
        for (int32_t u = hnext[s]; u != e;) { const int32_t w = hnext[u]; hnext[u] = hprev[u] = -1; u = w; }
        hnext[s] = p; hprev[p] = s; htri[s] = first_new;
        hnext[p] = e; hprev[e] = p; htri[p] = prev_new;
    }
    /* Lawson flips */
    int64_t sp = 0;
    for (int32_t t = 0; t < nt && !rc; ++t)
        for (int j = 0; j < 3; ++j) stack[sp++] = ((int64_t)t << 2) | j;
    while (sp > 0 && !rc) {
        const int64_t item = stack[--sp];
        const int32_t A = (int32_t)(item >> 2), ia = (int32_t)(item & 3);
        const int32_t B = T[A].nb[ia];
        if (B < 0) continue;
        const int32_t a = T[A].v[ia], b = T[A].v[(ia + 1) % 3], c = T[A].v[(ia + 2) % 3];
        const int32_t jb = slot_of(&T[B], b);   /* B = (.., c, b, ..) with d opposite */
        const int32_t ib = (jb + 1) % 3;        /* slot of d: after b comes d (B is CCW: c, b, d) */
        const int32_t d = T[B].v[ib];
        if (incircle(x, y, a, b, c, d) <= 0) continue;
        const int32_t n_ca = T[A].nb[(ia + 1) % 3], n_ab = T[A].nb[(ia + 2) % 3];
        const int32_t n_dc = T[B].nb[jb], n_bd = T[B].nb[(jb + 2) % 3];
        /* A <- (a, b, d), B <- (a, d, c) */
        T[A].v[0] = a; T[A].v[1] = b; T[A].v[2] = d;
        T[A].nb[0] = n_bd; T[A].nb[1] = B; T[A].nb[2] = n_ab;
        T[B].v[0] = a; T[B].v[1] = d; T[B].v[2] = c;
        T[B].nb[0] = n_dc; T[B].nb[1] = n_ca; T[B].nb[2] = A;
        relink(T, n_bd, B, A);
        relink(T, n_ca, A, B);
        if (sp + 4 > stack_cap) {
            int64_t* grown = (int64_t*)realloc(stack, (size_t)(2 * stack_cap) * sizeof(int64_t));
            if (!grown) { rc = -2; break; }
            stack = grown;
            stack_cap *= 2;
        }
        stack[sp++] = ((int64_t)A << 2) | 0;
        stack[sp++] = ((int64_t)A << 2) | 2;
        stack[sp++] = ((int64_t)B << 2) | 0;
        stack[sp++] = ((int64_t)B << 2) | 1;
    }
    if (!rc) {
        for (int32_t t = 0; t < nt; ++t)
            for (int j = 0; j < 3; ++j) tris_out[3 * (int64_t)t + j] = T[t].v[j];
        *n_tris_out = nt;
    }
    free(order); free(T); free(hnext); free(hprev); free(htri); free(stack);
    return rc;
}
