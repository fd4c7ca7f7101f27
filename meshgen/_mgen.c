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
