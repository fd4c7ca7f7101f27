/*
 * smartlap -- Smart Laplacian smoothing of 2D triangular meshes on MI355X.
 *
 * The operation (Zhao, Mei, Xu, Zhang, ICCS 2015, Sec. 2.1 and Sec. 3.3.4):
 * every free node is moved to the geometric centre of its neighbours
 * (eq. (2)); the move is kept only if the worst quality among the node's
 * incident triangles does not drop.  The quality of a triangle (p0,p1,p2),
 * taken in its stored vertex order, is
 *     q = (2*sqrt(3) * cr) / S,
 *     a = p1-p0, b = p2-p0, c = p2-p1,  cr = a.x*b.y - b.x*a.y,
 *     S = (|a|^2 + |c|^2) + |b|^2,      q = 0 when S == 0,
 * i.e. 4*sqrt(3)*A / sum(l^2) with A the signed area (1 for an equilateral
 * CCW triangle, negative for an inverted one).  Every operation is one
 * IEEE-754 double operation in the order written (no contraction), the
 * centroid sums the neighbour row in its stored order and divides once by
 * the neighbour count.
 *
 * Forms (Sec. 2.2): SL_JACOBI is Form A, eq. (2) -- every read comes from the
 * previous pass.  SL_INPLACE_COLORED is Form B, eq. (3) -- the free nodes are
 * coloured (greedy, in decreasing SplitMix64 priority of the node id, so no
 * two adjacent free nodes share a colour) and each pass runs the colour
 * classes in increasing colour, updating in place.
 *
 * Conventions for every entry point:
 *   - Return value: an sl_status; SL_OK is 0, errors are negative.  On any
 *     error a message is available from sl_last_error() (per thread), and
 *     output arrays are left untouched.
 *   - Ownership: the caller owns every array it passes.  The library copies
 *     or reads them before the call returns (or, for the *_async calls,
 *     before the work they queue completes) and keeps no pointer to them.
 *   - Device memory: what the library allocates for a call is given back
 *     when the call's work is done (for handles and servers: in the matching
 *     *_destroy call).  Given-back blocks are kept for reuse by later calls,
 *     up to 16 GiB per device, and memory the runtime's stream-ordered pool
 *     frees stays reserved in that pool; sl_release_cached_memory() returns
 *     both to the device.
 *   - Indices are 0-based int32.  Arrays are dense, no padding.
 */
#ifndef SMARTLAP_H
#define SMARTLAP_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define SL_API __attribute__((visibility("default")))
#else
#define SL_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SL_OK = 0,
    SL_EINVAL = -1,    /* null pointer, size <= 0, non-monotone ptr, index out of range,
                          iterations < 0, coordinate not finite or of magnitude >= 2^500
                          (2^61 in single precision: so that no squared length or sum
                          of them overflows), bad option value */
    SL_ETOPO = -2,     /* self neighbour, triangle with a repeated vertex, incident triangle
                          not containing its node, a vertex of an incident triangle missing
                          from the node's neighbour row, free node without neighbours,
                          valence > 127 (free nodes), asymmetric rows (coloured form) */
    SL_ENOMEM = -3,    /* device allocation failed or a budget would be exceeded */
    SL_EDEVICE = -4,   /* a HIP runtime error; text in sl_last_error() */
    SL_EBUSY = -5,     /* result not ready yet */
    SL_ECANCELED = -6, /* request was cancelled */
    SL_ETIMEOUT = -7   /* request passed its deadline */
} sl_status;

typedef enum { SL_JACOBI = 0, SL_INPLACE_COLORED = 1 } sl_form;
typedef enum {
    SL_ACCEPT_GE = 0,  /* accept iff new worst quality >= old worst quality (default) */
    SL_ACCEPT_GT = 1   /* accept iff it strictly increases */
} sl_accept;
typedef enum { SL_AOS = 0, SL_SOA = 1 } sl_layout;   /* coordinate stream on the device */
typedef enum {
    SL_F64 = 0,          /* every operation in IEEE double precision (default) */
    SL_F32 = 1           /* the paper's precision (Sec. 4): coordinates rounded to float once
                            on the device, every operation one IEEE float operation in the same
                            order, the constant the float nearest 2*sqrt(3); results returned
                            as doubles (exactly representable).  The squared displacement of
                            the convergence test is computed in float and compared in double.
                            Form A on the tile path only (SL_EINVAL otherwise). */
} sl_precision;
typedef enum { SL_REORDER_NONE = 0, SL_REORDER_HILBERT = 1 } sl_reorder;
typedef enum {
    SL_KERNEL_AUTO = 0,  /* Form A: the tile kernel when the mesh fits it, else the node kernel.
                            Form B: the resident kernel when the mesh fits it (never in a
                            server or on a handle), else the node kernel (faster there than
                            colour-class tiles, which SL_KERNEL_TILE asks for) */
    SL_KERNEL_NODE = 1,  /* one work-item per free node, neighbours gathered from HBM/L2 */
    SL_KERNEL_TILE = 2,  /* work-group per tile of free nodes staged in LDS: Form A's tiles of
                            consecutive free nodes, or Form B's tiles of one colour class each
                            (one launch per class, in place; double precision, at most 32
                            classes).  At most 16 neighbour entries and 16 incidences per node
                            on average over a tile, at most 4 (colour-class tiles: 8) distinct
                            outside neighbours per tile node, and the halo and rows must fit
                            in LDS; else the node kernel */
    SL_KERNEL_RESIDENT = 3, /* one work-group runs every sweep of the mesh in one launch, with
                               the coordinates, rows and fans in LDS (double precision, not in a
                               server): Form A keeps both buffers, Form B one, updated class by
                               class.  (32 or 16) n + 4 (n + 1) + 2 nbr_ptr[n] + 2 tri_ptr[n]
                               bytes must fit in 159 KB, n, nbr_ptr[n], tri_ptr[n] <= 65535 and
                               Form B has at most 32 colour classes; SL_EINVAL otherwise.  For
                               Form A one compute unit outpaces the tile kernel only on meshes
                               of a few hundred nodes, so it is never chosen automatically */
    SL_KERNEL_LANES = 4     /* a lane group of lane_width work-items of one wave per free node:
                               the group's lanes gather the node's neighbours and evaluate its
                               incident triangles side by side, and DPP moves inside the group
                               fold their minima; neighbours come from L2/HBM, no tiles.  Double
                               precision, either form (Form B: one launch per colour class).  It
                               issues each wave instruction for 64 / lane_width nodes instead of
                               64, so the tile kernel outruns it; never chosen automatically */
} sl_kernel;

typedef struct {
    int32_t form;        /* sl_form */
    int32_t accept;      /* sl_accept */
    int32_t layout;      /* sl_layout */
    int32_t reorder;     /* sl_reorder: node order used on the device; results do not depend on it */
    int32_t block_size;  /* node kernel work-group size: 0 = automatic, else 64/128/256 */
    int32_t kernel;      /* sl_kernel; results do not depend on it */
    int32_t tile_nodes;      /* free nodes per tile on the tile path.  Form A: 0 = automatic (the
                              * value sl_autotune chose on this device, else 512; a one-call
                              * smooth takes 256 on meshes of fewer than 2^19 nodes), or 256 or 512.
                              * Form B's colour-class tiles: 0 = automatic (512 on meshes of at
                              * least 2^20 nodes, else 256), or 128, 256 or 512.  Results do not
                              * depend on it */
    int32_t tile_wg_per_cu;  /* tile-kernel work-groups per compute unit: 0 = automatic (the
                              * value sl_autotune chose, else as many as fit, at most 4), or
                              * 1..8, capped by what fits in LDS; results do not depend on it */
    int32_t precision;       /* sl_precision */
    int32_t lane_width;      /* SL_KERNEL_LANES: work-items per free node, 0 = automatic (the
                              * value sl_autotune chose on this device, else 8), or 4, 8 or 16;
                              * results do not depend on it */
    /* Optional accept flags, nullable.  Size iterations * ((n_nodes + 7) / 8)
     * bytes; sweep k occupies bytes [k*((n+7)/8), (k+1)*((n+7)/8)); bit (i % 8)
     * of byte (i / 8) is 1 iff free node i accepted its move in sweep k
     * (0 for fixed nodes and for sweeps that did not run).  Host memory for
     * smooth_mesh, device memory for smooth_mesh_device. */
    uint8_t* flags_out;
} sl_options;

typedef struct {
    int32_t iterations_run;     /* sweeps executed (<= iterations) */
    int32_t n_colors;           /* colour classes (coloured form), else 0 */
    double max_disp_sq_last;    /* largest squared displacement in the last sweep run */
    int64_t accepted_last;      /* free nodes that accepted in the last sweep run */
    int64_t accepted_total;     /* summed over all sweeps run */
    double setup_ms;            /* device time: validation, reorder, relabel, fan build */
    double sweep_ms;            /* device time of the sweep loop only */
    double total_ms;            /* host wall time of the whole call */
    int32_t kernel_used;        /* SL_KERNEL_NODE, SL_KERNEL_TILE, SL_KERNEL_RESIDENT or SL_KERNEL_LANES */
    int32_t tile_nodes;         /* free nodes per tile on the tile path, else 0 */
} sl_report;

/* Fills *opts with the defaults: Jacobi, GE, AoS, Hilbert reorder, automatic
 * block size and kernel, no flags. */
SL_API void sl_options_default(sl_options* opts);

/*
 * smooth_mesh -- iterated Smart Laplacian on one mesh, host arrays.
 *
 * coords    in/out, n_nodes x 2 doubles, (x, y) interleaved.  Written only on SL_OK
 *           (a device failure during the final copy may leave it partly written).
 * n_nodes   >= 1.
 * nbr_ptr   n_nodes+1 offsets into nbr_idx (CSR node -> neighbour), nbr_ptr[0] = 0.
 * nbr_idx   nbr_ptr[n_nodes] neighbour ids; the order within a row is the
 *           summation order of the centroid.
 * tri_ptr   n_nodes+1 offsets into tri_idx (CSR node -> incident triangle).
 * tri_idx   tri_ptr[n_nodes] triangle ids; each must contain its node.  A
 *           node's tests use the triangles of its own row only.  The tile
 *           kernel needs each listed triangle to be listed by all of its
 *           free vertices; a mesh whose rows disagree runs on the node kernel
 *           (same results).
 * tris      n_tris x 3 vertex ids; the stored order is the evaluation order
 *           of the quality (CCW for a positive quality).
 * n_tris    >= 0.
 * boundary  n_nodes bytes, nonzero = fixed node (never moved, never evaluated).
 * iterations  cap on sweeps, >= 0.
 * tol       > 0: stop after the first sweep whose largest squared displacement
 *           of a node is below tol*tol; <= 0: run exactly `iterations` sweeps.
 * opts      nullable (defaults).  report: nullable.
 * The call is synchronous; it uses the current HIP device.
 */
SL_API sl_status smooth_mesh(double* coords, int32_t n_nodes, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                      const int32_t* tri_ptr, const int32_t* tri_idx, const int32_t* tris, int32_t n_tris,
                      const uint8_t* boundary, int32_t iterations, double tol, const sl_options* opts,
                      sl_report* report);

/*
 * smooth_mesh_device -- as smooth_mesh, but every array (coords, the CSR
 * arrays, tris, boundary, opts->flags_out) is device memory on the current
 * HIP device, and all work is queued on `stream` (a hipStream_t; NULL = the
 * null stream).  The input arrays are only read; coords is overwritten with
 * the result, and must be 16-byte aligned (SL_EINVAL otherwise: the (x, y)
 * pairs are moved as 16-byte units).  The call returns after the work on
 * `stream` has completed (the sweep count and the validation result are
 * needed on the host).
 */
SL_API sl_status smooth_mesh_device(double* coords, int32_t n_nodes, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                             const int32_t* tri_ptr, const int32_t* tri_idx, const int32_t* tris, int32_t n_tris,
                             const uint8_t* boundary, int32_t iterations, double tol, const sl_options* opts,
                             sl_report* report, void* stream);

/*
 * smooth_mesh_device_noalloc -- for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid allocation): the same
 * call, arguments, results and errors as smooth_mesh_device, but the library
 * allocates no device memory.  Every device array of the call -- the mesh's
 * reordered copy, tiles and coordinate buffers, the setup's temporaries, the
 * sweep state and accept bits -- is carved from one static workspace of
 * 256 MiB per device (a file-scope device array, held by each device the
 * library runs on until the process ends; about 1.5 million nodes of a mesh
 * of valence 6, fewer with flag output).  A mesh that needs more fails with
 * SL_ENOMEM before any work, coordinates untouched.  The workspace keeps
 * the last call's contents; each call clears what must start at zero.  Calls
 * on one device share it, so they must not overlap: within a process the
 * library runs them one at a time (the call returns only when its work on
 * `stream` is done); the sweep loop is launched directly, not through a
 * captured graph.  The first call on a device looks up the workspace's
 * device address and creates the call's four timing events.
 */
SL_API sl_status smooth_mesh_device_noalloc(double* coords, int32_t n_nodes, const int32_t* nbr_ptr,
                                     const int32_t* nbr_idx, const int32_t* tri_ptr, const int32_t* tri_idx,
                                     const int32_t* tris, int32_t n_tris, const uint8_t* boundary, int32_t iterations,
                                     double tol, const sl_options* opts, sl_report* report, void* stream);

/* One mesh of a batch or a served request: host arrays as for smooth_mesh.
 * coords is in/out (written on SL_OK only). */
typedef struct {
    double* coords;
    int32_t n_nodes;
    int32_t n_tris;
    const int32_t* nbr_ptr;
    const int32_t* nbr_idx;
    const int32_t* tri_ptr;
    const int32_t* tri_idx;
    const int32_t* tris;
    const uint8_t* boundary;
} sl_mesh_desc;

typedef struct {
    double setup_ms;            /* host wall time of uploads and per-mesh setup */
    double sweep_ms;            /* device time of the batched sweep loop */
    double total_ms;            /* host wall time of the whole call */
    int64_t node_updates;       /* sum over meshes of free nodes x sweeps run */
    int64_t tiles;              /* tiles in the batched work list */
    int32_t meshes_on_tile_path;
    int32_t graph_used;         /* 1 if the sweep loop ran as a captured HIP graph */
    double graph_ms;            /* host wall time of capturing and instantiating the graph */
    double results_ms;          /* host wall time of un-permuting and copying out the results */
    int32_t meshes_resident;    /* meshes run on the resident kernel (all their sweeps in one launch) */
    int32_t reserved;
} sl_batch_report;

/*
 * sl_batch_smooth -- the same smoothing as smooth_mesh, applied to n_meshes
 * independent meshes at once (host arrays).  All meshes are resident on the
 * device together; each sweep is one launch over the tiles of every mesh,
 * and the sweep loop runs as a captured HIP graph.  Every mesh gets exactly
 * the result a separate smooth_mesh call with the same options would give.
 * iterations and tol apply to every mesh (each stops on its own).
 * Device memory: the meshes' own arrays are taken as one allocation (about
 * 135 bytes per node in double precision), or one per mesh when that single
 * allocation fails; setup temporaries are per mesh and short-lived.
 * reports: nullable, n_meshes entries.  batch: nullable.
 * On an error in mesh i the message names i and no coords are written.
 */
SL_API sl_status sl_batch_smooth(const sl_mesh_desc* meshes, int32_t n_meshes, int32_t iterations, double tol,
                                 const sl_options* opts, sl_report* reports, sl_batch_report* batch);

/* ---- mesh handles --------------------------------------------------------
 * A mesh set up once -- validated, reordered and tiled on the device, as the
 * paper's mesh object holds vertices with their neighbours and incident
 * triangles (Sec. 3.2) -- and kept resident, so that it can be smoothed any
 * number of times, alone or batched with other handles, without uploading
 * or setting it up again.  Sweeps continue where the last call stopped:
 * k sweeps and then k more give exactly the result of 2k sweeps in one
 * smooth_mesh call.  Options are fixed at creation (automatic values
 * resolved then); flags_out is ignored and the resident kernel is not used
 * (Form B runs on the node kernel, or on colour-class tiles where the mesh
 * fits them when SL_KERNEL_TILE asks for them).  A handle belongs to the device that
 * was current at creation, and calls on it must be made with that device
 * current; it is not thread-safe (one call at a time per handle).  Work on
 * a handle is ordered across streams: each call's work runs after the
 * previous call's. */
typedef struct sl_mesh sl_mesh;

/* Creates a handle from host arrays (as for smooth_mesh; desc->coords gives
 * the initial positions and is not written).  Synchronous.  Device memory:
 * about 135 bytes per node in double precision, freed by sl_mesh_destroy. */
SL_API sl_status sl_mesh_create(const sl_mesh_desc* desc, const sl_options* opts, sl_mesh** out);

/* The same from device arrays (as for smooth_mesh_device), read on `stream`
 * (a hipStream_t, NULL = the null stream); returns when the handle is ready
 * and the arrays are no longer needed. */
SL_API sl_status sl_mesh_create_device(const double* coords, int32_t n_nodes, const int32_t* nbr_ptr,
                                       const int32_t* nbr_idx, const int32_t* tri_ptr, const int32_t* tri_idx,
                                       const int32_t* tris, int32_t n_tris, const uint8_t* boundary,
                                       const sl_options* opts, void* stream, sl_mesh** out);

/* Queues `iterations` more sweeps (>= 0) on `stream`.  tol <= 0: exactly
 * that many, and the call returns without waiting for the device.  tol > 0:
 * stop after the first sweep whose largest squared displacement is below
 * tol*tol; the call then reads the sweep state back after every 32 sweeps
 * and returns once the mesh has stopped (the device is idle for the mesh). */
SL_API sl_status sl_mesh_smooth_async(sl_mesh* mesh, int32_t iterations, double tol, void* stream);

/* Sweeps several handles together, `iterations` more sweeps each (tol as
 * for sl_mesh_smooth_async, each mesh stopping on its own): one launch per
 * sweep over the tiles of every handle, queued on `stream`.  Every handle
 * gets exactly the result of sweeping it alone.  The handles must share
 * form, accept rule, layout and precision, those on the tile path their
 * tile size; no handle may appear twice.  batch: nullable; filled with what
 * is known when the call returns (tiles, meshes on the tile path, node
 * updates, host time of the call; its device times are 0). */
SL_API sl_status sl_mesh_smooth_batch_async(sl_mesh* const* meshes, int32_t n_meshes, int32_t iterations,
                                            double tol, void* stream, sl_batch_report* batch);

/* Copies the current positions to host memory (n_nodes x 2 doubles, the
 * caller's node order) after the handle's queued work; report (nullable) is
 * filled with the handle's totals: sweeps run since creation, accepted
 * counts, the setup time and the device time of the last single-handle
 * smooth call.  Synchronous.  On an error coords is not written, except
 * that a device failure during the copy may leave it partly written. */
SL_API sl_status sl_mesh_download(sl_mesh* mesh, double* coords, sl_report* report);

/* The same into device memory (16-byte aligned), queued on `stream` after
 * the handle's queued work; returns without waiting. */
SL_API sl_status sl_mesh_download_device(sl_mesh* mesh, double* coords, void* stream);

/* The handle's totals as for sl_mesh_download, without the positions. */
SL_API sl_status sl_mesh_get_report(sl_mesh* mesh, sl_report* report);

/* Waits for the handle's queued work and frees its device memory.  NULL is
 * ignored. */
SL_API void sl_mesh_destroy(sl_mesh* mesh);

/* Frees the device blocks the library keeps for reuse on the current
 * device and trims the runtime's stream-ordered pool to what is in use.
 * Call it when another user of the device needs the memory; later calls
 * allocate again. */
SL_API sl_status sl_release_cached_memory(void);

/* ---- adjacency from a triangle list -------------------------------------
 * Builds the inputs the smoothing calls take from a bare triangle list, the
 * way the paper finds neighbours and constraints (Sec. 3.3.2, Sec. 3.3.3):
 *   tri_ptr/tri_idx  each node's incident triangles, in index order;
 *   nbr_ptr/nbr_idx  each node's distinct neighbours: the other two vertices
 *                    of its incident triangles, triangle by triangle in index
 *                    order and, inside a triangle (v1,v2,v3), v2,v3 for v1,
 *                    v1,v3 for v2 and v1,v2 for v3, each kept where it first
 *                    appears (this row order is the centroid's summation
 *                    order);
 *   boundary         0 for a node every neighbour of which was seen exactly
 *                    twice (every edge at the node lies in two triangles),
 *                    else 1 (also for a node in no triangle).
 * Sizes: nbr_ptr and tri_ptr n_nodes+1, tri_idx 3*n_tris, boundary n_nodes,
 * nbr_idx nbr_capacity entries (6*n_tris always suffices); n_tris at most
 * INT32_MAX/6.  *nnz receives nbr_ptr[n_nodes].  With nbr_idx NULL the call
 * is a size query: only *nnz is written.
 * Errors: SL_EINVAL for bad sizes, a null output, a vertex id out of range,
 * or nbr_capacity < *nnz (then *nnz holds the size needed); SL_ETOPO for a
 * triangle with a repeated vertex.  The other outputs are written only on
 * SL_OK.  Work runs on the device; the rows are sorted and deduplicated
 * there, one work-item per node.
 * sl_build_adjacency: host arrays, synchronous. */
SL_API sl_status sl_build_adjacency(const int32_t* tris, int32_t n_tris, int32_t n_nodes, int32_t* nbr_ptr,
                                    int32_t* nbr_idx, int64_t nbr_capacity, int32_t* tri_ptr, int32_t* tri_idx,
                                    uint8_t* boundary, int64_t* nnz);

/* The same with every array in device memory (nnz is a host pointer); work
 * runs on `stream` (a hipStream_t, NULL for the default stream) and is
 * complete when the call returns. */
SL_API sl_status sl_build_adjacency_device(const int32_t* tris, int32_t n_tris, int32_t n_nodes, int32_t* nbr_ptr,
                                           int32_t* nbr_idx, int64_t nbr_capacity, int32_t* tri_ptr,
                                           int32_t* tri_idx, uint8_t* boundary, int64_t* nnz, void* stream);

/* ---- autotuning ---------------------------------------------------------
 * The launch shape of the tile kernel -- free nodes per tile (256 or 512)
 * and work-groups per compute unit -- changes only speed, never results.
 * sl_autotune times sweeps of every candidate shape on the caller's meshes
 * (a deterministic sample of them, taken at a stride in index order, of at
 * most about 8M nodes), twice each, interleaved, and keeps the fastest as
 * the automatic choice of the current device -- or the default shape (512
 * nodes, 4 work-groups per CU; block size 256) when it is within 1% of the
 * fastest -- for the rest of the process: later calls whose options
 * leave tile_nodes / tile_wg_per_cu at 0 use it.  For Form B (coloured) the
 * node kernel's work-group size is tuned and used where block_size is 0 (the
 * node kernel is Form B's automatic choice beyond the resident kernel);
 * colour-class tiles are not tuned.  With opts->kernel == SL_KERNEL_LANES
 * (either form) the lane-group width (4, 8, 16; default 8) is tuned instead
 * and used where lane_width is 0.  Meshes are read, not written.  The
 * caller's opts give form, accept, layout and kernel; their tile, block and
 * lane fields are ignored.
 * out: nullable.  Thread-safe; a later call replaces the device's choice. */
typedef struct {
    int32_t tile_nodes;          /* chosen, 0 if no sampled mesh fits the tile path */
    int32_t tile_wg_per_cu;      /* chosen */
    int32_t block_size;          /* chosen node-kernel work-group size (Form B), else 0 */
    int32_t n_candidates;        /* entries of the table below that were timed */
    struct {
        int32_t tile_nodes;      /* 0 for a node-kernel or lane-group candidate */
        int32_t wg_per_cu;       /* or the node-kernel work-group size, or the lane-group width */
        double ns_per_update;    /* device time per free-node update */
    } candidates[16];
    int32_t sampled_meshes;
    int64_t sampled_free_nodes;
    double tune_ms;              /* host wall time of the call */
    int32_t lane_width;          /* chosen lane-group width (kernel SL_KERNEL_LANES), else 0 */
} sl_tuning;

SL_API sl_status sl_autotune(const sl_mesh_desc* meshes, int32_t n_meshes, const sl_options* opts, sl_tuning* out);

/* Forgets the current device's tuned choice (automatic values revert to the
 * built-in defaults). */
SL_API void sl_autotune_reset(void);

/* ---- serving ----------------------------------------------------------
 * A server takes smoothing requests as they arrive and sweeps the admitted
 * ones together (continuous batching): a request is admitted when a slot is
 * free and its estimated device footprint fits the HBM budget, joins the
 * next scheduling step after its setup, and leaves as soon as it reaches its
 * sweep cap or tolerance.  Its result is exactly that of smooth_mesh with the
 * same options.  One scheduler thread per server owns the device; the calls
 * below are thread-safe.
 * Ownership: the arrays a request's sl_mesh_desc points to are read by the
 * scheduler thread and must stay valid and unchanged until sl_server_poll
 * returns something other than SL_EBUSY for that request (or the server is
 * destroyed); desc->coords is not written (results go to poll's coords_out). */
typedef struct sl_server sl_server;

typedef struct {
    size_t hbm_budget_bytes;    /* admission limit on estimated footprints; 0 = 200 GiB */
    int32_t max_active;         /* requests swept together at most; 0 = 256 */
    int32_t sweeps_per_step;    /* sweeps between two scheduling decisions; 0 = 8 */
    int32_t setup_threads;      /* threads that upload and set up admitted requests; 0 = 4, at most 64 */
} sl_server_config;

typedef struct {
    double submitted_s;         /* server clock (seconds since sl_server_create) */
    double admitted_s;          /* slot and memory granted */
    double started_s;           /* setup done, first step next */
    double done_s;              /* result on the host (or failure recorded) */
} sl_request_times;

typedef struct {
    int64_t submitted, completed, failed, steps;
    int64_t node_updates;       /* free nodes x sweeps of completed requests */
    int32_t queued, active;
    size_t hbm_in_use;          /* sum of the admitted requests' estimated footprints */
} sl_server_stats;

SL_API void sl_server_config_default(sl_server_config* cfg);
/* opts: as for smooth_mesh (flags_out ignored); nullable. */
SL_API sl_status sl_server_create(const sl_server_config* cfg, const sl_options* opts, sl_server** out);
/* Queues a request; deadline_s > 0: fail with SL_ETIMEOUT if not done within
 * deadline_s seconds of submission.  *request_id identifies it. */
SL_API sl_status sl_server_submit(sl_server* srv, const sl_mesh_desc* mesh, int32_t iterations, double tol,
                                  double deadline_s, uint64_t* request_id);
/* SL_EBUSY while the request is queued or running.  Otherwise returns its
 * final status once (the id is then released): on SL_OK the positions are
 * copied to coords_out (n_nodes x 2, nullable) and report/times are filled
 * (nullable); SL_ECANCELED, SL_ETIMEOUT, SL_ENOMEM or a setup error otherwise
 * (times still filled). */
SL_API sl_status sl_server_poll(sl_server* srv, uint64_t request_id, double* coords_out, sl_report* report,
                                sl_request_times* times);
/* Asks for a request to stop; it ends with SL_ECANCELED at the next step. */
SL_API sl_status sl_server_cancel(sl_server* srv, uint64_t request_id);
SL_API sl_status sl_server_get_stats(sl_server* srv, sl_server_stats* stats);
/* Stops the scheduler and frees everything; pending requests are dropped. */
SL_API void sl_server_destroy(sl_server* srv);

/* Message describing the last failure on the calling thread ("" if none). */
SL_API const char* sl_last_error(void);

/* Library version string. */
SL_API const char* sl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SMARTLAP_H */
