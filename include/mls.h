/*
 * mls.h -- C ABI of the MI355X (gfx950) moving-least-squares projection
 * library (libmls.so).
 *
 * The operation: given a point cloud P = {p_i} sampled (with noise) from a
 * surface, project query points r near the surface onto the MLS surface of P
 * (Section 1.4, problem statement; Algorithm 1: input a point set, output a
 * surface represented by a point set). For every query the library
 *   1. finds the k nearest cloud points exactly (canonical FP64 squared
 *      distances, ties to the smaller original index) from a Morton-sorted
 *      uniform grid hash -- the neighbourhood search of Section 2 and
 *      Section 2.2, with k neighbours instead of a radius;
 *   2. weights them with theta(d) = exp(-d^2/h^2) (Section 1.4 asks for a
 *      smooth, positive, monotonically decreasing theta);
 *   3. fits the reference plane H (Eq. (1.1), one step with the weights
 *      centred at r): n = eigenvector of the smallest eigenvalue of the
 *      weighted 3x3 covariance; origin q = orthogonal projection of r on H;
 *   4. fits the heights over H with a weighted bivariate quadratic g in an
 *      orthonormal frame of H with origin q, weights theta(|p_i - q|)
 *      (Section 2.1, Algorithm 1);
 *   5. returns q + g(0,0) n, the projection of the point onto g
 *      (Section 2.1, Algorithm 1).
 * A query with fewer than `min_support` list entries within
 * `support_radius_h * h` is an outlier (Section 3.3) and is returned
 * unchanged with status MLS_PT_OUTLIER.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers unless marked (host). The caller
 *     owns every array and every workspace; the library allocates no device
 *     memory of its own (its one device array of fixed size is the scratch
 *     of mls_project_noalloc, in its code object).
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     Calls are stream-ordered. mls_build_grid synchronises `stream` twice
 *     (to size the grid); the other calls never block the host.
 *   - Argument errors are found on the host before anything is launched and
 *     are returned as codes; nothing aborts and no exception crosses the ABI.
 *     A failed launch or an earlier asynchronous device error is returned as
 *     MLS_ERR_HIP (the HIP error text is kept by mls_last_error()).
 *   - Per-point conditions are statuses, not errors (MLS_PT_*).
 *   - Points are FP32 xyz triples (n_points x 3, row-major). Queries and
 *     outputs are FP32 or FP64 triples (dtype).
 */
#ifndef MLS_H
#define MLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MLS_OK = 0,
  MLS_ERR_INVALID_ARGUMENT = 1,
  MLS_ERR_TOO_FEW_POINTS = 2,
  MLS_ERR_UNSUPPORTED = 3,
  MLS_ERR_WORKSPACE_TOO_SMALL = 4,
  MLS_ERR_OUT_OF_MEMORY = 5,
  MLS_ERR_HIP = 6
} mls_status;

typedef enum { MLS_F32 = 0, MLS_F64 = 1 } mls_dtype;

typedef enum {
  MLS_PREC_FP64 = 0,        /* moments, eigen-solve and Cholesky in FP64 */
  MLS_PREC_FP32_MOMENTS = 1 /* moments in FP32 on centred, h-scaled
                               coordinates with compensated block sums;
                               eigen-solve and Cholesky in FP64 */
} mls_precision;

/* Per-point status byte: low nibble is the status, bits 4 and 5 flags. */
enum {
  MLS_PT_OK = 0,         /* projected onto the local quadratic */
  MLS_PT_OUTLIER = 1,    /* fewer than min_support neighbours within
                            support_radius_h * h (Section 3.3); out = r */
  MLS_PT_PLANE_ONLY = 2, /* quadratic fit singular (support < 6 or a
                            Cholesky pivot <= 1e-12 * max diagonal); out = q */
  MLS_PT_NONFINITE = 3,  /* query has a NaN/Inf coordinate; out = NaN */
  MLS_PT_NO_MINIMUM = 4, /* levin = 1: the descent to Levin's plane left the
                            support radius (no local minimum of Eq. (1.1)
                            within reach); out = r */
  MLS_PT_FLAG_NORMAL_AMBIGUOUS = 0x10, /* lambda2 - lambda1 < 1e-6 lambda3 */
  MLS_PT_FLAG_TRUNCATED = 0x20         /* ball neighbourhood: every one of the
                                          k list entries lies within the
                                          radius, so the ball may hold more
                                          points than were used */
};

#define MLS_MAX_K 64
#define MLS_MAX_PLANE_ITERS 16

typedef struct mls_grid mls_grid; /* opaque, host-side handle */

/* Projection parameters (host struct). */
typedef struct {
  int32_t k;                /* neighbours per query, 1 <= k <= MLS_MAX_K and
                               k <= finite points of every cloud */
  int32_t precision;        /* mls_precision */
  double support_radius_h;  /* outlier radius in units of h (default 3.0) */
  int32_t min_support;      /* outlier threshold (default 3) */
  int32_t stages;           /* mls_stage bits; 0 = MLS_STAGE_ALL */
  int32_t search_extra;     /* extra neighbours the search keeps per query
                               beyond k (k + search_extra <= MLS_MAX_K), for
                               MLS_STAGE_REFRESH in later passes; 0 = none */
  int32_t plane_iters;      /* steps of the reference plane with the weights
                               of Eq. (1.1) at the plane's own projection
                               q = r + t n of the query (Section 1.4), from
                               the plane with the weights at r (t = 0);
                               0 <= plane_iters <= MLS_MAX_PLANE_ITERS; 0 =
                               the t = 0 plane. Forward only: the adjoint
                               returns MLS_ERR_UNSUPPORTED for a nonzero
                               value. */
  int32_t ball;             /* 0: the neighbourhood is the k nearest; 1: the
                               paper's neighbourhood of radius R (Section 1.4)
                               with R = support_radius_h * h, taken as the
                               k-nearest list entries within R (canonical
                               keys): exact when fewer than k entries lie
                               within R, else the status carries
                               MLS_PT_FLAG_TRUNCATED; 2: the same
                               neighbourhood without a count cap: every cloud
                               point whose canonical key to the query is at
                               most R^2, however many (k is unused; the call
                               must run all stages and return no lists, the
                               support count is the ball's size; plane_iters
                               and levin return MLS_ERR_UNSUPPORTED). Forward
                               only, like plane_iters. */
  int32_t levin;            /* 0: the reference plane of plane_iters; 1:
                               Levin's reference plane (Section 1.4): the
                               local minimum over the unit normal n and the
                               offset t of Eq. (1.1) with the weights at the
                               plane's own projection q = r + t n, reached by
                               Newton's method from the plane with the
                               weights at r (that start plane and the descent
                               in FP64 on both precision paths); a
                               descent that leaves |t| <= support_radius_h * h
                               gives MLS_PT_NO_MINIMUM. Excludes plane_iters
                               (MLS_ERR_INVALID_ARGUMENT); forward only
                               (the adjoint returns MLS_ERR_UNSUPPORTED). */
  int32_t slot_order;       /* mls_slot_order bits; 0 = the caller's order.
                               For queries aligned with the grid's points
                               only (query_offsets NULL, n_queries ==
                               n_points; else MLS_ERR_INVALID_ARGUMENT):
                               MLS_SLOT_QUERIES reads the query of sorted
                               position p (mls_grid_sorted_points) at
                               queries[p], MLS_SLOT_OUTPUTS writes its output,
                               status and list at p. Iterated passes keep
                               their intermediate points in that order and
                               read and write memory in sequence; the last
                               pass returns the caller's order (QUERIES
                               alone). MLS_SLOT_OWN_POINTS takes the grid's
                               own points as the queries (queries may be
                               NULL; dtype still gives the outputs' type),
                               the first pass of iterated passes. With
                               exactly one of QUERIES and OUTPUTS,
                               out_points must not alias queries. Not with
                               ball = 2 nor in the adjoint
                               (MLS_ERR_UNSUPPORTED). */
} mls_params;

/* Bits of mls_params.slot_order. */
typedef enum {
  MLS_SLOT_QUERIES = 1,
  MLS_SLOT_OUTPUTS = 2,
  MLS_SLOT_OWN_POINTS = 4
} mls_slot_order;

/* Stages of mls_project. MLS_STAGE_SEARCH leaves the neighbour lists and
 * support counts in the workspace; a later call with MLS_STAGE_FIT on the
 * same grid, queries, k, query_offsets and workspace (stream-ordered after
 * it) fits and projects from them, so one search can serve several fits.
 * MLS_STAGE_REFRESH (with MLS_STAGE_SEARCH) serves iterated passes (the
 * method moves the queries iteratively, Section 1.4), where the queries move
 * a little between passes and the cloud stays: instead of
 * searching every query afresh, the lists of k + search_extra points the
 * previous search left in this workspace (same grid, k, search_extra, query
 * slots) are re-ranked by the canonical key for the new query positions. A
 * list holds every point within the distance R of the query it was searched
 * for (R = its farthest entry's distance), so when the new k-th distance is
 * below R minus the query's displacement, the k nearest are in the list (triangle
 * inequality) and the re-ranked list is the exact result; every other query
 * is searched afresh (every query when the previous search kept no extra
 * entries, search_extra = 0). The result is the same as a fresh search.
 * The library records, per workspace, which search last wrote it: a call
 * with MLS_STAGE_FIT alone or with MLS_STAGE_REFRESH returns
 * MLS_ERR_INVALID_ARGUMENT (before launching anything, reason in
 * mls_last_error()) unless that search was on the same grid with the same k,
 * search_extra, n_queries and query_offsets (and, for MLS_STAGE_FIT alone,
 * the same support_radius_h). A workspace that no search has written, or
 * whose last writer was another grid's search, an mls_knn call with another
 * k, or an adjoint on caller lists, is rejected. The caller must not modify
 * the workspace between the calls. */
typedef enum {
  MLS_STAGE_ALL = 0,
  MLS_STAGE_SEARCH = 1,
  MLS_STAGE_FIT = 2,
  MLS_STAGE_REFRESH = 4
} mls_stage;

/* Library version string (host). */
const char *mls_version(void);
/* Text of a status code (host). */
const char *mls_status_string(mls_status s);
/* Text of the last HIP error seen by this thread ("" if none) (host). */
const char *mls_last_error(void);

/* ---- grid --------------------------------------------------------------
 * The grid is the spatial index of the cloud: points sorted by
 * (cloud, Morton code of their uniform-grid cell) -- Morton order is the
 * reordering the paper suggests for chaotic clouds (Section 2 introduction)
 * -- plus an open-addressing hash from cell to its contiguous range of
 * sorted points. It replaces the paper's per-process k-d tree (Section 2.2).
 *
 * Bytes of device workspace mls_build_grid needs for n_points points in
 * n_clouds clouds (host). */
size_t mls_grid_workspace_bytes(int64_t n_points, int32_t n_clouds);

/* Build the grid of one cloud or of a batch of clouds.
 *   points          n_points x 3 FP32 (device). Copied into the workspace
 *                   (Morton-sorted snapshot): later writes to `points` do not
 *                   affect the grid. Points with a NaN/Inf coordinate are kept
 *                   out of every neighbourhood.
 *   cloud_offsets   (host) n_clouds+1 ascending offsets into points, first 0,
 *                   last n_points; NULL means one cloud.
 *   h               (host) n_clouds Gaussian widths, finite and > 0.
 *   cell_size       (host) n_clouds edges of the finest cells, or NULL;
 *                   entries <= 0 select 1.25 h. The grid also indexes cells
 *                   of 2, 4, ..., 128 times that edge (each a contiguous
 *                   Morton range of the sorted points). The edge grows when
 *                   a cloud would need more than 2^19 cells along an axis.
 *   workspace       device buffer of at least mls_grid_workspace_bytes(),
 *                   256-byte aligned; it holds the grid and must outlive it.
 *   out_grid        (host) receives the handle.
 * Errors: INVALID_ARGUMENT (null pointers, n_points < 1, n_clouds < 1,
 * offsets not ascending or not spanning the points, h not finite and > 0,
 * misaligned workspace), WORKSPACE_TOO_SMALL, OUT_OF_MEMORY (host handle),
 * HIP. */
mls_status mls_build_grid(const float *points, int64_t n_points,
                          const int64_t *cloud_offsets, int32_t n_clouds,
                          const double *h, const double *cell_size,
                          void *workspace, size_t workspace_bytes, void *stream,
                          mls_grid **out_grid);

/* Rebuilds a built grid for new positions of its points (the same count,
 * clouds, h and cell sizes), without any host synchronisation, copy or
 * memset: every step is a kernel on `stream`, so a caller can capture a
 * rebuild in a HIP graph with the calls that use the grid (a training step
 * that moves the cloud, then searches and projects it again).
 *   points   n_points x 3 FP32 (device), the new positions.
 * The rebuild keeps the first build's grid geometry (origin, cell edges,
 * cells per axis) and table size: a point that moves out of the first
 * build's box is assigned to the nearest edge cell, which keeps every search
 * exact (a cell at the grid's edge is never behind a face the search
 * certifies against). The cell table takes, on the device, the longest
 * prefix of the first build's levels whose cells fill at most half of it; a
 * level left out finds nothing, which the search treats as an empty block
 * (exact, slower). Host-side facts (mls_get_grid_info: cell and non-finite
 * counts) are those of the first build. Workspaces whose lists came from
 * this grid can no longer serve MLS_STAGE_FIT, MLS_STAGE_REFRESH or reused
 * adjoint lists. Errors: INVALID_ARGUMENT (null arguments), HIP. */
mls_status mls_rebuild_grid(mls_grid *grid, const float *points, void *stream);

/* Frees the host handle only (the workspace is the caller's). */
mls_status mls_grid_destroy(mls_grid *grid);

/* Host-visible facts about a built grid (host). */
typedef struct {
  int64_t n_points;
  int32_t n_clouds;
  int32_t key_bits;       /* bits of the (cloud, Morton) sort key */
  int64_t n_cells;        /* non-empty cells over all clouds */
  int64_t hash_capacity;  /* slots of the cell hash */
  int64_t n_nonfinite;    /* points left out of every neighbourhood */
  int64_t min_cloud_finite; /* smallest number of finite points in a cloud */
} mls_grid_info;
mls_status mls_get_grid_info(const mls_grid *grid, mls_grid_info *info);

/* Per-cloud geometry the grid chose (host): origin xyz, cell edge, dims xyz
 * for cloud c. */
mls_status mls_get_cloud_grid(const mls_grid *grid, int32_t c, double origin[3],
                              double *cell, int32_t dims[3]);

/* Sorted-order view of the grid (device pointers into the workspace, for the
 * caller's inspection): xyzw with w = original index bits, and the inverse
 * permutation (original index -> sorted position). */
mls_status mls_grid_sorted_points(const mls_grid *grid, const void **xyzw,
                                  const int32_t **inverse_perm);

/* The grid's cell table (device pointers into the workspace, for the
 * caller's inspection): `capacity` slots of 16 bytes, each {tagged key low
 * word, high word, first sorted position, end sorted position} (the cell
 * holds sorted points [first, end)), empty slots with key ~0. A tagged key is
 * the level-l cell key (the level-0 key shifted right by 3 l) with l in bits
 * 60..62; a key sits at its home slot, the top log2(capacity) bits of
 * key * 0x9e3779b97f4a7c15 (mod 2^64), or the first free slot after it
 * (linear probing, wrapping). *levels (device int32) is the number of levels
 * in the table, 0 to 8, which a rebuild decides on the device. */
mls_status mls_grid_cell_table(const mls_grid *grid, const void **table, int64_t *capacity,
                               const int32_t **levels);

/* ---- projection --------------------------------------------------------
 * Queries belong to clouds. query_offsets (host, n_clouds+1, ascending,
 * spanning n_queries) gives each cloud's contiguous query range; NULL means
 * the queries are aligned with the grid's points (n_queries == n_points,
 * query i belongs to the cloud of point i) or, for one cloud, that every
 * query belongs to it.
 *
 * Processing order: queries aligned with the points are processed in the
 * grid's Morton order; other queries are first sorted by the key of their
 * cell (cloud, Morton code), so that queries sharing cells and neighbours
 * run together. The sort is part of every fresh search (mls_knn, a search
 * without MLS_STAGE_REFRESH, the adjoint without reused lists); the stages
 * that continue from a preceding search (MLS_STAGE_FIT alone,
 * MLS_STAGE_REFRESH, the adjoint's reused lists) keep its order, which the
 * workspace holds beside the lists. Results do not depend on the order.
 *
 * Bytes of device workspace mls_project / mls_knn need for n_queries
 * queries with k neighbours kept per query (for mls_project and
 * mls_project_backward: params->k + params->search_extra) (host). */
size_t mls_project_workspace_bytes(const mls_grid *grid, int32_t k,
                                   int64_t n_queries);

/* Exact k nearest neighbours of each query (step 1 alone).
 *   out_neighbors  n_queries x k int32 ORIGINAL point indices, ascending by
 *                  (FP64 squared distance, index); -1 pads a list when the
 *                  cloud has fewer than k finite points and for non-finite
 *                  queries.
 *   out_keys       nullable, n_queries x k FP64 squared distances. */
mls_status mls_knn(const mls_grid *grid, int32_t k, const void *queries,
                   mls_dtype dtype, int64_t n_queries,
                   const int64_t *query_offsets, int32_t *out_neighbors,
                   double *out_keys, void *workspace, size_t workspace_bytes,
                   void *stream);

/* One MLS projection pass (steps 1-5) of every query.
 *   out_points     n_queries x 3 in `dtype` (may alias `queries`: each output
 *                  is written after its own query has been read and no query
 *                  reads another query).
 *   out_status     n_queries status bytes (MLS_PT_*).
 *   out_neighbors  nullable; as in mls_knn. Keep it to run the backward pass
 *                  without recomputing the lists.
 * out_points and out_status may be NULL when params->stages is
 * MLS_STAGE_SEARCH alone.
 * Iterated passes (the surface is approached by moving the queries) call this
 * again with the outputs as queries and the same grid.
 * Graph capture: with query_offsets NULL the call only launches kernels on
 * `stream` (no host copy, allocation, memset or wait), so it can be captured
 * in a HIP graph and replayed; with query_offsets it first copies them to the
 * device from host memory. */
mls_status mls_project(const mls_grid *grid, const mls_params *params,
                       const void *queries, mls_dtype dtype, int64_t n_queries,
                       const int64_t *query_offsets, void *out_points,
                       uint8_t *out_status, int32_t *out_neighbors,
                       void *workspace, size_t workspace_bytes, void *stream);

/* mls_project plus the geometry of the MLS surface at each output point.
 * Near q the surface is the graph of the fitted quadratic g over the plane H
 * (Section 1.4 and Section 2.1): x -> q + h (x u + y v + g(x/h, y/h) n).
 *   out_normals     nullable, n_queries x 3 in `dtype`: the graph's unit
 *                   normal at the output, n - a_1 u - a_2 v normalised (its
 *                   sign is that of the fitted plane's normal, which is not
 *                   oriented).
 *   out_curvatures  nullable, n_queries x 2 in `dtype`: mean curvature H
 *                   (positive where the surface bends toward the returned
 *                   normal) and Gaussian curvature K, in units of 1/length
 *                   and 1/length^2 of the query coordinates.
 * PLANE_ONLY: the plane's normal and NaN curvatures; OUTLIER and NONFINITE:
 * NaN. Written by the fit stage (MLS_STAGE_FIT); the other arguments and
 * errors are those of mls_project. */
mls_status mls_project_geometry(const mls_grid *grid, const mls_params *params,
                                const void *queries, mls_dtype dtype, int64_t n_queries,
                                const int64_t *query_offsets, void *out_points,
                                uint8_t *out_status, int32_t *out_neighbors,
                                void *out_normals, void *out_curvatures, void *workspace,
                                size_t workspace_bytes, void *stream);

/* ---- projection without allocation -------------------------------------
 * For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): one whole mls_project pass (params->stages MLS_STAGE_ALL, or
 * MLS_STAGE_SEARCH | MLS_STAGE_FIT) whose projection workspace is a fixed
 * device array inside the library, MLS_NOALLOC_SCRATCH_BYTES per GPU, which
 * each GPU the call runs on holds until the process ends. The call
 * allocates nothing; it takes the array's device address once per device
 * (on its first call there, for the current device, which must be the
 * device of `stream`). Inputs and outputs are the caller's, exactly as for
 * mls_project, with the same results; the grid is built as usual.
 *   Limit: the workspace mls_project_workspace_bytes(grid, params->k +
 *   params->search_extra, n_queries) must fit the array (about 166 bytes per
 *   query at k = 32: some 400,000 queries); larger calls return
 *   MLS_ERR_WORKSPACE_TOO_SMALL before anything is launched, with the sizes
 *   in mls_last_error().
 *   Nothing in the array needs to start at zero: every call writes what it
 *   reads. All calls on one GPU share its array, so calls on one GPU whose
 *   work can overlap (different streams or threads without ordering between
 *   them) race and give undefined results; order them on one stream.
 *   The fit-only and refresh stages and the adjoint's reused lists cannot
 *   continue from this call (MLS_ERR_INVALID_ARGUMENT for other stages).
 * Errors: those of mls_project, and MLS_ERR_UNSUPPORTED for a device number
 * of 64 or more. */
#define MLS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
mls_status mls_project_noalloc(const mls_grid *grid, const mls_params *params,
                               const void *queries, mls_dtype dtype, int64_t n_queries,
                               const int64_t *query_offsets, void *out_points,
                               uint8_t *out_status, int32_t *out_neighbors, void *stream);

/* Bytes of device workspace mls_project_backward needs: the projection's
 * workspace plus a sorted-order accumulation buffer of 3 values per cloud
 * point (FP32 for MLS_PREC_FP32_MOMENTS, FP64 for MLS_PREC_FP64) (host).
 * Returns 0 for invalid arguments. */
size_t mls_project_backward_workspace_bytes(const mls_grid *grid, int32_t k,
                                            int64_t n_queries, int32_t precision);

/* Adjoint (vector-Jacobian product) of one mls_project pass with respect to
 * the query and point positions. Not in the paper, which has no derivative:
 * it is the reverse-mode derivative of the projection of Section 1.4, Eq.
 * (1.1) and Section 2.1 (plane by weighted covariance, quadratic height fit,
 * out = q + h a_0 n) with the neighbour lists and the statuses held fixed and
 * every per-query moment recomputed with the forward's own arithmetic
 * (params->precision). The derivative of the unit normal is that of the
 * simple smallest eigenvalue; where that eigenvalue is exactly repeated the
 * normal's contribution is dropped (those queries carry
 * MLS_PT_FLAG_NORMAL_AMBIGUOUS in the forward).
 *   queries        as in mls_project (same dtype, count, offsets).
 *   params         as in mls_project; params->stages selects the lists:
 *                  MLS_STAGE_ALL (0, or SEARCH|FIT): `neighbors` if given,
 *                  else a fresh search (the lists of mls_project);
 *                  MLS_STAGE_FIT: the lists that the last search on this same
 *                  workspace left there (mls_project with the same grid,
 *                  queries, k, search_extra and offsets, nothing else run on
 *                  the workspace since; checked on the host as for
 *                  mls_project's MLS_STAGE_FIT, MLS_ERR_INVALID_ARGUMENT
 *                  otherwise); `neighbors` must then be NULL.
 *   neighbors      device, nullable: n_queries x k ORIGINAL indices as
 *                  written by mls_project / mls_knn. An entry outside
 *                  [0, n_points) makes its query an outlier.
 *   grad_out       device, n_queries x 3 in `dtype`: dL/d out.
 *   grad_queries   device, n_queries x 3 in `dtype`, overwritten with dL/d r
 *                  (OUTLIER: grad_out; NONFINITE query: 0).
 *   grad_points    device, n_points x 3 in `dtype`, overwritten with dL/d p
 *                  for every point of the grid (sum over the queries whose
 *                  list holds the point; 0 for the others), written once
 *                  from the sums in the workspace.
 *   workspace      device, at least mls_project_backward_workspace_bytes,
 *                  256-byte aligned; required even when n_queries is 0. Must
 *                  be device memory from hipMalloc: the point gradients are
 *                  summed there in sorted order with hardware float atomics
 *                  (per-workgroup partial sums in FP64, then one atomic per
 *                  component and point and workgroup).
 * The summation order of the point gradients follows the hardware order of
 * atomic additions, so they can differ between runs in the last bits; the
 * query gradients are deterministic. Errors: MLS_ERR_INVALID_ARGUMENT for
 * null or inconsistent arguments, MLS_ERR_WORKSPACE_TOO_SMALL,
 * MLS_ERR_TOO_FEW_POINTS as in mls_project, MLS_ERR_HIP for a failed launch.
 * When the queries are the cloud's own points (the usual first pass), the
 * gradient with respect to the cloud is grad_queries + grad_points. */
mls_status mls_project_backward(const mls_grid *grid, const mls_params *params,
                                const void *queries, mls_dtype dtype,
                                int64_t n_queries, const int64_t *query_offsets,
                                const int32_t *neighbors, const void *grad_out,
                                void *grad_queries, void *grad_points,
                                void *workspace, size_t workspace_bytes,
                                void *stream);

/* ---- tuning --------------------------------------------------------------
 * Not in the paper: the grid hash replaces its k-d tree (Section 2.2), and
 * the search cost of the hash depends on the finest cell edge. The tuner
 * measures it.
 *
 * Bytes of device workspace mls_autotune_cell needs (host). */
size_t mls_autotune_workspace_bytes(int64_t n_points, int32_t n_clouds,
                                    int32_t k, int32_t stride);

/* Picks the cell edge factor f (cell = f * h of each cloud) with the fastest
 * neighbour search: for each candidate builds the grid and times (HIP events,
 * second of two runs) the search stage of k neighbours for a sample of
 * 1/stride of each cloud's points as FP32 queries: runs of 256 consecutive
 * points of that grid's Morton order, one run in every 256 x stride, so that
 * the sample meets the block reuse of a search over the whole cloud. Waits
 * for the stream (host).
 *   points, n_points, cloud_offsets, n_clouds, h   as in mls_build_grid.
 *   candidates      host, n_candidates factors > 0.
 *   best_factor     host out: the fastest candidate.
 *   ms_per_candidate host out, nullable: n_candidates search times in ms.
 * Errors as in mls_build_grid and mls_project. */
mls_status mls_autotune_cell(const float *points, int64_t n_points,
                             const int64_t *cloud_offsets, int32_t n_clouds,
                             const double *h, int32_t k,
                             const double *candidates, int32_t n_candidates,
                             int32_t stride, void *workspace,
                             size_t workspace_bytes, void *stream,
                             double *best_factor, float *ms_per_candidate);

#ifdef __cplusplus
}
#endif
#endif /* MLS_H */
