// mls_internal.h -- types and small device helpers shared by the kernels of
// libmls.so (grid build, neighbour search, forward and adjoint projection).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mls.h"

namespace mls {

constexpr int kWave = 64;
constexpr uint64_t kEmptyKey = ~0ull;  // hash slot marker and non-finite point key
constexpr int kMaxLevels = 8;           // grid levels: cell edges c, 2c, ..., 128c
constexpr int kLevelShift = 60;         // hash keys carry the level in bits 60..62

// Per-cloud geometry and parameters, resident in device memory.
struct CloudDev {
  double origin[3];  // grid origin (minimum corner of the cloud's box)
  double cell;       // cell edge
  double inv_cell;   // 1 / cell
  double h;          // Gaussian width
  int32_t dims[3];   // cells per axis
  int32_t bits;      // Morton bits per axis used by the key
  int64_t begin;     // first original point index of the cloud
  int64_t end;       // one past the last
  int64_t sbegin;    // sorted positions [sbegin, send) hold the cloud's finite points
  int64_t send;
};

// Canonical squared distance: sub, mul, mul, mul, add, add, no contraction.
__device__ __forceinline__ double canon_key(double px, double py, double pz, double rx,
                                            double ry, double rz) {
#pragma clang fp contract(off)
  const double dx = px - rx;
  const double dy = py - ry;
  const double dz = pz - rz;
  const double sx = dx * dx;
  const double sy = dy * dy;
  const double sz = dz * dz;
  return (sx + sy) + sz;
}

// Workgroups are dealt to the 8 XCDs in turn (XCD = id mod 8). Renumbering
// gives each XCD one contiguous range of block numbers, so work that is
// adjacent in Morton order (and shares cells, table lines and neighbours)
// runs on the same XCD and meets in its L2. A bijection of [0, nb) for any nb.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t x = b & 7, i = b >> 3;
  const uint32_t per = nb >> 3, rem = nb & 7;
  return x * per + (x < rem ? x : rem) + i;
}

// Device-resident view of a built grid, passed to kernels by value.
struct GridView {
  const float4 *pts;         // sorted points, w = original index bits
  const int32_t *inv_perm;   // original index -> sorted position
  const uint4 *table;        // hash slots: {key lo, key hi, start, end}, all levels
  const CloudDev *clouds;    // n_clouds entries
  uint64_t hash_mask;        // capacity - 1
  int32_t n_clouds;
  int32_t morton_bits;       // bits per axis of the level-0 key (same for all clouds)
  int64_t n_points;
  int32_t n_levels;          // levels the first build put in the hash (1..kMaxLevels)
  int32_t hash_shift;        // 64 - log2(capacity)
  const int32_t *levels;     // device: levels in the hash now (a rebuild
                             // decides it on the device; 0..n_levels)
};

// Levels whose cells are in the hash (uniform; a level beyond them finds
// nothing and must not be searched).
__device__ __forceinline__ int levels_of(const GridView &g) {
  const int l = g.levels ? *g.levels : g.n_levels;
  return l < g.n_levels ? (l > 0 ? l : 0) : g.n_levels;
}

// Host-side handle contents.
struct GridHost {
  GridView view;
  int64_t n_points;
  int32_t n_clouds;
  int32_t key_bits;
  int64_t n_cells;
  int64_t hash_capacity;
  int64_t n_nonfinite;
  int64_t min_cloud_finite;
  int64_t *offsets;          // host copy, n_clouds + 1
  int64_t *offsets_dev;      // device copy, in the workspace
  int64_t *finite_counts;    // host, n_clouds
  CloudDev *clouds_host;     // host copy of the device table
  CloudDev *clouds_dev;      // in the workspace
  void *workspace;
  size_t workspace_bytes;
};

// ---- small device helpers -------------------------------------------------

__device__ __forceinline__ uint64_t spread_bits3(uint32_t v) {
  // spread the low 21 bits of v to every third bit
  uint64_t x = v & 0x1fffffull;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint64_t cell_key(int32_t cloud, int32_t ix, int32_t iy,
                                             int32_t iz, int32_t bits) {
  uint64_t m = spread_bits3((uint32_t)ix) | (spread_bits3((uint32_t)iy) << 1) |
               (spread_bits3((uint32_t)iz) << 2);
  return ((uint64_t)cloud << (3 * bits)) | m;
}

// Hash key of the level-`level` cell (ix, iy, iz) (coordinates at that
// level): the level-0 key shifted right by 3*level -- a level-l cell is a
// contiguous range of the Morton-sorted points -- tagged with the level.
__device__ __forceinline__ uint64_t level_cell_key(int32_t cloud, int32_t ix, int32_t iy,
                                                   int32_t iz, int32_t bits, int level) {
  return cell_key(cloud, ix, iy, iz, bits - level) | ((uint64_t)level << kLevelShift);
}

__device__ __forceinline__ uint64_t level_key(uint64_t key0, int level) {
  return (key0 >> (3 * level)) | ((uint64_t)level << kLevelShift);
}

// Multiplicative (Fibonacci) hash: the high bits of key * 2^64/phi select
// the slot of a table of 2^(64 - shift) slots.
__device__ __forceinline__ uint64_t hash_slot(uint64_t key, int shift) {
  return (key * 0x9e3779b97f4a7c15ull) >> shift;
}

// Returns {start, count} of the cell, count 0 if the cell is empty.
__device__ __forceinline__ int2 lookup_cell(const GridView &g, uint64_t key) {
  uint64_t slot = hash_slot(key, g.hash_shift);
  for (uint64_t probe = 0; probe <= g.hash_mask; ++probe) {
    uint4 e = g.table[slot];
    uint64_t k = (uint64_t)e.x | ((uint64_t)e.y << 32);
    if (k == key) {
      // a cell range always lies inside the sorted array
      const int64_t st = (int64_t)e.z, en = (int64_t)e.w;
      if (en < st || en > g.n_points) return make_int2(0, 0);
      return make_int2((int)st, (int)(en - st));
    }
    if (k == kEmptyKey) return make_int2(0, 0);
    slot = (slot + 1) & g.hash_mask;
  }
  return make_int2(0, 0);
}

// Cell coordinate of a coordinate along one axis (no clamping).
__device__ __forceinline__ int64_t cell_coord(double x, double origin, double inv_cell) {
  return (int64_t)floor((x - origin) * inv_cell);
}

}  // namespace mls

// ---- host launchers (defined in the .hip files) -----------------------------
namespace mls {
// Bounding boxes: blocks per cloud write partial records (32 B each) that a
// second kernel reduces; at most max(kBboxPartsMax, n_clouds) records.
constexpr int kBboxPartsMax = 8192;
int bbox_parts(int64_t max_cloud, int32_t n_clouds);
hipError_t launch_bbox(const float *pts, const int64_t *offsets_dev, int32_t n_clouds,
                       int64_t max_cloud, uint4 *partial, uint32_t *bbox_bits,
                       unsigned long long *nonfinite, hipStream_t s);
hipError_t launch_keys(const float *pts, const CloudDev *clouds, int32_t n_clouds,
                       int64_t max_cloud, int32_t bits, uint64_t *keys, int32_t *vals,
                       hipStream_t s);
hipError_t launch_query_keys(const void *q, bool is_f64, int64_t n, const int32_t *qcloud,
                             const CloudDev *clouds, int32_t bits, uint64_t *keys, int32_t *vals,
                             hipStream_t s);
size_t radix_temp_bytes(int64_t n);
hipError_t radix_sort_pairs(uint64_t *keys, int32_t *vals, uint64_t *keys_alt, int32_t *vals_alt,
                            int64_t n, int32_t key_bits, void *temp, bool *result_in_alt,
                            hipStream_t s);
hipError_t launch_gather(const float *pts, const int32_t *vals, int64_t n, float4 *sorted,
                         int32_t *inv_perm, hipStream_t s);
hipError_t launch_count_cells(const uint64_t *keys, int64_t n, unsigned long long *counts,
                              hipStream_t s);
// Fills the table and inserts the cells of its first *levels_dev levels.
hipError_t launch_build_table(const uint64_t *keys, int64_t n, const int32_t *levels_dev,
                              uint4 *table, uint64_t capacity, hipStream_t s);
// Rebuild helpers (kernels only, no host round trip): clear n counters;
// recompute the clouds' sorted ranges from their non-finite counts; build the
// table with the levels whose cells fit half of the capacity (decided on the
// device from the per-level counts).
hipError_t launch_clear_u64(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_set_i32(int32_t *p, int32_t v, hipStream_t s);
hipError_t launch_cloud_ranges(CloudDev *clouds, int32_t n_clouds,
                               const unsigned long long *nonfinite, hipStream_t s);
hipError_t launch_table_dev_levels(const uint64_t *keys, int64_t n, int n_levels,
                                   const unsigned long long *counts, int32_t *levels_dev,
                                   uint4 *table, uint64_t capacity, hipStream_t s);

struct QueryView {
  const void *q;            // queries, n x 3
  int32_t is_f64;
  int64_t n;
  const int32_t *order;     // processing order -> query index, or null (identity)
  const int32_t *qcloud;    // per query cloud id, or null (cloud 0)
  int32_t aligned;          // queries aligned with points: order from the grid
  int32_t kstride;          // entries per query in the tile lists (k + search extra)
  int32_t slot_in;          // aligned queries given in the grid's sorted order (q[p])
  int32_t slot_out;         // results written in the grid's sorted order (out[p])
  int32_t in_f64;           // query coordinates are doubles (else floats)
  int32_t in_stride;        // elements from one query to the next: 3, or 4 when
                            // the queries are the grid's own sorted points
};

// Index of slot p's query in the query array and of its results in the
// result arrays (qi: the query's own index, the original point index for
// aligned queries).
__device__ __forceinline__ int64_t in_index(const QueryView &qv, int64_t p, int64_t qi) {
  return qv.slot_in ? p : qi;
}
__device__ __forceinline__ int64_t out_index(const QueryView &qv, int64_t p, int64_t qi) {
  return qv.slot_out ? p : qi;
}

// The query of slot p (qi: its own index).
__device__ __forceinline__ void load_slot_query(const GridView &g, const QueryView &qv,
                                                int64_t p, int64_t qi, double r[3]) {
  const int64_t i = in_index(qv, p, qi) * qv.in_stride;
  if (qv.in_f64) {
    const double *q = (const double *)qv.q + i;
    r[0] = q[0]; r[1] = q[1]; r[2] = q[2];
  } else {
    const float *q = (const float *)qv.q + i;
    r[0] = q[0]; r[1] = q[1]; r[2] = q[2];
  }
}

// Query index of slot p < qv.n for queries that are not the grid's points:
// the permutation of the search's sort (clamped, like list entries, so that
// a corrupted workspace cannot address outside the queries), or p.
__device__ __forceinline__ int64_t ordered_query(const QueryView &qv, int64_t p) {
  if (!qv.order) return p;
  const uint32_t v = (uint32_t)qv.order[p];
  return (int64_t)v < qv.n ? (int64_t)v : 0;
}

// Exact search of the k = qv.kstride nearest of every query into the tile
// lists (the first kfit of each list are the kfit nearest), with the slot's
// anchor and bound (4 doubles per slot) for later refreshes. With refresh,
// the lists of the previous search are re-ranked for the new queries first
// and only the slots they cannot certify (flag, 1 byte per slot) are searched.
hipError_t launch_knn(const GridView &g, const QueryView &qv, int32_t k, int32_t kfit,
                      double support_r_h, bool refresh, int32_t *nbr_tiles, uint8_t *support,
                      double *anchor, uint8_t *flag, int32_t *out_nbr, double *out_keys,
                      hipStream_t s);
hipError_t launch_mls_forward(const GridView &g, const QueryView &qv, int32_t k,
                              int32_t precision, int32_t min_support, int32_t plane_iters,
                              int32_t ball, int32_t levin, double support_radius_h,
                              const int32_t *nbr_tiles,
                              const uint8_t *support, void *out, uint8_t *status,
                              void *out_normals, void *out_curvatures, hipStream_t s);
// The projection over the radius-R ball without a count cap (one wave per
// query; no lists).
hipError_t launch_ball(const GridView &g, const QueryView &qv, int32_t precision,
                       int32_t min_support, double support_radius_h, void *out, uint8_t *status,
                       void *out_normals, void *out_curvatures, hipStream_t s);
hipError_t launch_lists_from_caller(const GridView &g, const QueryView &qv, int32_t k,
                                    const int32_t *user, int32_t *nbr_tiles, hipStream_t s);
hipError_t launch_mls_backward(const GridView &g, const QueryView &qv, int32_t k,
                               int32_t precision, double support_radius_h, int32_t min_support,
                               const int32_t *nbr_tiles, const void *grad_out, void *grad_q,
                               void *gp_sorted, void *grad_points, hipStream_t s);
// Bytes of the mls_project workspace (host).
size_t proj_workspace_bytes(int32_t n_clouds, int32_t k, int64_t n);
hipError_t launch_fill_cloud_ids(const int64_t *offsets_dev, int32_t n_clouds, int64_t n,
                                 int32_t *qcloud, hipStream_t s);
}  // namespace mls
