// abi.hip -- extern "C" entry points of libmls.so: argument validation on the
// host, workspace carving, and the launch sequence of each call.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "grid_access.h"
#include "mls_internal.h"

namespace {

thread_local char g_last_error[256] = "";

mls_status hip_fail(hipError_t e, const char *where) {
  snprintf(g_last_error, sizeof g_last_error, "%s: %s", where, hipGetErrorString(e));
  return MLS_ERR_HIP;
}

#define MLS_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #call);   \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Byte layout of the grid workspace.
struct GridLayout {
  size_t pts, inv_perm, keys_a, keys_b, vals_a, vals_b, radix, table, clouds, offsets, bbox,
      bbox_part, nonfinite, counter, levels, total;
  uint64_t table_cap_max;
};

GridLayout grid_layout(int64_t n, int32_t c) {
  GridLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
  L.pts = take(16 * (size_t)n);
  L.inv_perm = take(4 * (size_t)n);
  L.keys_a = take(8 * (size_t)n);
  L.keys_b = take(8 * (size_t)n);
  L.vals_a = take(4 * (size_t)n);
  L.vals_b = take(4 * (size_t)n);
  L.radix = take(mls::radix_temp_bytes(n));
  L.table_cap_max = next_pow2(std::max<uint64_t>(4 * (uint64_t)n, 64));
  L.table = take(16 * L.table_cap_max);
  L.clouds = take(sizeof(mls::CloudDev) * (size_t)c);
  L.offsets = take(8 * ((size_t)c + 1));
  L.bbox = take(24 * (size_t)c);
  L.bbox_part = take(32 * (size_t)std::max<int64_t>(mls::kBboxPartsMax, c));
  L.nonfinite = take(8 * (size_t)c);
  L.counter = take(64);
  L.levels = take(64);  // levels in the table after a rebuild (device)
  L.total = o;
  return L;
}

// Byte layout of the projection workspace.
struct ProjLayout {
  size_t nbr, support, qcloud, offsets, anchor, flag, order, total;
  // the sort of queries that are not the grid's points, inside `anchor`
  // (which the search writes only after the sort): two key buffers, one
  // value buffer (the other one is `order`) and the radix sort's scratch
  size_t skeys_a, skeys_b, svals, sradix;
};

// k_list: entries kept per query (k plus the search's extra neighbours).
ProjLayout proj_layout(int32_t n_clouds, int32_t k_list, int64_t n) {
  ProjLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
  // neighbour lists in tiles of 64 queries (the last tile padded)
  L.nbr = take(4 * (size_t)((n + 63) / 64) * 64 * (size_t)k_list);
  L.support = take((size_t)n);
  L.qcloud = take(n_clouds > 1 ? 4 * (size_t)n : 0);
  L.offsets = take(8 * ((size_t)n_clouds + 1));
  const size_t sort_bytes = 2 * align256(8 * (size_t)n) + align256(4 * (size_t)n) +
                            align256(mls::radix_temp_bytes(n));
  // per slot: the searched query and its bound
  L.anchor = take(std::max(32 * (size_t)n, sort_bytes));
  L.skeys_a = L.anchor;
  L.skeys_b = L.skeys_a + align256(8 * (size_t)n);
  L.svals = L.skeys_b + align256(8 * (size_t)n);
  L.sradix = L.svals + align256(4 * (size_t)n);
  L.flag = take((size_t)n);         // per slot: left to a fresh search
  L.order = take(4 * (size_t)n);    // per slot: the query it serves
  L.total = o;
  return L;
}

// The adjoint's workspace: the projection layout, then the sorted-order
// accumulation buffer of the point gradients (3 per point, in the type of the
// per-neighbour arithmetic).
size_t bwd_gp_offset(int32_t n_clouds, int32_t k, int64_t n) {
  return proj_layout(n_clouds, k, n).total;
}

size_t bwd_total(int32_t n_clouds, int32_t k, int64_t n, int64_t n_points, int32_t precision) {
  const size_t elem = precision == MLS_PREC_FP32_MOMENTS ? 4 : 8;
  return bwd_gp_offset(n_clouds, k, n) + align256(3 * elem * (size_t)n_points);
}

}  // namespace

namespace mls {
size_t proj_workspace_bytes(int32_t n_clouds, int32_t k, int64_t n) {
  return proj_layout(n_clouds, k, n).total;
}
}  // namespace mls

namespace {

bool offsets_ok(const int64_t *off, int32_t c, int64_t n) {
  if (off[0] != 0 || off[c] != n) return false;
  for (int32_t i = 0; i < c; ++i)
    if (off[i + 1] < off[i]) return false;
  return true;
}

float ordered_to_float(uint32_t o) {
  uint32_t b = (o & 0x80000000u) ? (o ^ 0x80000000u) : ~o;
  float f;
  memcpy(&f, &b, 4);
  return f;
}

mls_status check_async() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "earlier asynchronous error");
  return MLS_OK;
}

// ---- which search last wrote a projection workspace (host) ----------------
// The stages that continue from a preceding search (fit only, refresh, the
// adjoint's reused lists) read the lists, support counts and anchors that
// search left in the workspace. A record per workspace range (the calling
// grid, k, kept entries, query count, a digest of the query offsets and the
// support radius) lets them check, on the host and before any launch, that
// the workspace holds what they are about to read.
struct SearchRecord {
  uintptr_t lo, hi;         // workspace byte range written by the search
  const mls_grid *grid;
  int32_t k, k_list;
  int64_t n;
  uint64_t digest;          // query offsets (or their absence)
  double support_r_h;
};

std::mutex g_rec_mu;
constexpr int kMaxRecords = 64;
SearchRecord g_rec[kMaxRecords];
int g_rec_n = 0;

uint64_t offsets_digest(const int64_t *off, int32_t c, int64_t n) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the words below
  auto mix = [&](uint64_t v) {
    for (int b = 0; b < 8; ++b) {
      h ^= (v >> (8 * b)) & 0xff;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)n);
  mix(off ? 1u : 0u);
  if (off)
    for (int32_t i = 0; i <= c; ++i) mix((uint64_t)off[i]);
  return h;
}

// Drops every record whose range meets [lo, hi) (the caller holds the lock).
void drop_overlapping(uintptr_t lo, uintptr_t hi) {
  int w = 0;
  for (int i = 0; i < g_rec_n; ++i)
    if (g_rec[i].hi <= lo || g_rec[i].lo >= hi) g_rec[w++] = g_rec[i];
  g_rec_n = w;
}

void forget_workspace(const void *ws, size_t bytes) {
  std::lock_guard<std::mutex> lk(g_rec_mu);
  drop_overlapping((uintptr_t)ws, (uintptr_t)ws + std::max<size_t>(bytes, 1));
}

void record_search(const void *ws, size_t bytes, const mls_grid *grid, int32_t k, int32_t k_list,
                   int64_t n, uint64_t digest, double support_r_h) {
  std::lock_guard<std::mutex> lk(g_rec_mu);
  const uintptr_t lo = (uintptr_t)ws, hi = lo + std::max<size_t>(bytes, 1);
  drop_overlapping(lo, hi);
  if (g_rec_n == kMaxRecords) {  // drop the oldest
    for (int i = 1; i < g_rec_n; ++i) g_rec[i - 1] = g_rec[i];
    --g_rec_n;
  }
  g_rec[g_rec_n++] = SearchRecord{lo, hi, grid, k, k_list, n, digest, support_r_h};
}

void forget_grid(const mls_grid *grid) {
  std::lock_guard<std::mutex> lk(g_rec_mu);
  int w = 0;
  for (int i = 0; i < g_rec_n; ++i)
    if (g_rec[i].grid != grid) g_rec[w++] = g_rec[i];
  g_rec_n = w;
}

// MLS_OK when the last search that wrote `ws` was on `grid` with the same k,
// kept entries, query count and offsets (and support radius when asked);
// otherwise MLS_ERR_INVALID_ARGUMENT with the reason in mls_last_error().
mls_status require_search(const void *ws, const mls_grid *grid, int32_t k, int32_t k_list,
                          int64_t n, uint64_t digest, const double *support_r_h,
                          const char *stage) {
  std::lock_guard<std::mutex> lk(g_rec_mu);
  const SearchRecord *r = nullptr;
  for (int i = 0; i < g_rec_n; ++i)
    if (g_rec[i].lo == (uintptr_t)ws) r = &g_rec[i];
  const char *why = nullptr;
  if (!r) why = "no search on this grid has written this workspace";
  else if (r->grid != grid) why = "the workspace holds another grid's lists";
  else if (r->k != k) why = "the search used another k";
  else if (r->k_list != k_list) why = "the search kept another number of extra neighbours";
  else if (r->n != n || r->digest != digest) why = "the search had other query counts or offsets";
  else if (support_r_h && r->support_r_h != *support_r_h)
    why = "the search counted the support with another radius";
  if (!why) return MLS_OK;
  snprintf(g_last_error, sizeof g_last_error, "%s: %s", stage, why);
  return MLS_ERR_INVALID_ARGUMENT;
}

// ---- the fixed scratch of mls_project_noalloc ------------------------------
// The projection workspace of callers that cannot allocate: a device array of
// fixed size in this library's code object. Every GPU holds its own copy, at
// its own address, from the first use until the process ends. In host code
// the array's name is not a device address: host code uses only the address
// hipGetSymbolAddress returns on each device (taken once per device, with
// that device current).
constexpr size_t kScratchBytes = MLS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices];

mls_status scratch_of_current_device(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxScratchDevices) {
    snprintf(g_last_error, sizeof g_last_error, "mls_project_noalloc: device %d not supported",
             dev);
    return MLS_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || ((uintptr_t)p & 255) != 0) {
      snprintf(g_last_error, sizeof g_last_error, "mls_project_noalloc: bad scratch address");
      return MLS_ERR_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MLS_OK;
}

}  // namespace

struct mls_grid {
  mls::GridHost g;
};

namespace mls {
const GridHost &grid_host(const mls_grid *grid) { return grid->g; }
}  // namespace mls

extern "C" {

const char *mls_version(void) { return "mls-mi355x 0.1 (gfx950)"; }

const char *mls_status_string(mls_status s) {
  switch (s) {
    case MLS_OK: return "ok";
    case MLS_ERR_INVALID_ARGUMENT: return "invalid argument";
    case MLS_ERR_TOO_FEW_POINTS: return "a cloud has fewer finite points than k";
    case MLS_ERR_UNSUPPORTED: return "unsupported";
    case MLS_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case MLS_ERR_OUT_OF_MEMORY: return "out of host memory";
    case MLS_ERR_HIP: return "HIP error";
  }
  return "unknown status";
}

const char *mls_last_error(void) { return g_last_error; }

size_t mls_grid_workspace_bytes(int64_t n_points, int32_t n_clouds) {
  if (n_points < 1 || n_clouds < 1) return 0;
  return grid_layout(n_points, n_clouds).total;
}

mls_status mls_build_grid(const float *points, int64_t n_points, const int64_t *cloud_offsets,
                          int32_t n_clouds, const double *h, const double *cell_size,
                          void *workspace, size_t workspace_bytes, void *stream,
                          mls_grid **out_grid) {
  g_last_error[0] = 0;
  if (!out_grid) return MLS_ERR_INVALID_ARGUMENT;
  *out_grid = nullptr;
  if (!points || !h || !workspace || n_points < 1 || n_clouds < 1 ||
      n_points > 0x7fffffffll || n_clouds > 65535)
    return MLS_ERR_INVALID_ARGUMENT;
  if (((uintptr_t)workspace & 255) != 0) return MLS_ERR_INVALID_ARGUMENT;
  if (cloud_offsets ? !offsets_ok(cloud_offsets, n_clouds, n_points) : n_clouds != 1)
    return MLS_ERR_INVALID_ARGUMENT;
  for (int32_t c = 0; c < n_clouds; ++c) {
    if (!(h[c] > 0.0) || !isfinite(h[c])) return MLS_ERR_INVALID_ARGUMENT;
    if (cell_size && !isfinite(cell_size[c])) return MLS_ERR_INVALID_ARGUMENT;
  }
  const GridLayout L = grid_layout(n_points, n_clouds);
  if (workspace_bytes < L.total) return MLS_ERR_WORKSPACE_TOO_SMALL;
  mls_status st = check_async();
  if (st != MLS_OK) return st;

  mls_grid *G = new (std::nothrow) mls_grid();
  if (!G) return MLS_ERR_OUT_OF_MEMORY;
  mls::GridHost &gh = G->g;
  gh.offsets = (int64_t *)malloc(8 * ((size_t)n_clouds + 1));
  gh.finite_counts = (int64_t *)malloc(8 * (size_t)n_clouds);
  gh.clouds_host = (mls::CloudDev *)calloc((size_t)n_clouds, sizeof(mls::CloudDev));
  uint32_t *bbox_h = (uint32_t *)malloc(24 * (size_t)n_clouds);
  unsigned long long *nonfin_h = (unsigned long long *)malloc(8 * (size_t)n_clouds);
  auto cleanup = [&](mls_status s) {
    free(bbox_h);
    free(nonfin_h);
    if (s != MLS_OK) {
      free(gh.offsets);
      free(gh.finite_counts);
      free(gh.clouds_host);
      delete G;
    }
    return s;
  };
  if (!gh.offsets || !gh.finite_counts || !gh.clouds_host || !bbox_h || !nonfin_h)
    return cleanup(MLS_ERR_OUT_OF_MEMORY);
  if (cloud_offsets) memcpy(gh.offsets, cloud_offsets, 8 * ((size_t)n_clouds + 1));
  else { gh.offsets[0] = 0; gh.offsets[1] = n_points; }

  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  float4 *pts = (float4 *)(ws + L.pts);
  int32_t *inv_perm = (int32_t *)(ws + L.inv_perm);
  uint64_t *keys_a = (uint64_t *)(ws + L.keys_a), *keys_b = (uint64_t *)(ws + L.keys_b);
  int32_t *vals_a = (int32_t *)(ws + L.vals_a), *vals_b = (int32_t *)(ws + L.vals_b);
  uint4 *table = (uint4 *)(ws + L.table);
  mls::CloudDev *clouds = (mls::CloudDev *)(ws + L.clouds);
  int64_t *offsets_dev = (int64_t *)(ws + L.offsets);
  uint32_t *bbox = (uint32_t *)(ws + L.bbox);
  unsigned long long *nonfin = (unsigned long long *)(ws + L.nonfinite);
  unsigned long long *counter = (unsigned long long *)(ws + L.counter);

  int64_t max_cloud = 0;
  for (int32_t c = 0; c < n_clouds; ++c)
    max_cloud = std::max(max_cloud, gh.offsets[c + 1] - gh.offsets[c]);

  hipError_t e;
#define STEP(call)                                         \
  do {                                                     \
    e = (call);                                            \
    if (e != hipSuccess) return cleanup(hip_fail(e, #call)); \
  } while (0)
  STEP(hipMemcpyAsync(offsets_dev, gh.offsets, 8 * ((size_t)n_clouds + 1),
                      hipMemcpyHostToDevice, s));
  STEP(mls::launch_bbox(points, offsets_dev, n_clouds, max_cloud, (uint4 *)(ws + L.bbox_part),
                        bbox, nonfin, s));
  STEP(hipMemcpyAsync(bbox_h, bbox, 24 * (size_t)n_clouds, hipMemcpyDeviceToHost, s));
  STEP(hipMemcpyAsync(nonfin_h, nonfin, 8 * (size_t)n_clouds, hipMemcpyDeviceToHost, s));
  STEP(hipStreamSynchronize(s));

  // per-cloud geometry: origin at the box minimum, dims covering the box
  int cloud_bits = 0;
  while ((1ll << cloud_bits) < n_clouds) ++cloud_bits;
  // the level tag of the cell hash sits in bits 60..62 of the key
  const int max_bits = std::min(19, (59 - cloud_bits) / 3);
  int bits = 1;
  int64_t sorted_at = 0, nonfinite_total = 0, min_finite = INT64_MAX;
  for (int32_t c = 0; c < n_clouds; ++c) {
    mls::CloudDev &cd = gh.clouds_host[c];
    const int64_t cnt = gh.offsets[c + 1] - gh.offsets[c];
    const int64_t fin = cnt - (int64_t)nonfin_h[c];
    gh.finite_counts[c] = fin;
    nonfinite_total += (int64_t)nonfin_h[c];
    min_finite = std::min(min_finite, fin);
    cd.begin = gh.offsets[c];
    cd.end = gh.offsets[c + 1];
    cd.sbegin = sorted_at;
    cd.send = sorted_at + fin;
    sorted_at += fin;
    cd.h = h[c];
    double lo[3] = {0, 0, 0}, ext[3] = {0, 0, 0};
    if (fin > 0)
      for (int a = 0; a < 3; ++a) {
        lo[a] = (double)ordered_to_float(bbox_h[6 * c + a]);
        ext[a] = (double)ordered_to_float(bbox_h[6 * c + 3 + a]) - lo[a];
      }
    double cell = (cell_size && cell_size[c] > 0.0) ? cell_size[c] : 1.25 * h[c];
    const double max_ext = std::max(ext[0], std::max(ext[1], ext[2]));
    const double limit = (double)((1ll << max_bits) - 1);
    if (max_ext / cell >= limit) cell = max_ext / (limit - 1.0);
    cd.cell = cell;
    cd.inv_cell = 1.0 / cell;
    for (int a = 0; a < 3; ++a) {
      cd.origin[a] = lo[a];
      int64_t d = (int64_t)floor(ext[a] * cd.inv_cell) + 1;
      if (d < 1) d = 1;
      if (d > (1ll << max_bits)) d = 1ll << max_bits;
      cd.dims[a] = (int32_t)d;
      while ((1ll << bits) < d) ++bits;
    }
  }
  for (int32_t c = 0; c < n_clouds; ++c) gh.clouds_host[c].bits = bits;
  const int key_bits = 3 * bits + cloud_bits + 1;  // top bit separates non-finite keys

  STEP(hipMemcpyAsync(clouds, gh.clouds_host, sizeof(mls::CloudDev) * (size_t)n_clouds,
                      hipMemcpyHostToDevice, s));
  STEP(mls::launch_keys(points, clouds, n_clouds, max_cloud, bits, keys_a, vals_a, s));
  bool in_alt = false;
  STEP(mls::radix_sort_pairs(keys_a, vals_a, keys_b, vals_b, n_points, key_bits, ws + L.radix,
                             &in_alt, s));
  const uint64_t *skeys = in_alt ? keys_b : keys_a;
  const int32_t *svals = in_alt ? vals_b : vals_a;
  STEP(mls::launch_gather(points, svals, n_points, pts, inv_perm, s));
  STEP(hipMemsetAsync(counter, 0, 8 * mls::kMaxLevels, s));
  STEP(mls::launch_count_cells(skeys, n_points, counter, s));
  unsigned long long level_cells[mls::kMaxLevels] = {};
  STEP(hipMemcpyAsync(level_cells, counter, 8 * mls::kMaxLevels, hipMemcpyDeviceToHost, s));
  STEP(hipStreamSynchronize(s));
  // every level shares one hash, at a load factor of at most 1/8 where the
  // reserved table allows (the search's lookups then probe about one slot)
  // and never above 1/2 (coarse levels are dropped before that). The
  // reservation, next_pow2(4 n) slots, holds twice the level-0 cells (at
  // most n), so one level always fits; the check keeps every table write
  // inside the reservation regardless.
  int n_levels = mls::kMaxLevels;
  while (bits - (n_levels - 1) < 1) --n_levels;
  uint64_t cap = 0;
  for (;; --n_levels) {
    uint64_t total = 0;
    for (int l = 0; l < n_levels; ++l) total += level_cells[l];
    const uint64_t need = next_pow2(std::max<uint64_t>(2 * total, 64));
    if (need <= L.table_cap_max) {
      cap = std::min<uint64_t>(next_pow2(std::max<uint64_t>(8 * total, 64)), L.table_cap_max);
      break;
    }
    if (n_levels == 1) {
      snprintf(g_last_error, sizeof g_last_error, "cell table exceeds its reservation");
      return cleanup(MLS_ERR_WORKSPACE_TOO_SMALL);
    }
  }
  const unsigned long long ncells = level_cells[0];
  int32_t *levels_dev = (int32_t *)(ws + L.levels);
  STEP(mls::launch_set_i32(levels_dev, n_levels, s));
  STEP(mls::launch_build_table(skeys, n_points, levels_dev, table, cap, s));
#undef STEP

  gh.view.pts = pts;
  gh.view.inv_perm = inv_perm;
  gh.view.table = table;
  gh.view.clouds = clouds;
  gh.view.hash_mask = cap - 1;
  gh.view.n_clouds = n_clouds;
  gh.view.morton_bits = bits;
  gh.view.n_points = n_points;
  gh.view.n_levels = n_levels;
  gh.view.levels = levels_dev;
  {
    int shift = 64;
    for (uint64_t c = cap; c > 1; c >>= 1) --shift;
    gh.view.hash_shift = shift;
  }
  gh.n_points = n_points;
  gh.n_clouds = n_clouds;
  gh.key_bits = key_bits;
  gh.n_cells = (int64_t)ncells;
  gh.hash_capacity = (int64_t)cap;
  gh.n_nonfinite = nonfinite_total;
  gh.min_cloud_finite = min_finite;
  gh.clouds_dev = clouds;
  gh.offsets_dev = offsets_dev;
  gh.workspace = workspace;
  gh.workspace_bytes = workspace_bytes;
  *out_grid = G;
  return cleanup(MLS_OK);
}

mls_status mls_rebuild_grid(mls_grid *grid, const float *points, void *stream) {
  g_last_error[0] = 0;
  if (!grid || !points) return MLS_ERR_INVALID_ARGUMENT;
  mls_status st = check_async();
  if (st != MLS_OK) return st;
  mls::GridHost &gh = grid->g;
  const int64_t n = gh.n_points;
  const int32_t C = gh.n_clouds;
  const GridLayout L = grid_layout(n, C);
  char *ws = (char *)gh.workspace;
  float4 *pts = (float4 *)(ws + L.pts);
  int32_t *inv_perm = (int32_t *)(ws + L.inv_perm);
  uint64_t *keys_a = (uint64_t *)(ws + L.keys_a), *keys_b = (uint64_t *)(ws + L.keys_b);
  int32_t *vals_a = (int32_t *)(ws + L.vals_a), *vals_b = (int32_t *)(ws + L.vals_b);
  uint4 *table = (uint4 *)(ws + L.table);
  mls::CloudDev *clouds = (mls::CloudDev *)(ws + L.clouds);
  const int64_t *offsets_dev = (const int64_t *)(ws + L.offsets);
  uint32_t *bbox = (uint32_t *)(ws + L.bbox);
  unsigned long long *nonfin = (unsigned long long *)(ws + L.nonfinite);
  unsigned long long *counter = (unsigned long long *)(ws + L.counter);
  int32_t *levels = (int32_t *)(ws + L.levels);
  int64_t max_cloud = 0;
  for (int32_t c = 0; c < C; ++c) max_cloud = std::max(max_cloud, gh.offsets[c + 1] - gh.offsets[c]);
  hipStream_t s = (hipStream_t)stream;
  // lists that searches on this grid left in workspaces hold the old sorted
  // positions: no later stage may continue from them
  forget_grid(grid);
  MLS_HIP(mls::launch_bbox(points, offsets_dev, C, max_cloud, (uint4 *)(ws + L.bbox_part), bbox,
                           nonfin, s));
  MLS_HIP(mls::launch_cloud_ranges(clouds, C, nonfin, s));
  MLS_HIP(mls::launch_keys(points, clouds, C, max_cloud, gh.view.morton_bits, keys_a, vals_a, s));
  bool in_alt = false;
  MLS_HIP(mls::radix_sort_pairs(keys_a, vals_a, keys_b, vals_b, n, gh.key_bits, ws + L.radix,
                                &in_alt, s));
  const uint64_t *skeys = in_alt ? keys_b : keys_a;
  const int32_t *svals = in_alt ? vals_b : vals_a;
  MLS_HIP(mls::launch_gather(points, svals, n, pts, inv_perm, s));
  MLS_HIP(mls::launch_clear_u64(counter, mls::kMaxLevels, s));
  MLS_HIP(mls::launch_count_cells(skeys, n, counter, s));
  MLS_HIP(mls::launch_table_dev_levels(skeys, n, gh.view.n_levels, counter, levels, table,
                                       (uint64_t)gh.hash_capacity, s));
  return MLS_OK;
}

mls_status mls_grid_destroy(mls_grid *grid) {
  if (!grid) return MLS_ERR_INVALID_ARGUMENT;
  forget_grid(grid);
  free(grid->g.offsets);
  free(grid->g.finite_counts);
  free(grid->g.clouds_host);
  delete grid;
  return MLS_OK;
}

mls_status mls_get_grid_info(const mls_grid *grid, mls_grid_info *info) {
  if (!grid || !info) return MLS_ERR_INVALID_ARGUMENT;
  const mls::GridHost &g = grid->g;
  info->n_points = g.n_points;
  info->n_clouds = g.n_clouds;
  info->key_bits = g.key_bits;
  info->n_cells = g.n_cells;
  info->hash_capacity = g.hash_capacity;
  info->n_nonfinite = g.n_nonfinite;
  info->min_cloud_finite = g.min_cloud_finite;
  return MLS_OK;
}

mls_status mls_get_cloud_grid(const mls_grid *grid, int32_t c, double origin[3], double *cell,
                              int32_t dims[3]) {
  if (!grid || !origin || !cell || !dims || c < 0 || c >= grid->g.n_clouds)
    return MLS_ERR_INVALID_ARGUMENT;
  const mls::CloudDev &cd = grid->g.clouds_host[c];
  for (int a = 0; a < 3; ++a) {
    origin[a] = cd.origin[a];
    dims[a] = cd.dims[a];
  }
  *cell = cd.cell;
  return MLS_OK;
}

mls_status mls_grid_sorted_points(const mls_grid *grid, const void **xyzw,
                                  const int32_t **inverse_perm) {
  if (!grid || !xyzw || !inverse_perm) return MLS_ERR_INVALID_ARGUMENT;
  *xyzw = grid->g.view.pts;
  *inverse_perm = grid->g.view.inv_perm;
  return MLS_OK;
}

mls_status mls_grid_cell_table(const mls_grid *grid, const void **table, int64_t *capacity,
                               const int32_t **levels) {
  if (!grid || !table || !capacity || !levels) return MLS_ERR_INVALID_ARGUMENT;
  *table = grid->g.view.table;
  *capacity = grid->g.hash_capacity;
  *levels = grid->g.view.levels;
  return MLS_OK;
}

size_t mls_project_workspace_bytes(const mls_grid *grid, int32_t k, int64_t n_queries) {
  if (!grid || k < 1 || k > MLS_MAX_K || n_queries < 0) return 0;
  return proj_layout(grid->g.n_clouds, k, n_queries).total;
}

size_t mls_project_backward_workspace_bytes(const mls_grid *grid, int32_t k, int64_t n_queries,
                                            int32_t precision) {
  if (!grid || k < 1 || k > MLS_MAX_K || n_queries < 0) return 0;
  if (precision != MLS_PREC_FP64 && precision != MLS_PREC_FP32_MOMENTS) return 0;
  return bwd_total(grid->g.n_clouds, k, n_queries, grid->g.n_points, precision);
}

}  // extern "C"

namespace {

// Shared validation and set-up of mls_knn / mls_project / mls_project_backward.
mls_status prepare_queries(const mls_grid *grid, int32_t k, int32_t k_list, const void *queries,
                           mls_dtype dtype, int64_t n, const int64_t *query_offsets,
                           void *workspace, size_t workspace_bytes, bool sort, hipStream_t s,
                           mls::QueryView *qv, ProjLayout *L) {
  if (!grid || k < 1 || k > MLS_MAX_K || k_list < k || k_list > MLS_MAX_K || n < 0 ||
      n > 0x7fffffffll)
    return MLS_ERR_INVALID_ARGUMENT;
  if (dtype != MLS_F32 && dtype != MLS_F64) return MLS_ERR_INVALID_ARGUMENT;
  if (n > 0 && (!queries || !workspace)) return MLS_ERR_INVALID_ARGUMENT;
  const mls::GridHost &g = grid->g;
  if (k > g.min_cloud_finite) return MLS_ERR_TOO_FEW_POINTS;
  const int32_t C = g.n_clouds;
  const bool aligned = !query_offsets && n == g.n_points;
  if (query_offsets) {
    if (!offsets_ok(query_offsets, C, n)) return MLS_ERR_INVALID_ARGUMENT;
  } else if (C > 1 && !aligned) {
    return MLS_ERR_INVALID_ARGUMENT;
  }
  *L = proj_layout(C, k_list, n);
  if (n > 0 && ((uintptr_t)workspace & 255) != 0) return MLS_ERR_INVALID_ARGUMENT;
  if (n > 0 && workspace_bytes < L->total) return MLS_ERR_WORKSPACE_TOO_SMALL;
  mls_status st = check_async();
  if (st != MLS_OK) return st;
  char *ws = (char *)workspace;
  qv->q = queries;
  qv->is_f64 = dtype == MLS_F64;
  qv->n = n;
  qv->order = nullptr;
  qv->aligned = aligned ? 1 : 0;
  qv->qcloud = nullptr;
  qv->kstride = k_list;
  qv->slot_in = 0;
  qv->slot_out = 0;
  qv->in_f64 = qv->is_f64;
  qv->in_stride = 3;
  if (C > 1 && n > 0) {
    // queries aligned with the points take the grid's device offsets (no
    // host copy, so the call can be captured in a graph); explicit query
    // offsets are uploaded first
    int32_t *qcloud = (int32_t *)(ws + L->qcloud);
    const int64_t *off_dev = g.offsets_dev;
    if (query_offsets) {
      int64_t *up = (int64_t *)(ws + L->offsets);
      MLS_HIP(hipMemcpyAsync(up, query_offsets, 8 * ((size_t)C + 1), hipMemcpyHostToDevice, s));
      off_dev = up;
    }
    MLS_HIP(mls::launch_fill_cloud_ids(off_dev, C, n, qcloud, s));
    qv->qcloud = qcloud;
  }
  if (!aligned && n > 0) {
    // other queries are processed in the Morton order of their cells; a
    // search sorts them, and the stages that continue from a preceding
    // search (fit only, refresh) keep that search's slots
    int32_t *order = (int32_t *)(ws + L->order);
    qv->order = order;
    if (sort) {
      // the value buffer the sort starts from is `order` when the number of
      // 8-bit digit passes is even, so the result lands in `order` either way
      const int passes = (g.key_bits + 7) / 8;
      int32_t *svals = (int32_t *)(ws + L->svals);
      int32_t *v0 = (passes & 1) ? svals : order, *v1 = (passes & 1) ? order : svals;
      uint64_t *k0 = (uint64_t *)(ws + L->skeys_a), *k1 = (uint64_t *)(ws + L->skeys_b);
      MLS_HIP(mls::launch_query_keys(queries, dtype == MLS_F64, n, qv->qcloud, g.clouds_dev,
                                     g.view.morton_bits, k0, v0, s));
      bool in_alt = false;  // = passes odd
      MLS_HIP(mls::radix_sort_pairs(k0, v0, k1, v1, n, g.key_bits, ws + L->sradix, &in_alt, s));
    }
  }
  return MLS_OK;
}

}  // namespace

extern "C" {

mls_status mls_knn(const mls_grid *grid, int32_t k, const void *queries, mls_dtype dtype,
                   int64_t n_queries, const int64_t *query_offsets, int32_t *out_neighbors,
                   double *out_keys, void *workspace, size_t workspace_bytes, void *stream) {
  g_last_error[0] = 0;
  if (n_queries > 0 && !out_neighbors) return MLS_ERR_INVALID_ARGUMENT;
  hipStream_t s = (hipStream_t)stream;
  mls::QueryView qv;
  ProjLayout L;
  if (grid && workspace && n_queries > 0 && k >= 1 && k <= MLS_MAX_K)
    forget_workspace(workspace, proj_layout(grid->g.n_clouds, k, n_queries).total);
  mls_status st = prepare_queries(grid, k, k, queries, dtype, n_queries, query_offsets,
                                  workspace, workspace_bytes, true, s, &qv, &L);
  if (st != MLS_OK || n_queries == 0) return st;
  char *ws = (char *)workspace;
  MLS_HIP(mls::launch_knn(grid->g.view, qv, k, k, 3.0, false, (int32_t *)(ws + L.nbr),
                          (uint8_t *)(ws + L.support), (double *)(ws + L.anchor),
                          (uint8_t *)(ws + L.flag), out_neighbors, out_keys, s));
  record_search(workspace, L.total, grid, k, k, n_queries,
                offsets_digest(query_offsets, grid->g.n_clouds, n_queries), 3.0);
  return MLS_OK;
}

mls_status mls_project_geometry(const mls_grid *grid, const mls_params *params,
                                const void *queries, mls_dtype dtype, int64_t n_queries,
                                const int64_t *query_offsets, void *out_points,
                                uint8_t *out_status, int32_t *out_neighbors, void *out_normals,
                                void *out_curvatures, void *workspace, size_t workspace_bytes,
                                void *stream) {
  g_last_error[0] = 0;
  if (!params) return MLS_ERR_INVALID_ARGUMENT;
  if (params->precision != MLS_PREC_FP64 && params->precision != MLS_PREC_FP32_MOMENTS)
    return MLS_ERR_INVALID_ARGUMENT;
  if (!(params->support_radius_h > 0.0) || !isfinite(params->support_radius_h) ||
      params->min_support < 0 || params->stages < 0 || params->stages > 7 ||
      params->search_extra < 0 || params->search_extra > MLS_MAX_K ||
      params->plane_iters < 0 || params->plane_iters > MLS_MAX_PLANE_ITERS ||
      params->ball < 0 || params->ball > 2 || (params->levin != 0 && params->levin != 1) ||
      (params->levin && params->plane_iters) || params->slot_order < 0 || params->slot_order > 7)
    return MLS_ERR_INVALID_ARGUMENT;
  if (params->slot_order) {
    // sorted order exists for queries aligned with the grid's points only
    if (!grid || query_offsets || n_queries != grid->g.n_points) {
      snprintf(g_last_error, sizeof g_last_error,
               "slot_order needs queries aligned with the grid's points");
      return MLS_ERR_INVALID_ARGUMENT;
    }
    const bool own = (params->slot_order & MLS_SLOT_OWN_POINTS) != 0;
    const bool q_sorted = own || (params->slot_order & MLS_SLOT_QUERIES);
    if (!own && q_sorted != ((params->slot_order & MLS_SLOT_OUTPUTS) != 0) && n_queries > 0 &&
        queries == out_points)
      return MLS_ERR_INVALID_ARGUMENT;
    if (params->ball == 2) return MLS_ERR_UNSUPPORTED;
    // the grid's own points: `queries` is not read (only dtype, for the outputs)
    if (own) queries = grid->g.view.pts;
  }
  const int stages = params->stages == 0 ? (MLS_STAGE_SEARCH | MLS_STAGE_FIT) : params->stages;
  if ((stages & MLS_STAGE_REFRESH) && !(stages & MLS_STAGE_SEARCH))
    return MLS_ERR_INVALID_ARGUMENT;
  if (n_queries > 0 && (stages & MLS_STAGE_FIT) && (!out_points || !out_status))
    return MLS_ERR_INVALID_ARGUMENT;
  if (!grid) return MLS_ERR_INVALID_ARGUMENT;
  hipStream_t s = (hipStream_t)stream;
  mls::QueryView qv;
  ProjLayout L;
  if (params->ball == 2) {
    // the ball without a count cap: one kernel, no lists (k unused)
    if (stages != (MLS_STAGE_SEARCH | MLS_STAGE_FIT) || out_neighbors) {
      snprintf(g_last_error, sizeof g_last_error,
               "ball = 2 projects in one call (all stages) and returns no lists");
      return MLS_ERR_INVALID_ARGUMENT;
    }
    if (params->plane_iters || params->levin) return MLS_ERR_UNSUPPORTED;
    if (workspace && n_queries > 0)
      forget_workspace(workspace, proj_layout(grid->g.n_clouds, 1, n_queries).total);
    mls_status st = prepare_queries(grid, 1, 1, queries, dtype, n_queries, query_offsets,
                                    workspace, workspace_bytes, true, s, &qv, &L);
    if (st != MLS_OK || n_queries == 0) return st;
    MLS_HIP(mls::launch_ball(grid->g.view, qv, params->precision, params->min_support,
                             params->support_radius_h, out_points, out_status, out_normals,
                             out_curvatures, s));
    return MLS_OK;
  }
  const int32_t k_list = params->k + params->search_extra;
  // a fresh search sorts queries that are not the grid's points; refresh and
  // fit-only calls keep the slots of the preceding search, which must be the
  // last search that wrote this workspace, with the same grid, k, kept
  // entries and queries (checked here, before anything is launched)
  const bool sort = (stages & MLS_STAGE_SEARCH) && !(stages & MLS_STAGE_REFRESH);
  const bool fit_only = (stages & MLS_STAGE_FIT) && !(stages & MLS_STAGE_SEARCH);
  const uint64_t digest = offsets_digest(query_offsets, grid->g.n_clouds, n_queries);
  if (n_queries > 0 && (fit_only || (stages & MLS_STAGE_REFRESH))) {
    mls_status rs = require_search(workspace, grid, params->k, k_list, n_queries, digest,
                                   fit_only ? &params->support_radius_h : nullptr,
                                   fit_only ? "fit-only stage" : "refresh stage");
    if (rs != MLS_OK) return rs;
  }
  // a search (re)writes the lists: the workspace holds no complete search
  // until it has been launched
  if ((stages & MLS_STAGE_SEARCH) && workspace && n_queries > 0 && params->k >= 1 &&
      k_list <= MLS_MAX_K)
    forget_workspace(workspace, proj_layout(grid->g.n_clouds, k_list, n_queries).total);
  mls_status st = prepare_queries(grid, params->k, k_list, queries, dtype, n_queries,
                                  query_offsets, workspace, workspace_bytes, sort, s, &qv, &L);
  if (st != MLS_OK || n_queries == 0) return st;
  qv.slot_in = (params->slot_order & (MLS_SLOT_QUERIES | MLS_SLOT_OWN_POINTS)) ? 1 : 0;
  if (params->slot_order & MLS_SLOT_OWN_POINTS) {
    // the sorted points {x, y, z, index} as the queries in sorted order
    qv.q = grid->g.view.pts;
    qv.in_f64 = 0;
    qv.in_stride = 4;
  }
  qv.slot_out = (params->slot_order & MLS_SLOT_OUTPUTS) ? 1 : 0;
  char *ws = (char *)workspace;
  int32_t *nbr = (int32_t *)(ws + L.nbr);
  uint8_t *support = (uint8_t *)(ws + L.support);
  if (stages & MLS_STAGE_SEARCH) {
    MLS_HIP(mls::launch_knn(grid->g.view, qv, k_list, params->k, params->support_radius_h,
                            (stages & MLS_STAGE_REFRESH) != 0, nbr, support,
                            (double *)(ws + L.anchor), (uint8_t *)(ws + L.flag), out_neighbors,
                            nullptr, s));
    record_search(workspace, L.total, grid, params->k, k_list, n_queries, digest,
                  params->support_radius_h);
  }
  if (stages & MLS_STAGE_FIT)
    MLS_HIP(mls::launch_mls_forward(grid->g.view, qv, params->k, params->precision,
                                    params->min_support, params->plane_iters, params->ball,
                                    params->levin, params->support_radius_h, nbr, support, out_points,
                                    out_status, out_normals, out_curvatures, s));
  return MLS_OK;
}

mls_status mls_project(const mls_grid *grid, const mls_params *params, const void *queries,
                       mls_dtype dtype, int64_t n_queries, const int64_t *query_offsets,
                       void *out_points, uint8_t *out_status, int32_t *out_neighbors,
                       void *workspace, size_t workspace_bytes, void *stream) {
  return mls_project_geometry(grid, params, queries, dtype, n_queries, query_offsets, out_points,
                              out_status, out_neighbors, nullptr, nullptr, workspace,
                              workspace_bytes, stream);
}

mls_status mls_project_noalloc(const mls_grid *grid, const mls_params *params,
                               const void *queries, mls_dtype dtype, int64_t n_queries,
                               const int64_t *query_offsets, void *out_points,
                               uint8_t *out_status, int32_t *out_neighbors, void *stream) {
  g_last_error[0] = 0;
  if (!grid || !params) return MLS_ERR_INVALID_ARGUMENT;
  if (!(params->stages == MLS_STAGE_ALL ||
        params->stages == (MLS_STAGE_SEARCH | MLS_STAGE_FIT))) {
    snprintf(g_last_error, sizeof g_last_error,
             "mls_project_noalloc: only a whole pass (search and fit) is supported");
    return MLS_ERR_INVALID_ARGUMENT;
  }
  const int32_t k_list = params->k + params->search_extra;
  if (params->k < 1 || params->search_extra < 0 || k_list > MLS_MAX_K || n_queries < 0 ||
      n_queries > 0x7fffffffll)
    return MLS_ERR_INVALID_ARGUMENT;
  const size_t need = proj_layout(grid->g.n_clouds, k_list, n_queries).total;
  if (need > kScratchBytes) {
    snprintf(g_last_error, sizeof g_last_error,
             "mls_project_noalloc: %lld queries with %d list entries need %zu bytes of "
             "scratch, above the fixed %zu",
             (long long)n_queries, (int)k_list, need, kScratchBytes);
    return MLS_ERR_WORKSPACE_TOO_SMALL;
  }
  void *ws = nullptr;
  mls_status st = scratch_of_current_device(&ws);
  if (st != MLS_OK) return st;
  st = mls_project_geometry(grid, params, queries, dtype, n_queries, query_offsets, out_points,
                            out_status, out_neighbors, nullptr, nullptr, ws, kScratchBytes,
                            stream);
  // the scratch is private to this call: no later stage may continue from it
  forget_workspace(ws, kScratchBytes);
  return st;
}

mls_status mls_project_backward(const mls_grid *grid, const mls_params *params,
                                const void *queries, mls_dtype dtype, int64_t n_queries,
                                const int64_t *query_offsets, const int32_t *neighbors,
                                const void *grad_out, void *grad_queries, void *grad_points,
                                void *workspace, size_t workspace_bytes, void *stream) {
  g_last_error[0] = 0;
  if (!params || !grid) return MLS_ERR_INVALID_ARGUMENT;
  if (params->precision != MLS_PREC_FP64 && params->precision != MLS_PREC_FP32_MOMENTS)
    return MLS_ERR_INVALID_ARGUMENT;
  if (!(params->support_radius_h > 0.0) || !isfinite(params->support_radius_h) ||
      params->min_support < 0 || params->search_extra < 0 || params->search_extra > MLS_MAX_K)
    return MLS_ERR_INVALID_ARGUMENT;
  if (params->plane_iters != 0 || params->ball != 0 || params->levin != 0 ||
      params->slot_order != 0)
    return MLS_ERR_UNSUPPORTED;
  const int32_t k_list = params->k + params->search_extra;
  // stages: ALL = lists from `neighbors` or a fresh search; FIT = the lists a
  // preceding search left in this workspace
  const bool reuse = params->stages == MLS_STAGE_FIT;
  if (!(params->stages == MLS_STAGE_ALL || params->stages == (MLS_STAGE_SEARCH | MLS_STAGE_FIT) ||
        reuse) || (reuse && neighbors))
    return MLS_ERR_INVALID_ARGUMENT;
  if (n_queries > 0 && (!grad_out || !grad_queries)) return MLS_ERR_INVALID_ARGUMENT;
  // the point gradients are accumulated in the workspace even without queries
  if (!grad_points || !workspace) return MLS_ERR_INVALID_ARGUMENT;
  if (params->k >= 1 && k_list <= MLS_MAX_K && n_queries >= 0 &&
      workspace_bytes < bwd_total(grid->g.n_clouds, k_list, n_queries, grid->g.n_points,
                                  params->precision))
    return MLS_ERR_WORKSPACE_TOO_SMALL;
  hipStream_t s = (hipStream_t)stream;
  mls::QueryView qv;
  ProjLayout L;
  // reused lists: the last search that wrote this workspace must be this
  // grid's, with the same k, kept entries and queries
  const uint64_t digest = offsets_digest(query_offsets, grid->g.n_clouds, n_queries);
  if (reuse && n_queries > 0) {
    mls_status rs = require_search(workspace, grid, params->k, k_list, n_queries, digest,
                                   nullptr, "adjoint with reused lists");
    if (rs != MLS_OK) return rs;
  }
  if (!reuse && n_queries > 0 && params->k >= 1 && k_list <= MLS_MAX_K)
    forget_workspace(workspace, proj_layout(grid->g.n_clouds, k_list, n_queries).total);
  mls_status st = prepare_queries(grid, params->k, k_list, queries, dtype, n_queries,
                                  query_offsets, workspace, workspace_bytes, !reuse, s, &qv, &L);
  if (st != MLS_OK) return st;
  if (((uintptr_t)workspace & 255) != 0) return MLS_ERR_INVALID_ARGUMENT;
  char *ws = (char *)workspace;
  int32_t *nbr = (int32_t *)(ws + L.nbr);
  if (n_queries > 0 && !reuse) {
    if (neighbors) {
      MLS_HIP(mls::launch_lists_from_caller(grid->g.view, qv, params->k, neighbors, nbr, s));
    } else {
      MLS_HIP(mls::launch_knn(grid->g.view, qv, k_list, params->k, params->support_radius_h,
                              false, nbr, (uint8_t *)(ws + L.support), (double *)(ws + L.anchor),
                              (uint8_t *)(ws + L.flag), nullptr, nullptr, s));
      record_search(workspace, L.total, grid, params->k, k_list, n_queries, digest,
                    params->support_radius_h);
    }
  }
  void *gp = ws + bwd_gp_offset(grid->g.n_clouds, k_list, n_queries);
  MLS_HIP(mls::launch_mls_backward(grid->g.view, qv, params->k, params->precision,
                                   params->support_radius_h, params->min_support, nbr, grad_out,
                                   grad_queries, gp, grad_points, s));
  return MLS_OK;
}

}  // extern "C"

