// grid.hip -- build of the uniform-grid spatial index on the GPU.
//
// Steps (all stream-ordered, HBM-bound):
//   1. per-cloud bounding box and count of non-finite points (the paper's
//      k-d tree build also starts by finding the minimum and maximum along
//      each dimension, Section 2.2);
//   2. per-point key (cloud id, Morton code of the point's cell) -- Morton
//      order is the reordering the paper suggests for chaotic clouds;
//   3. stable LSD radix sort of (key, original index), 8-bit digits;
//   4. gather of the sorted points as float4 {x, y, z, original index};
//   5. open-addressing hash from each non-empty cell to its contiguous range
//      of sorted points.
#include "mls_internal.h"

namespace mls {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t float_to_ordered(float f) {
  uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ int64_t find_cloud(const int64_t *offsets, int32_t n_clouds, int64_t i) {
  int32_t lo = 0, hi = n_clouds;  // offsets[lo] <= i < offsets[hi]
  while (hi - lo > 1) {
    int32_t mid = (lo + hi) >> 1;
    if (offsets[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// ---- 1. bounding boxes --------------------------------------------------------
// grid: x over chunks of the largest cloud, y over clouds.
__global__ __launch_bounds__(kThreads) void k_bbox(const float *__restrict__ pts,
                                                   const int64_t *__restrict__ offsets,
                                                   uint32_t *__restrict__ bbox,
                                                   unsigned long long *__restrict__ nonfinite) {
  const int c = blockIdx.y;
  const int64_t b = offsets[c], e = offsets[c + 1];
  uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu};
  uint32_t mx[3] = {0u, 0u, 0u};
  uint32_t bad = 0;
  for (int64_t i = b + (int64_t)blockIdx.x * kThreads + threadIdx.x; i < e;
       i += (int64_t)gridDim.x * kThreads) {
    float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
      ++bad;
      continue;
    }
    uint32_t o[3] = {float_to_ordered(x), float_to_ordered(y), float_to_ordered(z)};
    for (int a = 0; a < 3; ++a) {
      mn[a] = min(mn[a], o[a]);
      mx[a] = max(mx[a], o[a]);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    for (int a = 0; a < 3; ++a) {
      mn[a] = min(mn[a], (uint32_t)__shfl_xor((int)mn[a], off));
      mx[a] = max(mx[a], (uint32_t)__shfl_xor((int)mx[a], off));
    }
    bad += (uint32_t)__shfl_xor((int)bad, off);
  }
  // one set of atomics per block (atomics on the cloud's 7 words serialise)
  __shared__ uint32_t part[kThreads / 64][7];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    for (int a = 0; a < 3; ++a) {
      part[w][a] = mn[a];
      part[w][3 + a] = mx[a];
    }
    part[w][6] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < kThreads / 64; ++v) {
      for (int a = 0; a < 3; ++a) {
        mn[a] = min(mn[a], part[v][a]);
        mx[a] = max(mx[a], part[v][3 + a]);
      }
      bad += part[v][6];
    }
    for (int a = 0; a < 3; ++a) {
      atomicMin(bbox + 6 * c + a, mn[a]);
      atomicMax(bbox + 6 * c + 3 + a, mx[a]);
    }
    if (bad) atomicAdd(nonfinite + c, (unsigned long long)bad);
  }
}

__global__ void k_bbox_init(uint32_t *bbox, unsigned long long *nonfinite, int32_t n_clouds) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 6 * n_clouds) bbox[i] = (i % 6) < 3 ? 0xffffffffu : 0u;
  if (i < n_clouds) nonfinite[i] = 0ull;
}

// ---- 2. keys ------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_keys(const float *__restrict__ pts,
                                                   const CloudDev *__restrict__ clouds,
                                                   int32_t bits, uint64_t *__restrict__ keys,
                                                   int32_t *__restrict__ vals) {
  const int c = blockIdx.y;
  const CloudDev cd = clouds[c];
  for (int64_t i = cd.begin + (int64_t)blockIdx.x * kThreads + threadIdx.x; i < cd.end;
       i += (int64_t)gridDim.x * kThreads) {
    float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
    uint64_t key = kEmptyKey;
    if (isfinite(x) && isfinite(y) && isfinite(z)) {
      double p[3] = {(double)x, (double)y, (double)z};
      int32_t ic[3];
      for (int a = 0; a < 3; ++a) {
        int64_t t = cell_coord(p[a], cd.origin[a], cd.inv_cell);
        t = t < 0 ? 0 : (t >= cd.dims[a] ? cd.dims[a] - 1 : t);
        ic[a] = (int32_t)t;
      }
      key = cell_key(c, ic[0], ic[1], ic[2], bits);
    }
    keys[i] = key;
    vals[i] = (int32_t)i;
  }
}

// Keys of queries that are not the grid's points: the cloud id and the
// Morton code of the query's cell in that cloud's grid (clamped to the grid,
// so a query outside the box takes the nearest boundary cell); non-finite
// queries sort last. Sorting the queries by these keys makes queries that
// share cells and neighbours adjacent in the processing order, as the sorted
// points are for queries aligned with them.
template <typename Q>
__global__ __launch_bounds__(kThreads) void k_query_keys(const Q *__restrict__ q, int64_t n,
                                                         const int32_t *__restrict__ qcloud,
                                                         const CloudDev *__restrict__ clouds,
                                                         int32_t bits, uint64_t *__restrict__ keys,
                                                         int32_t *__restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const double p[3] = {(double)q[3 * i], (double)q[3 * i + 1], (double)q[3 * i + 2]};
  uint64_t key = kEmptyKey;
  if (isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2])) {
    const int32_t c = qcloud ? qcloud[i] : 0;
    const CloudDev &cd = clouds[c];
    int32_t ic[3];
    for (int a = 0; a < 3; ++a) {
      // clamp in floating point: a far query's cell index may not fit an int
      double t = floor((p[a] - cd.origin[a]) * cd.inv_cell);
      t = t < 0.0 ? 0.0 : (t > (double)(cd.dims[a] - 1) ? (double)(cd.dims[a] - 1) : t);
      ic[a] = (int32_t)t;
    }
    key = cell_key(c, ic[0], ic[1], ic[2], bits);
  }
  keys[i] = key;
  vals[i] = (int32_t)i;
}

// ---- 3. radix sort --------------------------------------------------------------
constexpr int kRsItems = 16;
constexpr int kRsTile = kThreads * kRsItems;  // 4096 keys per block
constexpr int kScanItems = 8;
constexpr int kScanTile = kThreads * kScanItems;  // 2048 entries per scan block

__global__ __launch_bounds__(kThreads) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                      int shift, uint32_t *__restrict__ hist,
                                                      int64_t nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
  for (int i = 0; i < kRsItems; ++i) {
    int64_t idx = base + i * kThreads + threadIdx.x;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// block-local exclusive scan of 2048 entries, optional block sums
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t *lds, uint32_t *total) {
  // inclusive wave scan
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = (uint32_t)__shfl_up((int)x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) lds[w] = x;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
  for (int i = 0; i < kThreads / 64; ++i) {
    uint32_t s = lds[i];
    if (i < w) wbase += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return wbase + x - v;
}

__global__ __launch_bounds__(kThreads) void k_scan_sums(const uint32_t *__restrict__ in, int64_t n,
                                                        uint32_t *__restrict__ sums) {
  __shared__ uint32_t lds[kThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  uint32_t tot;
  block_scan_excl(s, lds, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void k_scan_apply(uint32_t *__restrict__ data, int64_t n,
                                                         const uint32_t *__restrict__ block_prefix) {
  __shared__ uint32_t lds[kThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? data[base + i] : 0u;
    s += v[i];
  }
  uint32_t tot;
  uint32_t run = block_scan_excl(s, lds, &tot) + (block_prefix ? block_prefix[blockIdx.x] : 0u);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) data[base + i] = run;
    run += v[i];
  }
}

// Stable scatter: every wave ranks its 64 x kRsItems sub-tile row by row with
// ballot-based digit matching, so equal digits keep their input order.
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                         const int32_t *__restrict__ vin,
                                                         uint64_t *__restrict__ kout,
                                                         int32_t *__restrict__ vout, int64_t n,
                                                         int shift,
                                                         const uint32_t *__restrict__ offs,
                                                         int64_t nblocks) {
  constexpr int kW = kThreads / 64;
  __shared__ uint32_t cnt[kW][256];
  __shared__ uint32_t woff[kW][256];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int i = tid; i < kW * 256; i += kThreads) (&cnt[0][0])[i] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)w * (64 * kRsItems);
  const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint64_t key[kRsItems];
  int32_t val[kRsItems];
  uint32_t loc[kRsItems];
#pragma unroll
  for (int i = 0; i < kRsItems; ++i) {
    const int64_t idx = base + i * 64 + lane;
    const bool valid = idx < n;
    key[i] = valid ? kin[idx] : 0ull;
    val[i] = valid ? vin[idx] : 0;
    const uint32_t d = (uint32_t)(key[i] >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
    const uint32_t c0 = cnt[w][d];
    loc[i] = c0 + below;
    __builtin_amdgcn_wave_barrier();
    if (valid && below == 0) cnt[w][d] = c0 + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  {
    const int d = tid;  // kThreads == 256 digits
    uint32_t s = 0;
#pragma unroll
    for (int ww = 0; ww < kW; ++ww) {
      const uint32_t c = cnt[ww][d];
      woff[ww][d] = s;
      s += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kRsItems; ++i) {
    const int64_t idx = base + i * 64 + lane;
    if (idx < n) {
      const uint32_t d = (uint32_t)(key[i] >> shift) & 255u;
      const uint32_t dst = offs[(int64_t)d * nblocks + blockIdx.x] + woff[w][d] + loc[i];
      if ((int64_t)dst < n) {  // always true when the histogram and scan agree
        kout[dst] = key[i];
        vout[dst] = val[i];
      }
    }
  }
}

// ---- 4. gather ----------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_gather(const float *__restrict__ pts,
                                                     const int32_t *__restrict__ vals, int64_t n,
                                                     float4 *__restrict__ sorted,
                                                     int32_t *__restrict__ inv_perm) {
  const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (s >= n) return;
  const int32_t v = vals[s];
  if (v < 0 || (int64_t)v >= n) return;  // cannot happen for a permutation
  sorted[s] = make_float4(pts[3 * (int64_t)v], pts[3 * (int64_t)v + 1], pts[3 * (int64_t)v + 2],
                          __int_as_float(v));
  inv_perm[v] = (int32_t)s;
}

// ---- 5. cells -------------------------------------------------------------------------
// A level-l cell is a run of equal (key >> 3l) in the sorted keys.
__device__ __forceinline__ bool is_run_start(const uint64_t *keys, int64_t s, int level) {
  const uint64_t k = keys[s];
  return k != kEmptyKey && (s == 0 || (keys[s - 1] >> (3 * level)) != (k >> (3 * level)));
}

__global__ __launch_bounds__(kThreads) void k_count_cells(const uint64_t *__restrict__ keys,
                                                          int64_t n, int n_levels,
                                                          unsigned long long *__restrict__ counts) {
  __shared__ uint32_t part[kMaxLevels][kThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t c[kMaxLevels] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * kThreads)
    for (int l = 0; l < n_levels; ++l) c[l] += is_run_start(keys, s, l) ? 1u : 0u;
  for (int l = 0; l < kMaxLevels; ++l) {
    uint32_t v = c[l];
    for (int off = 32; off > 0; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off);
    if (lane == 0) part[l][w] = v;
  }
  __syncthreads();
  if (threadIdx.x < kMaxLevels && threadIdx.x < n_levels) {
    uint32_t t = 0;
    for (int i = 0; i < kThreads / 64; ++i) t += part[threadIdx.x][i];
    if (t) atomicAdd(counts + threadIdx.x, (unsigned long long)t);
  }
}

__global__ void k_table_fill(uint4 *__restrict__ table, uint64_t capacity) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < capacity) table[i] = make_uint4(0xffffffffu, 0xffffffffu, 0u, 0u);
}

__global__ __launch_bounds__(kThreads) void k_table_insert(const uint64_t *__restrict__ keys,
                                                           int64_t n, int n_levels,
                                                           uint4 *__restrict__ table,
                                                           uint64_t mask, int shift) {
  const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (s >= n) return;
  for (int l = 0; l < n_levels; ++l) {
    if (!is_run_start(keys, s, l)) continue;
    const int sh = 3 * l;
    const uint64_t key = keys[s] >> sh;
    // end of the run: exponential then binary search for the first larger key
    int64_t lo = s, step = 1, hi;
    for (;;) {
      hi = lo + step;
      if (hi >= n || (keys[hi] >> sh) != key) break;
      lo = hi;
      step <<= 1;
    }
    if (hi > n) hi = n;
    while (hi - lo > 1) {  // keys[lo] in the run, keys[hi] past it (or hi == n)
      const int64_t mid = lo + ((hi - lo) >> 1);
      if ((keys[mid] >> sh) == key) lo = mid; else hi = mid;
    }
    const uint32_t count = (uint32_t)(hi - s);
    const uint64_t tagged = key | ((uint64_t)l << kLevelShift);
    uint64_t slot = hash_slot(tagged, shift);
    for (uint64_t probe = 0; probe <= mask; ++probe) {
      unsigned long long *kp = reinterpret_cast<unsigned long long *>(table + slot);
      const unsigned long long prev = atomicCAS(kp, (unsigned long long)kEmptyKey,
                                                (unsigned long long)tagged);
      if (prev == (unsigned long long)kEmptyKey) {
        uint32_t *vp = reinterpret_cast<uint32_t *>(table + slot);
        vp[2] = (uint32_t)s;
        vp[3] = count;
        break;
      }
      slot = (slot + 1) & mask;
    }
  }
}

// ---- rebuild ------------------------------------------------------------------------
// A rebuild keeps the first build's geometry and table size; what depends on
// the new points is decided on the device, so that no host round trip sits
// between the steps.

__global__ void k_set_i32(int32_t *p, int32_t v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

__global__ void k_clear_u64(unsigned long long *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Sorted ranges of the clouds' finite points (non-finite points sort last).
__global__ void k_cloud_ranges(CloudDev *__restrict__ clouds, int32_t n_clouds,
                               const unsigned long long *__restrict__ nonfinite) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int64_t at = 0;
  for (int32_t c = 0; c < n_clouds; ++c) {
    const int64_t fin = (clouds[c].end - clouds[c].begin) - (int64_t)nonfinite[c];
    clouds[c].sbegin = at;
    clouds[c].send = at + (fin > 0 ? fin : 0);
    at = clouds[c].send;
  }
}

// The levels of the table: the longest prefix of levels whose cells fill at
// most half of the capacity (a level left out is absent from the hash: its
// lookups find nothing, which the search treats as an empty block and
// widens, so results stay exact).
__global__ void k_levels_fit(const unsigned long long *__restrict__ counts, int n_levels,
                             uint64_t capacity, int32_t *__restrict__ levels_out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  uint64_t total = 0;
  int fit = 0;
  for (int l = 0; l < n_levels; ++l) {
    total += counts[l];
    if (2 * total > capacity) break;
    fit = l + 1;
  }
  *levels_out = fit;
}

__global__ __launch_bounds__(kThreads) void k_table_insert_dev(const uint64_t *__restrict__ keys,
                                                               int64_t n,
                                                               const int32_t *__restrict__ levels,
                                                               uint4 *__restrict__ table,
                                                               uint64_t mask, int shift) {
  const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (s >= n) return;
  const int n_levels = *levels;
  for (int l = 0; l < n_levels; ++l) {
    if (!is_run_start(keys, s, l)) continue;
    const int sh = 3 * l;
    const uint64_t key = keys[s] >> sh;
    int64_t lo = s, step = 1, hi;
    for (;;) {
      hi = lo + step;
      if (hi >= n || (keys[hi] >> sh) != key) break;
      lo = hi;
      step <<= 1;
    }
    if (hi > n) hi = n;
    while (hi - lo > 1) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if ((keys[mid] >> sh) == key) lo = mid; else hi = mid;
    }
    const uint32_t count = (uint32_t)(hi - s);
    const uint64_t tagged = key | ((uint64_t)l << kLevelShift);
    uint64_t slot = hash_slot(tagged, shift);
    for (uint64_t probe = 0; probe <= mask; ++probe) {
      unsigned long long *kp = reinterpret_cast<unsigned long long *>(table + slot);
      const unsigned long long prev = atomicCAS(kp, (unsigned long long)kEmptyKey,
                                                (unsigned long long)tagged);
      if (prev == (unsigned long long)kEmptyKey) {
        uint32_t *vp = reinterpret_cast<uint32_t *>(table + slot);
        vp[2] = (uint32_t)s;
        vp[3] = count;
        break;
      }
      slot = (slot + 1) & mask;
    }
  }
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_clear_u64(unsigned long long *p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_u64, dim3(blocks_for(n, 64)), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_set_i32(int32_t *p, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_cloud_ranges(CloudDev *clouds, int32_t n_clouds,
                               const unsigned long long *nonfinite, hipStream_t s) {
  hipLaunchKernelGGL(k_cloud_ranges, dim3(1), dim3(64), 0, s, clouds, n_clouds, nonfinite);
  return hipGetLastError();
}

hipError_t launch_table_dev_levels(const uint64_t *keys, int64_t n, int n_levels,
                                   const unsigned long long *counts, int32_t *levels_dev,
                                   uint4 *table, uint64_t capacity, hipStream_t s) {
  hipLaunchKernelGGL(k_levels_fit, dim3(1), dim3(64), 0, s, counts, n_levels, capacity,
                     levels_dev);
  hipLaunchKernelGGL(k_table_fill, dim3(blocks_for((int64_t)capacity, 256)), dim3(256), 0, s,
                     table, capacity);
  int shift = 64;
  for (uint64_t c = capacity; c > 1; c >>= 1) --shift;
  hipLaunchKernelGGL(k_table_insert_dev, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s,
                     keys, n, levels_dev, table, capacity - 1, shift);
  return hipGetLastError();
}

hipError_t launch_bbox(const float *pts, const int64_t *offsets_dev, int32_t n_clouds,
                       int64_t max_cloud, uint32_t *bbox_bits, unsigned long long *nonfinite,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_bbox_init, dim3(blocks_for(6 * n_clouds, 256)), dim3(256), 0, s, bbox_bits,
                     nonfinite, n_clouds);
  unsigned gx = blocks_for(max_cloud, kThreads * 32);
  if (gx < 1) gx = 1;
  if (gx > 512) gx = 512;
  hipLaunchKernelGGL(k_bbox, dim3(gx, n_clouds), dim3(kThreads), 0, s, pts, offsets_dev,
                     bbox_bits, nonfinite);
  return hipGetLastError();
}

hipError_t launch_keys(const float *pts, const CloudDev *clouds, int32_t n_clouds,
                       int64_t max_cloud, int32_t bits, uint64_t *keys, int32_t *vals,
                       hipStream_t s) {
  unsigned gx = blocks_for(max_cloud, kThreads * 4);
  if (gx < 1) gx = 1;
  if (gx > 4096) gx = 4096;
  hipLaunchKernelGGL(k_keys, dim3(gx, n_clouds), dim3(kThreads), 0, s, pts, clouds, bits, keys,
                     vals);
  return hipGetLastError();
}

hipError_t launch_query_keys(const void *q, bool is_f64, int64_t n, const int32_t *qcloud,
                             const CloudDev *clouds, int32_t bits, uint64_t *keys, int32_t *vals,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 grid(blocks_for(n, kThreads));
  if (is_f64)
    hipLaunchKernelGGL(k_query_keys<double>, grid, dim3(kThreads), 0, s, (const double *)q, n,
                       qcloud, clouds, bits, keys, vals);
  else
    hipLaunchKernelGGL(k_query_keys<float>, grid, dim3(kThreads), 0, s, (const float *)q, n,
                       qcloud, clouds, bits, keys, vals);
  return hipGetLastError();
}

static int64_t scan_levels_bytes(int64_t len) {
  int64_t total = 0;
  while (len > kScanTile) {
    len = (len + kScanTile - 1) / kScanTile;
    total += ((len * 4 + 255) / 256) * 256;
  }
  return total;
}

size_t radix_temp_bytes(int64_t n) {
  const int64_t nblocks = (n + kRsTile - 1) / kRsTile;
  const int64_t hist = 256 * nblocks;
  return (size_t)(((hist * 4 + 255) / 256) * 256 + scan_levels_bytes(hist));
}

// exclusive scan of `len` uint32 in place, using `temp` for the block sums
static hipError_t device_scan(uint32_t *data, int64_t len, uint32_t *temp, hipStream_t s) {
  if (len <= kScanTile) {
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kThreads), 0, s, data, len,
                       (const uint32_t *)nullptr);
    return hipGetLastError();
  }
  const int64_t nb = (len + kScanTile - 1) / kScanTile;
  uint32_t *sums = temp;
  uint32_t *next = temp + ((nb * 4 + 255) / 256) * 64;
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(kThreads), 0, s, data, len, sums);
  hipError_t e = device_scan(sums, nb, next, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, data, len,
                     (const uint32_t *)sums);
  return hipGetLastError();
}

hipError_t radix_sort_pairs(uint64_t *keys, int32_t *vals, uint64_t *keys_alt, int32_t *vals_alt,
                            int64_t n, int32_t key_bits, void *temp, bool *result_in_alt,
                            hipStream_t s) {
  const int64_t nblocks = (n + kRsTile - 1) / kRsTile;
  uint32_t *hist = (uint32_t *)temp;
  uint32_t *scan_tmp = hist + ((256 * nblocks * 4 + 255) / 256) * 64;
  uint64_t *ki = keys, *ko = keys_alt;
  int32_t *vi = vals, *vo = vals_alt;
  bool alt = false;
  for (int shift = 0; shift < key_bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nblocks), dim3(kThreads), 0, s, ki, n, shift,
                       hist, nblocks);
    hipError_t e = device_scan(hist, 256 * nblocks, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nblocks), dim3(kThreads), 0, s, ki, vi, ko,
                       vo, n, shift, hist, nblocks);
    uint64_t *tk = ki; ki = ko; ko = tk;
    int32_t *tv = vi; vi = vo; vo = tv;
    alt = !alt;
  }
  *result_in_alt = alt;
  return hipGetLastError();
}

hipError_t launch_gather(const float *pts, const int32_t *vals, int64_t n, float4 *sorted,
                         int32_t *inv_perm, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, pts, vals, n,
                     sorted, inv_perm);
  return hipGetLastError();
}

hipError_t launch_count_cells(const uint64_t *keys, int64_t n, int n_levels,
                              unsigned long long *counts, hipStream_t s) {
  unsigned blocks = blocks_for(n, kThreads * 8);
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_count_cells, dim3(blocks), dim3(kThreads), 0, s, keys, n, n_levels, counts);
  return hipGetLastError();
}

hipError_t launch_build_table(const uint64_t *keys, int64_t n, int n_levels, uint4 *table,
                              uint64_t capacity, hipStream_t s) {
  hipLaunchKernelGGL(k_table_fill, dim3(blocks_for((int64_t)capacity, 256)), dim3(256), 0, s,
                     table, capacity);
  int shift = 64;
  for (uint64_t c = capacity; c > 1; c >>= 1) --shift;
  hipLaunchKernelGGL(k_table_insert, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, keys, n,
                     n_levels, table, capacity - 1, shift);
  return hipGetLastError();
}

}  // namespace mls
