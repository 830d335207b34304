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
#include <algorithm>

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
// Two stages without atomics: every block reduces its share of one cloud
// into a partial record, then one block per cloud reduces the partials.
// grid: x over chunks of the largest cloud, y over clouds.
constexpr int kBboxUnroll = 4;

__device__ __forceinline__ void bbox_point(float x, float y, float z, uint32_t *mn, uint32_t *mx,
                                           uint32_t &bad) {
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
    ++bad;
    return;
  }
  const uint32_t o[3] = {float_to_ordered(x), float_to_ordered(y), float_to_ordered(z)};
  for (int a = 0; a < 3; ++a) {
    mn[a] = min(mn[a], o[a]);
    mx[a] = max(mx[a], o[a]);
  }
}

// Block-wide min / max / sum of the 7 words; the result is valid in thread 0.
__device__ __forceinline__ void bbox_block_reduce(uint32_t *mn, uint32_t *mx, uint32_t &bad) {
  for (int off = 32; off > 0; off >>= 1) {
    for (int a = 0; a < 3; ++a) {
      mn[a] = min(mn[a], (uint32_t)__shfl_xor((int)mn[a], off));
      mx[a] = max(mx[a], (uint32_t)__shfl_xor((int)mx[a], off));
    }
    bad += (uint32_t)__shfl_xor((int)bad, off);
  }
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
  if (threadIdx.x == 0)
    for (int v = 1; v < kThreads / 64; ++v) {
      for (int a = 0; a < 3; ++a) {
        mn[a] = min(mn[a], part[v][a]);
        mx[a] = max(mx[a], part[v][3 + a]);
      }
      bad += part[v][6];
    }
}

// partial record of block x of cloud c: {min bits x3, max bits x3, non-finite count, 0}
__global__ __launch_bounds__(kThreads) void k_bbox(const float *__restrict__ pts,
                                                   const int64_t *__restrict__ offsets,
                                                   uint4 *__restrict__ partial) {
  const int c = blockIdx.y;
  const int64_t b = offsets[c], e = offsets[c + 1];
  uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu};
  uint32_t mx[3] = {0u, 0u, 0u};
  uint32_t bad = 0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i0 = b + (int64_t)blockIdx.x * kThreads + threadIdx.x; i0 < e;
       i0 += kBboxUnroll * stride) {
    float v[kBboxUnroll][3];
#pragma unroll
    for (int u = 0; u < kBboxUnroll; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < e) {
        v[u][0] = pts[3 * i];
        v[u][1] = pts[3 * i + 1];
        v[u][2] = pts[3 * i + 2];
      }
    }
#pragma unroll
    for (int u = 0; u < kBboxUnroll; ++u)
      if (i0 + u * stride < e) bbox_point(v[u][0], v[u][1], v[u][2], mn, mx, bad);
  }
  bbox_block_reduce(mn, mx, bad);
  if (threadIdx.x == 0) {
    uint4 *r = partial + 2 * ((int64_t)c * gridDim.x + blockIdx.x);
    r[0] = make_uint4(mn[0], mn[1], mn[2], mx[0]);
    r[1] = make_uint4(mx[1], mx[2], bad, 0u);
  }
}

// one block per cloud: reduce the cloud's `parts` partial records
__global__ __launch_bounds__(kThreads) void k_bbox_reduce(const uint4 *__restrict__ partial,
                                                          int parts, uint32_t *__restrict__ bbox,
                                                          unsigned long long *__restrict__ nonfinite) {
  const int c = blockIdx.x;
  uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu};
  uint32_t mx[3] = {0u, 0u, 0u};
  uint32_t bad = 0;
  for (int j = threadIdx.x; j < parts; j += kThreads) {
    const uint4 *r = partial + 2 * ((int64_t)c * parts + j);
    const uint4 r0 = r[0], r1 = r[1];
    mn[0] = min(mn[0], r0.x);
    mn[1] = min(mn[1], r0.y);
    mn[2] = min(mn[2], r0.z);
    mx[0] = max(mx[0], r0.w);
    mx[1] = max(mx[1], r1.x);
    mx[2] = max(mx[2], r1.y);
    bad += r1.z;
  }
  bbox_block_reduce(mn, mx, bad);
  if (threadIdx.x == 0) {
    for (int a = 0; a < 3; ++a) {
      bbox[6 * c + a] = mn[a];
      bbox[6 * c + 3 + a] = mx[a];
    }
    nonfinite[c] = bad;
  }
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

// Tile of block b among nb: blocks are dealt to the 8 XCDs in turn, so each
// XCD is given a contiguous range of tiles; tiles next to each other then
// write the cache lines they share through the same L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

__global__ __launch_bounds__(kThreads) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                      int shift, uint32_t *__restrict__ hist,
                                                      int64_t nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t base = tile * kRsTile;
#pragma unroll
  for (int i = 0; i < kRsItems; ++i) {
    int64_t idx = base + i * kThreads + threadIdx.x;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + tile] = h[threadIdx.x];
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
// ballot-based digit matching, so equal digits keep their input order. The
// tile is then laid out in LDS in digit order and written from there, so
// that consecutive lanes store consecutive addresses of a digit's run.
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
  __shared__ int32_t gadj[256];  // global position of the digit's run minus its tile position
  __shared__ uint32_t scan_lds[kW];
  __shared__ uint64_t skey[kRsTile];
  __shared__ int32_t sval[kRsTile];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  for (int i = tid; i < kW * 256; i += kThreads) (&cnt[0][0])[i] = 0u;
  __syncthreads();
  const int64_t tbase = tile * kRsTile;
  const int64_t base = tbase + (int64_t)w * (64 * kRsItems);
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
    uint32_t tot = 0;
#pragma unroll
    for (int ww = 0; ww < kW; ++ww) {
      const uint32_t c = cnt[ww][d];
      woff[ww][d] = tot;
      tot += c;
    }
    uint32_t all;
    const uint32_t dstart = block_scan_excl(tot, scan_lds, &all);
#pragma unroll
    for (int ww = 0; ww < kW; ++ww) woff[ww][d] += dstart;
    gadj[d] = (int32_t)offs[(int64_t)d * nblocks + tile] - (int32_t)dstart;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kRsItems; ++i) {
    if (base + i * 64 + lane < n) {
      const uint32_t d = (uint32_t)(key[i] >> shift) & 255u;
      const uint32_t at = woff[w][d] + loc[i];
      skey[at] = key[i];
      sval[at] = val[i];
    }
  }
  __syncthreads();
  const int count = (int)min<int64_t>(kRsTile, n - tbase);
  for (int j = tid; j < count; j += kThreads) {
    const uint64_t k = skey[j];
    const int64_t dst = (int64_t)gadj[(uint32_t)(k >> shift) & 255u] + j;
    if (dst >= 0 && dst < n) {  // always true when the histogram and scan agree
      kout[dst] = k;
      vout[dst] = sval[j];
    }
  }
}

// ---- 4. gather ----------------------------------------------------------------------
struct Point3 {
  float x, y, z;
};

__global__ __launch_bounds__(kThreads) void k_gather(const float *__restrict__ pts,
                                                     const int32_t *__restrict__ vals, int64_t n,
                                                     float4 *__restrict__ sorted,
                                                     int32_t *__restrict__ inv_perm) {
  const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (s >= n) return;
  const int32_t v = vals[s];
  if (v < 0 || (int64_t)v >= n) return;  // cannot happen for a permutation
  const Point3 p = reinterpret_cast<const Point3 *>(pts)[v];
  sorted[s] = make_float4(p.x, p.y, p.z, __int_as_float(v));
  inv_perm[v] = (int32_t)s;
}

// ---- 5. cells -------------------------------------------------------------------------
// A level-l cell is a run of equal (key >> 3l) in the sorted keys, so the
// sorted position s starts a cell at level l exactly when the highest bit in
// which keys[s] and keys[s - 1] differ is at least 3l (position 0, and the
// end of the keys, bound runs at every level). Cells are nested: a start at
// level l is a start at every level below it. Non-finite keys sort last and
// differ from every finite key in the top bit, so they bound the last cell.

// Highest differing bit of keys[s] and its predecessor: 64 at s == 0 and at
// s >= n (a boundary at every level), -1 for equal keys.
__device__ __forceinline__ int boundary_bit(const uint64_t *keys, int64_t s, int64_t n,
                                            uint64_t key) {
  if (s == 0 || s >= n) return 64;
  const uint64_t d = key ^ keys[s - 1];
  return d ? 63 - __clzll((long long)d) : -1;
}

constexpr int kCountUnroll = 4;

// Cells per level (counts[l] += cells of level l), for the table's levels.
__global__ __launch_bounds__(kThreads) void k_count_cells(const uint64_t *__restrict__ keys,
                                                          int64_t n,
                                                          unsigned long long *__restrict__ counts) {
  __shared__ uint32_t part[kMaxLevels][kThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t c[kMaxLevels] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t s0 = (int64_t)blockIdx.x * kThreads + threadIdx.x; s0 < n;
       s0 += kCountUnroll * stride) {
    uint64_t k[kCountUnroll], p[kCountUnroll];
#pragma unroll
    for (int u = 0; u < kCountUnroll; ++u) {
      const int64_t s = s0 + u * stride;
      k[u] = s < n ? keys[s] : kEmptyKey;
      p[u] = (s > 0 && s < n) ? keys[s - 1] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < kCountUnroll; ++u) {
      const int64_t s = s0 + u * stride;
      if (s >= n || k[u] == kEmptyKey) continue;
      const uint64_t d = k[u] ^ p[u];
      const int hb = s == 0 ? 64 : (d ? 63 - __clzll((long long)d) : -1);
#pragma unroll
      for (int l = 0; l < kMaxLevels; ++l) c[l] += hb >= 3 * l ? 1u : 0u;
    }
  }
  for (int l = 0; l < kMaxLevels; ++l) {
    uint32_t v = c[l];
    for (int off = 32; off > 0; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off);
    if (lane == 0) part[l][w] = v;
  }
  __syncthreads();
  if (threadIdx.x < kMaxLevels) {
    uint32_t t = 0;
    for (int i = 0; i < kThreads / 64; ++i) t += part[threadIdx.x][i];
    if (t) atomicAdd(counts + threadIdx.x, (unsigned long long)t);
  }
}

__global__ void k_table_fill(uint4 *__restrict__ table, uint64_t capacity) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < capacity) table[i] = make_uint4(0xffffffffu, 0xffffffffu, 0u, 0u);
}

// Slot of a tagged key: the empty slot it claims or the slot another lane
// already claimed for it (linear probing from its home slot).
__device__ __forceinline__ uint32_t *claim_slot(uint4 *table, uint64_t tagged, uint64_t mask,
                                                int shift) {
  uint64_t slot = hash_slot(tagged, shift);
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    unsigned long long *kp = reinterpret_cast<unsigned long long *>(table + slot);
    const unsigned long long prev =
        atomicCAS(kp, (unsigned long long)kEmptyKey, (unsigned long long)tagged);
    if (prev == (unsigned long long)kEmptyKey || prev == (unsigned long long)tagged)
      return reinterpret_cast<uint32_t *>(table + slot);
    slot = (slot + 1) & mask;
  }
  return nullptr;  // a full table: cannot happen below a load factor of 1
}

// Insertion of every cell of the table's levels (*levels of them) as
// {tagged key, first sorted position, end}. A wave takes 64 consecutive
// positions and ballots give each level's run boundaries. A cell starting in
// the wave writes its start, and its end when the run ends inside the wave;
// the first boundary of each level in the wave writes the end of the run
// that began in an earlier wave (whichever of the two writers comes first
// claims the slot). The wave's writes are spread over its lanes, about one
// compare-and-swap round per wave, with no search for run ends.
__global__ __launch_bounds__(kThreads) void k_table_insert(const uint64_t *__restrict__ keys,
                                                           int64_t n,
                                                           const int32_t *__restrict__ levels,
                                                           uint4 *__restrict__ table,
                                                           uint64_t mask, int shift) {
  constexpr int kW = kThreads / 64;
  constexpr int kTasks = 64 * kMaxLevels;
  __shared__ uint16_t task[kW][kTasks];  // (lane << 3) | level
  __shared__ int32_t task_end[kW][kTasks];  // end of the run, -1 past the wave
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t base = ((int64_t)blockIdx.x * kW + w) * 64;
  const int64_t s = base + lane;
  const int nl = min(max(*levels, 0), kMaxLevels);
  const uint64_t key = s < n ? keys[s] : kEmptyKey;
  const int hb = boundary_bit(keys, s, n, key);
  const bool finite = s < n && key != kEmptyKey;
  const uint64_t above = lane == 63 ? 0ull : (~0ull << (lane + 1));  // lanes after this one
  int starts = 0;  // levels this lane starts a cell at: 0 .. starts - 1
  int first_bnd = -1;  // lane l: first boundary of level l in the wave
  uint64_t bnd[kMaxLevels];
#pragma unroll
  for (int l = 0; l < kMaxLevels; ++l) {
    const bool b = hb >= 3 * l;
    bnd[l] = __ballot(b);
    starts += (b && finite && l < nl) ? 1 : 0;
    if (lane == l && bnd[l]) first_bnd = __ffsll((long long)bnd[l]) - 1;
  }
  // exclusive prefix of the start writes over the wave
  int incl = starts;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  const int first = incl - starts;
  const int total = __shfl(incl, 63);
#pragma unroll
  for (int l = 0; l < kMaxLevels; ++l) {
    if (l < starts) {
      const uint64_t after = bnd[l] & above;
      task[w][first + l] = (uint16_t)((lane << 3) | l);
      task_end[w][first + l] = after ? (int32_t)(base + __ffsll((long long)after) - 1) : -1;
    }
  }
  __syncthreads();
  for (int t = lane; t < total; t += 64) {
    const int info = task[w][t];
    const int l = info & 7;
    const int64_t start = base + (info >> 3);
    const int32_t end = task_end[w][t];
    uint32_t *vp = claim_slot(table, (keys[start] >> (3 * l)) | ((uint64_t)l << kLevelShift),
                              mask, shift);
    if (!vp) continue;
    if (end >= 0) {
      *reinterpret_cast<uint2 *>(vp + 2) = make_uint2((uint32_t)start, (uint32_t)end);
    } else {
      vp[2] = (uint32_t)start;
    }
  }
  // lane l < nl: the run of level l that ends at the wave's first boundary
  // began before the wave (no start precedes the first boundary)
  if (lane < nl && first_bnd >= 0) {
    const int64_t last = base + first_bnd - 1;  // the run's last position
    if (last >= 0 && last < n) {
      const uint64_t k = keys[last];
      if (k != kEmptyKey) {
        uint32_t *vp = claim_slot(table, (k >> (3 * lane)) | ((uint64_t)lane << kLevelShift),
                                  mask, shift);
        if (vp) vp[3] = (uint32_t)(base + first_bnd);
      }
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

static int hash_shift_of(uint64_t capacity) {
  int shift = 64;
  for (uint64_t c = capacity; c > 1; c >>= 1) --shift;
  return shift;
}

hipError_t launch_table_dev_levels(const uint64_t *keys, int64_t n, int n_levels,
                                   const unsigned long long *counts, int32_t *levels_dev,
                                   uint4 *table, uint64_t capacity, hipStream_t s) {
  hipLaunchKernelGGL(k_levels_fit, dim3(1), dim3(64), 0, s, counts, n_levels, capacity,
                     levels_dev);
  return launch_build_table(keys, n, levels_dev, table, capacity, s);
}

int bbox_parts(int64_t max_cloud, int32_t n_clouds) {
  int64_t gx = (max_cloud + kThreads * 16 - 1) / (kThreads * 16);
  const int64_t cap = std::max<int64_t>(1, kBboxPartsMax / n_clouds);
  return (int)std::max<int64_t>(1, std::min(gx, cap));
}

hipError_t launch_bbox(const float *pts, const int64_t *offsets_dev, int32_t n_clouds,
                       int64_t max_cloud, uint4 *partial, uint32_t *bbox_bits,
                       unsigned long long *nonfinite, hipStream_t s) {
  const int gx = bbox_parts(max_cloud, n_clouds);
  hipLaunchKernelGGL(k_bbox, dim3(gx, n_clouds), dim3(kThreads), 0, s, pts, offsets_dev, partial);
  hipLaunchKernelGGL(k_bbox_reduce, dim3(n_clouds), dim3(kThreads), 0, s, partial, gx, bbox_bits,
                     nonfinite);
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

hipError_t launch_count_cells(const uint64_t *keys, int64_t n, unsigned long long *counts,
                              hipStream_t s) {
  unsigned blocks = blocks_for(n, kThreads * 16);
  if (blocks < 1) blocks = 1;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_count_cells, dim3(blocks), dim3(kThreads), 0, s, keys, n, counts);
  return hipGetLastError();
}

hipError_t launch_build_table(const uint64_t *keys, int64_t n, const int32_t *levels_dev,
                              uint4 *table, uint64_t capacity, hipStream_t s) {
  hipLaunchKernelGGL(k_table_fill, dim3(blocks_for((int64_t)capacity, 256)), dim3(256), 0, s,
                     table, capacity);
  // waves cover positions 0 .. n: the wave holding position n ends the last run
  hipLaunchKernelGGL(k_table_insert, dim3(blocks_for(n + 1, kThreads)), dim3(kThreads), 0, s, keys,
                     n, levels_dev, table, capacity - 1, hash_shift_of(capacity));
  return hipGetLastError();
}

}  // namespace mls
