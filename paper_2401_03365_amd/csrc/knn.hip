// knn.hip -- exact k-nearest-neighbour search on the uniform grid.
//
// The k-nearest set is defined on canonical FP64 keys
//     key = ((dx*dx + dy*dy) + dz*dz),  d = p - r,
// each operation a binary64 round-to-nearest with no fused multiply-add (this
// file is compiled with contraction off), ties to the smaller original index,
// so the set is unique and equals a brute-force search over the whole cloud.
// Keys of non-negative doubles order like their bit patterns.
//
// Work layout: one wavefront owns a chunk of consecutive queries in
// processing order (Morton order: the grid's order for queries aligned with
// the points, a sort by cell key for other queries), so consecutive queries
// usually fall in the same cell. The grid indexes cells at several levels
// (edges c, 2c, 4c, 8c: a coarse cell is a contiguous Morton range of the
// sorted points). For each query the wave
// uses the 3x3x3 or 5x5x5 block of cells around the query's cell at a level
// chosen so that the block holds the k nearest (the level follows the
// previous query's k-th distance, so it adapts to the local density). The
// block's cells are staged nearest first -- cell lookups and their prefix
// sum in LDS -- and its first 192 candidates (coordinates, positions,
// indices) are gathered once into registers (lanes x slots) and reused by
// every following query of the chunk in the same block: per query the FP64
// keys and the selection of those, then the rest of a larger block 64
// candidates at a time, each entering only below the k-th pair so far.
//
// Certification: the distance beta from the query to the boundary of the
// visited box (faces beyond the cloud's grid count as infinitely far; a
// margin of cell * 2^-20 covers the rounding of the cell assignment) bounds
// every unvisited point from below, and the list is final once the k-th key
// is strictly below beta^2. Queries that no level certifies take the
// general path: shells of growing Chebyshev radius L around the query's
// level-0 cell, then an exhaustive scan of the cloud beyond kMaxRing.
//
// Selection (k of up to 256 pairs): keys are bucketed by a monotone map
// b = floor(key * scale) into 256 bins; an LDS histogram and its prefix sum
// give the bin b* holding the k-th pair; bins below b* are kept and inside b*
// the needed number of smallest pairs is found by ranking (small bins) or by
// bisection on the key bits and then on the index (large bins, i.e. ties).
#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kSlots = 4;                 // slot 0 = running top-k, 1..3 = candidates
constexpr int kNew = (kSlots - 1) * 64;   // candidates per batch
constexpr int kMaxRing = 12;
constexpr int kChunk = 64;                // consecutive queries per wave task

// The queries of a wave's chunk, loaded together at the chunk's start.
struct alignas(16) ChunkQueries {
  double x[kChunk], y[kChunk], z[kChunk];
  int32_t qi[kChunk];
  int32_t cloud[kChunk];
};

// List entries of up to 8 consecutive queries (entry j of the g-th query of
// the group at [g][j]), flushed to the tiles as 32-byte segments per entry
// (a smaller group leaves the LDS room for 5 blocks per CU).
constexpr int kListGroup = 8;
struct alignas(16) ListGroup {
  int32_t e[kListGroup][64];
};

struct alignas(16) WaveLds {
  uint32_t cstart[128];
  uint32_t cexcl[128];
  uint64_t ck[64];
  int32_t cpos[64];
  int32_t cidx[64];
  uint32_t hist[256];
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t dbits(double d) { return (uint64_t)__double_as_longlong(d); }
__device__ __forceinline__ double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

__device__ __forceinline__ bool pair_lt(uint64_t ka, int32_t ia, uint64_t kb, int32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

__device__ __forceinline__ uint32_t popc(uint64_t m) { return (uint32_t)__popcll(m); }

// Cross-lane moves on the DPP and permlane paths of the VALU (no LDS round
// trip). dpp<ctrl, rows>: lanes whose source is outside their row, or whose
// row is masked off, get `fill`.
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowShl4 = 0x104, kRowRor8 = 0x128, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E;  // quad_perm [1,0,3,2], [2,3,0,1]

template <int ctrl, int rows = 0xf>
__device__ __forceinline__ uint32_t dpp(uint32_t v, uint32_t fill) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, ctrl, rows, 0xf, false);
}

// Value of lane ^ s (s a power of two up to 32, known at compile time once
// unrolled).
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, int s, int lane) {
  switch (s) {
    case 1: return dpp<kQuadXor1>(v, v);
    case 2: return dpp<kQuadXor2>(v, v);
    case 4: {
      const uint32_t up = dpp<kRowShl4>(v, v), down = dpp<kRowShr4>(v, v);
      return (lane & 4) ? down : up;
    }
    case 8: return dpp<kRowRor8>(v, v);
    case 16: {
      const auto q = __builtin_amdgcn_permlane16_swap(v, v, false, false);
      return (lane & 16) ? q[0] : q[1];
    }
    default: {
      const auto q = __builtin_amdgcn_permlane32_swap(v, v, false, false);
      return (lane & 32) ? q[0] : q[1];
    }
  }
}

__device__ __forceinline__ uint64_t xor_lane_u64(uint64_t v, int s, int lane) {
  return ((uint64_t)xor_lane((uint32_t)(v >> 32), s, lane) << 32) | xor_lane((uint32_t)v, s, lane);
}

// Inclusive prefix sum over the wave's lanes.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += dpp<kRowShr1>(x, 0u);
  x += dpp<kRowShr2>(x, 0u);
  x += dpp<kRowShr4>(x, 0u);
  x += dpp<kRowShr8>(x, 0u);
  x += dpp<kRowBcast15, 0xa>(x, 0u);
  x += dpp<kRowBcast31, 0xc>(x, 0u);
  return x;
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), l) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
}

// A wave-uniform double held in scalar registers.
__device__ __forceinline__ double uniform_f64(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int ctrl, int rows = 0xf>
__device__ __forceinline__ uint64_t max_step(uint64_t v) {
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  const uint64_t o = ((uint64_t)dpp<ctrl, rows>(hi, hi) << 32) | dpp<ctrl, rows>(lo, lo);
  return o > v ? o : v;
}

// Maximum over the wave (inclusive max-scan; lane 63 holds the maximum).
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  v = max_step<kRowShr1>(v);
  v = max_step<kRowShr2>(v);
  v = max_step<kRowShr4>(v);
  v = max_step<kRowShr8>(v);
  v = max_step<kRowBcast15, 0xa>(v);
  v = max_step<kRowBcast31, 0xc>(v);
  return readlane_u64(v, 63);
}

struct Slots {
  uint64_t key[kSlots];
  int32_t pos[kSlots];
  int32_t idx[kSlots];
};

// Among the entries flagged by `in`, keep the `need` smallest (key, index)
// pairs: bisection on the key bits, then on the index among equal keys.
__device__ void select_in_set(const Slots &s, const bool in[kSlots], uint32_t need,
                              bool keep[kSlots]) {
  uint64_t mx = 0;
#pragma unroll
  for (int i = 0; i < kSlots; ++i) mx = (in[i] && s.key[i] > mx) ? s.key[i] : mx;
  mx = wave_max_u64(mx);
  uint64_t lo = 0, hi = mx + 1;
  uint32_t clo = 0, chi = 0;
#pragma unroll
  for (int i = 0; i < kSlots; ++i) chi += popc(__ballot(in[i]));
  while (hi - lo > 1 && chi - clo > 1) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kSlots; ++i) c += popc(__ballot(in[i] && s.key[i] < mid));
    if (c < need) { lo = mid; clo = c; } else { hi = mid; chi = c; }
  }
  uint64_t K = lo;
  if (hi - lo > 1) {  // exactly one flagged entry in [lo, hi): it is the need-th
    uint64_t found = 0;
#pragma unroll
    for (int i = 0; i < kSlots; ++i)
      found = (in[i] && s.key[i] >= lo && s.key[i] < hi) ? s.key[i] : found;
    K = wave_max_u64(found);
  }
  uint32_t c_lt = 0, c_le = 0;
#pragma unroll
  for (int i = 0; i < kSlots; ++i) {
    c_lt += popc(__ballot(in[i] && s.key[i] < K));
    c_le += popc(__ballot(in[i] && s.key[i] <= K));
  }
  const uint32_t at_k = need - c_lt;  // entries with key == K to keep
  if (c_le - c_lt == at_k) {
#pragma unroll
    for (int i = 0; i < kSlots; ++i) keep[i] = in[i] && s.key[i] <= K;
    return;
  }
  int64_t ilo = -1, ihi = 0x7fffffff;  // count(idx <= ilo) < at_k <= count(idx <= ihi)
  while (ihi - ilo > 1) {
    const int64_t mid = ilo + ((ihi - ilo) >> 1);
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kSlots; ++i)
      c += popc(__ballot(in[i] && s.key[i] == K && s.idx[i] <= mid));
    if (c < at_k) ilo = mid; else ihi = mid;
  }
#pragma unroll
  for (int i = 0; i < kSlots; ++i)
    keep[i] = in[i] && (s.key[i] < K || (s.key[i] == K && s.idx[i] <= (int32_t)ihi));
}

// Flags the min(k, total) smallest valid pairs. scale maps keys to buckets
// (keys beyond 255/scale share the last bucket). Returns the bucket holding
// the k-th pair, or -1 when every valid entry is kept.
__device__ int select_topk(const Slots &s, int k, double scale, WaveLds &L, int lane,
                           bool keep[kSlots], uint32_t *total_out) {
  uint32_t total = 0;
#pragma unroll
  for (int i = 0; i < kSlots; ++i) total += popc(__ballot(s.key[i] != kEmptyKey));
  *total_out = total;
  if ((int)total <= k) {
#pragma unroll
    for (int i = 0; i < kSlots; ++i) keep[i] = s.key[i] != kEmptyKey;
    return -1;
  }
  reinterpret_cast<uint4 *>(L.hist)[lane] = make_uint4(0u, 0u, 0u, 0u);
  wave_sync();
  int bkt[kSlots];
#pragma unroll
  for (int i = 0; i < kSlots; ++i) {
    const bool v = s.key[i] != kEmptyKey;
    const double x = bitsd(v ? s.key[i] : 0ull) * scale;
    const int b = x < 255.0 ? (int)x : 255;
    bkt[i] = v ? b : 256;
    if (v) atomicAdd(&L.hist[b], 1u);
  }
  wave_sync();
  const uint4 hv = reinterpret_cast<const uint4 *>(L.hist)[lane];
  const uint32_t s4 = hv.x + hv.y + hv.z + hv.w;
  const uint32_t incl = wave_incl_scan(s4);
  const uint32_t e0 = incl - s4, e1 = e0 + hv.x, e2 = e1 + hv.y, e3 = e2 + hv.z;
  const uint32_t ku = (uint32_t)k;
  int mybin = -1;
  uint32_t mybelow = 0, mycnt = 0;
  if (e0 < ku && ku <= e1) { mybin = 0; mybelow = e0; mycnt = hv.x; }
  if (e1 < ku && ku <= e2) { mybin = 1; mybelow = e1; mycnt = hv.y; }
  if (e2 < ku && ku <= e3) { mybin = 2; mybelow = e2; mycnt = hv.z; }
  if (e3 < ku && ku <= incl) { mybin = 3; mybelow = e3; mycnt = hv.w; }
  const uint64_t who = __ballot(mybin >= 0);
  const int src = (int)__builtin_ctzll(who);
  const int bstar = 4 * src + __builtin_amdgcn_readlane(mybin, src);
  const uint32_t below = (uint32_t)__builtin_amdgcn_readlane((int)mybelow, src);
  const uint32_t m = (uint32_t)__builtin_amdgcn_readlane((int)mycnt, src);
  const uint32_t need = ku - below;
  bool in[kSlots];
#pragma unroll
  for (int i = 0; i < kSlots; ++i) in[i] = bkt[i] == bstar;
  if (need == m) {
#pragma unroll
    for (int i = 0; i < kSlots; ++i) keep[i] = bkt[i] <= bstar;
    return bstar;
  }
  bool kin[kSlots];
  if (m <= 16) {
    // rank every entry of the bucket against the others
#pragma unroll
    for (int i = 0; i < kSlots; ++i) kin[i] = false;
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      uint64_t mask = __ballot(in[sl]);
      while (mask) {
        const int l = (int)__builtin_ctzll(mask);
        mask &= mask - 1;
        const uint64_t ke = readlane_u64(s.key[sl], l);
        const int32_t ie = __builtin_amdgcn_readlane(s.idx[sl], l);
        uint32_t rank = 0;
#pragma unroll
        for (int i = 0; i < kSlots; ++i)
          rank += popc(__ballot(in[i] && pair_lt(s.key[i], s.idx[i], ke, ie)));
        kin[sl] = (lane == l) ? (rank < need) : kin[sl];
      }
    }
  } else {
    select_in_set(s, in, need, kin);
  }
#pragma unroll
  for (int i = 0; i < kSlots; ++i) keep[i] = bkt[i] < bstar || kin[i];
  return bstar;
}

// Moves the kept entries into slot 0 (lanes 0..count-1) and clears the
// candidate slots' keys (their positions and indices stay). Returns the count.
__device__ int compact(Slots &s, const bool keep[kSlots], WaveLds &L, int lane) {
  const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t base = 0;
#pragma unroll
  for (int i = 0; i < kSlots; ++i) {
    const uint64_t msk = __ballot(keep[i]);
    if (keep[i]) {
      const uint32_t o = base + popc(msk & lt_mask);
      L.ck[o] = s.key[i];
      L.cpos[o] = s.pos[i];
      L.cidx[o] = s.idx[i];
    }
    base += popc(msk);
  }
  wave_sync();
  const int ntop = (int)base;
  const bool have = lane < ntop;
  const uint64_t ck = L.ck[lane];
  const int32_t cp = L.cpos[lane], ci = L.cidx[lane];
  wave_sync();
  s.key[0] = have ? ck : kEmptyKey;
  s.pos[0] = have ? cp : 0;
  s.idx[0] = have ? ci : 0x7fffffff;
#pragma unroll
  for (int i = 1; i < kSlots; ++i) s.key[i] = kEmptyKey;
  return ntop;
}

// Sorts the (key, index, position) triples held one per lane ascending by
// (key, index) across the wave (bitonic network over 64 lanes).
__device__ __forceinline__ void sort_lanes(uint64_t &mk, int32_t &mi, int32_t &mp, int lane) {
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const uint64_t ok = xor_lane_u64(mk, stride, lane);
      const int32_t oi = (int32_t)xor_lane((uint32_t)mi, stride, lane);
      const int32_t op = (int32_t)xor_lane((uint32_t)mp, stride, lane);
      const bool up = (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      const bool olt = pair_lt(ok, oi, mk, mi);
      const bool ogt = pair_lt(mk, mi, ok, oi);
      const bool take = (lower == up) ? olt : ogt;
      mk = take ? ok : mk;
      mi = take ? oi : mi;
      mp = take ? op : mp;
    }
  }
}

// Moves the kfit smallest (key, index) pairs of the lane entries (lanes
// 0..ntop-1) to lanes 0..kfit-1 and the rest after them, each part in lane
// order, and returns the largest key. A list that keeps extra entries needs
// only this split: the fit takes its first kfit, and a refresh re-ranks the
// whole list. The kfit smallest are found by the histogram selection, here
// over the lane entries alone (about a third of the instructions of the
// bitonic sort of the same 64 lanes).
__device__ uint64_t partition_lanes(uint64_t &mk, int32_t &mi, int32_t &mp, int ntop, int kfit,
                                    WaveLds &L, int lane) {
  const bool valid = lane < ntop;
  const uint64_t kmax = wave_max_u64(valid ? mk : 0ull);
  if (ntop <= kfit) return kmax;
  Slots t;
  t.key[0] = valid ? mk : kEmptyKey;
  t.idx[0] = mi;
  t.pos[0] = mp;
#pragma unroll
  for (int i = 1; i < kSlots; ++i) {
    t.key[i] = kEmptyKey;
    t.idx[i] = 0x7fffffff;
    t.pos[i] = 0;
  }
  const double mx = bitsd(kmax);
  bool keep[kSlots];
  uint32_t total;
  select_topk(t, kfit, mx > 0.0 ? 255.0 / mx : 1.0, L, lane, keep, &total);
  const uint64_t km = __ballot(keep[0]);
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const uint32_t dest = keep[0] ? popc(km & lt) : popc(km) + popc(~km & lt);
  if (valid) {
    L.ck[dest] = mk;
    L.cpos[dest] = mp;
    L.cidx[dest] = mi;
  }
  wave_sync();
  if (valid) {
    mk = L.ck[lane];
    mp = L.cpos[lane];
    mi = L.cidx[lane];
  }
  wave_sync();
  return kmax;
}

template <int ctrl, int rows = 0xf>
__device__ __forceinline__ void pair_max_step(uint64_t &mk, int32_t &mi) {
  const uint32_t lo = (uint32_t)mk, hi = (uint32_t)(mk >> 32);
  const uint64_t ok = ((uint64_t)dpp<ctrl, rows>(hi, hi) << 32) | dpp<ctrl, rows>(lo, lo);
  const int32_t oi = (int32_t)dpp<ctrl, rows>((uint32_t)mi, (uint32_t)mi);
  const bool t = pair_lt(mk, mi, ok, oi);
  mk = t ? ok : mk;
  mi = t ? oi : mi;
}

// Largest (key, index) pair of the running top-k (uniform result).
__device__ void top_max(const Slots &s, int ntop, int lane, uint64_t &kmax, int32_t &imax) {
  uint64_t mk = lane < ntop ? s.key[0] : 0;
  int32_t mi = lane < ntop ? s.idx[0] : -1;
  pair_max_step<kRowShr1>(mk, mi);
  pair_max_step<kRowShr2>(mk, mi);
  pair_max_step<kRowShr4>(mk, mi);
  pair_max_step<kRowShr8>(mk, mi);
  pair_max_step<kRowBcast15, 0xa>(mk, mi);
  pair_max_step<kRowBcast31, 0xc>(mk, mi);
  kmax = readlane_u64(mk, 63);
  imax = __builtin_amdgcn_readlane(mi, 63);
}

// Distance from r to the boundary of the box of cells [c0 - L, c0 + L]
// (faces beyond the cloud's grid are at infinity), minus the assignment
// margin. Returns +inf when the box covers the whole grid.
__device__ __forceinline__ double box_clearance(const CloudDev &cd, const double r[3],
                                                const int32_t c0[3], int L, int level = 0) {
  double beta = __longlong_as_double(0x7ff0000000000000ll);
  const double cell = ldexp(cd.cell, level);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int32_t lo = c0[a] - L, hi = c0[a] + L;
    const int32_t dims = ((cd.dims[a] - 1) >> level) + 1;
    if (lo > 0) beta = fmin(beta, r[a] - (cd.origin[a] + (double)lo * cell));
    if (hi < dims - 1) beta = fmin(beta, (cd.origin[a] + (double)(hi + 1) * cell) - r[a]);
  }
  if (!isinf(beta)) beta -= cell * 0x1p-20;
  return beta;
}

// Squared bound a k-th key must stay strictly below: beta^2 rounded down.
__device__ __forceinline__ double cert_bound(double beta) {
  if (isinf(beta)) return beta;
  return beta > 0.0 ? beta * beta * (1.0 - 0x1p-40) : 0.0;
}

// Sorted position of candidate ci of the concatenated cell ranges staged in
// LDS (128 entries: exclusive prefix `cexcl`, starts `cstart`).
__device__ __forceinline__ int32_t cand_pos(const WaveLds &L, int32_t ci) {
  int lo = 0, hi = 128;  // largest c with cexcl[c] <= ci
#pragma unroll
  for (int it = 0; it < 7; ++it) {
    const int mid = (lo + hi) >> 1;
    const bool le = (int32_t)L.cexcl[mid] <= ci;
    lo = le ? mid : lo;
    hi = le ? hi : mid;
  }
  return (int32_t)L.cstart[lo] + (ci - (int32_t)L.cexcl[lo]);
}

__device__ __forceinline__ int2 lookup_if(const GridView &g, int cloud, const CloudDev &cd,
                                          bool has, int32_t cx, int32_t cy, int32_t cz,
                                          int level) {
  if (has && cx >= 0 && cy >= 0 && cz >= 0 && cx <= ((cd.dims[0] - 1) >> level) &&
      cy <= ((cd.dims[1] - 1) >> level) && cz <= ((cd.dims[2] - 1) >> level))
    return lookup_cell(g, level_cell_key(cloud, cx, cy, cz, g.morton_bits, level));
  return make_int2(0, 0);
}

// Stages up to 128 cell ranges (entry lane and entry 64 + lane) and their
// exclusive prefix in LDS; returns the candidate total.
__device__ __forceinline__ int32_t stage_ranges(int2 a, int2 b, WaveLds &L, int lane) {
  const uint32_t xa = wave_incl_scan((uint32_t)a.y);
  const uint32_t ta = (uint32_t)__builtin_amdgcn_readlane((int)xa, 63);
  const uint32_t xb = wave_incl_scan((uint32_t)b.y);
  const uint32_t tb = (uint32_t)__builtin_amdgcn_readlane((int)xb, 63);
  wave_sync();
  L.cstart[lane] = (uint32_t)a.x;
  L.cexcl[lane] = xa - (uint32_t)a.y;
  L.cstart[64 + lane] = (uint32_t)b.x;
  L.cexcl[64 + lane] = ta + xb - (uint32_t)b.y;
  wave_sync();
  return (int32_t)(ta + tb);
}

// One cell per lane (count 0 for lanes without a cell).
__device__ __forceinline__ int32_t stage_cells(const GridView &g, int cloud, const CloudDev &cd,
                                               bool has, int32_t cx, int32_t cy, int32_t cz,
                                               WaveLds &L, int lane, int level = 0) {
  return stage_ranges(lookup_if(g, cloud, cd, has, cx, cy, cz, level), make_int2(0, 0), L, lane);
}

// Cell offsets of a (2 half + 1)^3 block in order of their squared distance
// from the centre cell (nearest first), so that the first candidates of a
// staged block are those of the cells nearest the query.
struct CellOrder {
  int8_t d[125][3];
};
constexpr CellOrder make_cell_order(int half) {
  CellOrder o{};
  int n = 0;
  for (int r2 = 0; r2 <= 3 * half * half; ++r2)
    for (int z = -half; z <= half; ++z)
      for (int y = -half; y <= half; ++y)
        for (int x = -half; x <= half; ++x)
          if (x * x + y * y + z * z == r2) {
            o.d[n][0] = (int8_t)x;
            o.d[n][1] = (int8_t)y;
            o.d[n][2] = (int8_t)z;
            ++n;
          }
  return o;
}
__constant__ CellOrder kCellOrder3 = make_cell_order(1);
__constant__ CellOrder kCellOrder5 = make_cell_order(2);

// The (2 half + 1)^3 block of level-`level` cells around cell cl (half 1 or
// 2), nearest cells first.
__device__ __forceinline__ int32_t stage_block(const GridView &g, int cloud, const CloudDev &cd,
                                               const int32_t cl[3], int half, int level,
                                               WaveLds &L, int lane) {
  const int w = 2 * half + 1;
  const int n = w * w * w;
  const CellOrder &ord = half == 1 ? kCellOrder3 : kCellOrder5;
  // both lanes' cells probe their home slots together (two loads in flight),
  // then the rare collisions walk on
  int2 ab[2];
  uint64_t key[2], slot[2];
  bool need[2];
  uint4 e4[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int t = lane + 64 * e;
    const int tt = t < n ? t : 0;
    const int32_t cx = cl[0] + ord.d[tt][0], cy = cl[1] + ord.d[tt][1], cz = cl[2] + ord.d[tt][2];
    need[e] = t < n && cx >= 0 && cy >= 0 && cz >= 0 && cx <= ((cd.dims[0] - 1) >> level) &&
              cy <= ((cd.dims[1] - 1) >> level) && cz <= ((cd.dims[2] - 1) >> level);
    key[e] = level_cell_key(cloud, cx, cy, cz, g.morton_bits, level);
    slot[e] = hash_slot(key[e], g.hash_shift);
    ab[e] = make_int2(0, 0);
  }
#pragma unroll
  for (int e = 0; e < 2; ++e) e4[e] = need[e] ? g.table[slot[e]] : make_uint4(~0u, ~0u, 0u, 0u);
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    for (uint64_t probe = 0; need[e] && probe <= g.hash_mask; ++probe) {
      const uint64_t kk = (uint64_t)e4[e].x | ((uint64_t)e4[e].y << 32);
      if (kk == key[e]) {
        const int64_t st = (int64_t)e4[e].z, en = (int64_t)e4[e].w;
        if (en >= st && en <= g.n_points) ab[e] = make_int2((int)st, (int)(en - st));
        need[e] = false;
      } else if (kk == kEmptyKey) {
        need[e] = false;
      } else {
        slot[e] = (slot[e] + 1) & g.hash_mask;
        e4[e] = g.table[slot[e]];
      }
    }
  }
  return stage_ranges(ab[0], ab[1], L, lane);
}

// Candidate at sorted position pos into slot sl if it can still enter the
// top-k (branch-free: position and index are always written, only the key
// marks the entry valid).
__device__ __forceinline__ void put_candidate(const GridView &g, int32_t pos, bool present,
                                              const double r[3], int ntop, int k, uint64_t kmax,
                                              int32_t imax, Slots &s, int sl) {
  float4 P = make_float4(0.f, 0.f, 0.f, 0.f);
  if (present) P = g.pts[pos];
  const uint64_t key = dbits(canon_key((double)P.x, (double)P.y, (double)P.z, r[0], r[1], r[2]));
  const int32_t idx = __float_as_int(P.w);
  const bool take = present && ((ntop < k) || pair_lt(key, idx, kmax, imax));
  s.pos[sl] = pos;
  s.idx[sl] = idx;
  s.key[sl] = take ? key : kEmptyKey;
}

// Merge the filled candidate slots into the top-k (general path).
__device__ void merge_general(Slots &s, int &ntop, int k, uint64_t &kmax, int32_t &imax,
                              WaveLds &L, int lane) {
  uint64_t mx;
  if (ntop == k) {
    mx = kmax;  // new entries were filtered below the current k-th pair
  } else {
    mx = 0;
#pragma unroll
    for (int i = 0; i < kSlots; ++i) mx = (s.key[i] != kEmptyKey && s.key[i] > mx) ? s.key[i] : mx;
    mx = wave_max_u64(mx);
  }
  const double scale = 255.99 / fmax(bitsd(mx), 1e-300);
  bool keep[kSlots];
  uint32_t total;
  select_topk(s, k, scale, L, lane, keep, &total);
  ntop = compact(s, keep, L, lane);
  if (ntop == k) top_max(s, ntop, lane, kmax, imax);
}

// General search for one query from scratch: rings of growing Chebyshev
// radius around the query's cell at the coarsest level, then the exhaustive
// scan. Returns ntop.
__device__ int search_general(const GridView &g, int cloud, const CloudDev &cd, const double r[3],
                              const int32_t cq[3], int k, Slots &s, WaveLds &L, int lane) {
  // the coarsest level in the hash; with none, the exhaustive scan
  const int nlev = levels_of(g);
  const int lev = nlev > 0 ? nlev - 1 : 0;
  const double cellc = ldexp(cd.cell, lev);
  int32_t c0[3];
  int32_t lmin = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // floor division of the level-0 cell by 2^lev (cq may be negative)
    c0[a] = cq[a] >= 0 ? (cq[a] >> lev) : -((-cq[a] + (1 << lev) - 1) >> lev);
    const int32_t dims = ((cd.dims[a] - 1) >> lev) + 1;
    lmin = max(lmin, max(-c0[a], c0[a] - (dims - 1)));
  }
  (void)cellc;
#pragma unroll
  for (int i = 0; i < kSlots; ++i) { s.key[i] = kEmptyKey; s.pos[i] = 0; s.idx[i] = 0x7fffffff; }
  int ntop = 0;
  uint64_t kmax = kEmptyKey;
  int32_t imax = 0x7fffffff;
  bool brute = nlev == 0 || lmin > kMaxRing;
  const int L0 = lmin < 1 ? 1 : lmin;
  bool done = false;
  for (int ring = L0; !done && !brute; ++ring) {
    const int w = 2 * ring + 1;
    const int32_t ncells = w * w * w;
    for (int32_t t0 = 0; t0 < ncells; t0 += 64) {
      const int32_t t = t0 + lane;
      const int32_t dx = t % w - ring, dy = (t / w) % w - ring, dz = t / (w * w) - ring;
      const int cheb = max(abs(dx), max(abs(dy), abs(dz)));
      const bool has = t < ncells && (ring == L0 || cheb == ring);
      const int32_t total =
          stage_cells(g, cloud, cd, has, c0[0] + dx, c0[1] + dy, c0[2] + dz, L, lane, lev);
      for (int32_t b0 = 0; b0 < total; b0 += kNew) {
#pragma unroll
        for (int sl = 1; sl < kSlots; ++sl) {
          const int32_t ci = b0 + (sl - 1) * 64 + lane;
          const bool present = ci < total;
          const int32_t pos = present ? cand_pos(L, ci) : 0;
          const bool inb = pos >= 0 && (int64_t)pos < g.n_points;
          put_candidate(g, inb ? pos : 0, present && inb, r, ntop, k, kmax, imax, s, sl);
        }
        bool any = false;
#pragma unroll
        for (int sl = 1; sl < kSlots; ++sl) any |= __ballot(s.key[sl] != kEmptyKey) != 0ull;
        if (any) merge_general(s, ntop, k, kmax, imax, L, lane);
      }
    }
    const double beta = box_clearance(cd, r, c0, ring, lev);
    if (isinf(beta)) {
      done = true;  // every cell of the cloud visited
    } else {
      if (ntop == k && bitsd(kmax) < cert_bound(beta)) done = true;
      if (!done && ring >= kMaxRing) brute = true;
    }
  }
  if (brute) {
#pragma unroll
    for (int i = 0; i < kSlots; ++i) { s.key[i] = kEmptyKey; s.idx[i] = 0x7fffffff; }
    ntop = 0;
    kmax = kEmptyKey;
    imax = 0x7fffffff;
    const int64_t total = cd.send - cd.sbegin;
    for (int64_t b0 = 0; b0 < total; b0 += kNew) {
#pragma unroll
      for (int sl = 1; sl < kSlots; ++sl) {
        const int64_t ci = b0 + (sl - 1) * 64 + lane;
        const bool present = ci < total;
        put_candidate(g, present ? (int32_t)(cd.sbegin + ci) : 0, present, r, ntop, k, kmax,
                      imax, s, sl);
      }
      bool any = false;
#pragma unroll
      for (int sl = 1; sl < kSlots; ++sl) any |= __ballot(s.key[sl] != kEmptyKey) != 0ull;
      if (any) merge_general(s, ntop, k, kmax, imax, L, lane);
    }
  }
  return ntop;
}

// Block options o = 0 .. 2 levels - 1: level o / 2, half-width 1 + o % 2, in
// increasing block volume ((2 half + 1) 2^level)^3; each guarantees a
// clearance of about half * 2^level cells of the finest level.

// Searches the k (= kfit + extra) nearest of every query slot (only the
// slots flagged in slot_flag when it is given). The tile list of a slot holds
// its k entries, sorted by (key, index) whenever k > kfit or sorted output is
// wanted, so that the first kfit are the kfit nearest; the support count and
// the caller's lists cover the first kfit. The slot's anchor (the query) and
// bound (the k-th key: every point outside the list is at least that far, in
// squared distance, from the anchor; +inf when the list holds the whole
// cloud; -1 for a non-finite query or a list without extra entries, which a
// refresh then searches afresh) serve later refreshes.
// kMode: kPlain (k == kfit, every slot searched, no caller lists: the
// common case), kExtra (k > kfit, every slot, no caller lists: a search that
// keeps entries for a refresh), kFlagged (the slots a refresh left, no
// caller lists) or kAny; each compiled without the branches of the others.
constexpr int kPlain = 0, kExtra = 1, kFlagged = 2, kAny = 3;
template <int kMode>
// The full-search variants run 5 waves per SIMD (96 VGPRs, a few spills
// outside the hot loops): the extra wave hides more of the staging's global
// round trips than the registers would save; the others keep 4.
__global__ __launch_bounds__(64 * kWavesPerBlock, (kMode == kFlagged || kMode == kAny) ? 4 : 5)
void k_knn(GridView g, QueryView qv, int32_t k, int32_t kfit, double support_r_h,
           int32_t *__restrict__ nbr, uint8_t *__restrict__ support, double *__restrict__ anchor,
           const uint8_t *__restrict__ slot_flag, int32_t *__restrict__ out_nbr,
           double *__restrict__ out_keys) {
  __shared__ WaveLds lds[kWavesPerBlock];
  __shared__ ChunkQueries chq[kWavesPerBlock];
  __shared__ ListGroup lgr[kWavesPerBlock];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  WaveLds &L = lds[wv];
  ChunkQueries &Q = chq[wv];
  ListGroup &LG = lgr[wv];
  // every slot is searched: lists are gathered per group of queries and
  // written as whole segments (a refresh leaves other slots' rows as they are)
  const bool grouped = kMode == kPlain || kMode == kExtra || (kMode == kAny && !slot_flag);
  if (kMode != kAny) {
    if (kMode == kPlain) kfit = k;
    if (kMode != kFlagged) slot_flag = nullptr;
    out_nbr = nullptr;
    out_keys = nullptr;
  }
  const int64_t nchunks = (qv.n + kChunk - 1) / kChunk;
  const int nopt = 2 * levels_of(g);
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  for (int64_t task = blk * kWavesPerBlock + wv; task < nchunks;
       task += (int64_t)gridDim.x * kWavesPerBlock) {
    // cache of the staged block: its cell, option and cloud, the candidate
    // count and the candidate coordinates (positions and indices live in the
    // candidate slots of s)
    int32_t cc0[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    int ccloud = -1, copt = -1;
    int32_t ncand = -1;
    double rho_est = 0.0;  // k-th distance of the previous query of the chunk
    float cx[kSlots], cy[kSlots], cz[kSlots];
    Slots s;
#pragma unroll
    for (int i = 0; i < kSlots; ++i) {
      s.key[i] = kEmptyKey; s.pos[i] = 0; s.idx[i] = 0x7fffffff;
      cx[i] = cy[i] = cz[i] = 0.f;
    }
    const int64_t p0 = task * kChunk;
    const int64_t pend = min(p0 + kChunk, qv.n);
    // the chunk's slots to search: all, or those a refresh left (one flag
    // load per lane instead of one dependent load per slot)
    uint64_t todo = ~0ull;
    if (slot_flag) {
      todo = __ballot(p0 + lane < pend && slot_flag[p0 + lane] != 0);
      if (todo == 0) continue;
    }
    // for the slots a refresh left: lane j holds slot p0 + j's hint
    double hint_l = 0.0;
    {
      // lane j loads query slot p0 + j (one round trip for the chunk)
      const int64_t p = p0 + lane;
      int32_t qi = 0, cl = 0;
      double x = 0.0, y = 0.0, z = 0.0;
      if (p < pend && ((todo >> lane) & 1)) {
        if (slot_flag) hint_l = anchor[4 * p + 3];
        if (qv.aligned) qi = __float_as_int(g.pts[p].w);
        else qi = (int32_t)ordered_query(qv, p);
        double rq[3];
        load_slot_query(g, qv, p, qi, rq);
        x = rq[0]; y = rq[1]; z = rq[2];
        cl = qv.qcloud ? qv.qcloud[qi] : 0;
        qi = (int32_t)out_index(qv, p, qi);  // where the caller's lists go
      }
      wave_sync();
      Q.x[lane] = x; Q.y[lane] = y; Q.z[lane] = z;
      Q.qi[lane] = qi;
      Q.cloud[lane] = cl;
      wave_sync();
    }
    for (int64_t p = p0; p < pend; ++p) {
      if (!((todo >> (p - p0)) & 1)) continue;
      if (slot_flag) {
        // the refresh left the squared distance of the old list's farthest
        // entry from the moved query (its k nearest lie within it); that
        // bound is loose, so the block targets the smaller of it and the
        // previous query's k-th distance
        const double hint = readlane_f64(hint_l, (int)(p - p0));
        if (hint > 0.0 && isfinite(hint))
          rho_est = rho_est > 0.0 ? fmin(rho_est, sqrt(hint)) : sqrt(hint);
      }
      const int j = (int)(p - p0);
      const int64_t qi = __builtin_amdgcn_readfirstlane(Q.qi[j]);
      const double r[3] = {uniform_f64(Q.x[j]), uniform_f64(Q.y[j]), uniform_f64(Q.z[j])};
      const int cloud = __builtin_amdgcn_readfirstlane(Q.cloud[j]);
      const CloudDev &cd = g.clouds[cloud];
      const bool finite = isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]);
      int ntop = 0;
      if (finite && cd.send > cd.sbegin) {
        int32_t c0[3];
        int32_t lmin = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          double t = floor((r[a] - cd.origin[a]) * cd.inv_cell);
          t = fmin(fmax(t, -1073741824.0), 1073741824.0);
          c0[a] = (int32_t)t;
          lmin = max(lmin, max(-c0[a], c0[a] - (cd.dims[a] - 1)));
        }
        bool solved = false;
        if (lmin == 0 && nopt > 0) {
          double target = 1.05 * rho_est;
          // the query's offset in its level-0 cell, in cell units (FP32: it
          // only steers the choice of block, never the certification)
          float u[3];
#pragma unroll
          for (int a = 0; a < 3; ++a)
            u[a] = (float)((r[a] - cd.origin[a]) * cd.inv_cell - (double)c0[a]);
          for (int att = 0; att < 2 * kMaxLevels + 2 && !solved; ++att) {
            // smallest block whose clearance (half-width plus the query's
            // interior clearance in its cell) reaches the target; option o
            // is level o / 2 with half-width 1 + o % 2
            const float tgt = (float)(target * cd.inv_cell);
            int opt = nopt - 1;
            for (int o = 0; o < nopt; ++o) {
              const int l = o >> 1;
              const float w = (float)(1 << l);
              float f = w;
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                const float off = (float)(c0[a] & ((1 << l) - 1)) + u[a];
                f = fminf(f, fminf(off, w - off));
              }
              if ((float)(1 + (o & 1)) * w + fmaxf(f, 0.f) >= tgt) { opt = o; break; }
            }
            const int lt = opt >> 1, half = 1 + (opt & 1);
            const int32_t cl[3] = {c0[0] >> lt, c0[1] >> lt, c0[2] >> lt};
            if (cl[0] != cc0[0] || cl[1] != cc0[1] || cl[2] != cc0[2] || cloud != ccloud ||
                opt != copt) {
              // stage the block (and cache its candidates when they fit)
              cc0[0] = cl[0]; cc0[1] = cl[1]; cc0[2] = cl[2];
              ccloud = cloud;
              copt = opt;
              ncand = stage_block(g, cloud, cd, cl, half, lt, L, lane);
              // the slots cache the first kNew candidates (the nearest cells'):
              // all of them, or the part a larger block's queries keep and
              // complete from the rest of the block per query
#pragma unroll
              for (int sl = 1; sl < kSlots; ++sl) {
                if ((sl - 1) * 64 < ncand) {
                  const int32_t ci = (sl - 1) * 64 + lane;
                  int32_t pos = ci < ncand ? cand_pos(L, ci) : 0;
                  pos = (pos >= 0 && (int64_t)pos < g.n_points) ? pos : 0;
                  const float4 P = g.pts[pos];
                  cx[sl] = P.x; cy[sl] = P.y; cz[sl] = P.z;
                  s.pos[sl] = pos;
                  s.idx[sl] = __float_as_int(P.w);
                }
              }
            }
            const double beta = box_clearance(cd, r, cl, half, lt);
            const double bound = cert_bound(beta);
            const bool inf = isinf(bound);
            if (ncand < k && !inf) {
              // too few points in the block: need a wider one
              if (opt == nopt - 1) break;
              target = fmax(target, 1.5 * fmax(beta, 0.0) + 1e-300);
              continue;
            }
            uint64_t kmax = kEmptyKey;
            int32_t imax = 0x7fffffff;
            bool exact_max = false;
            {
              const bool partial = ncand > kNew;
#pragma unroll
              for (int sl = 1; sl < kSlots; ++sl) {
                if ((sl - 1) * 64 < ncand) {
                  const bool present = (sl - 1) * 64 + lane < ncand;
                  const uint64_t key = dbits(canon_key((double)cx[sl], (double)cy[sl],
                                                       (double)cz[sl], r[0], r[1], r[2]));
                  s.key[sl] = present ? key : kEmptyKey;
                } else {
                  s.key[sl] = kEmptyKey;
                }
              }
              s.key[0] = kEmptyKey;
              double scale;
              if (inf) {
                uint64_t mx = 0;
#pragma unroll
                for (int i = 1; i < kSlots; ++i)
                  mx = (s.key[i] != kEmptyKey && s.key[i] > mx) ? s.key[i] : mx;
                scale = 255.99 / fmax(bitsd(wave_max_u64(mx)), 1e-300);
              } else {
                scale = 255.99 / fmax(bound, 1e-300);
              }
              bool keep[kSlots];
              uint32_t total;
              const int bstar = select_topk(s, k, scale, L, lane, keep, &total);
              ntop = compact(s, keep, L, lane);
              if (!partial && bstar >= 0 && bstar < 255 && !inf) {
                kmax = dbits((double)(bstar + 1) / scale);  // upper bound of the k-th key
              } else {
                top_max(s, ntop, lane, kmax, imax);
                exact_max = true;
              }
              // the rest of a large block, 64 candidates at a time, each
              // entering only below the current k-th pair
              for (int32_t b0 = kNew; b0 < ncand; b0 += 64) {
                const int32_t ci = b0 + lane;
                const bool present = ci < ncand;
                const int32_t pos = present ? cand_pos(L, ci) : 0;
                const bool inb = pos >= 0 && (int64_t)pos < g.n_points;
                float4 P = make_float4(0.f, 0.f, 0.f, 0.f);
                if (present && inb) P = g.pts[pos];
                const uint64_t key =
                    dbits(canon_key((double)P.x, (double)P.y, (double)P.z, r[0], r[1], r[2]));
                const int32_t idx = __float_as_int(P.w);
                const bool take = present && inb && (ntop < k || pair_lt(key, idx, kmax, imax));
                if (__ballot(take) == 0ull) continue;
                Slots t;
                t.key[0] = s.key[0]; t.pos[0] = s.pos[0]; t.idx[0] = s.idx[0];
                t.key[1] = take ? key : kEmptyKey; t.pos[1] = pos; t.idx[1] = idx;
#pragma unroll
                for (int i = 2; i < kSlots; ++i) {
                  t.key[i] = kEmptyKey; t.pos[i] = 0; t.idx[i] = 0x7fffffff;
                }
                merge_general(t, ntop, k, kmax, imax, L, lane);
                s.key[0] = t.key[0]; s.pos[0] = t.pos[0]; s.idx[0] = t.idx[0];
              }
              if (partial) exact_max = ntop == k;
            }
            const bool done = ntop == k ? (inf || bitsd(kmax) < bound) : inf;
            if (done) {
              solved = true;
              rho_est = ntop == k ? sqrt(bitsd(kmax)) : 0.0;
            } else {
              if (opt == nopt - 1) break;
              // the block holds k points within sqrt(kmax): a clearance above
              // that certifies
              const double rk = exact_max ? sqrt(bitsd(kmax)) : sqrt(fmax(bound, 0.0));
              target = fmax(1.05 * rk, 1.05 * sqrt(fmax(bound, 0.0)));
            }
          }
        }
        if (!solved) {
          ntop = search_general(g, cloud, cd, r, c0, k, s, L, lane);
          cc0[0] = INT32_MIN;  // the general path reused the candidate slots
          copt = -1;
        }
      }

      const double rad = support_r_h * cd.h;
      const double rad2 = rad * rad;
      uint64_t mk = lane < ntop ? s.key[0] : kEmptyKey;
      int32_t mi = lane < ntop ? s.idx[0] : 0x7fffffff;
      int32_t mp = lane < ntop ? s.pos[0] : -1;
      // a list that keeps extra entries leads with the kfit nearest; lists
      // returned to the caller are sorted
      uint64_t klast = 0ull;
      if ((kMode == kExtra || kMode == kFlagged) && k > kfit)
        klast = partition_lanes(mk, mi, mp, ntop, kfit, L, lane);
      if (kMode == kAny && (k > kfit || out_nbr || out_keys)) {
        sort_lanes(mk, mi, mp, lane);  // valid entries first
        klast = readlane_u64(mk, k - 1);
      }
      const bool valid = lane < ntop;
      const uint32_t m = popc(__ballot(valid && lane < kfit && bitsd(mk) <= rad2));
      // lists are stored per tile of 64 consecutive queries, neighbour-major:
      // entry j of query p at [(p / 64) * 64 k + j * 64 + p % 64]; entries
      // past the cloud's size are -1
      if (lane < k) {
        const int32_t e = valid ? mp : -1;
        if (grouped) LG.e[j & (kListGroup - 1)][lane] = e;
        else nbr[(p >> 6) * 64 * k + lane * 64 + (p & 63)] = e;
      }
      if (grouped && ((j & (kListGroup - 1)) == kListGroup - 1 || p == pend - 1)) {
        // the group's row segments, 8 entries (32 B) per list row; rows of
        // slots past the last query hold -1
        wave_sync();
        const int g0 = j & ~(kListGroup - 1), gn = (j & (kListGroup - 1)) + 1;
        if (lane < k) {
          int4 *dst = reinterpret_cast<int4 *>(nbr + (p >> 6) * 64 * k + lane * 64 +
                                               ((p0 + g0) & 63));
#pragma unroll
          for (int q4 = 0; q4 < kListGroup / 4; ++q4) {
            int32_t v[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
              v[t] = (4 * q4 + t < gn) ? LG.e[4 * q4 + t][lane] : -1;
            dst[q4] = make_int4(v[0], v[1], v[2], v[3]);
          }
        }
        wave_sync();
      }
      // the bound of a list with extra entries: its largest key (used when
      // the list is full, ntop == k)
      const uint64_t kth = klast;
      if (lane == 0) {
        support[p] = (uint8_t)((finite && ntop >= kfit) ? m : 0);
        double *an = anchor + 4 * p;
        if (kMode == kPlain) {
          an[3] = -1.0;  // no extra entries: a refresh searches afresh
        } else {
          an[0] = r[0]; an[1] = r[1]; an[2] = r[2];
          an[3] = (!finite || k == kfit) ? -1.0
                  : (ntop < k ? __longlong_as_double(0x7ff0000000000000ll) : bitsd(kth));
        }
      }
      if (lane < kfit) {
        if (out_nbr) out_nbr[qi * kfit + lane] = valid ? mi : -1;
        if (out_keys) out_keys[qi * kfit + lane] = valid ? bitsd(mk) : bitsd(0x7ff8000000000000ull);
      }
    }
  }
}

// Refresh with few changes, one lane per slot. The first kfit entries of a
// list are the kfit nearest of the list for the query it was searched for;
// for the moved query only entries near the kfit-th distance can change
// sides. The lane keeps the kSwap largest (key, index) pairs among the first
// kfit and the kSwap smallest among the others; when fewer than kSwap pairs
// are out of order, swapping them gives the kfit nearest of the list, and
// with the certification of the re-ranking refresh the list is final (only
// the swapped rows and the support count are rewritten). Other slots are
// flagged 2 for the re-ranking refresh.
constexpr int kSwap = 4;

// kSwap (key, index, row, position) entries held in registers (one array
// per field, so that every access is static after unrolling).
struct Ents {
  uint64_t key[kSwap];
  int32_t idx[kSwap], row[kSwap], pos[kSwap];
};

// Inserts e into the ordered entries, dropping the last: descending when
// `desc` (largest first), else ascending. Branch-free selects.
template <bool desc>
__device__ __forceinline__ void ents_insert(Ents &a, uint64_t ek, int32_t ei, int32_t er,
                                            int32_t ep) {
  bool c[kSwap];
#pragma unroll
  for (int i = 0; i < kSwap; ++i)
    c[i] = desc ? pair_lt(a.key[i], a.idx[i], ek, ei) : pair_lt(ek, ei, a.key[i], a.idx[i]);
#pragma unroll
  for (int i = kSwap - 1; i > 0; --i) {
    const bool from_prev = c[i] && c[i - 1];
    const bool here = c[i] && !c[i - 1];
    a.key[i] = from_prev ? a.key[i - 1] : (here ? ek : a.key[i]);
    a.idx[i] = from_prev ? a.idx[i - 1] : (here ? ei : a.idx[i]);
    a.row[i] = from_prev ? a.row[i - 1] : (here ? er : a.row[i]);
    a.pos[i] = from_prev ? a.pos[i - 1] : (here ? ep : a.pos[i]);
  }
  a.key[0] = c[0] ? ek : a.key[0];
  a.idx[0] = c[0] ? ei : a.idx[0];
  a.row[0] = c[0] ? er : a.row[0];
  a.pos[0] = c[0] ? ep : a.pos[0];
}

__global__ __launch_bounds__(256) void k_knn_refresh_lane(GridView g, QueryView qv, int32_t k,
                                                          int32_t kfit, double support_r_h,
                                                          int32_t *__restrict__ nbr,
                                                          uint8_t *__restrict__ support,
                                                          const double *__restrict__ anchor,
                                                          uint8_t *__restrict__ slot_flag) {
  const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (p >= qv.n) return;
  int64_t qi;
  if (qv.aligned) qi = __float_as_int(g.pts[p].w);
  else qi = ordered_query(qv, p);
  double r[3];
  load_slot_query(g, qv, p, qi, r);
  const double *an = anchor + 4 * p;
  const double bound = an[3];
  const bool finite = isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]);
  if (!finite || !(bound >= 0.0) || kfit < kSwap) {
    slot_flag[p] = 2;
    return;
  }
  const double rad = support_r_h * g.clouds[qv.qcloud ? qv.qcloud[qi] : 0].h;
  const double rad2 = rad * rad;
  int32_t *row = nbr + (p >> 6) * 64 * k + (p & 63);
  Ents hi, lo;  // hi descending (largest first), lo ascending
#pragma unroll
  for (int i = 0; i < kSwap; ++i) {
    hi.key[i] = 0ull; hi.idx[i] = -1; hi.row[i] = 0; hi.pos[i] = 0;
    lo.key[i] = kEmptyKey; lo.idx[i] = 0x7fffffff; lo.row[i] = 0; lo.pos[i] = 0;
  }
  int m = 0;
  bool valid = true;
  // positions and points of 4 entries are loaded ahead of their use
  constexpr int kAhead = 4;
  int32_t pq[kAhead];
  float4 Pq[kAhead];
#pragma unroll
  for (int a = 0; a < kAhead; ++a) pq[a] = a < k ? row[a * 64] : -1;
#pragma unroll
  for (int a = 0; a < kAhead; ++a) {
    const bool hv = pq[a] >= 0 && (int64_t)pq[a] < g.n_points;
    Pq[a] = g.pts[hv ? pq[a] : 0];
  }
  for (int j0 = 0; j0 < k; j0 += kAhead) {
    int32_t pn[kAhead];
#pragma unroll
    for (int a = 0; a < kAhead; ++a)
      pn[a] = j0 + kAhead + a < k ? row[(j0 + kAhead + a) * 64] : -1;
#pragma unroll
    for (int a = 0; a < kAhead; ++a) {
      const int j = j0 + a;
      if (j >= k) break;
      const int32_t pos = pq[a];
      const bool have = pos >= 0 && (int64_t)pos < g.n_points;
      const float4 P = Pq[a];
      const uint64_t key = dbits(canon_key((double)P.x, (double)P.y, (double)P.z, r[0], r[1], r[2]));
      const int32_t idx = __float_as_int(P.w);
      if (j < kfit) {
        valid = valid && have;
        m += (have && bitsd(key) <= rad2) ? 1 : 0;
        ents_insert<true>(hi, key, idx, j, pos);
      } else if (have) {
        ents_insert<false>(lo, key, idx, j, pos);
      }
    }
#pragma unroll
    for (int a = 0; a < kAhead; ++a) {
      pq[a] = pn[a];
      const bool hv = pq[a] >= 0 && (int64_t)pq[a] < g.n_points;
      Pq[a] = g.pts[hv ? pq[a] : 0];
    }
  }
  // pairs out of order: lo[i] < hi[i] holds for i < s (both sides monotone)
  int s = 0;
#pragma unroll
  for (int i = 0; i < kSwap; ++i) s += pair_lt(lo.key[i], lo.idx[i], hi.key[i], hi.idx[i]) ? 1 : 0;
  bool ok = valid && s < kSwap;
  // the kfit-th pair after the swaps: the larger of the largest kept inside
  // entry and the largest entry swapped in
  uint64_t kk = hi.key[0];
  int32_t ki = hi.idx[0];
#pragma unroll
  for (int i = 1; i < kSwap; ++i) {
    kk = (s == i) ? hi.key[i] : kk;
    ki = (s == i) ? hi.idx[i] : ki;
  }
#pragma unroll
  for (int i = 0; i < kSwap; ++i) {
    const bool up = i == s - 1 && pair_lt(kk, ki, lo.key[i], lo.idx[i]);
    kk = up ? lo.key[i] : kk;
    ki = up ? lo.idx[i] : ki;
  }
  if (ok && !isinf(bound)) {
    const double dx = r[0] - an[0], dy = r[1] - an[1], dz = r[2] - an[2];
    const double delta = sqrt(dx * dx + dy * dy + dz * dz) * (1.0 + 0x1p-40);
    const double reach = sqrt(bound) * (1.0 - 0x1p-40) - delta;
    ok = reach > 0.0 && bitsd(kk) < reach * reach * (1.0 - 0x1p-40);
  }
  if (ok) {
#pragma unroll
    for (int i = 0; i < kSwap; ++i) {
      if (i < s) {
        row[hi.row[i] * 64] = lo.pos[i];
        row[lo.row[i] * 64] = hi.pos[i];
        m += (bitsd(lo.key[i]) <= rad2 ? 1 : 0) - (bitsd(hi.key[i]) <= rad2 ? 1 : 0);
      }
    }
    support[p] = (uint8_t)m;
  }
  slot_flag[p] = ok ? 0 : 2;
}

// Re-ranks the previous search's list of every slot for the slot's new
// query. The list (k entries, positions) holds every point within
// sqrt(bound) of the anchor, so a point outside it is at least
// sqrt(bound) - |r - anchor| from the new query r (triangle inequality); when
// the new kfit-th distance is below that, the kfit nearest are in the list
// and the re-ranked list is final. Other slots are flagged for a fresh search.
__global__ __launch_bounds__(256) void k_knn_refresh(GridView g, QueryView qv, int32_t k,
                                                     int32_t kfit, double support_r_h,
                                                     int32_t *__restrict__ nbr,
                                                     uint8_t *__restrict__ support,
                                                     double *__restrict__ anchor,
                                                     uint8_t *__restrict__ slot_flag,
                                                     bool pending_only,
                                                     int32_t *__restrict__ out_nbr,
                                                     double *__restrict__ out_keys) {
  __shared__ WaveLds lds[4];
  const int lane = threadIdx.x & 63;
  WaveLds &L = lds[threadIdx.x >> 6];
  const int64_t nchunks = (qv.n + kChunk - 1) / kChunk;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  for (int64_t task = blk * 4 + (threadIdx.x >> 6); task < nchunks;
       task += (int64_t)gridDim.x * 4) {
    const int64_t p0 = task * kChunk;
    const int64_t pend = min(p0 + kChunk, qv.n);
    // the chunk's slots left by the lane pass (one flag load per lane)
    uint64_t todo = ~0ull;
    if (pending_only) {
      todo = __ballot(p0 + lane < pend && slot_flag[p0 + lane] == 2);
      if (todo == 0) continue;
    }
    // lane j holds slot p0 + j's query index, query and anchor (one round
    // trip for the chunk; each slot then reads them across the lanes)
    int32_t lqi = 0;
    double lr[3] = {0.0, 0.0, 0.0}, lan[4] = {0.0, 0.0, 0.0, -1.0};
    if (p0 + lane < pend && ((todo >> lane) & 1)) {
      const int64_t pl = p0 + lane;
      lqi = qv.aligned ? __float_as_int(g.pts[pl].w) : (int32_t)ordered_query(qv, pl);
      load_slot_query(g, qv, pl, lqi, lr);
#pragma unroll
      for (int c = 0; c < 4; ++c) lan[c] = anchor[4 * pl + c];
    }
    // the list row of the next slot to refresh, and its points, are loaded
    // while the current one is ranked
    auto next_slot = [&](int64_t from) {
      const uint64_t rest = from - p0 < 64 ? todo & (~0ull << (from - p0)) : 0ull;
      return rest ? p0 + (int64_t)__builtin_ctzll(rest) : pend;
    };
    int64_t pn = next_slot(p0);
    int32_t pos_n = -1;
    float4 P_n = make_float4(0.f, 0.f, 0.f, 0.f);
    if (pn < pend) {
      pos_n = lane < k ? nbr[(pn >> 6) * 64 * k + lane * 64 + (pn & 63)] : -1;
      const bool hv = pos_n >= 0 && (int64_t)pos_n < g.n_points;
      P_n = g.pts[hv ? pos_n : 0];
    }
    for (int64_t p = pn; p < pend; p = pn) {
      const int32_t pos_c = pos_n;
      const float4 P_c = P_n;
      pn = next_slot(p + 1);
      if (pn < pend) {
        pos_n = lane < k ? nbr[(pn >> 6) * 64 * k + lane * 64 + (pn & 63)] : -1;
        const bool hv = pos_n >= 0 && (int64_t)pos_n < g.n_points;
        P_n = g.pts[hv ? pos_n : 0];
      }
      const int jl = (int)(p - p0);
      const int64_t qi = __builtin_amdgcn_readlane(lqi, jl);
      const double r[3] = {readlane_f64(lr[0], jl), readlane_f64(lr[1], jl),
                           readlane_f64(lr[2], jl)};
      const bool finite = isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]);
      const double an[4] = {readlane_f64(lan[0], jl), readlane_f64(lan[1], jl),
                            readlane_f64(lan[2], jl), readlane_f64(lan[3], jl)};
      const double bound = an[3];
      int32_t *row = nbr + (p >> 6) * 64 * k + (p & 63);
      if (!finite) {
        if (lane < k) row[lane * 64] = -1;
        if (lane == 0) {
          support[p] = 0;
          slot_flag[p] = 0;
        }
        if (lane < kfit) {
          if (out_nbr) out_nbr[out_index(qv, p, qi) * kfit + lane] = -1;
          if (out_keys) out_keys[out_index(qv, p, qi) * kfit + lane] = bitsd(0x7ff8000000000000ull);
        }
        continue;
      }
      const int32_t pos = pos_c;
      const bool have = pos >= 0 && (int64_t)pos < g.n_points;
      const float4 P = P_c;
      uint64_t mk = have ? dbits(canon_key((double)P.x, (double)P.y, (double)P.z, r[0], r[1], r[2]))
                         : kEmptyKey;
      int32_t mi = have ? __float_as_int(P.w) : 0x7fffffff;
      int32_t mp = have ? pos : -1;
      const uint64_t vmask = __ballot(have);
      const uint32_t nvalid = popc(vmask);
      uint64_t kth, klast;
      if (!out_nbr && !out_keys && vmask == (nvalid == 64 ? ~0ull : (1ull << nvalid) - 1)) {
        // the list's entries lead (as the search writes them): split at kfit
        klast = partition_lanes(mk, mi, mp, (int)nvalid, kfit, L, lane);
        kth = wave_max_u64(lane < kfit && have ? mk : 0ull);
      } else {
        // sorted for the caller (or entries out of place)
        sort_lanes(mk, mi, mp, lane);
        kth = readlane_u64(mk, kfit - 1);
        klast = readlane_u64(mk, k - 1);
      }
      // certification (bound < 0: no usable list; +inf: the list is the cloud)
      bool ok = bound >= 0.0 && nvalid >= (uint32_t)kfit;
      if (ok && !isinf(bound)) {
        const double dx = r[0] - an[0], dy = r[1] - an[1], dz = r[2] - an[2];
        const double delta = sqrt(dx * dx + dy * dy + dz * dz) * (1.0 + 0x1p-40);
        const double reach = sqrt(bound) * (1.0 - 0x1p-40) - delta;
        ok = reach > 0.0 && bitsd(kth) < reach * reach * (1.0 - 0x1p-40);
      }
      if (ok) {
        const double rad = support_r_h * g.clouds[qv.qcloud ? qv.qcloud[qi] : 0].h;
        const double rad2 = rad * rad;
        const uint32_t m = popc(__ballot(lane < kfit && bitsd(mk) <= rad2));
        if (lane < k) row[lane * 64] = mp;
        if (lane < kfit) {
          if (out_nbr) out_nbr[out_index(qv, p, qi) * kfit + lane] = mi;
          if (out_keys) out_keys[out_index(qv, p, qi) * kfit + lane] = bitsd(mk);
        }
        if (lane == 0) support[p] = (uint8_t)m;
      }
      if (lane == 0) {
        slot_flag[p] = ok ? 0 : 1;
        // a slot left to the fresh search keeps, in place of its bound, the
        // squared distance of the list's farthest entry from the new query:
        // its k nearest lie within it, which steers the search's block
        if (!ok) anchor[4 * p + 3] = nvalid == (uint32_t)k ? bitsd(klast) : 0.0;
      }
    }
  }
}

__global__ void k_fill_cloud_ids(const int64_t *__restrict__ offsets, int32_t n_clouds, int64_t n,
                                 int32_t *__restrict__ qcloud) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int lo = 0, hi = n_clouds;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offsets[mid] <= i) lo = mid; else hi = mid;
  }
  qcloud[i] = lo;
}

}  // namespace

hipError_t launch_knn(const GridView &g, const QueryView &qv, int32_t k, int32_t kfit,
                      double support_r_h, bool refresh, int32_t *nbr, uint8_t *support,
                      double *anchor, uint8_t *flag, int32_t *out_nbr, double *out_keys,
                      hipStream_t s) {
  if (qv.n == 0) return hipSuccess;
  const int64_t tasks = (qv.n + kChunk - 1) / kChunk;
  int64_t blocks = (tasks + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > 65536) blocks = 65536;
  // launches that search or re-rank only the slots a refresh left take one
  // resident grid (4 blocks per CU) looping over the chunks: with a block
  // per chunk, the many chunks without such slots end at once and the
  // dispatch of their blocks, not the work, sets the pace
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  const int64_t sparse_blocks = std::min<int64_t>(blocks, 4 * (int64_t)cus);
  if (refresh) {
    // lists that need no re-ranking are settled one lane per slot; sorted
    // output for the caller takes the re-ranking path for every slot
    const bool lane_pass = !out_nbr && !out_keys;
    if (lane_pass)
      hipLaunchKernelGGL(k_knn_refresh_lane, dim3((unsigned)((qv.n + 255) / 256)), dim3(256), 0,
                         s, g, qv, k, kfit, support_r_h, nbr, support, anchor, flag);
    hipLaunchKernelGGL(k_knn_refresh, dim3((unsigned)(lane_pass ? sparse_blocks : blocks)),
                       dim3(256), 0, s, g, qv, k, kfit, support_r_h, nbr, support, anchor, flag,
                       lane_pass, out_nbr, out_keys);
  }
  const bool own = !refresh && !out_nbr && !out_keys;
  if (own && k == kfit)
    hipLaunchKernelGGL(k_knn<kPlain>, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, s, g,
                       qv, k, kfit, support_r_h, nbr, support, anchor, nullptr, nullptr, nullptr);
  else if (own)
    hipLaunchKernelGGL(k_knn<kExtra>, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, s, g,
                       qv, k, kfit, support_r_h, nbr, support, anchor, nullptr, nullptr, nullptr);
  else if (refresh && !out_nbr && !out_keys)
    hipLaunchKernelGGL(k_knn<kFlagged>, dim3((unsigned)sparse_blocks), dim3(64 * kWavesPerBlock), 0, s,
                       g, qv, k, kfit, support_r_h, nbr, support, anchor, flag, nullptr, nullptr);
  else
    hipLaunchKernelGGL(k_knn<kAny>, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, s, g,
                       qv, k, kfit, support_r_h, nbr, support, anchor, refresh ? flag : nullptr,
                       out_nbr, out_keys);
  return hipGetLastError();
}

hipError_t launch_fill_cloud_ids(const int64_t *offsets_dev, int32_t n_clouds, int64_t n,
                                 int32_t *qcloud, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_cloud_ids, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     offsets_dev, n_clouds, n, qcloud);
  return hipGetLastError();
}

}  // namespace mls
