// knn.hip -- exact k-nearest-neighbour search on the uniform grid.
//
// One wavefront per query; lanes range over candidate points. The k-nearest
// set is defined on canonical FP64 keys
//     key = ((dx*dx + dy*dy) + dz*dz),  d = p - r,
// each operation a binary64 round-to-nearest with no fused multiply-add, and
// ties go to the smaller original index, so the set is unique and equal to a
// brute-force search over the whole cloud. Keys of non-negative doubles order
// like their bit patterns, so selection works on uint64.
//
// Search: the 3x3x3 block of cells around the query's cell first, then
// shells of growing Chebyshev radius L. After each round the distance beta
// from the query to the boundary of the visited box (minus a margin that
// covers the rounding of the cell assignment) bounds every unvisited point
// from below; the search stops when the k-th key is strictly below beta^2.
// Beyond kMaxRing rings the cloud is scanned exhaustively. The running top-k
// lives in one register slot per lane (lane j holds entry j); each batch of
// new candidates is merged by finding the k-th smallest (key, index) pair with
// a ballot/popcount bisection and compacting the survivors through LDS.
#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kSlots = 4;      // slot 0 = running top-k, slots 1..3 = new candidates
constexpr int kNew = (kSlots - 1) * 64;
constexpr int kMaxRing = 12;

struct alignas(16) WaveLds {
  uint32_t cstart[64];
  uint32_t cexcl[65];
  uint32_t pad[3];
  uint64_t ck[64];
  int32_t cpos[64];
  int32_t cidx[64];
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Canonical squared distance; contraction must stay off so that the rounding
// sequence is exactly sub, mul, mul, mul, add, add.
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

__device__ __forceinline__ uint64_t dbits(double d) { return (uint64_t)__double_as_longlong(d); }

__device__ __forceinline__ bool pair_lt(uint64_t ka, int32_t ia, uint64_t kb, int32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

__device__ __forceinline__ uint32_t popc(uint64_t m) { return (uint32_t)__popcll(m); }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  return (uint64_t)__shfl_xor((long long)v, m);
}

struct Slots {
  uint64_t key[kSlots];
  int32_t pos[kSlots];
  int32_t idx[kSlots];
};

__device__ __forceinline__ uint32_t count_lt(const Slots &s, uint64_t x) {
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < kSlots; ++i) c += popc(__ballot(s.key[i] < x));
  return c;
}

// Merge the new candidates (slots 1..) into the running top-k (slot 0,
// lanes < ntop). Invalid entries carry key ~0. On return slot 0 holds
// min(k, total) entries and ntop/kmax/imax describe it.
__device__ void merge(Slots &s, int &ntop, int k, uint64_t &kmax, int32_t &imax, WaveLds &L,
                      int lane) {
  const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t total = 0;
#pragma unroll
  for (int i = 0; i < kSlots; ++i) total += popc(__ballot(s.key[i] != kEmptyKey));
  bool keep[kSlots];
  if ((int)total <= k) {
#pragma unroll
    for (int i = 0; i < kSlots; ++i) keep[i] = s.key[i] != kEmptyKey;
  } else {
    // k-th smallest key value K: count_lt(K) < k <= count_lt(K + 1)
    uint64_t mx = 0;
#pragma unroll
    for (int i = 0; i < kSlots; ++i)
      if (s.key[i] != kEmptyKey && s.key[i] > mx) mx = s.key[i];
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t o = shfl_xor_u64(mx, off);
      mx = o > mx ? o : mx;
    }
    uint64_t lo = 0, hi = mx + 1;
    uint32_t clo = 0, chi = total;
    while (hi - lo > 1 && chi - clo > 1) {
      const uint64_t mid = lo + ((hi - lo) >> 1);
      const uint32_t c = count_lt(s, mid);
      if ((int)c < k) { lo = mid; clo = c; } else { hi = mid; chi = c; }
    }
    uint64_t K = lo;
    if (hi - lo > 1) {
      // exactly one entry in [lo, hi): it is the k-th
      uint64_t found = 0;
#pragma unroll
      for (int i = 0; i < kSlots; ++i)
        if (s.key[i] >= lo && s.key[i] < hi) found = s.key[i];
      for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = shfl_xor_u64(found, off);
        found = o > found ? o : found;
      }
      K = found;
    }
    const uint32_t c_lt = count_lt(s, K);
    const uint32_t c_le = count_lt(s, K + 1);
    const uint32_t need = (uint32_t)k - c_lt;  // entries with key == K to keep
    if (c_le - c_lt == need) {
#pragma unroll
      for (int i = 0; i < kSlots; ++i) keep[i] = s.key[i] <= K;
    } else {
      // ties at K: keep the `need` smallest original indices
      int64_t ilo = -1, ihi = 0x7fffffff;  // count(idx <= ilo) < need <= count(idx <= ihi)
      while (ihi - ilo > 1) {
        const int64_t mid = ilo + ((ihi - ilo) >> 1);
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < kSlots; ++i) c += popc(__ballot(s.key[i] == K && s.idx[i] <= mid));
        if (c < need) ilo = mid; else ihi = mid;
      }
#pragma unroll
      for (int i = 0; i < kSlots; ++i)
        keep[i] = s.key[i] < K || (s.key[i] == K && s.idx[i] <= (int32_t)ihi);
    }
  }
  // compact kept entries into LDS, slot-major then lane order
  uint32_t base = 0;
#pragma unroll
  for (int i = 0; i < kSlots; ++i) {
    const uint64_t m = __ballot(keep[i]);
    if (keep[i]) {
      const uint32_t o = base + popc(m & lt_mask);
      L.ck[o] = s.key[i];
      L.cpos[o] = s.pos[i];
      L.cidx[o] = s.idx[i];
    }
    base += popc(m);
  }
  wave_sync();
  ntop = (int)base;
  {
    const bool have = lane < ntop;
    const uint64_t ck = L.ck[lane];
    const int32_t cp = L.cpos[lane], ci = L.cidx[lane];
    s.key[0] = have ? ck : kEmptyKey;
    s.pos[0] = have ? cp : 0;
    s.idx[0] = have ? ci : 0x7fffffff;
  }
  wave_sync();
#pragma unroll
  for (int i = 1; i < kSlots; ++i) s.key[i] = kEmptyKey;
  if (ntop == k) {
    uint64_t mk = lane < ntop ? s.key[0] : 0;
    int32_t mi = lane < ntop ? s.idx[0] : -1;
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t ok = shfl_xor_u64(mk, off);
      const int32_t oi = __shfl_xor(mi, off);
      const bool t = pair_lt(mk, mi, ok, oi);
      mk = t ? ok : mk;
      mi = t ? oi : mi;
    }
    kmax = mk;
    imax = mi;
  }
}

// Load candidate `ci` (an index into the batch's concatenated cell ranges)
// into slot `sl` if it can enter the top-k.
__device__ __forceinline__ void load_candidate(const GridView &g, const WaveLds &L, int64_t ci,
                                               int64_t total, bool from_cells, int64_t range_base,
                                               double rx, double ry, double rz, int ntop, int k,
                                               uint64_t kmax, int32_t imax, Slots &s, int sl) {
  s.key[sl] = kEmptyKey;
  if (ci >= total) return;
  int64_t pos;
  if (from_cells) {
    int lo = 0, hi = 64;  // largest c with cexcl[c] <= ci
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if ((int64_t)L.cexcl[mid] <= ci) lo = mid; else hi = mid;
    }
    pos = (int64_t)L.cstart[lo] + (ci - (int64_t)L.cexcl[lo]);
  } else {
    pos = range_base + ci;
  }
  if (pos < 0 || pos >= g.n_points) return;
  const float4 P = g.pts[pos];
  const uint64_t key = dbits(canon_key((double)P.x, (double)P.y, (double)P.z, rx, ry, rz));
  const int32_t idx = __float_as_int(P.w);
  // branch-free: position and index are written unconditionally and only the
  // key marks the entry valid
  const bool take = (ntop < k) || pair_lt(key, idx, kmax, imax);
  s.pos[sl] = (int32_t)pos;
  s.idx[sl] = idx;
  s.key[sl] = take ? key : kEmptyKey;
}

__global__ __launch_bounds__(64 * kWavesPerBlock) void k_knn(GridView g, QueryView qv, int32_t k,
                                                            double support_r_h,
                                                            int32_t *__restrict__ nbr,
                                                            uint8_t *__restrict__ support,
                                                            int32_t *__restrict__ out_nbr,
                                                            double *__restrict__ out_keys) {
  __shared__ WaveLds lds[kWavesPerBlock];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  WaveLds &L = lds[wv];
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t p = (int64_t)blockIdx.x * kWavesPerBlock + wv; p < qv.n; p += nwaves) {
    int64_t qi;
    if (qv.aligned) qi = __float_as_int(g.pts[p].w);
    else qi = qv.order ? qv.order[p] : p;
    qi = __builtin_amdgcn_readfirstlane((int)qi);
    double rx, ry, rz;
    if (qv.is_f64) {
      const double *q = (const double *)qv.q + 3 * qi;
      rx = q[0]; ry = q[1]; rz = q[2];
    } else {
      const float *q = (const float *)qv.q + 3 * qi;
      rx = q[0]; ry = q[1]; rz = q[2];
    }
    const int cloud = qv.qcloud ? qv.qcloud[qi] : 0;
    const CloudDev &cd = g.clouds[cloud];
    const bool finite = isfinite(rx) && isfinite(ry) && isfinite(rz);

    Slots s;
#pragma unroll
    for (int i = 0; i < kSlots; ++i) { s.key[i] = kEmptyKey; s.pos[i] = 0; s.idx[i] = 0x7fffffff; }
    int ntop = 0;
    uint64_t kmax = kEmptyKey;
    int32_t imax = 0x7fffffff;

    if (finite && cd.send > cd.sbegin) {
      const double r[3] = {rx, ry, rz};
      int64_t c0[3];
      int64_t lmin = 0;
      for (int a = 0; a < 3; ++a) {
        int64_t t = cell_coord(r[a], cd.origin[a], cd.inv_cell);
        t = t < -(1ll << 40) ? -(1ll << 40) : (t > (1ll << 40) ? (1ll << 40) : t);
        c0[a] = t;
        int64_t out_lo = -t, out_hi = t - (cd.dims[a] - 1);
        lmin = max(lmin, max(out_lo, out_hi));
      }
      bool brute = lmin > kMaxRing;
      int L0 = (int)(lmin < 1 ? 1 : lmin);
      bool done = false;
      for (int ring = L0; !done && !brute; ++ring) {
        // cells of this round: the whole box at the first round, a shell after
        const int w = 2 * ring + 1;
        const int64_t ncand_cells = (int64_t)w * w * w;
        for (int64_t t0 = 0; t0 < ncand_cells; t0 += 64) {
          const int64_t t = t0 + lane;
          int2 sc = make_int2(0, 0);
          if (t < ncand_cells) {
            const int dx = (int)(t % w) - ring;
            const int dy = (int)((t / w) % w) - ring;
            const int dz = (int)(t / ((int64_t)w * w)) - ring;
            const int cheb = max(abs(dx), max(abs(dy), abs(dz)));
            const int64_t cx = c0[0] + dx, cy = c0[1] + dy, cz = c0[2] + dz;
            const bool in_round = (ring == L0) || cheb == ring;
            if (in_round && cx >= 0 && cy >= 0 && cz >= 0 && cx < cd.dims[0] && cy < cd.dims[1] &&
                cz < cd.dims[2])
              sc = lookup_cell(g, cell_key(cloud, (int)cx, (int)cy, (int)cz, g.morton_bits));
          }
          // exclusive scan of counts over the wave
          uint32_t x = (uint32_t)sc.y;
          for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)x, off);
            if (lane >= off) x += y;
          }
          const uint32_t total = (uint32_t)__shfl((int)x, 63);
          if (total == 0) continue;
          L.cstart[lane] = (uint32_t)sc.x;
          L.cexcl[lane] = x - (uint32_t)sc.y;
          wave_sync();
          for (int64_t b0 = 0; b0 < total; b0 += kNew) {
#pragma unroll
            for (int sl = 1; sl < kSlots; ++sl)
              load_candidate(g, L, b0 + (sl - 1) * 64 + lane, total, true, 0, rx, ry, rz, ntop, k,
                             kmax, imax, s, sl);
            bool any = false;
#pragma unroll
            for (int sl = 1; sl < kSlots; ++sl) any |= __ballot(s.key[sl] != kEmptyKey) != 0ull;
            if (any) merge(s, ntop, k, kmax, imax, L, lane);
          }
          wave_sync();
        }
        // termination: k-th key strictly below the squared distance to the
        // unvisited region (minus the cell-assignment margin)
        double beta = __longlong_as_double(0x7ff0000000000000ll);  // +inf
        for (int a = 0; a < 3; ++a) {
          const int64_t lo_cell = c0[a] - ring, hi_cell = c0[a] + ring;
          if (lo_cell > 0) beta = fmin(beta, r[a] - (cd.origin[a] + (double)lo_cell * cd.cell));
          if (hi_cell < cd.dims[a] - 1)
            beta = fmin(beta, (cd.origin[a] + (double)(hi_cell + 1) * cd.cell) - r[a]);
        }
        if (isinf(beta)) {
          done = true;  // every cell of the cloud visited
        } else {
          beta -= cd.cell * 0x1p-20;
          if (ntop == k && beta > 0.0) {
            const double bound = beta * beta * (1.0 - 0x1p-40);
            if (__longlong_as_double((long long)kmax) < bound) done = true;
          }
          if (!done && ring >= kMaxRing) brute = true;
        }
      }
      if (brute) {
        // exhaustive scan of the cloud's sorted range
#pragma unroll
        for (int i = 0; i < kSlots; ++i) { s.key[i] = kEmptyKey; s.idx[i] = 0x7fffffff; }
        ntop = 0;
        kmax = kEmptyKey;
        imax = 0x7fffffff;
        const int64_t total = cd.send - cd.sbegin;
        for (int64_t b0 = 0; b0 < total; b0 += kNew) {
#pragma unroll
          for (int sl = 1; sl < kSlots; ++sl)
            load_candidate(g, L, b0 + (sl - 1) * 64 + lane, total, false, cd.sbegin, rx, ry, rz,
                           ntop, k, kmax, imax, s, sl);
          bool any = false;
#pragma unroll
          for (int sl = 1; sl < kSlots; ++sl) any |= __ballot(s.key[sl] != kEmptyKey) != 0ull;
          if (any) merge(s, ntop, k, kmax, imax, L, lane);
        }
      }
    }

    // ascending (key, index) order of the top-k: bitonic sort across lanes
    uint64_t mk = s.key[0];
    int32_t mi = s.idx[0], mp = s.pos[0];
    for (int size = 2; size <= 64; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        const uint64_t ok = shfl_xor_u64(mk, stride);
        const int32_t oi = __shfl_xor(mi, stride);
        const int32_t op = __shfl_xor(mp, stride);
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
    const double rad = support_r_h * cd.h;
    const double rad2 = rad * rad;
    const bool valid = lane < ntop;
    const uint32_t m = popc(__ballot(valid && __longlong_as_double((long long)mk) <= rad2));
    if (lane < k) {
      nbr[p * k + lane] = valid ? mp : 0;
      if (out_nbr) out_nbr[qi * k + lane] = valid ? mi : -1;
      if (out_keys)
        out_keys[qi * k + lane] = valid ? __longlong_as_double((long long)mk)
                                        : __longlong_as_double(0x7ff8000000000000ll);
    }
    if (lane == 0) support[p] = (uint8_t)((finite && ntop == k) ? m : 0);
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

hipError_t launch_knn(const GridView &g, const QueryView &qv, int32_t k, double support_r_h,
                      int32_t *nbr, uint8_t *support, int32_t *out_nbr, double *out_keys,
                      hipStream_t s) {
  if (qv.n == 0) return hipSuccess;
  int64_t blocks = (qv.n + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_knn, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, s, g, qv, k,
                     support_r_h, nbr, support, out_nbr, out_keys);
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
