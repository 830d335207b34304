// ball.hip -- the MLS projection over the paper's radius-R neighbourhood
// without a count cap (Section 1.4: the points within R of r; Section 3.3:
// fewer than 3 of them make the point an outlier), one wavefront per query.
//
// The ball is every cloud point whose canonical FP64 key to r is at most R^2
// (R = support_radius_h * h), however many there are. The wave stages the
// grid cells that cover the box [r - R, r + R] at the finest level where it
// spans at most 5 cells per axis (their ranges in LDS), and its lanes walk
// the cells' points: each point's key decides membership, and the members'
// weighted moments are summed per lane (FP32 compensated or FP64, as in the
// fit kernel) and then across the wave in FP64. The per-query algebra (plane,
// frame, quadratic fit, output, geometry) is the fit kernel's. A box that no
// level covers with 5 cells per axis (R beyond the coarsest cells) is walked
// as the whole cloud.
#include "mls_fit.h"

namespace mls {
namespace {

constexpr int kBallWaves = 4;
constexpr int kBallSpan = 5;    // cells per axis of a staged box
constexpr int kBallCells = 128; // >= kBallSpan^3

struct alignas(16) BallLds {
  uint32_t cstart[kBallCells];
  uint32_t cexcl[kBallCells];  // exclusive prefix of the counts; padding ~0u
};

__device__ __forceinline__ double xor_lane_f64(double v, int off) {
  const long long b = __double_as_longlong(v);
  const int lo = __shfl_xor((int)(b & 0xffffffff), off);
  const int hi = __shfl_xor((int)(b >> 32), off);
  return __longlong_as_double(((long long)hi << 32) | (long long)(uint32_t)lo);
}

// Sum over the wave by a butterfly: every lane ends with the same value (an
// addition and its mirror are the same IEEE operation).
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += xor_lane_f64(v, off);
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off);
  return v;
}

// Largest staged cell c with cexcl[c] <= ci.
__device__ __forceinline__ int32_t ball_cand_pos(const BallLds &L, int32_t ci) {
  int lo = 0;
#pragma unroll
  for (int step = kBallCells / 2; step > 0; step >>= 1)
    lo = (L.cexcl[lo + step] <= (uint32_t)ci) ? lo + step : lo;
  return (int32_t)L.cstart[lo] + (ci - (int32_t)L.cexcl[lo]);
}

// Stages the level-`lev` cells [lo, hi] (at most kBallCells) of `cloud`;
// returns the point count.
__device__ int32_t stage_box(const GridView &g, int cloud, const int32_t lo[3],
                             const int32_t hi[3], int lev, BallLds &L, int lane) {
  const int32_t nx = hi[0] - lo[0] + 1, ny = hi[1] - lo[1] + 1, nz = hi[2] - lo[2] + 1;
  const int32_t total = nx * ny * nz;
  uint32_t base = 0;
  // the previous query's reads of the ranges are complete before they are
  // overwritten
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int32_t t0 = 0; t0 < kBallCells; t0 += 64) {
    const int32_t t = t0 + lane;
    int2 rc = make_int2(0, 0);
    if (t < total) {
      const int32_t x = lo[0] + t % nx, y = lo[1] + (t / nx) % ny, z = lo[2] + t / (nx * ny);
      rc = lookup_cell(g, level_cell_key(cloud, x, y, z, g.morton_bits, lev));
    }
    // inclusive scan of the counts over the lanes
    uint32_t incl = (uint32_t)rc.y;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t o = (uint32_t)__shfl_up((int)incl, off);
      incl += lane >= off ? o : 0u;
    }
    L.cstart[t] = (uint32_t)rc.x;
    // empty cells get an excl equal to the next cell's, so the search skips them
    L.cexcl[t] = t < total ? base + incl - (uint32_t)rc.y : ~0u;
    base += (uint32_t)__shfl((int)incl, 63);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return (int32_t)base;
}

__device__ __forceinline__ void store_geometry(void *normals, void *curv, int is_f64, int64_t qi,
                                               const double N[3], double H, double K) {
  if (normals) store_vec(normals, is_f64, qi, N);
  if (curv) {
    if (is_f64) {
      double *d = (double *)curv + 2 * qi;
      d[0] = H; d[1] = K;
    } else {
      float *f = (float *)curv + 2 * qi;
      f[0] = (float)H; f[1] = (float)K;
    }
  }
}

template <bool kF32>
__global__ __launch_bounds__(64 * kBallWaves) void k_ball(GridView g, QueryView qv,
                                                          double support_r_h, int32_t min_support,
                                                          void *__restrict__ out,
                                                          uint8_t *__restrict__ status,
                                                          void *__restrict__ out_normals,
                                                          void *__restrict__ out_curv) {
  __shared__ BallLds lds[kBallWaves];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  BallLds &L = lds[wv];
  using T = Real<kF32>;
  const double nanv = __longlong_as_double(0x7ff8000000000000ll);
  const int64_t first = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBallWaves + wv;
  for (int64_t p = first; p < qv.n; p += (int64_t)gridDim.x * kBallWaves) {
    const int64_t qi = __builtin_amdgcn_readfirstlane((int)query_of_slot(g, qv, p));
    const int64_t qo = out_index(qv, p, qi);  // where the results go
    double r[3];
    load_slot_query(g, qv, p, qi, r);
    const bool lead = lane == 0;
    if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]))) {
      const double o[3] = {nanv, nanv, nanv};
      if (lead) {
        store_vec(out, qv.is_f64, qo, o);
        status[qo] = MLS_PT_NONFINITE;
        store_geometry(out_normals, out_curv, qv.is_f64, qo, o, nanv, nanv);
      }
      continue;
    }
    const int cloud = qv.qcloud ? qv.qcloud[qi] : 0;
    const CloudDev &cd = g.clouds[cloud];
    const double h = cd.h;
    const double R = support_r_h * h;
    const double R2 = R * R;
    // the finest level at which [r - R, r + R] spans at most kBallSpan cells
    // per axis (clamped to the grid)
    int lev = -1;
    int32_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    const int nlev = levels_of(g);
#pragma clang loop vectorize(disable) interleave(disable)
    for (int l = 0; l < nlev && lev < 0 && cd.send > cd.sbegin; ++l) {
      const double icell = ldexp(cd.inv_cell, -l);
      bool fits = true;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int32_t dims = ((cd.dims[a] - 1) >> l) + 1;
        double a0 = floor((r[a] - R - cd.origin[a]) * icell);
        double a1 = floor((r[a] + R - cd.origin[a]) * icell);
        a0 = fmin(fmax(a0, 0.0), (double)(dims - 1));
        a1 = fmin(fmax(a1, 0.0), (double)(dims - 1));
        lo[a] = (int32_t)a0;
        hi[a] = (int32_t)a1;
        fits = fits && (hi[a] - lo[a] + 1) <= kBallSpan;
      }
      if (fits) lev = l;
    }
    int32_t ncand;
    bool brute = false;
    if (cd.send <= cd.sbegin) {
      ncand = 0;
    } else if (lev >= 0) {
      ncand = stage_box(g, cloud, lo, hi, lev, L, lane);
    } else {
      // R beyond the coarsest cells: the whole cloud
      brute = true;
      ncand = (int32_t)(cd.send - cd.sbegin);
    }
    const Rel<kF32> rel(r, 1.0 / h);
    // pass 1: membership, support count and the 10 moments (weights at r)
    Acc<kF32, 10> A;
    A.zero();
    uint32_t m_lane = 0;
    int folded = 0;
    for (int32_t c = lane; c < ncand; c += 64) {
      int32_t pos = brute ? (int32_t)(cd.sbegin + c) : ball_cand_pos(L, c);
      pos = (pos >= 0 && (int64_t)pos < g.n_points) ? pos : 0;
      const float4 P = g.pts[pos];
      const double key = canon_key((double)P.x, (double)P.y, (double)P.z, r[0], r[1], r[2]);
      if (key <= R2) {
        ++m_lane;
        T dx, dy, dz;
        rel.d(P, dx, dy, dz);
        const T w = wexp(-(dx * dx + dy * dy + dz * dz));
        const T wx = w * dx, wy = w * dy, wz = w * dz;
        A.blk[0] += w;
        A.blk[1] += wx; A.blk[2] += wy; A.blk[3] += wz;
        A.blk[4] += wx * dx; A.blk[5] += wx * dy; A.blk[6] += wx * dz;
        A.blk[7] += wy * dy; A.blk[8] += wy * dz; A.blk[9] += wz * dz;
        if (++folded == kBatch) { A.fold(); folded = 0; }
      }
    }
    A.fold();
    const uint32_t m = wave_sum_u32(m_lane);
    if ((int)m < min_support) {
      if (lead) {
        store_vec(out, qv.is_f64, qo, r);
        status[qo] = MLS_PT_OUTLIER;
        const double o[3] = {nanv, nanv, nanv};
        store_geometry(out_normals, out_curv, qv.is_f64, qo, o, nanv, nanv);
      }
      continue;
    }
    double S0 = wave_sum_f64(A.value(0)), S1[3], S2[6];
    for (int a = 0; a < 3; ++a) S1[a] = wave_sum_f64(A.value(1 + a));
    for (int a = 0; a < 6; ++a) S2[a] = wave_sum_f64(A.value(4 + a));
    const PlaneFit pf = plane_from_moments(S0, S1, S2, r, h);
    // pass 2: the 21 sums of the quadratic fit, weights at q
    const FrameT<kF32> fr(pf);
    Acc<kF32, 21> B;
    B.zero();
    folded = 0;
    for (int32_t c = lane; c < ncand; c += 64) {
      int32_t pos = brute ? (int32_t)(cd.sbegin + c) : ball_cand_pos(L, c);
      pos = (pos >= 0 && (int64_t)pos < g.n_points) ? pos : 0;
      const float4 P = g.pts[pos];
      const double key = canon_key((double)P.x, (double)P.y, (double)P.z, r[0], r[1], r[2]);
      if (key <= R2) {
        T dx, dy, dz;
        rel.d(P, dx, dy, dz);
        const T e0 = dx - fr.tn[0], e1 = dy - fr.tn[1], e2 = dz - fr.tn[2];
        const T x = fr.u[0] * e0 + fr.u[1] * e1 + fr.u[2] * e2;
        const T y = fr.v[0] * e0 + fr.v[1] * e1 + fr.v[2] * e2;
        const T f = fr.n[0] * e0 + fr.n[1] * e1 + fr.n[2] * e2;
        const T w = wexp(-(e0 * e0 + e1 * e1 + e2 * e2));
        const T xx = x * x, xy = x * y, yy = y * y;
        const T wx = w * x, wy = w * y, wxx = w * xx, wxy = w * xy, wyy = w * yy;
        B.blk[0] += w; B.blk[1] += wx; B.blk[2] += wy;
        B.blk[3] += wxx; B.blk[4] += wxy; B.blk[5] += wyy;
        B.blk[6] += wxx * x; B.blk[7] += wxx * y; B.blk[8] += wyy * x; B.blk[9] += wyy * y;
        B.blk[10] += wxx * xx; B.blk[11] += wxx * xy; B.blk[12] += wxx * yy;
        B.blk[13] += wyy * xy; B.blk[14] += wyy * yy;
        B.blk[15] += w * f; B.blk[16] += wx * f; B.blk[17] += wy * f;
        B.blk[18] += wxx * f; B.blk[19] += wxy * f; B.blk[20] += wyy * f;
        if (++folded == kBatch) { B.fold(); folded = 0; }
      }
    }
    B.fold();
    QuadSums qs;
    for (int i = 0; i < 15; ++i) qs.s[i] = wave_sum_f64(B.value(i));
    for (int i = 0; i < 6; ++i) qs.b[i] = wave_sum_f64(B.value(15 + i));
    double a[6];
    const bool full = (m >= 6) && quad_solve(qs, 1e-12, a);
    double o[3];
    uint8_t st;
    if (full) {
      const double ha = h * a[0];
      for (int c = 0; c < 3; ++c) o[c] = pf.q[c] + ha * pf.n[c];
      st = MLS_PT_OK;
    } else {
      for (int c = 0; c < 3; ++c) o[c] = pf.q[c];
      st = MLS_PT_PLANE_ONLY;
    }
    if (lead) {
      store_vec(out, qv.is_f64, qo, o);
      status[qo] = st | pf.flags;
      if (out_normals || out_curv) {
        double N[3] = {pf.n[0], pf.n[1], pf.n[2]};
        double H = nanv, K = nanv;
        if (full) {
          for (int c = 0; c < 3; ++c) N[c] = pf.n[c] - a[1] * pf.u[c] - a[2] * pf.v[c];
          const double nn = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
          for (int c = 0; c < 3; ++c) N[c] /= nn;
          const double fx = a[1], fy = a[2];
          const double fxx = 2.0 * a[3] / h, fxy = a[4] / h, fyy = 2.0 * a[5] / h;
          const double W = 1.0 + fx * fx + fy * fy;
          H = ((1.0 + fy * fy) * fxx - 2.0 * fx * fy * fxy + (1.0 + fx * fx) * fyy) /
              (2.0 * W * sqrt(W));
          K = (fxx * fyy - fxy * fxy) / (W * W);
        }
        store_geometry(out_normals, out_curv, qv.is_f64, qo, N, H, K);
      }
    }
  }
}

}  // namespace

hipError_t launch_ball(const GridView &g, const QueryView &qv, int32_t precision,
                       int32_t min_support, double support_radius_h, void *out, uint8_t *status,
                       void *out_normals, void *out_curvatures, hipStream_t s) {
  if (qv.n == 0) return hipSuccess;
  int64_t blocks = (qv.n + kBallWaves - 1) / kBallWaves;
  if (blocks > 65536) blocks = 65536;
  if (precision == MLS_PREC_FP32_MOMENTS)
    hipLaunchKernelGGL(k_ball<true>, dim3((unsigned)blocks), dim3(64 * kBallWaves), 0, s, g, qv,
                       support_radius_h, min_support, out, status, out_normals, out_curvatures);
  else
    hipLaunchKernelGGL(k_ball<false>, dim3((unsigned)blocks), dim3(64 * kBallWaves), 0, s, g, qv,
                       support_radius_h, min_support, out, status, out_normals, out_curvatures);
  return hipGetLastError();
}

}  // namespace mls
