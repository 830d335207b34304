// mls_fwd.hip -- forward MLS projection, one lane per query.
//
// For query r with its k neighbours (sorted positions from the neighbour
// search) and Gaussian width h:
//   pass 1  d_i = (p_i - r)/h, w_i = exp(-|d_i|^2); S0, S1 = sum w d,
//           S2 = sum w d d^T (10 sums)                       [Section 1.4, Eq. (1.1)]
//   plane   C = S2/S0 - mu mu^T, n = smallest eigenvector, q = r + h <n,mu> n
//   frame   u, v orthonormal on the plane                    [Section 1.4]
//   pass 2  e_i = d_i - <n,mu> n (= (p_i - q)/h), x = <u,e>, y = <v,e>,
//           f = <n,e>, w'_i = exp(-|e_i|^2); 15 monomial sums + 6 sums of f
//           phi (21 sums)                                    [Section 2.1]
//   fit     6x6 Cholesky with the pivot rule, a = M^-1 b
//   output  out = q + h a_0 n                                [Section 2.1, Algorithm 1]
// Outlier rule (Section 3.3): fewer than min_support list entries within
// support_radius_h * h (counted by the neighbour search) -> out = r.
//
// Precision: FP64 accumulates every moment in double. The FP32-moments
// variant forms d, e, weights and products in FP32 on the centred, h-scaled
// coordinates, sums them in blocks of 8 neighbours and folds every block sum
// into a compensated (hi, lo) FP32 pair with TwoSum; the eigen-solve and the
// Cholesky stay FP64 in both.
#include "mls_internal.h"
#include "mls_math.h"

namespace mls {
namespace {

constexpr int kBlock = 256;
constexpr int kChunk = 8;  // neighbours per compensated block

template <int N>
struct CompSum {  // N compensated FP32 accumulators
  float hi[N], lo[N], blk[N];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < N; ++i) { hi[i] = 0.f; lo[i] = 0.f; blk[i] = 0.f; }
  }
  __device__ __forceinline__ void fold() {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float s = hi[i] + blk[i];
      const float z = s - hi[i];
      const float e = (hi[i] - (s - z)) + (blk[i] - z);  // TwoSum error
      hi[i] = s;
      lo[i] += e;
      blk[i] = 0.f;
    }
  }
  __device__ __forceinline__ double value(int i) const { return (double)hi[i] + (double)lo[i]; }
};

__device__ __forceinline__ void load_query(const QueryView &qv, int64_t qi, double r[3]) {
  if (qv.is_f64) {
    const double *q = (const double *)qv.q + 3 * qi;
    r[0] = q[0]; r[1] = q[1]; r[2] = q[2];
  } else {
    const float *q = (const float *)qv.q + 3 * qi;
    r[0] = q[0]; r[1] = q[1]; r[2] = q[2];
  }
}

__device__ __forceinline__ void store_out(void *out, int is_f64, int64_t qi, const double o[3]) {
  if (is_f64) {
    double *d = (double *)out + 3 * qi;
    d[0] = o[0]; d[1] = o[1]; d[2] = o[2];
  } else {
    float *f = (float *)out + 3 * qi;
    f[0] = (float)o[0]; f[1] = (float)o[1]; f[2] = (float)o[2];
  }
}

// Plane from the pass-1 moments; fills n, q, t = <n, mu>, the frame and flags.
struct PlaneFit {
  double n[3], u[3], v[3], t, q[3];
  uint8_t flags;
};

__device__ __forceinline__ PlaneFit plane_from_moments(double S0, const double S1[3],
                                                       const double S2[6], const double r[3],
                                                       double h) {
  PlaneFit pf;
  const double i0 = 1.0 / S0;
  const double mu0 = S1[0] * i0, mu1 = S1[1] * i0, mu2 = S1[2] * i0;
  Sym3 C;
  C.a00 = S2[0] * i0 - mu0 * mu0;
  C.a01 = S2[1] * i0 - mu0 * mu1;
  C.a02 = S2[2] * i0 - mu0 * mu2;
  C.a11 = S2[3] * i0 - mu1 * mu1;
  C.a12 = S2[4] * i0 - mu1 * mu2;
  C.a22 = S2[5] * i0 - mu2 * mu2;
  const Eig3 e = smallest_eigenpair(C);
  pf.n[0] = e.n[0]; pf.n[1] = e.n[1]; pf.n[2] = e.n[2];
  pf.flags = (e.lam[1] - e.lam[0] < 1e-6 * e.lam[2]) ? (uint8_t)MLS_PT_FLAG_NORMAL_AMBIGUOUS : 0;
  pf.t = pf.n[0] * mu0 + pf.n[1] * mu1 + pf.n[2] * mu2;
  for (int a = 0; a < 3; ++a) pf.q[a] = r[a] + h * pf.t * pf.n[a];
  plane_frame(pf.n, pf.u, pf.v);
  return pf;
}

// neighbour positions come from the search kernel and are always in range;
// the clamp keeps a corrupted list from reading outside the sorted array
__device__ __forceinline__ int64_t clamp_pos(int32_t v, int64_t n) {
  return (v >= 0 && (int64_t)v < n) ? v : 0;
}

constexpr int kBatch = kChunk;  // neighbour coordinates fetched together

// Issues the loads of neighbours j0 .. j0 + kBatch - 1 (fewer at the end of
// the list) before any of them is used, so their latencies overlap.
__device__ __forceinline__ void load_batch(const GridView &g, const int32_t *nb, int j0, int k,
                                           float4 PB[kBatch]) {
  int32_t id[kBatch];
#pragma unroll
  for (int b = 0; b < kBatch; ++b) id[b] = (j0 + b < k) ? nb[(j0 + b) * 64] : 0;
#pragma unroll
  for (int b = 0; b < kBatch; ++b) PB[b] = g.pts[clamp_pos(id[b], g.n_points)];
}

template <bool kF32>
__global__ __launch_bounds__(kBlock) void k_mls_forward(GridView g, QueryView qv, int32_t k,
                                                        int32_t min_support,
                                                        const int32_t *__restrict__ nbr,
                                                        const uint8_t *__restrict__ support,
                                                        void *__restrict__ out,
                                                        uint8_t *__restrict__ status) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= qv.n) return;
  int64_t qi;
  if (qv.aligned) qi = __float_as_int(g.pts[p].w);
  else qi = qv.order ? qv.order[p] : p;
  double r[3];
  load_query(qv, qi, r);
  if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]))) {
    const double nanv = __longlong_as_double(0x7ff8000000000000ll);
    const double o[3] = {nanv, nanv, nanv};
    store_out(out, qv.is_f64, qi, o);
    status[qi] = MLS_PT_NONFINITE;
    return;
  }
  const int m = support[p];
  if (m < min_support) {
    store_out(out, qv.is_f64, qi, r);
    status[qi] = MLS_PT_OUTLIER;
    return;
  }
  const int cloud = qv.qcloud ? qv.qcloud[qi] : 0;
  const double h = g.clouds[cloud].h;
  const double ih = 1.0 / h;
  // neighbour j of query p: nb[j * 64] (tile layout of the search kernel)
  const int32_t *nb = nbr + (p >> 6) * 64 * k + (p & 63);

  // ---- pass 1 -------------------------------------------------------------
  double S0, S1[3], S2[6];
  if constexpr (!kF32) {
    S0 = 0.0;
    for (int a = 0; a < 3; ++a) S1[a] = 0.0;
    for (int a = 0; a < 6; ++a) S2[a] = 0.0;
    for (int j0 = 0; j0 < k; j0 += kBatch) {
      float4 PB[kBatch];
      load_batch(g, nb, j0, k, PB);
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
      if (j0 + b >= k) break;
      const float4 P = PB[b];
      const double dx = ((double)P.x - r[0]) * ih;
      const double dy = ((double)P.y - r[1]) * ih;
      const double dz = ((double)P.z - r[2]) * ih;
      const double w = exp(-(dx * dx + dy * dy + dz * dz));
      const double wx = w * dx, wy = w * dy, wz = w * dz;
      S0 += w;
      S1[0] += wx; S1[1] += wy; S1[2] += wz;
      S2[0] += wx * dx; S2[1] += wx * dy; S2[2] += wx * dz;
      S2[3] += wy * dy; S2[4] += wy * dz; S2[5] += wz * dz;
      }
    }
  } else {
    const float rx = (float)r[0], ry = (float)r[1], rz = (float)r[2];
    // the query may be FP64: keep its FP32 rounding residual in the difference
    const float ex = (float)(r[0] - (double)rx), ey = (float)(r[1] - (double)ry),
                ez = (float)(r[2] - (double)rz);
    const float ihf = (float)ih;
    CompSum<10> A;
    A.zero();
    for (int j0 = 0; j0 < k; j0 += kChunk) {
      float4 PB[kBatch];
      load_batch(g, nb, j0, k, PB);
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        if (j0 + b >= k) break;
        const float4 P = PB[b];
        const float dx = ((P.x - rx) - ex) * ihf;
        const float dy = ((P.y - ry) - ey) * ihf;
        const float dz = ((P.z - rz) - ez) * ihf;
        const float w = __expf(-(dx * dx + dy * dy + dz * dz));
        const float wx = w * dx, wy = w * dy, wz = w * dz;
        A.blk[0] += w;
        A.blk[1] += wx; A.blk[2] += wy; A.blk[3] += wz;
        A.blk[4] += wx * dx; A.blk[5] += wx * dy; A.blk[6] += wx * dz;
        A.blk[7] += wy * dy; A.blk[8] += wy * dz; A.blk[9] += wz * dz;
      }
      A.fold();
    }
    S0 = A.value(0);
    for (int a = 0; a < 3; ++a) S1[a] = A.value(1 + a);
    for (int a = 0; a < 6; ++a) S2[a] = A.value(4 + a);
  }

  const PlaneFit pf = plane_from_moments(S0, S1, S2, r, h);

  // ---- pass 2 -------------------------------------------------------------
  QuadSums qs;
  if constexpr (!kF32) {
    for (int i = 0; i < 15; ++i) qs.s[i] = 0.0;
    for (int i = 0; i < 6; ++i) qs.b[i] = 0.0;
    const double tn0 = pf.t * pf.n[0], tn1 = pf.t * pf.n[1], tn2 = pf.t * pf.n[2];
    for (int j0 = 0; j0 < k; j0 += kBatch) {
      float4 PB[kBatch];
      load_batch(g, nb, j0, k, PB);
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
      if (j0 + b >= k) break;
      const float4 P = PB[b];
      const double e0 = ((double)P.x - r[0]) * ih - tn0;
      const double e1 = ((double)P.y - r[1]) * ih - tn1;
      const double e2 = ((double)P.z - r[2]) * ih - tn2;
      const double x = pf.u[0] * e0 + pf.u[1] * e1 + pf.u[2] * e2;
      const double y = pf.v[0] * e0 + pf.v[1] * e1 + pf.v[2] * e2;
      const double f = pf.n[0] * e0 + pf.n[1] * e1 + pf.n[2] * e2;
      const double w = exp(-(e0 * e0 + e1 * e1 + e2 * e2));
      const double xx = x * x, xy = x * y, yy = y * y;
      const double wx = w * x, wy = w * y, wxx = w * xx, wxy = w * xy, wyy = w * yy;
      qs.s[0] += w; qs.s[1] += wx; qs.s[2] += wy;
      qs.s[3] += wxx; qs.s[4] += wxy; qs.s[5] += wyy;
      qs.s[6] += wxx * x; qs.s[7] += wxx * y; qs.s[8] += wyy * x; qs.s[9] += wyy * y;
      qs.s[10] += wxx * xx; qs.s[11] += wxx * xy; qs.s[12] += wxx * yy;
      qs.s[13] += wyy * xy; qs.s[14] += wyy * yy;
      qs.b[0] += w * f; qs.b[1] += wx * f; qs.b[2] += wy * f;
      qs.b[3] += wxx * f; qs.b[4] += wxy * f; qs.b[5] += wyy * f;
      }
    }
  } else {
    const float rx = (float)r[0], ry = (float)r[1], rz = (float)r[2];
    const float ex = (float)(r[0] - (double)rx), ey = (float)(r[1] - (double)ry),
                ez = (float)(r[2] - (double)rz);
    const float ihf = (float)ih;
    const float tn0 = (float)(pf.t * pf.n[0]), tn1 = (float)(pf.t * pf.n[1]),
                tn2 = (float)(pf.t * pf.n[2]);
    const float u0 = (float)pf.u[0], u1 = (float)pf.u[1], u2 = (float)pf.u[2];
    const float v0 = (float)pf.v[0], v1 = (float)pf.v[1], v2 = (float)pf.v[2];
    const float n0 = (float)pf.n[0], n1 = (float)pf.n[1], n2 = (float)pf.n[2];
    CompSum<21> A;
    A.zero();
    for (int j0 = 0; j0 < k; j0 += kChunk) {
      float4 PB[kBatch];
      load_batch(g, nb, j0, k, PB);
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        if (j0 + b >= k) break;
        const float4 P = PB[b];
        const float e0 = ((P.x - rx) - ex) * ihf - tn0;
        const float e1 = ((P.y - ry) - ey) * ihf - tn1;
        const float e2 = ((P.z - rz) - ez) * ihf - tn2;
        const float x = u0 * e0 + u1 * e1 + u2 * e2;
        const float y = v0 * e0 + v1 * e1 + v2 * e2;
        const float f = n0 * e0 + n1 * e1 + n2 * e2;
        const float w = __expf(-(e0 * e0 + e1 * e1 + e2 * e2));
        const float xx = x * x, xy = x * y, yy = y * y;
        const float wx = w * x, wy = w * y, wxx = w * xx, wxy = w * xy, wyy = w * yy;
        A.blk[0] += w; A.blk[1] += wx; A.blk[2] += wy;
        A.blk[3] += wxx; A.blk[4] += wxy; A.blk[5] += wyy;
        A.blk[6] += wxx * x; A.blk[7] += wxx * y; A.blk[8] += wyy * x; A.blk[9] += wyy * y;
        A.blk[10] += wxx * xx; A.blk[11] += wxx * xy; A.blk[12] += wxx * yy;
        A.blk[13] += wyy * xy; A.blk[14] += wyy * yy;
        A.blk[15] += w * f; A.blk[16] += wx * f; A.blk[17] += wy * f;
        A.blk[18] += wxx * f; A.blk[19] += wxy * f; A.blk[20] += wyy * f;
      }
      A.fold();
    }
    for (int i = 0; i < 15; ++i) qs.s[i] = A.value(i);
    for (int i = 0; i < 6; ++i) qs.b[i] = A.value(15 + i);
  }

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
  store_out(out, qv.is_f64, qi, o);
  status[qi] = st | pf.flags;
}

}  // namespace

hipError_t launch_mls_forward(const GridView &g, const QueryView &qv, int32_t k,
                              int32_t precision, int32_t min_support, const int32_t *nbr,
                              const uint8_t *support, void *out, uint8_t *status, hipStream_t s) {
  if (qv.n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((qv.n + kBlock - 1) / kBlock);
  if (precision == MLS_PREC_FP32_MOMENTS)
    hipLaunchKernelGGL(k_mls_forward<true>, dim3(blocks), dim3(kBlock), 0, s, g, qv, k,
                       min_support, nbr, support, out, status);
  else
    hipLaunchKernelGGL(k_mls_forward<false>, dim3(blocks), dim3(kBlock), 0, s, g, qv, k,
                       min_support, nbr, support, out, status);
  return hipGetLastError();
}

}  // namespace mls
