// mls_fit.h -- the per-neighbour passes of the MLS fit, shared by the forward
// kernel and the adjoint kernel so that the adjoint recomputes exactly the
// moments, plane, frame and quadratic fit of the forward pass.
//
// Both passes exist in two arithmetic variants selected by a template flag:
//   kF32 = false  every per-neighbour quantity and every sum in FP64;
//   kF32 = true   per-neighbour quantities in FP32 on the centred, h-scaled
//                 coordinates (the FP64 query's FP32 rounding residual kept
//                 in the difference), summed in blocks of kBatch neighbours,
//                 each block sum folded into a compensated (hi, lo) FP32 pair
//                 with TwoSum.
// The per-query algebra (eigen-solve, frame, Cholesky) is FP64 in both.
#pragma once

#include <type_traits>

#include "mls_internal.h"
#include "mls_math.h"

namespace mls {

constexpr int kBatch = 8;  // neighbours fetched together and summed per block

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

template <int N>
struct PlainSum {  // N FP64 accumulators (fold is a no-op)
  double blk[N];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < N; ++i) blk[i] = 0.0;
  }
  __device__ __forceinline__ void fold() {}
  __device__ __forceinline__ double value(int i) const { return blk[i]; }
};

template <bool kF32, int N>
using Acc = typename std::conditional<kF32, CompSum<N>, PlainSum<N>>::type;
template <bool kF32>
using Real = typename std::conditional<kF32, float, double>::type;

__device__ __forceinline__ float wexp(float x) { return __expf(x); }
__device__ __forceinline__ double wexp(double x) { return exp(x); }

// d = (p - r) / h in the pass's arithmetic.
template <bool kF32>
struct Rel;

template <>
struct Rel<true> {
  float rx, ry, rz, ex, ey, ez, ih;
  __device__ __forceinline__ Rel(const double r[3], double ihd) {
    rx = (float)r[0]; ry = (float)r[1]; rz = (float)r[2];
    // the query may be FP64: keep its FP32 rounding residual in the difference
    ex = (float)(r[0] - (double)rx);
    ey = (float)(r[1] - (double)ry);
    ez = (float)(r[2] - (double)rz);
    ih = (float)ihd;
  }
  __device__ __forceinline__ void d(const float4 &P, float &dx, float &dy, float &dz) const {
    dx = ((P.x - rx) - ex) * ih;
    dy = ((P.y - ry) - ey) * ih;
    dz = ((P.z - rz) - ez) * ih;
  }
};

template <>
struct Rel<false> {
  double r0, r1, r2, ih;
  __device__ __forceinline__ Rel(const double r[3], double ihd) {
    r0 = r[0]; r1 = r[1]; r2 = r[2];
    ih = ihd;
  }
  __device__ __forceinline__ void d(const float4 &P, double &dx, double &dy, double &dz) const {
    dx = ((double)P.x - r0) * ih;
    dy = ((double)P.y - r1) * ih;
    dz = ((double)P.z - r2) * ih;
  }
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

__device__ __forceinline__ void load_vec(const void *base, int is_f64, int64_t i, double v[3]) {
  if (is_f64) {
    const double *d = (const double *)base + 3 * i;
    v[0] = d[0]; v[1] = d[1]; v[2] = d[2];
  } else {
    const float *f = (const float *)base + 3 * i;
    v[0] = f[0]; v[1] = f[1]; v[2] = f[2];
  }
}

__device__ __forceinline__ void store_vec(void *out, int is_f64, int64_t i, const double o[3]) {
  if (is_f64) {
    double *d = (double *)out + 3 * i;
    d[0] = o[0]; d[1] = o[1]; d[2] = o[2];
  } else {
    float *f = (float *)out + 3 * i;
    f[0] = (float)o[0]; f[1] = (float)o[1]; f[2] = (float)o[2];
  }
}

// Query index of processing slot p (slot order = the order of the lists).
__device__ __forceinline__ int64_t query_of_slot(const GridView &g, const QueryView &qv,
                                                 int64_t p) {
  if (qv.aligned) return __float_as_int(g.pts[p].w);
  return ordered_query(qv, p);
}

// Plane of the pass-1 moments: the weighted covariance, its smallest
// eigenpair, t = <n, mu>, the plane origin q and the frame.
struct PlaneFit {
  double mu[3];
  Sym3 C;
  double lam[3];
  double n[3], u[3], v[3], t, q[3];
  uint8_t flags;
};

__device__ __forceinline__ PlaneFit plane_from_moments(double S0, const double S1[3],
                                                       const double S2[6], const double r[3],
                                                       double h) {
  PlaneFit pf;
  const double i0 = 1.0 / S0;
  pf.mu[0] = S1[0] * i0; pf.mu[1] = S1[1] * i0; pf.mu[2] = S1[2] * i0;
  const double mu0 = pf.mu[0], mu1 = pf.mu[1], mu2 = pf.mu[2];
  Sym3 &C = pf.C;
  C.a00 = S2[0] * i0 - mu0 * mu0;
  C.a01 = S2[1] * i0 - mu0 * mu1;
  C.a02 = S2[2] * i0 - mu0 * mu2;
  C.a11 = S2[3] * i0 - mu1 * mu1;
  C.a12 = S2[4] * i0 - mu1 * mu2;
  C.a22 = S2[5] * i0 - mu2 * mu2;
  const Eig3 e = smallest_eigenpair(C);
  for (int a = 0; a < 3; ++a) { pf.n[a] = e.n[a]; pf.lam[a] = e.lam[a]; }
  pf.flags = (e.lam[1] - e.lam[0] < 1e-6 * e.lam[2]) ? (uint8_t)MLS_PT_FLAG_NORMAL_AMBIGUOUS : 0;
  pf.t = pf.n[0] * mu0 + pf.n[1] * mu1 + pf.n[2] * mu2;
  for (int a = 0; a < 3; ++a) pf.q[a] = r[a] + h * pf.t * pf.n[a];
  plane_frame(pf.n, pf.u, pf.v);
  return pf;
}

// neighbour positions come from the search kernel (or the index conversion of
// caller lists) and are in range; the clamp keeps a corrupted list from
// reading outside the sorted array
__device__ __forceinline__ int64_t clamp_pos(int32_t v, int64_t n) {
  return (v >= 0 && (int64_t)v < n) ? v : 0;
}

// Issues the loads of neighbours j0 .. j0 + kBatch - 1 (fewer at the end of
// the list) before any of them is used, so their latencies overlap. nb points
// at entry 0 of the query's list; entry j is nb[j * 64] (tile layout).
__device__ __forceinline__ void load_batch(const GridView &g, const int32_t *nb, int j0, int k,
                                           float4 PB[kBatch], int32_t id[kBatch]) {
#pragma unroll
  for (int b = 0; b < kBatch; ++b) id[b] = (j0 + b < k) ? nb[(j0 + b) * 64] : 0;
#pragma unroll
  for (int b = 0; b < kBatch; ++b) PB[b] = g.pts[clamp_pos(id[b], g.n_points)];
}

__device__ __forceinline__ void load_batch(const GridView &g, const int32_t *nb, int j0, int k,
                                           float4 PB[kBatch]) {
  int32_t id[kBatch];
  load_batch(g, nb, j0, k, PB, id);
}

// Pass 1: S0 = sum w, S1 = sum w d, S2 = sum w d d^T (packed 00 01 02 11 12 22).
// With kSupport it also counts the list entries whose canonical FP64 key to r
// is at most rad2 (into *m) and clears *valid if an entry is not a position.
// With kMask, list entry j takes part only if bit j of mask is set.
template <bool kF32, bool kSupport = false, bool kMask = false>
__device__ __forceinline__ void pass1_moments(const GridView &g, const int32_t *nb, int k,
                                              const Rel<kF32> &rel, double &S0, double S1[3],
                                              double S2[6], const double *r = nullptr,
                                              double rad2 = 0.0, int *m = nullptr,
                                              bool *valid = nullptr, uint64_t mask = ~0ull) {
  using T = Real<kF32>;
  Acc<kF32, 10> A;
  A.zero();
  for (int j0 = 0; j0 < k; j0 += kBatch) {
    float4 PB[kBatch];
    int32_t id[kBatch];
    load_batch(g, nb, j0, k, PB, id);
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      if (j0 + b >= k) break;
      if constexpr (kSupport) {
        *valid = *valid && id[b] >= 0 && (int64_t)id[b] < g.n_points;
        const double key = canon_key((double)PB[b].x, (double)PB[b].y, (double)PB[b].z, r[0],
                                     r[1], r[2]);
        *m += key <= rad2 ? 1 : 0;
      }
      T dx, dy, dz;
      rel.d(PB[b], dx, dy, dz);
      T w = wexp(-(dx * dx + dy * dy + dz * dz));
      if constexpr (kMask) w = ((mask >> (j0 + b)) & 1ull) ? w : (T)0;
      const T wx = w * dx, wy = w * dy, wz = w * dz;
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

// The moments of pass 1 (about r) with the weights centred at q = r + h tn
// instead of r: w_i = exp(-|d_i - tn|^2), tn = t n in units of h (a step of
// the reference plane toward the plane whose weights sit at its own
// projection of r, Section 1.4).
template <bool kF32, bool kMask = false>
__device__ __forceinline__ void plane_moments_at(const GridView &g, const int32_t *nb, int k,
                                                 const Rel<kF32> &rel, const Real<kF32> tn[3],
                                                 double &S0, double S1[3], double S2[6],
                                                 uint64_t mask = ~0ull) {
  using T = Real<kF32>;
  Acc<kF32, 10> A;
  A.zero();
  for (int j0 = 0; j0 < k; j0 += kBatch) {
    float4 PB[kBatch];
    int32_t id[kBatch];
    load_batch(g, nb, j0, k, PB, id);
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      if (j0 + b >= k) break;
      T dx, dy, dz;
      rel.d(PB[b], dx, dy, dz);
      const T ex = dx - tn[0], ey = dy - tn[1], ez = dz - tn[2];
      T w = wexp(-(ex * ex + ey * ey + ez * ez));
      if constexpr (kMask) w = ((mask >> (j0 + b)) & 1ull) ? w : (T)0;
      const T wx = w * dx, wy = w * dy, wz = w * dz;
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

// The plane quantities of pass 2 in the pass's arithmetic.
template <bool kF32>
struct FrameT {
  Real<kF32> tn[3], u[3], v[3], n[3];
  __device__ __forceinline__ explicit FrameT(const PlaneFit &pf) {
    for (int a = 0; a < 3; ++a) {
      tn[a] = (Real<kF32>)(pf.t * pf.n[a]);
      u[a] = (Real<kF32>)pf.u[a];
      v[a] = (Real<kF32>)pf.v[a];
      n[a] = (Real<kF32>)pf.n[a];
    }
  }
};

// Pass 2: the 15 monomial sums of M and the 6 sums of b, weights at q.
template <bool kF32, bool kMask = false>
__device__ __forceinline__ void pass2_sums(const GridView &g, const int32_t *nb, int k,
                                           const Rel<kF32> &rel, const FrameT<kF32> &fr,
                                           QuadSums &qs, uint64_t mask = ~0ull) {
  using T = Real<kF32>;
  Acc<kF32, 21> A;
  A.zero();
  for (int j0 = 0; j0 < k; j0 += kBatch) {
    float4 PB[kBatch];
    load_batch(g, nb, j0, k, PB);
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      if (j0 + b >= k) break;
      T dx, dy, dz;
      rel.d(PB[b], dx, dy, dz);
      const T e0 = dx - fr.tn[0], e1 = dy - fr.tn[1], e2 = dz - fr.tn[2];
      const T x = fr.u[0] * e0 + fr.u[1] * e1 + fr.u[2] * e2;
      const T y = fr.v[0] * e0 + fr.v[1] * e1 + fr.v[2] * e2;
      const T f = fr.n[0] * e0 + fr.n[1] * e1 + fr.n[2] * e2;
      T w = wexp(-(e0 * e0 + e1 * e1 + e2 * e2));
      if constexpr (kMask) w = ((mask >> (j0 + b)) & 1ull) ? w : (T)0;
      const T xx = x * x, xy = x * y, yy = y * y;
      const T wx = w * x, wy = w * y, wxx = w * xx, wxy = w * xy, wyy = w * yy;
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

}  // namespace mls
