// mls_fwd.hip -- forward MLS projection, one lane per query.
//
// For query r with its k neighbours (sorted positions from the neighbour
// search) and Gaussian width h:
//   pass 1  d_i = (p_i - r)/h, w_i = exp(-|d_i|^2); S0, S1 = sum w d,
//           S2 = sum w d d^T (10 sums)                       [Section 1.4, Eq. (1.1)]
//   plane   C = S2/S0 - mu mu^T, n = smallest eigenvector, q = r + h <n,mu> n;
//           with plane_iters > 0, that many more planes from the moments with
//           the weights centred at the current q (Section 1.4: the weights
//           of Eq. (1.1) belong to the projection of r onto the plane)
//           or, with levin = 1, Levin's plane: the local minimum of Eq. (1.1)
//           over (n, t) with the weights at q = r + t n, by Newton's method
//           from this plane (mls_levin.h); none within the support radius
//           -> status NO_MINIMUM, out = r
// With ball = 1 every sum runs over the list entries whose canonical key to r
// is at most (support_radius_h h)^2 (the paper's radius-R neighbourhood); a
// list wholly inside that radius is flagged TRUNCATED.
// Geometry (when asked): the graph q + h (x u + y v + g n) has at the output
// the unit normal (n - a_1 u - a_2 v) / |.| and, with f_x = a_1, f_y = a_2,
// f_xx = 2 a_3 / h, f_xy = a_4 / h, f_yy = 2 a_5 / h, W = 1 + f_x^2 + f_y^2,
// the mean curvature ((1 + f_y^2) f_xx - 2 f_x f_y f_xy + (1 + f_x^2) f_yy) /
// (2 W^1.5) and the Gaussian curvature (f_xx f_yy - f_xy^2) / W^2.
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
#include "mls_fit.h"
#include "mls_levin.h"

namespace mls {
namespace {

constexpr int kBlock = 256;

// Normal (3 values) and curvatures (H, K) of query qi in the query dtype;
// either array may be null.
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

// kExt: the variant with plane steps and the ball neighbourhood (runtime
// plane_iters and ball); the plain variant has neither.
template <bool kF32, bool kExt>
__global__ __launch_bounds__(kBlock) void k_mls_forward(GridView g, QueryView qv, int32_t k,
                                                        int32_t min_support, int32_t plane_iters,
                                                        int32_t ball, int32_t levin,
                                                        double support_radius_h,
                                                        void *__restrict__ out_normals,
                                                        void *__restrict__ out_curv,
                                                        const int32_t *__restrict__ nbr,
                                                        const uint8_t *__restrict__ support,
                                                        void *__restrict__ out,
                                                        uint8_t *__restrict__ status) {
  const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (p >= qv.n) return;
  const int64_t qi = query_of_slot(g, qv, p);
  const int64_t qo = out_index(qv, p, qi);  // where the results go
  double r[3];
  load_slot_query(g, qv, p, qi, r);
  if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]))) {
    const double nanv = __longlong_as_double(0x7ff8000000000000ll);
    const double o[3] = {nanv, nanv, nanv};
    store_vec(out, qv.is_f64, qo, o);
    status[qo] = MLS_PT_NONFINITE;
    if (kExt) store_geometry(out_normals, out_curv, qv.is_f64, qo, o, nanv, nanv);
    return;
  }
  const int m = support[p];
  if (m < min_support) {
    store_vec(out, qv.is_f64, qo, r);
    status[qo] = MLS_PT_OUTLIER;
    if (kExt) {
      const double nanv = __longlong_as_double(0x7ff8000000000000ll);
      const double o[3] = {nanv, nanv, nanv};
      store_geometry(out_normals, out_curv, qv.is_f64, qo, o, nanv, nanv);
    }
    return;
  }
  const int cloud = qv.qcloud ? qv.qcloud[qi] : 0;
  const double h = g.clouds[cloud].h;
  // neighbour j of query p: nb[j * 64] (tile layout of the search kernel)
  const int32_t *nb = nbr + (p >> 6) * 64 * qv.kstride + (p & 63);
  const Rel<kF32> rel(r, 1.0 / h);

  double S0, S1[3], S2[6];
  PlaneFit pf;
  QuadSums qs;
  uint8_t extra_flags = 0;
  if (kExt) {
    // the ball: list entries within the support radius (canonical keys, as
    // the search counted them)
    uint64_t mask = ~0ull;
    if (ball) {
      const double rad = support_radius_h * h;
      const double rad2 = rad * rad;
      mask = 0ull;
      for (int j = 0; j < k; ++j) {
        const float4 P = g.pts[clamp_pos(nb[j * 64], g.n_points)];
        const double key = canon_key((double)P.x, (double)P.y, (double)P.z, r[0], r[1], r[2]);
        mask |= (key <= rad2 ? 1ull : 0ull) << j;
      }
      if (m >= k) extra_flags = MLS_PT_FLAG_TRUNCATED;
    }
    if (kF32 && levin) {
      // the start of the descent decides which local minimum it reaches, so
      // the FP32-moment path starts it from the FP64 plane as well
      const Rel<false> rel64(r, 1.0 / h);
      pass1_moments<false, false, true>(g, nb, k, rel64, S0, S1, S2, nullptr, 0.0, nullptr,
                                        nullptr, mask);
    } else {
      pass1_moments<kF32, false, true>(g, nb, k, rel, S0, S1, S2, nullptr, 0.0, nullptr,
                                       nullptr, mask);
    }
    pf = plane_from_moments(S0, S1, S2, r, h);
    if (levin) {
      double n[3] = {pf.n[0], pf.n[1], pf.n[2]};
      double tau = pf.t;
      if (!levin_descend(g, nb, k, r, 1.0 / h, support_radius_h, mask, n, tau)) {
        store_vec(out, qv.is_f64, qo, r);
        status[qo] = MLS_PT_NO_MINIMUM | pf.flags | extra_flags;
        const double nanv = __longlong_as_double(0x7ff8000000000000ll);
        const double o[3] = {nanv, nanv, nanv};
        store_geometry(out_normals, out_curv, qv.is_f64, qo, o, nanv, nanv);
        return;
      }
      pf = plane_of(n, tau, r, h, pf.flags);
    }
    for (int it = 0; it < plane_iters; ++it) {
      const Real<kF32> tn[3] = {(Real<kF32>)(pf.t * pf.n[0]), (Real<kF32>)(pf.t * pf.n[1]),
                                (Real<kF32>)(pf.t * pf.n[2])};
      plane_moments_at<kF32, true>(g, nb, k, rel, tn, S0, S1, S2, mask);
      pf = plane_from_moments(S0, S1, S2, r, h);
    }
    pass2_sums<kF32, true>(g, nb, k, rel, FrameT<kF32>(pf), qs, mask);
  } else {
    pass1_moments<kF32>(g, nb, k, rel, S0, S1, S2);
    pf = plane_from_moments(S0, S1, S2, r, h);
    pass2_sums<kF32>(g, nb, k, rel, FrameT<kF32>(pf), qs);
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
  store_vec(out, qv.is_f64, qo, o);
  status[qo] = st | pf.flags | extra_flags;
  if (kExt && (out_normals || out_curv)) {
    const double nanv = __longlong_as_double(0x7ff8000000000000ll);
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

}  // namespace

hipError_t launch_mls_forward(const GridView &g, const QueryView &qv, int32_t k,
                              int32_t precision, int32_t min_support, int32_t plane_iters,
                              int32_t ball, int32_t levin, double support_radius_h,
                              const int32_t *nbr, const uint8_t *support, void *out,
                              uint8_t *status, void *out_normals, void *out_curvatures,
                              hipStream_t s) {
  if (qv.n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((qv.n + kBlock - 1) / kBlock);
  const bool f32 = precision == MLS_PREC_FP32_MOMENTS;
  const bool ext = plane_iters != 0 || ball != 0 || levin != 0 || out_normals ||
                   out_curvatures;
  if (f32 && !ext)
    hipLaunchKernelGGL((k_mls_forward<true, false>), dim3(blocks), dim3(kBlock), 0, s, g, qv, k,
                       min_support, 0, 0, 0, support_radius_h, nullptr, nullptr, nbr, support, out,
                       status);
  else if (f32)
    hipLaunchKernelGGL((k_mls_forward<true, true>), dim3(blocks), dim3(kBlock), 0, s, g, qv, k,
                       min_support, plane_iters, ball, levin, support_radius_h, out_normals,
                       out_curvatures, nbr, support, out, status);
  else if (!ext)
    hipLaunchKernelGGL((k_mls_forward<false, false>), dim3(blocks), dim3(kBlock), 0, s, g, qv,
                       k, min_support, 0, 0, 0, support_radius_h, nullptr, nullptr, nbr, support,
                       out, status);
  else
    hipLaunchKernelGGL((k_mls_forward<false, true>), dim3(blocks), dim3(kBlock), 0, s, g, qv,
                       k, min_support, plane_iters, ball, levin, support_radius_h, out_normals,
                       out_curvatures, nbr, support, out, status);
  return hipGetLastError();
}

}  // namespace mls
