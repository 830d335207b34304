// mls_levin.h -- Levin's reference plane (Section 1.4, Eq. (1.1) with the
// weights at the plane's own projection q = r + t n of the query), one lane
// per query.
//
// The plane minimises, over the unit normal n and the offset t,
//   F(n, t) = sum_i (<n, p_i - r> - t)^2 theta(|p_i - r - t n|),
// a local minimum, the one near r that gives the local tangent plane. It is
// reached by Newton's method from the plane with the weights centred at r
// (the t = 0 plane of the default path, itself the tangent plane estimate
// near r). In units of h (d_i = (p_i - r)/h, tau = t/h) a summand is
//   f(a, tau) = s^2 E,  a = <n, d>, s = a - tau, E = exp(-|d - tau n|^2).
// The variables are (alpha, beta, tau) with n = normalize(n0 + alpha u +
// beta v) on the frame (u, v) of the current n0; at alpha = beta = 0 the
// derivatives of a are x = <u, d>, y = <v, d> and the second ones -a (both
// tangent directions, no mixed term). With dE/da = 2 tau E and dE/dtau =
// 2 s E:
//   f_a  = 2 E s (1 + tau s)            f_t  = 2 E s (s^2 - 1)
//   f_aa = 2 E (1 + 4 tau s + 2 tau^2 s^2)
//   f_at = 2 E (3 s^2 + 2 tau s^3 - 1 - 2 tau s)
//   f_tt = 2 E (2 s^4 - 5 s^2 + 1)
// so grad F = sum (f_a x, f_a y, f_t) and the Hessian is
//   [sum f_aa x^2 - A, sum f_aa x y, sum f_at x;
//    ...,              sum f_aa y^2 - A, sum f_at y;
//    ...,              ...,              sum f_tt],  A = sum f_a a.
//
// Step rule (the same on every path, so that the same minimum is reached):
// the Newton direction of the Hessian, shifted by mu I where it is not
// positive definite (mu from 1e-3 of its largest diagonal magnitude,
// doubling), at most 0.5 long; far from the minimum (shifted Hessian, or a
// direction of 1e-4 or more) the step halves until F falls by at least 1e-4
// of the step times the slope; near it (positive definite, shorter than
// 1e-4) the full step is taken. The descent ends when the direction is at
// most 1e-15 long, when a full step is no shorter than the one before, or
// when no step length lowers F; |tau| beyond the support radius (in units of
// h) means no minimum within reach (status NO_MINIMUM). The terms are summed
// in FP64 on both precision paths, and the FP32-moment path starts from the
// FP64 plane: which local minimum the descent reaches depends on its start
// and path, and for queries well off the surface FP32 moments move the start
// enough to change it.
#pragma once

#include "mls_fit.h"

namespace mls {

struct LevinTerms {
  double F;
  double g[3];   // dF / d(alpha, beta, tau)
  double H[6];   // packed aa, ab, bb, at, bt, tt
};

// F, its gradient and Hessian at (n, tau) over the list entries of `mask`.
// r is the query; ih = 1 / h.
__device__ inline LevinTerms levin_terms(const GridView &g, const int32_t *nb, int k,
                                         const double r[3], double ih, const double n[3],
                                         double tau, uint64_t mask) {
  double u[3], v[3];
  plane_frame(n, u, v);
  LevinTerms T;
  T.F = 0.0;
  for (int i = 0; i < 3; ++i) T.g[i] = 0.0;
  for (int i = 0; i < 6; ++i) T.H[i] = 0.0;
  double A = 0.0;
  for (int j0 = 0; j0 < k; j0 += kBatch) {
    float4 PB[kBatch];
    load_batch(g, nb, j0, k, PB);
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      if (j0 + b >= k) break;
      if (!((mask >> (j0 + b)) & 1ull)) continue;
      const double d0 = ((double)PB[b].x - r[0]) * ih;
      const double d1 = ((double)PB[b].y - r[1]) * ih;
      const double d2 = ((double)PB[b].z - r[2]) * ih;
      const double a = n[0] * d0 + n[1] * d1 + n[2] * d2;
      const double x = u[0] * d0 + u[1] * d1 + u[2] * d2;
      const double y = v[0] * d0 + v[1] * d1 + v[2] * d2;
      const double e0 = d0 - tau * n[0], e1 = d1 - tau * n[1], e2 = d2 - tau * n[2];
      const double E = exp(-(e0 * e0 + e1 * e1 + e2 * e2));
      const double s = a - tau, s2 = s * s, ts = tau * s;
      const double E2 = 2.0 * E;
      const double fa = E2 * s * (1.0 + ts);
      const double ft = E2 * s * (s2 - 1.0);
      const double faa = E2 * (1.0 + 4.0 * ts + 2.0 * ts * ts);
      const double fat = E2 * (3.0 * s2 + 2.0 * ts * s2 - 1.0 - 2.0 * ts);
      const double ftt = E2 * (2.0 * s2 * s2 - 5.0 * s2 + 1.0);
      T.F += E * s2;
      T.g[0] += fa * x;
      T.g[1] += fa * y;
      T.g[2] += ft;
      T.H[0] += faa * x * x;
      T.H[1] += faa * x * y;
      T.H[2] += faa * y * y;
      T.H[3] += fat * x;
      T.H[4] += fat * y;
      T.H[5] += ftt;
      A += fa * a;
    }
  }
  T.H[0] -= A;
  T.H[2] -= A;
  return T;
}

// Newton direction p = -(H + mu I)^-1 grad by the LDL^T factorisation of
// the shifted Hessian; mu = 0 first, then 1e-3 of the largest diagonal
// magnitude, doubling until every pivot is positive. Returns whether H
// itself was positive definite.
__device__ inline bool levin_direction(const LevinTerms &T, double p[3]) {
  const double h00 = T.H[0], h01 = T.H[1], h11 = T.H[2], h02 = T.H[3], h12 = T.H[4],
               h22 = T.H[5];
  double scale = fmax(fabs(h00), fmax(fabs(h11), fabs(h22)));
  if (!(scale > 0.0)) scale = 1.0;
  double mu = 0.0;
  for (int attempt = 0; attempt < 200; ++attempt) {
    // LDL^T of [h00+mu h01 h02; h01 h11+mu h12; h02 h12 h22+mu]
    const double D0 = h00 + mu;
    if (D0 > 0.0) {
      const double l10 = h01 / D0, l20 = h02 / D0;
      const double D1 = (h11 + mu) - l10 * h01;
      if (D1 > 0.0) {
        const double l21 = (h12 - l20 * h01) / D1;
        const double D2 = (h22 + mu) - l20 * h02 - l21 * (h12 - l20 * h01);
        if (D2 > 0.0) {
          // L z = -g, D w = z, L^T p = w
          const double z0 = -T.g[0];
          const double z1 = -T.g[1] - l10 * z0;
          const double z2 = -T.g[2] - l20 * z0 - l21 * z1;
          p[2] = z2 / D2;
          p[1] = z1 / D1 - l21 * p[2];
          p[0] = z0 / D0 - l10 * p[1] - l20 * p[2];
          return mu == 0.0;
        }
      }
    }
    mu = mu == 0.0 ? 1e-3 * scale : 2.0 * mu;
  }
  for (int a = 0; a < 3; ++a) p[a] = -T.g[a] / scale;
  return false;
}

// Descends from the plane (n, tau) (in place) to the local minimum of F.
// Returns false when |tau| leaves [0, tmax].
__device__ inline bool levin_descend(const GridView &g, const int32_t *nb, int k,
                                     const double r[3], double ih, double tmax, uint64_t mask,
                                     double n[3], double &tau) {
  LevinTerms T = levin_terms(g, nb, k, r, ih, n, tau, mask);
  double last = __longlong_as_double(0x7ff0000000000000ll);
  for (int it = 0; it < 200; ++it) {
    double p[3];
    const bool pd = levin_direction(T, p);
    const double len = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    if (len <= 1e-15) break;
    if (len > 0.5) {
      const double c = 0.5 / len;
      p[0] *= c; p[1] *= c; p[2] *= c;
    }
    const bool newton_region = pd && len < 1e-4;
    if (newton_region && len >= last) break;
    last = len;
    const double slope = T.g[0] * p[0] + T.g[1] * p[1] + T.g[2] * p[2];
    double u[3], v[3];
    plane_frame(n, u, v);
    bool moved = false;
    double step = 1.0;
    for (int bt = 0; bt < 60 && !moved; ++bt, step *= 0.5) {
      double m[3];
      for (int a = 0; a < 3; ++a) m[a] = n[a] + step * (p[0] * u[a] + p[1] * v[a]);
      const double inv = 1.0 / sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
      for (int a = 0; a < 3; ++a) m[a] *= inv;
      const double tt = tau + step * p[2];
      const LevinTerms Tt = levin_terms(g, nb, k, r, ih, m, tt, mask);
      if (newton_region || Tt.F <= T.F + 1e-4 * step * slope) {
        for (int a = 0; a < 3; ++a) n[a] = m[a];
        tau = tt;
        T = Tt;
        moved = true;
      }
    }
    if (!moved) break;
    if (fabs(tau) > tmax) return false;
  }
  return fabs(tau) <= tmax;
}

// The PlaneFit of the plane (n, tau): origin q = r + h tau n and its frame.
__device__ inline PlaneFit plane_of(const double n[3], double tau, const double r[3], double h,
                                    uint8_t flags) {
  PlaneFit pf;
  for (int a = 0; a < 3; ++a) {
    pf.n[a] = n[a];
    pf.q[a] = r[a] + h * tau * n[a];
    pf.mu[a] = 0.0;
    pf.lam[a] = 0.0;
  }
  pf.t = tau;
  pf.C = Sym3{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  pf.flags = flags;
  plane_frame(pf.n, pf.u, pf.v);
  return pf;
}

}  // namespace mls
