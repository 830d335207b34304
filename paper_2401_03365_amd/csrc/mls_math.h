// mls_math.h -- per-query dense algebra of the MLS projection, in FP64,
// shared by the forward and adjoint kernels: the smallest eigenpair of the
// weighted 3x3 covariance, the local frame, and the 6x6 Cholesky solve of the
// quadratic height fit.
#pragma once

#include <hip/hip_runtime.h>

namespace mls {

struct Sym3 {
  double a00, a01, a02, a11, a12, a22;
};

struct Eig3 {
  double n[3];    // unit eigenvector of the smallest eigenvalue
  double lam[3];  // eigenvalues ascending
};

// Unit vector along the dominant column of adj(A - l I) (every nonzero
// column is parallel to the eigenvector of a simple eigenvalue l), polished
// by one more application of the adjugate. Returns false when the adjugate
// vanishes (l is a repeated eigenvalue).
__device__ inline bool adjugate_vector(double a00, double a01, double a02, double a11,
                                       double a12, double a22, double l, double v[3]) {
  const double b00 = a00 - l, b11 = a11 - l, b22 = a22 - l;
  const double j00 = b11 * b22 - a12 * a12;
  const double j11 = b00 * b22 - a02 * a02;
  const double j22 = b00 * b11 - a01 * a01;
  const double j01 = a02 * a12 - a01 * b22;
  const double j02 = a01 * a12 - a02 * b11;
  const double j12 = a01 * a02 - b00 * a12;
  double v0, v1, v2;
  if (j00 >= j11 && j00 >= j22) { v0 = j00; v1 = j01; v2 = j02; }
  else if (j11 >= j22)          { v0 = j01; v1 = j11; v2 = j12; }
  else                          { v0 = j02; v1 = j12; v2 = j22; }
  const double nn = v0 * v0 + v1 * v1 + v2 * v2;
  if (!(nn > 1e-200)) return false;
  double inv = 1.0 / sqrt(nn);
  v0 *= inv; v1 *= inv; v2 *= inv;
  const double w0 = j00 * v0 + j01 * v1 + j02 * v2;
  const double w1 = j01 * v0 + j11 * v1 + j12 * v2;
  const double w2 = j02 * v0 + j12 * v1 + j22 * v2;
  const double ww = w0 * w0 + w1 * w1 + w2 * w2;
  if (ww > 1e-200) {
    inv = 1.0 / sqrt(ww);
    v0 = w0 * inv; v1 = w1 * inv; v2 = w2 * inv;
  }
  v[0] = v0; v[1] = v1; v[2] = v2;
  return true;
}

// Smallest eigenpair of a symmetric positive semi-definite 3x3 matrix.
// lambda1 by Newton's method on p(l) = det(A - l I) from the left (p is
// positive, decreasing and convex below the smallest root, so the iterates
// increase monotonically to it); lambda2, lambda3 from the trace and the sum
// of principal minors. When lambda1 is at least as well separated from
// lambda2 as lambda3 is, the eigenvector comes from the adjugate of
// A - lambda1 I; otherwise the eigenvector of lambda3 is found that way and
// n is the smaller eigenvector of A restricted to its orthogonal complement
// (2x2, closed form), which stays a true eigenvector when lambda1 = lambda2.
__device__ inline Eig3 smallest_eigenpair(const Sym3 &C) {
  Eig3 r;
  double s = fmax(fmax(fabs(C.a00), fabs(C.a11)), fmax(fabs(C.a22), fmax(fabs(C.a01),
                                                        fmax(fabs(C.a02), fabs(C.a12)))));
  if (!(s > 0.0)) {
    r.n[0] = 1.0; r.n[1] = 0.0; r.n[2] = 0.0;
    r.lam[0] = r.lam[1] = r.lam[2] = 0.0;
    return r;
  }
  const double is = 1.0 / s;
  const double a00 = C.a00 * is, a01 = C.a01 * is, a02 = C.a02 * is;
  const double a11 = C.a11 * is, a12 = C.a12 * is, a22 = C.a22 * is;
  const double tr = a00 + a11 + a22;
  const double m2 = (a11 * a22 - a12 * a12) + (a00 * a22 - a02 * a02) + (a00 * a11 - a01 * a01);
  // start below the smallest eigenvalue: Gershgorin bound, capped at a small
  // negative value when the matrix is close to semi-definite
  const double g = fmin(a00 - fabs(a01) - fabs(a02),
                        fmin(a11 - fabs(a01) - fabs(a12), a22 - fabs(a02) - fabs(a12)));
  double l = fmax(g, -1e-5);
  {
    const double b00 = a00 - l, b11 = a11 - l, b22 = a22 - l;
    const double p = b00 * (b11 * b22 - a12 * a12) - a01 * (a01 * b22 - a12 * a02) +
                     a02 * (a01 * a12 - b11 * a02);
    if (!(p > 0.0)) l = g;  // the cap was not below the root
  }
  for (int it = 0; it < 64; ++it) {
    const double b00 = a00 - l, b11 = a11 - l, b22 = a22 - l;
    const double c00 = b11 * b22 - a12 * a12, c11 = b00 * b22 - a02 * a02,
                 c22 = b00 * b11 - a01 * a01;
    const double p = b00 * c00 - a01 * (a01 * b22 - a12 * a02) + a02 * (a01 * a12 - b11 * a02);
    const double dp = -(c00 + c11 + c22);
    if (!(p > 0.0) || !(dp < 0.0)) break;
    const double step = -p / dp;
    const double ln = l + step;
    if (!(ln > l)) break;
    l = ln;
    if (step <= 1e-17 * (fabs(l) + 1e-300)) break;
  }
  const double sr = tr - l;
  const double pr = m2 - l * sr;
  const double disc = sqrt(fmax(sr * sr - 4.0 * pr, 0.0));
  const double l2 = 0.5 * (sr - disc);
  const double l3 = sr - l2;
  double n[3] = {1.0, 0.0, 0.0};
  bool done = false;
  if (l2 - l >= l3 - l2) done = adjugate_vector(a00, a01, a02, a11, a12, a22, l, n);
  if (!done) {
    double v3[3];
    if (adjugate_vector(a00, a01, a02, a11, a12, a22, l3, v3)) {
      // orthonormal basis (e1, e2) of the complement of v3
      int ax = 0;
      if (fabs(v3[1]) < fabs(v3[ax])) ax = 1;
      if (fabs(v3[2]) < fabs(v3[ax])) ax = 2;
      double e1[3];
      if (ax == 0) { e1[0] = 0.0; e1[1] = -v3[2]; e1[2] = v3[1]; }
      else if (ax == 1) { e1[0] = v3[2]; e1[1] = 0.0; e1[2] = -v3[0]; }
      else { e1[0] = -v3[1]; e1[1] = v3[0]; e1[2] = 0.0; }
      const double i1 = 1.0 / sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
      e1[0] *= i1; e1[1] *= i1; e1[2] *= i1;
      const double e2[3] = {v3[1] * e1[2] - v3[2] * e1[1], v3[2] * e1[0] - v3[0] * e1[2],
                            v3[0] * e1[1] - v3[1] * e1[0]};
      const double Ae1[3] = {a00 * e1[0] + a01 * e1[1] + a02 * e1[2],
                             a01 * e1[0] + a11 * e1[1] + a12 * e1[2],
                             a02 * e1[0] + a12 * e1[1] + a22 * e1[2]};
      const double Ae2[3] = {a00 * e2[0] + a01 * e2[1] + a02 * e2[2],
                             a01 * e2[0] + a11 * e2[1] + a12 * e2[2],
                             a02 * e2[0] + a12 * e2[1] + a22 * e2[2]};
      const double b11 = e1[0] * Ae1[0] + e1[1] * Ae1[1] + e1[2] * Ae1[2];
      const double b12 = e1[0] * Ae2[0] + e1[1] * Ae2[1] + e1[2] * Ae2[2];
      const double b22 = e2[0] * Ae2[0] + e2[1] * Ae2[1] + e2[2] * Ae2[2];
      const double hd = 0.5 * (b11 - b22);
      const double mu = 0.5 * (b11 + b22) - sqrt(hd * hd + b12 * b12);
      // eigenvector of the smaller eigenvalue of [[b11, b12], [b12, b22]]
      double c1 = b12, c2 = mu - b11;
      const double d1 = mu - b22, d2 = b12;
      if (d1 * d1 + d2 * d2 > c1 * c1 + c2 * c2) { c1 = d1; c2 = d2; }
      const double cc = c1 * c1 + c2 * c2;
      if (!(cc > 1e-200)) { c1 = 1.0; c2 = 0.0; }
      for (int a = 0; a < 3; ++a) n[a] = c1 * e1[a] + c2 * e2[a];
    }
  }
  const double nv = 1.0 / sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  r.n[0] = n[0] * nv; r.n[1] = n[1] * nv; r.n[2] = n[2] * nv;
  r.lam[0] = l * s;
  r.lam[1] = l2 * s;
  r.lam[2] = l3 * s;
  return r;
}

// Frame on the plane: u = normalize(e_a x n) with a the axis of smallest
// |n_a| (lowest index on ties), v = n x u.
__device__ inline void plane_frame(const double n[3], double u[3], double v[3]) {
  int a = 0;
  if (fabs(n[1]) < fabs(n[a])) a = 1;
  if (fabs(n[2]) < fabs(n[a])) a = 2;
  double x0, x1, x2;  // e_a x n
  if (a == 0) { x0 = 0.0; x1 = -n[2]; x2 = n[1]; }
  else if (a == 1) { x0 = n[2]; x1 = 0.0; x2 = -n[0]; }
  else { x0 = -n[1]; x1 = n[0]; x2 = 0.0; }
  const double inv = 1.0 / sqrt(x0 * x0 + x1 * x1 + x2 * x2);
  u[0] = x0 * inv; u[1] = x1 * inv; u[2] = x2 * inv;
  v[0] = n[1] * u[2] - n[2] * u[1];
  v[1] = n[2] * u[0] - n[0] * u[2];
  v[2] = n[0] * u[1] - n[1] * u[0];
}

// Weighted sums of the quadratic fit: the 15 distinct monomials x^a y^b
// (a + b <= 4) and the 6 right-hand-side sums of f * phi.
struct QuadSums {
  double s[15];  // 1 x y xx xy yy xxx xxy xyy yyy xxxx xxxy xxyy xyyy yyyy
  double b[6];   // f*(1 x y xx xy yy)
};

// Index into s[] of M(i, j) for phi = (1, x, y, x^2, xy, y^2).
__device__ __forceinline__ int quad_index(int i, int j) {
  // monomial exponents of phi
  const int ex[6] = {0, 1, 0, 2, 1, 0};
  const int ey[6] = {0, 0, 1, 0, 1, 2};
  const int a = ex[i] + ex[j], b = ey[i] + ey[j];
  const int d = a + b;             // degree 0..4
  const int base[5] = {0, 1, 3, 6, 10};
  return base[d] + b;              // within degree ordered by the power of y
}

// Cholesky factor M = L L^T of the quadratic fit's normal matrix, with the
// pivot rule of the method: every pivot L_jj^2 must exceed tol * max_j M_jj
// (ok is false otherwise).
struct Chol6 {
  double L[6][6];  // lower triangle below the diagonal
  double inv[6];   // 1 / L_jj
  bool ok;

  __device__ inline void factor(const QuadSums &q, double tol) {
    double M[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j) M[i][j] = q.s[quad_index(i, j)];
    double maxdiag = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) maxdiag = fmax(maxdiag, M[i][i]);
    ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double s = M[j][j];
#pragma unroll
      for (int c = 0; c < j; ++c) s -= L[j][c] * L[j][c];
      ok = ok && (s > tol * maxdiag);
      const double d = sqrt(fmax(s, 1e-300));
      inv[j] = 1.0 / d;
#pragma unroll
      for (int i = j + 1; i < 6; ++i) {
        double z = M[i][j];
#pragma unroll
        for (int c = 0; c < j; ++c) z -= L[i][c] * L[j][c];
        L[i][j] = z * inv[j];
      }
    }
  }

  // x = M^-1 rhs by forward and back substitution.
  __device__ inline void solve(const double rhs[6], double x[6]) const {
    double y[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double z = rhs[i];
#pragma unroll
      for (int c = 0; c < i; ++c) z -= L[i][c] * y[c];
      y[i] = z * inv[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
      double z = y[i];
#pragma unroll
      for (int c = i + 1; c < 6; ++c) z -= L[c][i] * x[c];
      x[i] = z * inv[i];
    }
  }
};

// Solves the quadratic fit; on success writes a = M^-1 b and returns true.
__device__ inline bool quad_solve(const QuadSums &q, double tol, double a[6]) {
  Chol6 ch;
  ch.factor(q, tol);
  ch.solve(q.b, a);
  return ch.ok;
}

}  // namespace mls
