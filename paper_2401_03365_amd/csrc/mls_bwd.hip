// mls_bwd.hip -- adjoint of the MLS projection with respect to the query and
// point positions, one lane per query.
//
// The projection of one query (Section 1.4, Eq. (1.1); Section 2.1) is
//   d_i = (p_i - r)/h, w_i = exp(-|d_i|^2), S0 = sum w, S1 = sum w d,
//   S2 = sum w d d^T, mu = S1/S0, C = S2/S0 - mu mu^T,
//   n = smallest eigenvector of C, t = <n, mu>, e_i = d_i - t n,
//   u = (e_a x n)/|e_a x n| (a = axis of the smallest |n_a|), v = n x u,
//   x_i = <u,e_i>, y_i = <v,e_i>, f_i = <n,e_i>, om_i = exp(-|e_i|^2),
//   phi = (1, x, y, x^2, xy, y^2), M = sum om phi phi^T, b = sum om f phi,
//   a = M^-1 b, out = r + h (t + a_0) n    (PLANE_ONLY: a = 0; OUTLIER: out = r).
// With the neighbour lists and the statuses held fixed, the kernel recomputes
// every moment with the forward's own code and runs reverse mode from
// gbar = dL/d out:
//   s = t + a_0: nbar = h s gbar, tbar = h <gbar, n>, abar_0 = tbar;
//   bbar = M^-1 (abar_0 e_0); each neighbour adds
//     ombar = <bbar,phi>(f - <a,phi>), fbar = om <bbar,phi>,
//     phibar = om ((f - <a,phi>) bbar - <bbar,phi> a)
//   and ebar_i = -2 om ombar e + xbar u + ybar v + fbar n, with
//   ubar += xbar e, vbar += ybar e, nbar += fbar e - t ebar, tbar -= <n, ebar>;
//   frame: nbar += u x vbar, ubar += vbar x n, then through the normalisation
//   of e_a x n; t = <n, mu>: nbar += tbar mu, mubar = tbar n;
//   eigenvector: dn = -(C - l1 I)^+ dC n, so Cbar = -sym(z n^T) with
//   z = (C - l1 I)^+ nbar, solved on the plane's frame (C maps span(u, v) to
//   itself);
//   C, mu -> S0bar, S1bar, S2bar; each neighbour adds
//     wbar = S0bar + <S1bar, d> + d^T S2bar d,
//     dbar_i += w (S1bar + 2 S2bar d) - 2 w wbar d.
// Finally pbar_i = dbar_i / h (summed per block in LDS, then added with
// atomics into a sorted-order buffer) and rbar = gbar - sum_i dbar_i / h.
//
// The per-neighbour adjoint runs in the precision of the forward's moments
// (FP32 with compensated sums, or FP64); the per-query algebra is FP64.
#include "mls_fit.h"

namespace mls {
namespace {

constexpr int kBlock = 256;

// Per-neighbour pass-2 adjoint quantities (shared by both adjoint loops).
template <typename T>
struct Pass2Adj {
  T e[3], xb, yb, fb, eb[3];
};

template <bool kF32>
__device__ __forceinline__ Pass2Adj<Real<kF32>> pass2_adjoint_one(const Real<kF32> d[3],
                                                                  const FrameT<kF32> &fr,
                                                                  const Real<kF32> a[6],
                                                                  const Real<kF32> bb[6]) {
  using T = Real<kF32>;
  Pass2Adj<T> o;
  o.e[0] = d[0] - fr.tn[0];
  o.e[1] = d[1] - fr.tn[1];
  o.e[2] = d[2] - fr.tn[2];
  const T x = fr.u[0] * o.e[0] + fr.u[1] * o.e[1] + fr.u[2] * o.e[2];
  const T y = fr.v[0] * o.e[0] + fr.v[1] * o.e[1] + fr.v[2] * o.e[2];
  const T f = fr.n[0] * o.e[0] + fr.n[1] * o.e[1] + fr.n[2] * o.e[2];
  const T w = wexp(-(o.e[0] * o.e[0] + o.e[1] * o.e[1] + o.e[2] * o.e[2]));
  const T xx = x * x, xy = x * y, yy = y * y;
  const T beta = bb[0] + bb[1] * x + bb[2] * y + bb[3] * xx + bb[4] * xy + bb[5] * yy;
  const T rho = f - (a[0] + a[1] * x + a[2] * y + a[3] * xx + a[4] * xy + a[5] * yy);
  const T gx = a[1] + (T)2 * a[3] * x + a[4] * y;   // d<a,phi>/dx
  const T gy = a[2] + a[4] * x + (T)2 * a[5] * y;   // d<a,phi>/dy
  const T hx = bb[1] + (T)2 * bb[3] * x + bb[4] * y;
  const T hy = bb[2] + bb[4] * x + (T)2 * bb[5] * y;
  o.xb = w * (rho * hx - beta * gx);
  o.yb = w * (rho * hy - beta * gy);
  o.fb = w * beta;
  const T c = (T)-2 * w * beta * rho;  // -2 om ombar
#pragma unroll
  for (int q = 0; q < 3; ++q)
    o.eb[q] = c * o.e[q] + o.xb * fr.u[q] + o.yb * fr.v[q] + o.fb * fr.n[q];
  return o;
}

// First adjoint loop: sums of xbar e, ybar e, fbar e and ebar over the list.
template <bool kF32>
__device__ __forceinline__ void pass2_adjoint_sums(const GridView &g, const int32_t *nb, int k,
                                                   const Rel<kF32> &rel, const FrameT<kF32> &fr,
                                                   const Real<kF32> a[6],
                                                   const Real<kF32> bb[6], double U[3],
                                                   double V[3], double F[3], double E[3]) {
  using T = Real<kF32>;
  Acc<kF32, 12> A;
  A.zero();
  for (int j0 = 0; j0 < k; j0 += kBatch) {
    float4 PB[kBatch];
    load_batch(g, nb, j0, k, PB);
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      if (j0 + b >= k) break;
      T d[3];
      rel.d(PB[b], d[0], d[1], d[2]);
      const Pass2Adj<T> o = pass2_adjoint_one<kF32>(d, fr, a, bb);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        A.blk[q] += o.xb * o.e[q];
        A.blk[3 + q] += o.yb * o.e[q];
        A.blk[6 + q] += o.fb * o.e[q];
        A.blk[9 + q] += o.eb[q];
      }
    }
    A.fold();
  }
  for (int q = 0; q < 3; ++q) {
    U[q] = A.value(q);
    V[q] = A.value(3 + q);
    F[q] = A.value(6 + q);
    E[q] = A.value(9 + q);
  }
}

// Second adjoint loop: dbar_i of both passes, pbar_i = dbar_i / h scattered
// into gp (sorted order, xyz interleaved); returns sum_i dbar_i.
// Block-level aggregation of the point gradients: an open-addressing table in
// LDS keyed by sorted position (keys only inserted during the phase; probe
// step kStride), flushed to the global buffer with one atomic per component and
// distinct point. The 256 queries of a block are consecutive in Morton order
// and share most neighbours (about 800 distinct points for 12k list entries
// at k = 48), so the table removes most global atomics. An entry that finds
// no slot within kProbes goes straight to global memory. The table sums in
// FP64 for both paths: on gfx950 the LDS FP32 add (ds_add_f32) is several
// times slower than the FP64 one, and the FP32-moment kernel's three adds per
// list entry took 4 ms of a 10 ms adjoint at 10M points, k = 48; FP64 slots
// are larger, so that kernel's table has fewer of them (kSlots: 1,408 and
// 39 KB, so 4 blocks still fit a CU's LDS; 2,048 for the FP64 kernel).
constexpr uint32_t gcd_u32(uint32_t a, uint32_t b) { return b ? gcd_u32(b, a % b) : a; }

template <bool kF32>
struct ScatterTable {
  using T = Real<kF32>;
  static constexpr uint32_t kSlots = kF32 ? 1408 : 2048;
  static constexpr int kProbes = 32;
  static constexpr uint32_t kStride = 523;  // coprime with kSlots: visits every slot
  static_assert(gcd_u32(kStride, kSlots) == 1, "the probe must reach every slot");
  static_assert(!kF32 || 4 * kSlots * (sizeof(int32_t) + 3 * sizeof(double)) <= 160 * 1024,
                "four FP32-moment blocks must fit a CU's LDS");
  int32_t *key;  // kSlots, -1 = empty
  double *val;   // 3 x kSlots
  T *gp;         // global, sorted order, xyz interleaved

  __device__ __forceinline__ void add(int32_t pos, T v0, T v1, T v2) const {
    // positions of a block's neighbours come in runs: consecutive positions
    // take consecutive slots, and a collision jumps away from the run
    uint32_t s = (uint32_t)pos % kSlots;
#pragma unroll 1
    for (int probe = 0; probe < kProbes; ++probe) {
      int32_t cur = __hip_atomic_load(key + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (cur == -1) {
        cur = -1;
        __hip_atomic_compare_exchange_strong(key + s, &cur, pos, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        // cur is now the slot's key before the exchange (-1 if ours won)
        if (cur == -1) cur = pos;
      }
      if (cur == pos) {
        __hip_atomic_fetch_add(val + s, (double)v0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(val + kSlots + s, (double)v1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(val + 2 * kSlots + s, (double)v2, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        return;
      }
      s += kStride;
      if (s >= kSlots) s -= kSlots;
    }
    T *dst = gp + 3 * (int64_t)pos;
    unsafeAtomicAdd(dst + 0, v0);
    unsafeAtomicAdd(dst + 1, v1);
    unsafeAtomicAdd(dst + 2, v2);
  }
};

template <bool kF32>
__device__ __forceinline__ void final_adjoint(const GridView &g, const int32_t *nb, int k,
                                              const Rel<kF32> &rel, const FrameT<kF32> &fr,
                                              const Real<kF32> a[6], const Real<kF32> bb[6],
                                              Real<kF32> Sb0, const Real<kF32> Sb1[3],
                                              const Real<kF32> Sb2[6], Real<kF32> ih,
                                              const ScatterTable<kF32> &tab, double D[3]) {
  using T = Real<kF32>;
  Acc<kF32, 3> A;
  A.zero();
  for (int j0 = 0; j0 < k; j0 += kBatch) {
    float4 PB[kBatch];
    int32_t id[kBatch];
    load_batch(g, nb, j0, k, PB, id);
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      if (j0 + b >= k) break;
      T d[3];
      rel.d(PB[b], d[0], d[1], d[2]);
      const T w = wexp(-(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]));
      const T s2d0 = Sb2[0] * d[0] + Sb2[1] * d[1] + Sb2[2] * d[2];
      const T s2d1 = Sb2[1] * d[0] + Sb2[3] * d[1] + Sb2[4] * d[2];
      const T s2d2 = Sb2[2] * d[0] + Sb2[4] * d[1] + Sb2[5] * d[2];
      const T wb = Sb0 + Sb1[0] * d[0] + Sb1[1] * d[1] + Sb1[2] * d[2] +
                   (d[0] * s2d0 + d[1] * s2d1 + d[2] * s2d2);
      const T c = (T)-2 * wb;
      T db[3];
      db[0] = w * (Sb1[0] + (T)2 * s2d0 + c * d[0]);
      db[1] = w * (Sb1[1] + (T)2 * s2d1 + c * d[1]);
      db[2] = w * (Sb1[2] + (T)2 * s2d2 + c * d[2]);
      const Pass2Adj<T> o = pass2_adjoint_one<kF32>(d, fr, a, bb);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        db[q] += o.eb[q];
        A.blk[q] += db[q];
      }
      tab.add((int32_t)clamp_pos(id[b], g.n_points), db[0] * ih, db[1] * ih, db[2] * ih);
    }
    A.fold();
  }
  for (int q = 0; q < 3; ++q) D[q] = A.value(q);
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Adds to nbar the adjoint of u = (e_a x n) / |e_a x n| for the axis choice of
// plane_frame (held fixed), given ubar.
__device__ __forceinline__ void frame_u_adjoint(const double n[3], const double u[3],
                                                const double ubar[3], double nbar[3]) {
  int ax = 0;
  if (fabs(n[1]) < fabs(n[ax])) ax = 1;
  if (fabs(n[2]) < fabs(n[ax])) ax = 2;
  double ut[3];  // e_a x n
  if (ax == 0) { ut[0] = 0.0; ut[1] = -n[2]; ut[2] = n[1]; }
  else if (ax == 1) { ut[0] = n[2]; ut[1] = 0.0; ut[2] = -n[0]; }
  else { ut[0] = -n[1]; ut[1] = n[0]; ut[2] = 0.0; }
  const double inv = 1.0 / sqrt(dot3(ut, ut));
  const double uu = dot3(u, ubar);
  double tb[3];
  for (int q = 0; q < 3; ++q) tb[q] = (ubar[q] - u[q] * uu) * inv;
  // d/dn of <tb, e_a x n> = tb x e_a
  if (ax == 0) { nbar[1] += tb[2]; nbar[2] -= tb[1]; }
  else if (ax == 1) { nbar[0] -= tb[2]; nbar[2] += tb[0]; }
  else { nbar[0] += tb[1]; nbar[1] -= tb[0]; }
}

// Adjoint of the query in slot p; point gradients go through the table.
template <bool kF32>
__device__ __forceinline__ void backward_one(const GridView &g, const QueryView &qv, int32_t k,
                                             double support_radius_h, int32_t min_support,
                                             const int32_t *__restrict__ nbr,
                                             const void *__restrict__ grad_out,
                                             void *__restrict__ grad_q,
                                             const ScatterTable<kF32> &tab, int64_t p) {
  using T = Real<kF32>;
  const int64_t qi = query_of_slot(g, qv, p);
  double r[3], gb[3];
  load_query(qv, qi, r);
  load_vec(grad_out, qv.is_f64, qi, gb);
  if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]))) {
    const double z[3] = {0.0, 0.0, 0.0};
    store_vec(grad_q, qv.is_f64, qi, z);
    return;
  }
  const int cloud = qv.qcloud ? qv.qcloud[qi] : 0;
  const double h = g.clouds[cloud].h;
  const int32_t *nb = nbr + (p >> 6) * 64 * qv.kstride + (p & 63);

  // statuses of the forward: support on canonical keys (counted during pass
  // 1), any invalid entry makes the query an outlier
  const double rad = support_radius_h * h;
  int m = 0;
  bool valid = true;
  const Rel<kF32> rel(r, 1.0 / h);
  double S0, S1[3], S2[6];
  pass1_moments<kF32, true>(g, nb, k, rel, S0, S1, S2, r, rad * rad, &m, &valid);
  if (!valid || m < min_support) {  // out = r
    store_vec(grad_q, qv.is_f64, qi, gb);
    return;
  }

  // ---- forward recompute ----------------------------------------------------
  const PlaneFit pf = plane_from_moments(S0, S1, S2, r, h);
  const FrameT<kF32> fr(pf);
  double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double bb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double gn = dot3(gb, pf.n);
  double s = pf.t;
  {
    QuadSums qs;
    pass2_sums<kF32>(g, nb, k, rel, fr, qs);
    Chol6 ch;
    ch.factor(qs, 1e-12);
    if (m >= 6 && ch.ok) {
      ch.solve(qs.b, a);
      s += a[0];
      const double rhs[6] = {h * gn, 0.0, 0.0, 0.0, 0.0, 0.0};
      ch.solve(rhs, bb);  // bbar = M^-1 abar_0 e_0
    }
  }
  T aT[6], bbT[6];
  for (int i = 0; i < 6; ++i) { aT[i] = (T)a[i]; bbT[i] = (T)bb[i]; }

  // ---- out = r + h s n --------------------------------------------------------
  double nbar[3], tbar = h * gn;
  for (int q = 0; q < 3; ++q) nbar[q] = h * s * gb[q];

  // ---- pass-2 adjoint ---------------------------------------------------------
  {
    double U[3], V[3], F[3], E[3];
    pass2_adjoint_sums<kF32>(g, nb, k, rel, fr, aT, bbT, U, V, F, E);
    for (int q = 0; q < 3; ++q) nbar[q] += F[q] - pf.t * E[q];
    tbar -= dot3(pf.n, E);
    // v = n x u
    double c1[3], ubar[3];
    cross3(pf.u, V, c1);
    cross3(V, pf.n, ubar);
    for (int q = 0; q < 3; ++q) {
      nbar[q] += c1[q];
      ubar[q] += U[q];
    }
    frame_u_adjoint(pf.n, pf.u, ubar, nbar);
  }

  // ---- t = <n, mu> --------------------------------------------------------------
  double mubar[3];
  for (int q = 0; q < 3; ++q) {
    nbar[q] += tbar * pf.mu[q];
    mubar[q] = tbar * pf.n[q];
  }

  // ---- eigenvector: z = (C - l1 I)^+ nbar on span(u, v) -------------------------
  const Sym3 &C = pf.C;
  auto Cmul = [&](const double x[3], double y[3]) {
    y[0] = C.a00 * x[0] + C.a01 * x[1] + C.a02 * x[2];
    y[1] = C.a01 * x[0] + C.a11 * x[1] + C.a12 * x[2];
    y[2] = C.a02 * x[0] + C.a12 * x[1] + C.a22 * x[2];
  };
  double Cn[3], Cu[3], Cv[3];
  Cmul(pf.n, Cn);
  Cmul(pf.u, Cu);
  Cmul(pf.v, Cv);
  const double l1 = dot3(pf.n, Cn);
  const double b00 = dot3(pf.u, Cu) - l1, b01 = dot3(pf.u, Cv), b11 = dot3(pf.v, Cv) - l1;
  const double det = b00 * b11 - b01 * b01;
  const double cu = dot3(pf.u, nbar), cv = dot3(pf.v, nbar);
  double zu = (b11 * cu - b01 * cv) / det;
  double zv = (b00 * cv - b01 * cu) / det;
  if (!(isfinite(zu) && isfinite(zv))) { zu = 0.0; zv = 0.0; }  // repeated smallest eigenvalue
  double z[3];
  for (int q = 0; q < 3; ++q) z[q] = zu * pf.u[q] + zv * pf.v[q];
  // Cbar = G = -(z n^T + n z^T) / 2 (symmetric, full-matrix convention)
  double G[6];
  G[0] = -z[0] * pf.n[0];
  G[1] = -0.5 * (z[0] * pf.n[1] + pf.n[0] * z[1]);
  G[2] = -0.5 * (z[0] * pf.n[2] + pf.n[0] * z[2]);
  G[3] = -z[1] * pf.n[1];
  G[4] = -0.5 * (z[1] * pf.n[2] + pf.n[1] * z[2]);
  G[5] = -z[2] * pf.n[2];
  // C = S2/S0 - mu mu^T: mubar -= 2 G mu
  const double *mu = pf.mu;
  mubar[0] -= 2.0 * (G[0] * mu[0] + G[1] * mu[1] + G[2] * mu[2]);
  mubar[1] -= 2.0 * (G[1] * mu[0] + G[3] * mu[1] + G[4] * mu[2]);
  mubar[2] -= 2.0 * (G[2] * mu[0] + G[4] * mu[1] + G[5] * mu[2]);
  const double i0 = 1.0 / S0;
  const double GS2 = G[0] * S2[0] + G[3] * S2[3] + G[5] * S2[5] +
                     2.0 * (G[1] * S2[1] + G[2] * S2[2] + G[4] * S2[4]);
  const double Sb0 = -GS2 * i0 * i0 - dot3(mubar, mu) * i0;
  T Sb1[3], Sb2[6];
  for (int q = 0; q < 3; ++q) Sb1[q] = (T)(mubar[q] * i0);
  for (int q = 0; q < 6; ++q) Sb2[q] = (T)(G[q] * i0);

  // ---- both passes' per-neighbour adjoint, scatter -------------------------------
  double D[3];
  final_adjoint<kF32>(g, nb, k, rel, fr, aT, bbT, (T)Sb0, Sb1, Sb2, (T)(1.0 / h), tab, D);
  const double ih = 1.0 / h;
  double rb[3];
  for (int q = 0; q < 3; ++q) rb[q] = gb[q] - D[q] * ih;
  store_vec(grad_q, qv.is_f64, qi, rb);
}

// FP32 moments: 4 waves per SIMD (the 39 KB LDS table allows 4 blocks per
// CU; the neighbour loops are latency-bound and gain more from the waves than
// they lose to the spills of the FP64 solve state); FP64: the 56 KB table
// allows 2.
template <bool kF32>
__global__ __launch_bounds__(kBlock, kF32 ? 4 : 2) void k_mls_backward(GridView g, QueryView qv, int32_t k,
                                                         double support_radius_h,
                                                         int32_t min_support,
                                                         const int32_t *__restrict__ nbr,
                                                         const void *__restrict__ grad_out,
                                                         void *__restrict__ grad_q,
                                                         Real<kF32> *__restrict__ gp) {
  using T = Real<kF32>;
  using Tab = ScatterTable<kF32>;
  __shared__ int32_t skey[Tab::kSlots];
  __shared__ double sval[3 * Tab::kSlots];
  for (int i = threadIdx.x; i < (int)Tab::kSlots; i += kBlock) {
    skey[i] = -1;
    sval[i] = 0.0;
    sval[Tab::kSlots + i] = 0.0;
    sval[2 * Tab::kSlots + i] = 0.0;
  }
  __syncthreads();
  const Tab tab{skey, sval, gp};
  const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (p < qv.n)
    backward_one<kF32>(g, qv, k, support_radius_h, min_support, nbr, grad_out, grad_q, tab, p);
  __syncthreads();
  for (int i = threadIdx.x; i < (int)Tab::kSlots; i += kBlock) {
    const int32_t pos = skey[i];
    if (pos >= 0) {
      T *dst = gp + 3 * (int64_t)pos;
      unsafeAtomicAdd(dst + 0, (T)sval[i]);
      unsafeAtomicAdd(dst + 1, (T)sval[Tab::kSlots + i]);
      unsafeAtomicAdd(dst + 2, (T)sval[2 * Tab::kSlots + i]);
    }
  }
}

// Caller lists (original indices, row-major per query, k each) -> sorted
// positions in the tile layout (qv.kstride rows per tile); entries outside
// [0, n_points) and rows past k become -1.
__global__ void k_lists_from_caller(GridView g, QueryView qv, int32_t k,
                                    const int32_t *__restrict__ user,
                                    int32_t *__restrict__ nbr) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tiles = (qv.n + 63) / 64;
  const int64_t ks = qv.kstride;
  if (o >= tiles * 64 * ks) return;
  const int64_t tile = o / (64 * ks);
  const int64_t within = o - tile * 64 * ks;
  const int64_t p = tile * 64 + (within & 63);
  const int64_t j = within >> 6;
  int32_t pos = -1;
  if (p < qv.n && j < k) {
    const int64_t qi = query_of_slot(g, qv, p);
    const int32_t v = user[qi * k + j];
    if (v >= 0 && (int64_t)v < g.n_points) pos = g.inv_perm[v];
  }
  nbr[o] = pos;
}

template <typename T>
__global__ void k_zero(T *__restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (T)0;
}

// grad_points[original index] = sorted-order accumulation.
template <typename TS, typename TO>
__global__ void k_unsort_grad(GridView g, const TS *__restrict__ gs, TO *__restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.n_points) return;
  const int64_t o = __float_as_int(g.pts[s].w);
  out[3 * o + 0] = (TO)gs[3 * s + 0];
  out[3 * o + 1] = (TO)gs[3 * s + 1];
  out[3 * o + 2] = (TO)gs[3 * s + 2];
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_lists_from_caller(const GridView &g, const QueryView &qv, int32_t k,
                                    const int32_t *user, int32_t *nbr, hipStream_t s) {
  const int64_t total = (qv.n + 63) / 64 * 64 * (int64_t)qv.kstride;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lists_from_caller, dim3(blocks_for(total, 256)), dim3(256), 0, s, g, qv,
                     k, user, nbr);
  return hipGetLastError();
}

hipError_t launch_mls_backward(const GridView &g, const QueryView &qv, int32_t k,
                               int32_t precision, double support_radius_h, int32_t min_support,
                               const int32_t *nbr, const void *grad_out, void *grad_q,
                               void *gp_sorted, void *grad_points, hipStream_t s) {
  // the sorted-order scatter buffer holds the per-neighbour arithmetic's type;
  // grad_points has the dtype of the queries
  const bool f32 = precision == MLS_PREC_FP32_MOMENTS;
  const int64_t n3 = 3 * g.n_points;
  const dim3 b256(256);
  if (n3 > 0) {
    if (f32)
      hipLaunchKernelGGL(k_zero<float>, dim3(blocks_for(n3, 256)), b256, 0, s,
                         (float *)gp_sorted, n3);
    else
      hipLaunchKernelGGL(k_zero<double>, dim3(blocks_for(n3, 256)), b256, 0, s,
                         (double *)gp_sorted, n3);
  }
  if (qv.n > 0) {
    const dim3 grid(blocks_for(qv.n, kBlock));
    if (f32)
      hipLaunchKernelGGL(k_mls_backward<true>, grid, dim3(kBlock), 0, s, g, qv, k,
                         support_radius_h, min_support, nbr, grad_out, grad_q,
                         (float *)gp_sorted);
    else
      hipLaunchKernelGGL(k_mls_backward<false>, grid, dim3(kBlock), 0, s, g, qv, k,
                         support_radius_h, min_support, nbr, grad_out, grad_q,
                         (double *)gp_sorted);
  }
  if (n3 > 0) {
    const dim3 gb(blocks_for(g.n_points, 256));
    if (f32 && qv.is_f64)
      hipLaunchKernelGGL((k_unsort_grad<float, double>), gb, b256, 0, s, g,
                         (const float *)gp_sorted, (double *)grad_points);
    else if (f32)
      hipLaunchKernelGGL((k_unsort_grad<float, float>), gb, b256, 0, s, g,
                         (const float *)gp_sorted, (float *)grad_points);
    else if (qv.is_f64)
      hipLaunchKernelGGL((k_unsort_grad<double, double>), gb, b256, 0, s, g,
                         (const double *)gp_sorted, (double *)grad_points);
    else
      hipLaunchKernelGGL((k_unsort_grad<double, float>), gb, b256, 0, s, g,
                         (const double *)gp_sorted, (float *)grad_points);
  }
  return hipGetLastError();
}

}  // namespace mls
