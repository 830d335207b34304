"""Pins of the oracle's Levin reference plane (``levin``; Section 1.4,
Eq. (1.1) with q = r + t n): a local minimum over unit n and t of
F(n, t) = sum_i (<n, p_i - r> - t)^2 theta(|p_i - r - t n|), the one that
descent reaches from the weighted-PCA plane with the weights at r (the
tangent-plane estimate near r; the paper's local minimum with the smallest
t that gives the local tangent plane near r).

Independent checks (none reuses the oracle's hand-written derivatives): F is
written out here in numpy, its derivatives are taken by the complex step (F
at a complex argument; the imaginary part over the step is the derivative
to rounding), roots by scipy's brentq, descent by scipy's BFGS.

- Axially symmetric cap, query on the axis: symmetry keeps n on the axis and
  the operator reduces to the local minimum of a function of t alone in the
  basin of the start (the weighted mean height), found by walking downhill
  and brentq on the complex-step derivative; the oracle must agree to
  1e-12 h. The frozen-weight steps of ``plane_iters`` (which leave out the
  weights' dependence on (n, t)) land measurably elsewhere on the same cap.
- Generic noisy clouds: at the oracle's (n, t) the complex-step gradient of F
  in (tangent angles, t) vanishes and the finite-difference Hessian is
  positive definite (a local minimum); scipy's BFGS on the numpy F from the
  same start (weighted PCA in numpy) reaches the same plane.
- Planes: the orthogonal foot, exactly; a minimum beyond the range
  (support_radius_h * h) gives NO_MINIMUM and out = r.
- Equivariance under dyadic translation and scaling by 4 (h scaled)."""
import numpy as np
import pytest
from scipy.optimize import brentq, minimize

from paper_2401_03365_amd import synth

from test_oracle_plane_iters import symmetric_cap
from test_oracle_project import grid_cloud, load_golden, plane_case


def F_numpy(D, n, tau):
    """F in units of h for the neighbour offsets D (m x 3, units of h); n and
    tau may be complex (complex-step derivatives)."""
    a = D @ n
    E = D - tau * n[None, :]
    return np.sum((a - tau) ** 2 * np.exp(-np.sum(E * E, axis=1)))


def tangent(n):
    ax = np.argmin(np.abs(n))
    e = np.zeros(3)
    e[ax] = 1.0
    u = np.cross(e, n)
    u /= np.linalg.norm(u)
    return u, np.cross(n, u)


def F_local(D, n0, u, v, x):
    """F at n = normalize(n0 + x0 u + x1 v), tau = x2 (complex-safe)."""
    m = n0 + x[0] * u + x[1] * v
    m = m / np.sqrt(np.sum(m * m))
    return F_numpy(D, m, x[2])


def grad_cs(fun, x, step=1e-30):
    g = np.zeros(len(x))
    for i in range(len(x)):
        xc = np.array(x, dtype=complex)
        xc[i] += 1j * step
        g[i] = fun(xc).imag / step
    return g


def offsets(P, nb, r, h):
    return (P[nb] - r) / h


def G_slope(D, n, tau):
    """dG/dtau at tau: n minimised (scipy, from n), then dF/dtau by the
    complex step. Returns (slope, minimiser)."""
    u, v = tangent(n)
    res = minimize(lambda x: F_local(D, n, u, v, np.array([x[0], x[1], tau])).real,
                   np.zeros(2), method="BFGS", options={"gtol": 1e-13, "maxiter": 400})
    m = n + res.x[0] * u + res.x[1] * v
    m /= np.linalg.norm(m)
    s = F_numpy(D, m.astype(complex), tau + 1e-30j).imag / 1e-30
    return s, m


def pca_start(D):
    """The weighted-PCA plane with the weights at r (numpy): normal and t/h."""
    w = np.exp(-np.sum(D * D, axis=1))
    mu = (w[:, None] * D).sum(0) / w.sum()
    C = (w[:, None, None] * D[:, :, None] * D[:, None, :]).sum(0) / w.sum() - np.outer(mu, mu)
    n = np.linalg.eigh(C)[1][:, 0]
    return n, float(n @ mu)


@pytest.mark.parametrize("offset_h", [0.6, -0.8, 1.7, -2.2])
def test_axisymmetric_cap_against_scalar_minimisation(orc, offset_h):
    P = symmetric_cap()
    h = 0.06
    k = P.shape[0]
    r = np.array([0.0, 0.0, 1.0 + offset_h * h])
    nbr = np.arange(k, dtype=np.int32)[None, :]
    D = (P - r) / h
    ez = np.array([0.0, 0.0, 1.0])
    dG = lambda t: F_numpy(D, ez.astype(complex), t + 1e-30j).imag / 1e-30
    n0, t0 = pca_start(D)
    assert abs(abs(n0[2]) - 1.0) < 1e-12
    t0 *= np.sign(n0[2])  # the start's t along +z
    # walk downhill from the start to the first sign change of the slope
    step = -np.sign(dG(t0)) * 1e-3
    t = t0
    while np.sign(dG(t + step)) == np.sign(dG(t)):
        t += step
    root = brentq(dG, min(t, t + step), max(t, t + step), xtol=1e-15, rtol=1e-15, maxiter=200)
    _, st, dg = orc.project(P, r[None, :], k, h, nbr=nbr, diag=True, levin=True)
    assert st[0] & 0x0F == orc.PT_OK
    n = dg[0, 0:3]
    assert abs(abs(n[2]) - 1.0) < 1e-13
    q = dg[0, 6:9]
    assert abs(q[0]) < 1e-13 and abs(q[1]) < 1e-13
    assert abs(q[2] - (r[2] + root * h)) < 1e-12 * h, (q[2] - r[2]) / h - root
    # the frozen-weight steps reach another plane on the same data
    _, _, dg28 = orc.project(P, r[None, :], k, h, nbr=nbr, diag=True, plane_iters=60)
    assert abs(dg28[0, 8] - q[2]) > 5e-6 * h, abs(dg28[0, 8] - q[2]) / h


def noisy_sphere_case(seed=43, n=4000, k=32, count=24):
    P = synth.sphere(n, 0.01, seed=seed).astype(np.float64)
    h = synth.mean_nn_h(P.astype(np.float32))
    rng = np.random.default_rng(seed + 1)
    Q = P[rng.choice(P.shape[0], count, replace=False)]
    # move half of the queries off the cloud along the radius
    Q[: count // 2] *= (1.0 + rng.uniform(-1.0, 1.0, count // 2) * h)[:, None]
    return P, h, k, Q


def test_oracle_plane_is_a_local_minimum(orc):
    P, h, k, Q = noisy_sphere_case()
    nbr, _ = orc.knn(P, Q, k)
    _, st, dg = orc.project(P, Q, k, h, nbr=nbr, diag=True, levin=True)
    checked = 0
    for j in range(Q.shape[0]):
        if st[j] & 0x0F not in (orc.PT_OK, orc.PT_PLANE_ONLY) or st[j] & 0x10:
            continue
        D = offsets(P, nbr[j], Q[j], h)
        n0 = dg[j, 0:3]
        tau = (dg[j, 6:9] - Q[j]) @ n0 / h
        u, v = tangent(n0)
        fun = lambda x: F_local(D, n0, u, v, x)
        x0 = np.array([0.0, 0.0, tau])
        g = grad_cs(fun, x0)
        scale = np.sum(np.exp(-np.sum(D * D, axis=1))) + 1e-300
        assert np.abs(g).max() <= 1e-9 * scale, (j, g)
        H = np.zeros((3, 3))
        e = 1e-5
        for i in range(3):
            xp, xm = x0.copy(), x0.copy()
            xp[i] += e
            xm[i] -= e
            H[i] = (grad_cs(fun, xp) - grad_cs(fun, xm)) / (2 * e)
        lam = np.linalg.eigvalsh(0.5 * (H + H.T))
        assert lam[0] > 0, (j, lam)
        checked += 1
    assert checked >= 18


def test_independent_descent_reaches_the_same_plane(orc):
    # scipy's BFGS on the numpy F, in the tangent coordinates of the numpy
    # weighted-PCA start, converges to the oracle's (n, t)
    P, h, k, Q = noisy_sphere_case(seed=47, count=16)
    nbr, _ = orc.knn(P, Q, k)
    _, st, dg = orc.project(P, Q, k, h, nbr=nbr, diag=True, levin=True)
    checked = 0
    for j in range(Q.shape[0]):
        if st[j] & 0x0F not in (orc.PT_OK, orc.PT_PLANE_ONLY) or st[j] & 0x10:
            continue
        D = offsets(P, nbr[j], Q[j], h)
        n0, t0 = pca_start(D)
        u, v = tangent(n0)
        res = minimize(lambda x: F_local(D, n0, u, v, x).real, np.array([0.0, 0.0, t0]),
                       jac=lambda x: grad_cs(lambda y: F_local(D, n0, u, v, y), x),
                       method="BFGS", options={"gtol": 1e-14, "maxiter": 2000})
        m = n0 + res.x[0] * u + res.x[1] * v
        m /= np.linalg.norm(m)
        n = dg[j, 0:3]
        tau = (dg[j, 6:9] - Q[j]) @ n / h
        assert abs(abs(m @ n) - 1.0) < 1e-9, (j, m, n)
        assert abs(res.x[2] * np.sign(m @ n) - tau) < 1e-8, (j, res.x[2], tau)
        checked += 1
    assert checked >= 12


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_plane_feet_exact(orc, idx):
    c = load_golden()["planes"][idx]
    P, Q, feet, n = plane_case(c)
    out, st, dg = orc.project(P, Q, c["k"], c["h"], diag=True, levin=True)
    assert np.all((st & 0x0F) == orc.PT_OK)
    assert np.abs(out - feet).max() < 1e-13
    assert np.all(np.abs(np.abs(dg[:, 0:3] @ n) - 1.0) < 1e-14)


def test_minimum_beyond_the_range(orc):
    # plane z = 0; the feet of the queries lie 2.5 h and 1.3 h away
    rng = np.random.default_rng(61)
    xy = rng.integers(-32, 33, (3000, 2)) / 64.0
    P = np.column_stack([xy, np.zeros(3000)])
    h = 0.125
    Q = np.array([[0.0, 0.0, 2.5 * h], [0.01, 0.0, -1.3 * h]])
    out, st = orc.project(P, Q, 40, h, levin=True)
    assert np.all(st & 0x0F == orc.PT_OK) and np.abs(out[:, 2]).max() < 1e-13
    # the same minima lie beyond a range of 1.2 h (no support required)
    out, st = orc.project(P, Q, 40, h, levin=True, support_radius_h=1.2, min_support=0)
    np.testing.assert_array_equal(st & 0x0F, [orc.PT_NO_MINIMUM, orc.PT_NO_MINIMUM])
    np.testing.assert_array_equal(out, Q)
    out, st = orc.project(P, Q, 40, h, levin=True, support_radius_h=2.6, min_support=0)
    np.testing.assert_array_equal(st & 0x0F, [orc.PT_OK, orc.PT_OK])


@pytest.mark.parametrize("transform", ["translate", "scale"])
def test_equivariance(orc, transform):
    P = grid_cloud(46)
    h = synth.mean_nn_h(P)
    k = 20
    nbr, _ = orc.knn(P, P, k)
    out, st = orc.project(P, P, k, h, nbr=nbr, levin=True)
    if transform == "translate":
        t = np.array([0.5, -1.0, 0.25])
        P2, h2, f = P + t, h, lambda x: x + t
    else:
        P2, h2, f = P * 4.0, h * 4.0, lambda x: x * 4.0
    out2, st2 = orc.project(P2, P2, k, h2, nbr=nbr, levin=True)
    np.testing.assert_array_equal(st2, st)
    ok = (st & 0x0F) != orc.PT_NO_MINIMUM
    np.testing.assert_allclose(out2[ok], f(out)[ok], rtol=0, atol=1e-12 * max(1.0, h2 / h))
