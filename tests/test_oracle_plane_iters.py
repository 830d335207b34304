"""Pins of the oracle's self-consistent reference plane (Section 1.4: the
weights of Eq. (1.1) are taken at the projection q = r + t n of r onto the
plane itself; ``plane_iters`` steps from the t = 0 plane).

- Axially symmetric data: with the query on the axis, symmetry fixes the
  normal to the axis, and the self-consistent plane is the root of a scalar
  equation (q_z equals the weighted mean height with the weights centred at
  q_z), found here with scipy's brentq; the oracle's iterated q must converge
  to that root. Weights left at r, a wrong sign of t or a dropped term give a
  different height.
- Planes: the fitted plane does not depend on the weights, so every step
  count reproduces the orthogonal foot exactly.
- Stationarity at convergence: the weighted covariance with the weights at
  the oracle's final q has the oracle's normal as its smallest eigenvector
  (numpy eigh), and q is r's projection onto that plane.
- Zero steps leave the one-step result bit for bit; equivariance holds with
  steps as well."""
import numpy as np
import pytest
from scipy.optimize import brentq

from paper_2401_03365_amd import synth

from test_oracle_project import grid_cloud, load_golden, plane_case


def symmetric_cap(rings=14, per_ring=36, dtheta=0.02):
    """Unit-sphere cap sampled in rings around the z axis (FP32-exact), plus
    the pole."""
    pts = [[0.0, 0.0, 1.0]]
    for j in range(1, rings + 1):
        th = j * dtheta
        for a in range(per_ring):
            ph = 2 * np.pi * a / per_ring
            pts.append([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    P = np.array(pts).astype(np.float32).astype(np.float64)
    return P


@pytest.mark.parametrize("offset_h", [0.6, -0.8])
def test_axisymmetric_fixed_point_matches_scalar_root(orc, offset_h):
    P = symmetric_cap()
    h = 0.06
    k = P.shape[0]
    r = np.array([[0.0, 0.0, 1.0 + offset_h * h]])
    nbr = np.arange(k, dtype=np.int32)[None, :]

    def g(qz):
        w = np.exp(-np.sum((P - np.array([0.0, 0.0, qz])) ** 2, axis=1) / h ** 2)
        return np.sum(w * P[:, 2]) / np.sum(w) - qz

    lo, hi = P[:, 2].min(), P[:, 2].max()
    root = brentq(g, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=200)
    _, _, dg0 = orc.project(P, r, k, h, nbr=nbr, diag=True, plane_iters=0)
    _, _, dg = orc.project(P, r, k, h, nbr=nbr, diag=True, plane_iters=60)
    n = dg[0, 0:3]
    assert abs(abs(n[2]) - 1.0) < 1e-13          # normal along the axis
    q = dg[0, 6:9]
    assert abs(q[0]) < 1e-13 and abs(q[1]) < 1e-13
    assert abs(q[2] - root) < 1e-12 * h
    # the one-step plane (weights at r) is measurably elsewhere
    assert abs(dg0[0, 8] - root) > 1e-7 * h


@pytest.mark.parametrize("idx", [0, 1])
@pytest.mark.parametrize("iters", [1, 4])
def test_plane_feet_exact_for_any_step_count(orc, idx, iters):
    c = load_golden()["planes"][idx]
    P, Q, feet, n = plane_case(c)
    out, st = orc.project(P, Q, c["k"], c["h"], plane_iters=iters)
    assert np.all((st & 0x0F) == orc.PT_OK)
    assert np.abs(out - feet).max() < 1e-13


def test_stationary_at_convergence(orc):
    P = synth.sphere(4000, 0.01, seed=43).astype(np.float64)
    h = synth.mean_nn_h(P.astype(np.float32))
    k = 32
    rng = np.random.default_rng(44)
    Q = P[rng.choice(P.shape[0], 40, replace=False)]
    nbr, _ = orc.knn(P, Q, k)
    _, st, dg = orc.project(P, Q, k, h, nbr=nbr, diag=True, plane_iters=80)
    for j in range(Q.shape[0]):
        if st[j] & 0x10:
            continue
        X = P[nbr[j]]
        q = dg[j, 6:9]
        w = np.exp(-np.sum((X - q) ** 2, axis=1) / h ** 2)
        c = (w[:, None] * X).sum(0) / w.sum()
        D = X - c
        C = (w[:, None, None] * (D[:, :, None] * D[:, None, :])).sum(0) / w.sum()
        _, V = np.linalg.eigh(C)
        n_ref = V[:, 0]
        n = dg[j, 0:3]
        assert abs(abs(n @ n_ref) - 1.0) < 1e-10
        # q is the foot of r on the plane through c with that normal
        r = Q[j]
        foot = r - ((r - c) @ n_ref) * n_ref
        assert np.abs(q - foot).max() < 1e-10 * h


def test_zero_steps_is_the_one_step_projection(orc):
    P = synth.sphere(3000, 0.01, seed=45).astype(np.float64)
    h = synth.mean_nn_h(P.astype(np.float32))
    a = orc.project(P, P[:300], 24, h)
    b = orc.project(P, P[:300], 24, h, plane_iters=0)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("transform", ["translate", "scale"])
def test_equivariance_with_steps(orc, transform):
    P = grid_cloud(46)
    h = synth.mean_nn_h(P)
    k = 20
    nbr, _ = orc.knn(P, P, k)
    out, st = orc.project(P, P, k, h, nbr=nbr, plane_iters=3)
    if transform == "translate":
        t = np.array([0.5, -1.0, 0.25])
        P2, h2, f = P + t, h, lambda x: x + t
    else:
        P2, h2, f = P * 4.0, h * 4.0, lambda x: x * 4.0
    out2, st2 = orc.project(P2, P2, k, h2, nbr=nbr, plane_iters=3)
    np.testing.assert_array_equal(st2, st)
    np.testing.assert_allclose(out2, f(out), rtol=0, atol=1e-13 * max(1.0, h2 / h))
