"""Pins of the oracle's finite-difference adjoint (central differences of the
projection with the neighbour lists fixed), against:
  * an independent reverse-mode derivative: the projection written a second
    time in plain PyTorch FP64 CPU ops (eigh, solve) and differentiated by
    autograd;
  * the closed form for a plane: d out / d r = I - n n^T;
  * the exact invariants of a rigid motion applied to queries and points
    together (translation: sum of all Jacobians = I; rotation: the cross
    product identity below);
  * the trivial statuses (an outlier's output is its query)."""
import numpy as np
import pytest
import torch

from paper_2401_03365_amd import synth


def torch_project(Pn, r, h):
    """The projection of one query from its k neighbours Pn (k x 3), in the
    steps of the method: weighted moments at r, smallest eigenvector of the
    weighted covariance, q = r + h <n, mu> n, frame (u from the axis of the
    smallest |n_a|), weighted quadratic fit at q, out = q + h a_0 n."""
    d = (Pn - r) / h
    w = torch.exp(-(d * d).sum(1))
    S0 = w.sum()
    mu = (w[:, None] * d).sum(0) / S0
    C = (w[:, None, None] * d[:, :, None] * d[:, None, :]).sum(0) / S0 - torch.outer(mu, mu)
    lam, V = torch.linalg.eigh(C)
    n = V[:, 0]
    t = torch.dot(n, mu)
    ax = int(torch.argmin(torch.abs(n.detach())))
    ea = torch.zeros(3, dtype=Pn.dtype)
    ea[ax] = 1.0
    u = torch.linalg.cross(ea, n)
    u = u / torch.linalg.norm(u)
    v = torch.linalg.cross(n, u)
    e = d - t * n
    x, y, f = e @ u, e @ v, e @ n
    om = torch.exp(-(e * e).sum(1))
    phi = torch.stack([torch.ones_like(x), x, y, x * x, x * y, y * y], 1)
    M = (om[:, None, None] * phi[:, :, None] * phi[:, None, :]).sum(0)
    b = (om[:, None] * f[:, None] * phi).sum(0)
    a = torch.linalg.solve(M, b)
    return r + h * (t + a[0]) * n


def torch_vjp(P, Q, nbr, h, gout):
    """(gq, gp) of sum_j <gout_j, out_j> by autograd, lists fixed."""
    Pt = torch.tensor(P, dtype=torch.float64, requires_grad=True)
    Qt = torch.tensor(Q, dtype=torch.float64, requires_grad=True)
    G = torch.tensor(gout, dtype=torch.float64)
    L = 0.0
    for j in range(Q.shape[0]):
        idx = torch.tensor(nbr[j].astype(np.int64))
        L = L + torch.dot(G[j], torch_project(Pt[idx], Qt[j], h))
    L.backward()
    return Qt.grad.numpy(), Pt.grad.numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_fd_matches_autograd_of_independent_implementation(orc):
    P = synth.sphere_cap(3000, 0.01, seed=11).astype(np.float64)
    h = synth.mean_nn_h(P.astype(np.float32))
    rng = np.random.default_rng(12)
    sel = rng.choice(P.shape[0], 25, replace=False)
    Q = P[sel] + rng.normal(0, 0.2 * h, (25, 3))
    k = 24
    nbr, _ = orc.knn(P, Q, k)
    _, st = orc.project(P, Q, k, h, nbr=nbr)
    assert np.all((st & 0x0F) == 0) and np.all((st & 0x10) == 0)
    gout = rng.normal(size=Q.shape)
    gq, gp = orc.grad_fd(P, Q, k, h, nbr, gout)
    aq, ap = torch_vjp(P, Q, nbr, h, gout)
    assert rel(gq, aq) < 1e-6, rel(gq, aq)
    assert rel(gp, ap) < 1e-6, rel(gp, ap)


def test_fd_plane_closed_form(orc):
    # samples exactly on a tilted plane, queries off it: out is the foot, so
    # the Jacobian in r is the projector I - n n^T
    rng = np.random.default_rng(21)
    xy = rng.integers(-64, 65, (4000, 2)) / 64.0
    P = np.column_stack([xy, 0.25 * xy[:, 0] - 0.5 * xy[:, 1] + 0.125])
    n = np.array([-0.25, 0.5, 1.0])
    n /= np.linalg.norm(n)
    h = synth.mean_nn_h(P.astype(np.float32))
    Q = P[:50] + rng.uniform(-0.5, 0.5, (50, 1)) * h * n
    nbr, _ = orc.knn(P, Q, 24)
    gout = rng.normal(size=Q.shape)
    gq, gp = orc.grad_fd(P, Q, 24, h, nbr, gout)
    expect = gout - (gout @ n)[:, None] * n
    assert np.abs(gq - expect).max() < 1e-7


def test_fd_rigid_motion_invariants(orc):
    # out(r + c, p + c) = out + c  =>  sum_j gq_j + sum_i gp_i = sum_j g_j
    # out(R r, R p) = R out        =>  sum_j r_j x gq_j + sum_i p_i x gp_i
    #                                   = sum_j out_j x g_j
    P = synth.sphere(3000, 0.01, seed=13).astype(np.float64)
    h = synth.mean_nn_h(P.astype(np.float32))
    rng = np.random.default_rng(14)
    Q = P[rng.choice(P.shape[0], 40, replace=False)]
    nbr, _ = orc.knn(P, Q, 32)
    out, st = orc.project(P, Q, 32, h, nbr=nbr)
    gout = rng.normal(size=Q.shape)
    gq, gp = orc.grad_fd(P, Q, 32, h, nbr, gout)
    np.testing.assert_allclose(gq.sum(0) + gp.sum(0), gout.sum(0), atol=1e-6 * np.abs(gout).sum())
    lhs = np.cross(Q, gq).sum(0) + np.cross(P, gp).sum(0)
    rhs = np.cross(out, gout).sum(0)
    np.testing.assert_allclose(lhs, rhs, atol=1e-6 * np.abs(gout).sum())


def test_fd_outlier_is_identity(orc):
    P = synth.sphere(2000, 0.01, seed=15).astype(np.float64)
    h = synth.mean_nn_h(P.astype(np.float32))
    Q = np.array([[5.0, 5.0, 5.0]])
    nbr, _ = orc.knn(P, Q, 16)
    gout = np.array([[0.3, -0.2, 0.7]])
    gq, gp = orc.grad_fd(P, Q, 16, h, nbr, gout)
    np.testing.assert_array_equal(gq, gout)
    assert not gp.any()
