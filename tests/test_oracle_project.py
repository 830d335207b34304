"""Pins of the oracle's MLS projection against what the mathematics fixes:
closed forms (planes, symmetric quadric patches), library routines for the
sub-steps (eigh for the weighted covariance, lstsq for the weighted quadratic
fit), the O(h^4) convergence on a sphere, equivariance under exact
transforms, the status rules, and the paper's qualitative denoising claim."""
import json
import math
import os

import numpy as np
import pytest

from paper_2401_03365_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def load_golden():
    with open(GOLDEN) as f:
        return json.load(f)


def plane_case(c):
    """Samples exactly on z = a x + b y + c0 (dyadic) and FP32-exact queries
    offset along the normal. Returns (P, Q, expected feet, unit normal)."""
    a, b, c0 = c["z_coeffs"]
    rng = np.random.default_rng(c["seed"])
    steps = int(round(c["extent"] / c["grid_step"]))
    xy = rng.integers(-steps, steps + 1, (c["n"], 2)) * c["grid_step"]
    P = np.column_stack([xy, a * xy[:, 0] + b * xy[:, 1] + c0])
    assert np.array_equal(P.astype(np.float32).astype(np.float64), P)
    n = np.array([-a, -b, 1.0])
    n /= np.linalg.norm(n)
    lo, hi = c["query_offset_h"]
    off = rng.uniform(lo, hi, c["n"]) * c["h"]
    Q = (P + off[:, None] * n).astype(np.float32).astype(np.float64)
    # orthogonal foot of each query on the plane through (0, 0, c0)
    p0 = np.array([0.0, 0.0, c0])
    feet = Q - ((Q - p0) @ n)[:, None] * n
    return P, Q, feet, n


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_plane_reproduced_exactly(orc, idx):
    c = load_golden()["planes"][idx]
    P, Q, feet, n = plane_case(c)
    out, st, dg = orc.project(P, Q, c["k"], c["h"], diag=True)
    assert np.all((st & 0x0F) == orc.PT_OK)
    assert np.abs(out - feet).max() < 1e-13
    # the fitted normal is the plane's normal (up to sign)
    cosang = np.abs(dg[:, 0:3] @ n)
    assert np.all(cosang > 1 - 1e-14)
    # heights are zero, so every coefficient vanishes
    assert np.abs(dg[:, 15:21]).max() < 1e-10


def quadric_case(c):
    c0, c3, c4, c5 = c["coeffs_c0_c3_c4_c5"]
    half, s = c["lattice_half"], c["spacing"]
    g = np.arange(-half, half + 1) * s
    x, y = np.meshgrid(g, g, indexing="ij")
    x, y = x.ravel(), y.ravel()
    P = np.column_stack([x, y, c0 + c3 * x * x + c4 * x * y + c5 * y * y])
    assert np.array_equal(P.astype(np.float32).astype(np.float64), P)
    return P, np.array([[0.0, 0.0, c["query_z"]]])


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_symmetric_quadric_apex_exact(orc, idx):
    c = load_golden()["quadric_apex"][idx]
    P, Q = quadric_case(c)
    k = P.shape[0]  # the whole patch, so the neighbourhood is symmetric
    out, st, dg = orc.project(P, Q, k, c["h"], diag=True)
    assert (st[0] & 0x0F) == orc.PT_OK
    np.testing.assert_allclose(out[0], c["expected"], rtol=0, atol=1e-14)
    assert abs(abs(dg[0, 2]) - 1.0) < 1e-14  # normal along z


def weighted_cov_eigh(P, r, nb, h):
    d = (P[nb] - r) / h
    w = np.exp(-np.sum(d * d, axis=1))
    mu = (w[:, None] * d).sum(0) / w.sum()
    C = (w[:, None, None] * d[:, :, None] * d[:, None, :]).sum(0) / w.sum() - np.outer(mu, mu)
    lam, V = np.linalg.eigh(C)
    return lam, V, mu


def test_plane_fit_matches_eigh(orc):
    P = synth.sphere(4000, 0.02, seed=21).astype(np.float64)
    h = synth.mean_nn_h(P)
    k = 24
    nbr, _ = orc.knn(P, P[:300], k)
    out, st, dg = orc.project(P, P[:300], k, h, nbr=nbr, diag=True)
    for j in range(300):
        lam, V, mu = weighted_cov_eigh(P, P[j], nbr[j], h)
        np.testing.assert_allclose(dg[j, 3:6], lam, rtol=0, atol=1e-13 * lam[-1])
        gap = lam[1] - lam[0]
        assert abs(abs(dg[j, 0:3] @ V[:, 0]) - 1.0) < 1e-13 / max(gap / lam[-1], 1e-3)
        # q is the orthogonal projection of r onto the plane through r + h mu
        n = dg[j, 0:3]
        c = P[j] + h * mu
        q_ref = P[j] - ((P[j] - c) @ n) * n
        np.testing.assert_allclose(dg[j, 6:9], q_ref, rtol=0, atol=1e-15)


def test_quadratic_fit_matches_lstsq(orc):
    P = synth.torus(6000, sigma=0.01, seed=22).astype(np.float64)
    h = synth.mean_nn_h(P)
    k = 32
    Q = P[:200]
    nbr, _ = orc.knn(P, Q, k)
    out, st, dg = orc.project(P, Q, k, h, nbr=nbr, diag=True)
    for j in range(200):
        if (st[j] & 0x0F) != orc.PT_OK:
            continue
        n, q, u, v = dg[j, 0:3], dg[j, 6:9], dg[j, 9:12], dg[j, 12:15]
        # frame is orthonormal and right-handed
        F = np.stack([u, v, n])
        np.testing.assert_allclose(F @ F.T, np.eye(3), atol=1e-14)
        assert np.linalg.det(F) > 0
        e = (P[nbr[j]] - q) / h
        x, y, f = e @ u, e @ v, e @ n
        # weights as a function of the distance to q (Section 1.4)
        sw = np.sqrt(np.exp(-np.sum(e * e, axis=1)))
        A = np.column_stack([np.ones_like(x), x, y, x * x, x * y, y * y]) * sw[:, None]
        a_ref = np.linalg.lstsq(A, f * sw, rcond=None)[0]
        cond = np.linalg.cond(A)
        np.testing.assert_allclose(dg[j, 15:21], a_ref, rtol=0, atol=1e-15 * cond * cond)
        np.testing.assert_allclose(out[j], q + h * a_ref[0] * n, rtol=0, atol=1e-14)


def cap_max_error(orc, h_target, n_cap=4000, k=32, seed=0):
    theta = h_target * math.sqrt(n_cap / math.pi)
    rng = np.random.default_rng(seed)
    cz = rng.uniform(math.cos(theta), 1.0, n_cap)
    phi = rng.uniform(0, 2 * math.pi, n_cap)
    s = np.sqrt(1 - cz * cz)
    P = np.column_stack([s * np.cos(phi), s * np.sin(phi), cz])  # FP64, noise-free
    h = synth.mean_nn_h(P)
    Q = P[np.arccos(np.clip(P[:, 2], -1, 1)) < 5 * h]
    out, st = orc.project(P, Q, k, h)
    assert np.all((st & 0x0F) == orc.PT_OK)
    return h, np.abs(np.linalg.norm(out, axis=1) - 1.0).max()


def test_sphere_cap_convergence_order_four(orc):
    hs, errs = [], []
    for ht in (1.3e-2, 6.5e-3, 3.2e-3):
        h, e = cap_max_error(orc, ht)
        hs.append(h)
        errs.append(e)
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert 3.3 < slope < 4.7, (hs, errs, slope)
    # noise-free sphere projected to radius 1 within 1e-10 at h <= 3.2e-3
    assert hs[-1] <= 3.3e-3 and errs[-1] < 1e-10, (hs, errs)


def test_statuses(orc):
    # an isolated sample: fewer than 3 list entries within 3h -> OUTLIER, unchanged
    P = np.vstack([synth.lattice(6, 6, 1, spacing=0.1), [[5.0, 5.0, 5.0]]]).astype(np.float64)
    out, st = orc.project(P, P, 8, 0.1)
    assert (st[-1] & 0x0F) == orc.PT_OUTLIER
    np.testing.assert_array_equal(out[-1], P[-1])
    # collinear neighbours: the quadratic normal matrix is singular -> PLANE_ONLY, out = q
    L = synth.lattice(40, 1, 1, spacing=0.05).astype(np.float64)
    out, st, dg = orc.project(L, L[10:30], 12, 0.1, diag=True)
    assert np.all((st & 0x0F) == orc.PT_PLANE_ONLY)
    np.testing.assert_array_equal(out, dg[:, 6:9])
    # non-finite query -> NONFINITE, NaN output
    Q = np.array([[np.nan, 0, 0], [0.1, 0.1, np.inf]])
    out, st = orc.project(P, Q, 8, 0.1)
    assert np.all(st == orc.PT_NONFINITE) and np.all(np.isnan(out))


def grid_cloud(seed, n=1500):
    """Random points on a 2^-12 grid (exact under dyadic translation)."""
    rng = np.random.default_rng(seed)
    P = synth.sphere(n, 0.02, seed=seed).astype(np.float64)
    return np.round(P * 4096) / 4096


@pytest.mark.parametrize("transform", ["translate", "scale", "flip", "permute"])
def test_equivariance(orc, transform):
    P = grid_cloud(31)
    h = synth.mean_nn_h(P)
    k = 20
    nbr, key = orc.knn(P, P, k)
    out, st = orc.project(P, P, k, h, nbr=nbr)
    if transform == "translate":
        t = np.array([0.5, -1.0, 0.25])
        P2, h2, f = P + t, h, lambda x: x + t
    elif transform == "scale":
        P2, h2, f = P * 4.0, h * 4.0, lambda x: x * 4.0
    elif transform == "flip":
        s = np.array([-1.0, 1.0, -1.0])
        P2, h2, f = P * s, h, lambda x: x * s
    else:
        perm = [2, 0, 1]
        P2, h2, f = P[:, perm], h, lambda x: x[:, perm]
    nbr2, key2 = orc.knn(P2, P2, k)
    np.testing.assert_array_equal(nbr2, nbr)
    out2, st2 = orc.project(P2, P2, k, h2, nbr=nbr2)
    np.testing.assert_array_equal(st2, st)
    np.testing.assert_allclose(out2, f(out), rtol=0, atol=1e-13 * max(1.0, h2 / h))


def test_plane_idempotent_and_noisy_relative_idempotency(orc):
    c = load_golden()["planes"][0]
    P, Q, feet, n = plane_case(c)
    out, _ = orc.project(P, Q, c["k"], c["h"])
    out2, _ = orc.project(P, out, c["k"], c["h"])
    assert np.abs(out2 - out).max() < 1e-13
    P = synth.sphere(20000, 0.01, seed=1).astype(np.float64)
    h = synth.mean_nn_h(P)
    Q = P[:2000]
    o1, _ = orc.project(P, Q, 32, h)
    o2, _ = orc.project(P, o1, 32, h)
    ratio = np.linalg.norm(o2 - o1, axis=1) / np.linalg.norm(o1 - Q, axis=1)
    assert np.median(ratio) < 0.05


def test_denoising_on_noisy_sphere(orc):
    """The paper's qualitative finding (Section 3.3 tables): MLS lowers the
    mean deviation from the reference surface."""
    P = synth.sphere(20000, 0.01, seed=1).astype(np.float64)
    h = synth.mean_nn_h(P)
    out, st = orc.project(P, P, 32, h)
    before = np.abs(np.linalg.norm(P, axis=1) - 1)
    after = np.abs(np.linalg.norm(out, axis=1) - 1)
    assert after.mean() < 0.6 * before.mean()
    assert np.all((st & 0x0F) == orc.PT_OK)


def test_iterated_passes_keep_outliers(orc):
    P, mask = synth.torus(3000, sigma=0.005, n_outliers=30, seed=2, return_mask=True)
    P = P.astype(np.float64)
    h = synth.mean_nn_h(P)
    out, st = orc.project_passes(P, P, 16, h, 3)
    o = (st & 0x0F) == orc.PT_OUTLIER
    np.testing.assert_array_equal(out[o], P[o])
    assert o[mask].mean() > 0.2 and o[~mask].mean() < 0.01
