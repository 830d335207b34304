"""Pins of the oracle's NORMAL_AMBIGUOUS flag (reading A17: the status byte
carries 0x10 when lambda2 - lambda1 < 1e-6 lambda3 for the eigenvalues
lambda1 <= lambda2 <= lambda3 of the plane's weighted covariance, Section
1.4, Eq. (1.1) at t = 0).

The neighbourhoods are built so that the answer is fixed by construction:
a star of points on three orthogonal axes around the query (rotated, FP32),
whose weighted covariance has the eigenvalues 2 w(a) a^2 / S0 along the axis
of half-length a, so that its gap can be placed anywhere -- equal
eigenvalues (isotropic star), a collinear set (lambda1 = lambda2 = 0), a
disc (lambda2 = lambda3, flag clear), and gaps 10 % either side of the
threshold. The reference gap is recomputed with numpy.linalg.eigvalsh from
the same FP32 coordinates. A wrong threshold constant, a wrong eigenvalue
order (lambda3 - lambda2), or a gap taken relative to lambda1 fails one of
these."""
import numpy as np
import pytest

from paper_2401_03365_amd import synth

H = 1.0


def rotation(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return q


def axis_star(a, b, c, seed=0):
    """FP32 star: the origin plus +-a, +-b, +-c along the columns of a random
    rotation. Negation is exact in FP32, so the pairs stay symmetric and the
    weighted mean about the origin is exactly zero."""
    R = rotation(seed)
    half = np.array([a * R[:, 0], b * R[:, 1], c * R[:, 2]]).astype(np.float32)
    return np.vstack([np.zeros((1, 3), np.float32), half, -half])


def line(n_side=3, step=0.3, seed=0):
    R = rotation(seed)
    t = np.arange(-n_side, n_side + 1) * step
    return (t[:, None] * R[:, 0][None, :]).astype(np.float32)


def numpy_gap(P32, r, h=H):
    """(lambda2 - lambda1) / lambda3 of the weighted covariance about r,
    weights exp(-|p - r|^2 / h^2) (independent numpy computation)."""
    d = (P32.astype(np.float64) - r) / h
    w = np.exp(-np.sum(d * d, axis=1))
    mu = (w[:, None] * d).sum(0) / w.sum()
    C = (w[:, None, None] * d[:, :, None] * d[:, None, :]).sum(0) / w.sum() - np.outer(mu, mu)
    lam = np.linalg.eigvalsh(C)
    return (lam[1] - lam[0]) / lam[2]


def star_with_gap(g, seed=0, a=0.5, c=1.0):
    """Star whose smallest two eigenvalues differ by about g * lambda3 (the
    half-length b of the middle axis solves 2 w(b) b^2 - 2 w(a) a^2 =
    g * 2 w(c) c^2 by bisection, then rounds to FP32)."""
    f = lambda x: x * x * np.exp(-x * x)
    target = f(a) + g * f(c)
    lo, hi = a, 1.0  # f increases on [a, 1]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) < target else (lo, mid)
    return axis_star(a, 0.5 * (lo + hi), c, seed)


def flag_of(orc, P32, k=None):
    P = P32.astype(np.float64)
    k = P.shape[0] if k is None else k
    _, st, dg = orc.project(P, np.zeros((1, 3)), k, H, diag=True)
    return int(st[0]), dg[0, 3:6]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_isotropic_star_is_flagged(orc, seed):
    st, lam = flag_of(orc, axis_star(0.5, 0.5, 0.5, seed))
    assert numpy_gap(axis_star(0.5, 0.5, 0.5, seed), np.zeros(3)) < 1e-6
    assert st & orc.PT_FLAG_AMBIGUOUS
    assert st & 0x0F != orc.PT_OUTLIER


@pytest.mark.parametrize("seed", [0, 3])
def test_collinear_support_is_flagged(orc, seed):
    # lambda1 = lambda2 = 0 < 1e-6 lambda3: flagged (and no quadratic fit)
    st, lam = flag_of(orc, line(seed=seed))
    assert st & orc.PT_FLAG_AMBIGUOUS
    assert st & 0x0F == orc.PT_PLANE_ONLY
    assert lam[2] > 0 and lam[1] < 1e-12 * lam[2]


@pytest.mark.parametrize("seed", [0, 4])
def test_disc_is_not_flagged(orc, seed):
    # lambda2 = lambda3 (isotropic in the plane), lambda1 well apart: clear
    P = axis_star(0.2, 0.7, 0.7, seed)
    assert numpy_gap(P, np.zeros(3)) > 0.5
    st, lam = flag_of(orc, P)
    assert not st & orc.PT_FLAG_AMBIGUOUS
    assert abs(lam[2] - lam[1]) < 1e-6 * lam[2]  # equal up to the FP32 rounding


@pytest.mark.parametrize("g,seed", [(0.9e-6, 0), (0.9e-6, 5), (1.1e-6, 0), (1.1e-6, 5)])
def test_threshold_either_side(orc, g, seed):
    P = star_with_gap(g, seed)
    gap = numpy_gap(P, np.zeros(3))
    # the FP32 rounding of the middle axis moves the gap by about 1e-7
    assert abs(gap - g) < 0.06e-6, gap
    st, lam = flag_of(orc, P)
    assert bool(st & orc.PT_FLAG_AMBIGUOUS) == (gap < 1e-6), (gap, lam)
    # the oracle's eigenvalues give the same gap
    assert abs((lam[1] - lam[0]) / lam[2] - gap) < 1e-12


def test_flag_follows_the_query(orc):
    # the same star seen from an off-centre query is an ordinary anisotropic
    # neighbourhood: the flag clears
    P = axis_star(0.5, 0.5, 0.5, 0)
    _, st, dg = orc.project(P.astype(np.float64), np.array([[0.3, 0.1, -0.2]]), 7, H, diag=True)
    assert not st[0] & orc.PT_FLAG_AMBIGUOUS


@pytest.mark.parametrize("maker,k", [(lambda: synth.sphere(20000, 0.01, seed=1), 32),
                                     (lambda: synth.heightfield(30000, sigma=1e-3, seed=3), 48)])
def test_smooth_surfaces_are_rarely_flagged(orc, maker, k):
    # on clouds sampled from smooth surfaces the normal is well defined
    P = maker()
    h = synth.mean_nn_h(P)
    P64 = P.astype(np.float64)
    _, st, dg = orc.project(P64, P64, k, h, diag=True)
    flagged = (st & orc.PT_FLAG_AMBIGUOUS) != 0
    lam = dg[:, 3:6]
    gap = (lam[:, 1] - lam[:, 0]) / lam[:, 2]
    np.testing.assert_array_equal(flagged, gap < 1e-6)
    assert flagged.mean() <= 0.01
