"""Pins of the oracle's surface geometry at the projected point (O11: unit
normal of the fitted graph, mean and Gaussian curvature).

- Symmetric quadric patches (golden, exact reproduction): the apex has
  slope zero, so K = 4 c3 c5 - c4^2 and H N_z = c3 + c5 exactly.
- Planes: the normal is the plane's, both curvatures vanish.
- Noise-free sphere caps of radius rho: K -> 1/rho^2 and |H| -> 1/rho with
  an error that falls at least like h^2 as the sampling densifies; the
  normal is radial, also at the cap's rim where the fitted plane is tilted
  (the slope terms of the normal undo the tilt).
- Scaling the cloud and h by 4 leaves N, divides H by 4 and K by 16.
- Statuses: PLANE_ONLY gives the plane normal and no curvature, OUTLIER
  nothing."""
import numpy as np
import pytest

from paper_2401_03365_amd import synth

from test_oracle_project import grid_cloud, load_golden, plane_case, quadric_case


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_quadric_apex_curvatures_exact(orc, idx):
    c = load_golden()["quadric_apex"][idx]
    P, Q = quadric_case(c)
    c0, c3, c4, c5 = c["coeffs_c0_c3_c4_c5"]
    out, st, geo = orc.project(P, Q, P.shape[0], c["h"], geometry=True)
    assert (st[0] & 0x0F) == orc.PT_OK
    N, H, K = geo[0, :3], geo[0, 3], geo[0, 4]
    assert abs(abs(N[2]) - 1.0) < 1e-14
    assert abs(K - (4 * c3 * c5 - c4 * c4)) < 1e-11
    assert abs(H * N[2] - (c3 + c5)) < 1e-11


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_plane_geometry(orc, idx):
    c = load_golden()["planes"][idx]
    P, Q, feet, n = plane_case(c)
    out, st, geo = orc.project(P, Q, c["k"], c["h"], geometry=True)
    assert np.all((st & 0x0F) == orc.PT_OK)
    assert np.all(np.abs(np.abs(geo[:, :3] @ n) - 1.0) < 1e-14)
    assert np.abs(geo[:, 3:5]).max() < 1e-9


def cap64(n, cap_angle, rho, seed):
    """Area-uniform samples of a sphere cap in FP64 (an FP32-rounded cloud
    would add input noise that dominates the curvature of small patches)."""
    rng = np.random.default_rng(seed)
    cz = rng.uniform(np.cos(cap_angle), 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - cz * cz)
    return rho * np.stack([s * np.cos(phi), s * np.sin(phi), cz], axis=1)


@pytest.mark.parametrize("rho", [1.0, 2.0])
def test_sphere_cap_curvatures_converge(orc, rho):
    errs = []
    for n in (20000, 80000):
        P = cap64(n, 0.3, rho, seed=5)
        h = synth.mean_nn_h(P)
        # queries near the pole, away from the cap's rim
        Q = P[P[:, 2] > rho * np.cos(0.1)][:200]
        out, st, geo = orc.project(P, Q, 32, h, geometry=True)
        assert np.all((st & 0x0F) == orc.PT_OK)
        radial = out / np.linalg.norm(out, axis=1, keepdims=True)
        assert np.all(np.abs(np.abs(np.sum(geo[:, :3] * radial, axis=1)) - 1.0) < 1e-6)
        eK = np.abs(geo[:, 4] * rho ** 2 - 1.0).max()
        eH = np.abs(np.abs(geo[:, 3]) * rho - 1.0).max()
        errs.append((h, max(eK, eH)))
    (h1, e1), (h2, e2) = errs
    assert e2 < 1e-3
    assert e2 <= e1 * (h2 / h1) ** 2 * 1.5  # at least second order


def test_normal_corrects_the_plane_tilt(orc):
    # at the cap's rim the one-sided neighbourhood tilts the fitted plane;
    # the graph's normal at the output (slope terms included) is radial
    P = cap64(80000, 0.3, 1.0, 5)
    h = synth.mean_nn_h(P)
    Q = P[P[:, 2] < np.cos(0.295)][:100]
    out, st, dg, geo = orc.project(P, Q, 32, h, diag=True, geometry=True)
    radial = out / np.linalg.norm(out, axis=1, keepdims=True)
    dev_plane = 1.0 - np.abs(np.sum(dg[:, 0:3] * radial, axis=1))
    dev_surf = 1.0 - np.abs(np.sum(geo[:, :3] * radial, axis=1))
    assert np.median(dev_plane) > 1e-8
    assert dev_surf.max() < 1e-11


def test_scaling_by_four(orc):
    P = grid_cloud(55)
    h = synth.mean_nn_h(P)
    k = 20
    nbr, _ = orc.knn(P, P, k)
    _, st, geo = orc.project(P, P, k, h, nbr=nbr, geometry=True)
    _, st2, geo2 = orc.project(P * 4.0, P * 4.0, k, h * 4.0, nbr=nbr, geometry=True)
    np.testing.assert_array_equal(st, st2)
    ok = (st & 0x0F) == orc.PT_OK
    np.testing.assert_allclose(geo2[ok, :3], geo[ok, :3], rtol=0, atol=1e-13)
    np.testing.assert_allclose(geo2[ok, 3] * 4.0, geo[ok, 3], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(geo2[ok, 4] * 16.0, geo[ok, 4], rtol=1e-12, atol=1e-12)


def test_status_geometry(orc):
    # four coplanar-ish points: fewer than 6 in the support -> PLANE_ONLY
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [50, 50, 50]], dtype=np.float64)
    Q = np.array([[0.5, 0.5, 0.1], [50, 50, 50.01]])
    out, st, geo = orc.project(P, Q, 4, 1.0, geometry=True)
    assert (st[0] & 0x0F) == orc.PT_PLANE_ONLY
    assert abs(abs(geo[0, 2]) - 1.0) < 1e-14 and np.all(np.isnan(geo[0, 3:5]))
    assert (st[1] & 0x0F) == orc.PT_OUTLIER
    assert np.all(np.isnan(geo[1]))
