"""GPU parity of the surface geometry at the projected points (unit normal
of the fitted graph, mean and Gaussian curvature) against the FP64 oracle,
also for upsampling (queries four times denser than the samples).

The normal's sign follows the fitted plane's normal, which is not oriented:
normals are compared up to sign and H is compared after the same sign.
Bars, in units of h: FP64 path |dN| <= 1e-10, |dH| h <= 1e-9, |dK| h^2 <=
1e-9 on every point; FP32-moment path RMS |dN| <= 1e-4, RMS |dH| h <= 1e-3,
RMS |dK| h^2 <= 1e-3 (second-derivative coefficients carry the moment
rounding divided by the square of the support in units of h, a few hundred
times the 1e-5 h of the positions). PLANE_ONLY and OUTLIER give NaN
curvatures (and an OUTLIER a NaN normal) on both sides."""
import numpy as np
import pytest
import torch

from paper_2401_03365_amd import synth
from tests.parity import check_errors, check_status, oracle_ref, position_errors

pytestmark = pytest.mark.gpu


def api():
    from paper_2401_03365_amd import api as a
    return a


def compare(orc, P, k, h, precision, res, Q=None, **kw):
    out, st, nrm, curv = (t.cpu().numpy().astype(np.float64) if t.dtype != torch.uint8
                          else t.cpu().numpy() for t in res)
    P64 = P.astype(np.float64)
    Q64 = P64 if Q is None else Q
    ref, ref_st, lam, geo = oracle_ref(orc, P64, Q64, k, h, geometry=True, **kw)
    check_status(st, ref_st, lam)
    check_errors(position_errors(out, ref, ref_st, h), precision)
    # NaN patterns
    np.testing.assert_array_equal(np.isnan(nrm), np.isnan(geo[:, :3]))
    np.testing.assert_array_equal(np.isnan(curv), np.isnan(geo[:, 3:5]))
    ok = ((ref_st & 0x0F) == 0) & ((ref_st & 0x10) == 0)
    s = np.sign(np.sum(nrm[ok] * geo[ok, :3], axis=1))
    dN = np.linalg.norm(nrm[ok] - s[:, None] * geo[ok, :3], axis=1)
    dH = np.abs(curv[ok, 0] * s - geo[ok, 3]) * h
    dK = np.abs(curv[ok, 1] - geo[ok, 4]) * h * h
    if precision == "fp64":
        assert dN.max() <= 1e-10, dN.max()
        assert dH.max() <= 1e-9, dH.max()
        assert dK.max() <= 1e-9, dK.max()
    else:
        rms = lambda x: float(np.sqrt((x ** 2).mean()))
        assert rms(dN) <= 1e-4, rms(dN)
        assert rms(dH) <= 1e-3, rms(dH)
        assert rms(dK) <= 1e-3, rms(dK)
    return ok.sum()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sphere_geometry(orc, precision):
    P = synth.sphere(20000, 0.01, seed=1)
    h = synth.mean_nn_h(P)
    g = api().Grid(torch.from_numpy(P).cuda(), h)
    res = g.project(torch.from_numpy(P).cuda().double(), 32, precision, geometry=True)
    torch.cuda.synchronize()
    assert compare(orc, P, 32, h, precision, res) > 19000


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_torus_geometry_with_statuses_and_options(orc, precision):
    # outliers (NaN geometry) and the plane steps together
    P = synth.torus(20000, sigma=0.005, n_outliers=200, seed=57)
    h = synth.mean_nn_h(P)
    g = api().Grid(torch.from_numpy(P).cuda(), h)
    res = g.project(torch.from_numpy(P).cuda().double(), 32, precision, geometry=True,
                    plane_iters=2)
    torch.cuda.synchronize()
    compare(orc, P, 32, h, precision, res, plane_iters=2)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_upsampling_queries(orc, precision):
    # queries are not the samples: four per sample, jittered by up to 0.4 h
    # (a denser set projected onto the surface of the sparse one)
    P = synth.sphere(20000, 0.01, seed=1)
    h = synth.mean_nn_h(P)
    rng = np.random.default_rng(59)
    Q = (np.repeat(P.astype(np.float64), 4, axis=0) +
         rng.uniform(-0.4, 0.4, (4 * P.shape[0], 3)) * h)
    g = api().Grid(torch.from_numpy(P).cuda(), h)
    res = g.project(torch.from_numpy(Q).cuda(), 32, precision, geometry=True)
    torch.cuda.synchronize()
    assert compare(orc, P, 32, h, precision, res, Q=Q) > 0.95 * Q.shape[0]


def test_geometry_leaves_the_projection_unchanged(orc):
    P = synth.sphere(20000, 0.01, seed=1)
    h = synth.mean_nn_h(P)
    Pt = torch.from_numpy(P).cuda()
    g = api().Grid(Pt, h)
    o0, s0 = g.project(Pt.double(), 32, "fp32")
    o1, s1, _, _ = g.project(Pt.double(), 32, "fp32", geometry=True)
    torch.cuda.synchronize()
    assert torch.equal(s0, s1)
    assert (o0 - o1).abs().max().item() <= 1e-12 * h


def test_curvature_of_a_sphere(orc):
    # radius 1: K ~ 1 and |H| ~ 1 at every projected point, normals radial
    P = synth.sphere(200_000, 0.0, seed=58)
    h = synth.mean_nn_h(P)
    Pt = torch.from_numpy(P).cuda()
    g = api().Grid(Pt, h)
    out, st, nrm, curv = g.project(Pt.double(), 32, "fp64", geometry=True)
    torch.cuda.synchronize()
    out, nrm, curv = out.cpu().numpy(), nrm.cpu().numpy(), curv.cpu().numpy()
    radial = out / np.linalg.norm(out, axis=1, keepdims=True)
    assert np.median(np.abs(np.sum(nrm * radial, axis=1))) > 1 - 1e-6
    assert abs(np.median(curv[:, 1]) - 1.0) < 0.05
    assert abs(np.median(np.abs(curv[:, 0])) - 1.0) < 0.05
