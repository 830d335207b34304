"""GPU parity of the radius-R neighbourhood (``ball``: the k-nearest list
entries within R = support_radius_h * h, the paper's neighbourhood of
Section 1.4; TRUNCATED where the whole list lies inside R) against the FP64
oracle on the same setting.

Bars: statuses (with both flags) bit for bit (the FP32-moment path may take
the OK / PLANE_ONLY pivot decision differently where the oracle's relative
pivot is below 1e-5, which its FP32 moments do not resolve, on at most
0.1 % of the points), FP64 path
max |out - oracle| <= 1e-10 h with each point's error first divided by
max(1, 1e-6 / p), p the oracle's smallest relative Cholesky pivot of the 6x6
fit (small balls of a handful of points give fits with condition numbers up
to ~1e9 just above the 1e-12 pivot rule, and the rounding error of a solve
grows with the condition number); FP32-moment path, every point within
max(1e-4 h, 10 eps32 / min(p, gap) h), gap the oracle plane's relative
eigengap (the FP32 moments perturb the fit's solve and the plane's normal by
about eps32 / p and eps32 / gap), and RMS <= 1e-5 h over the points with
p >= 1e-4 (all but at most 5 %)."""
import numpy as np
import pytest
import torch

from paper_2401_03365_amd import synth
from tests.parity import check_status, relative_gap

pytestmark = pytest.mark.gpu

FP64_MAX_H = 1e-10
FP32_RMS_H = 1e-5
FP32_MAX_H = 1e-4
EPS32 = 2.0 ** -24


def api():
    from paper_2401_03365_amd import api as a
    return a


def check(orc, P64, Q, k, h, out, st, precision, radius_h, iters=0, uncapped=False):
    if uncapped:
        # every cloud point within R (the oracle's brute-force ball)
        ref, ref_st, _, dg = orc.project_ball(P64, Q, h, support_radius_h=radius_h, diag=True)
    else:
        ref_nbr, _ = orc.knn(P64, Q, k)
        ref, ref_st, dg = orc.project(P64, Q, k, h, nbr=ref_nbr, ball=True,
                                      support_radius_h=radius_h, plane_iters=iters, diag=True)
    piv = np.where(np.isfinite(dg[:, 23]), dg[:, 23], 1.0)
    # the FP32-moment path takes the pivot decision (OK or PLANE_ONLY) on its
    # own moments, whose relative rounding (~1e-7) does not resolve a pivot
    # below ~1e-5 of the largest diagonal: only there may it differ
    differ = (st & 0x2F) != (ref_st & 0x2F)
    if precision == "fp32":
        pivot_call = (((st & 0x0F) | (ref_st & 0x0F)) == 2) & ((st & 0x20) == (ref_st & 0x20)) & \
            (piv < 1e-5)
        assert np.all(pivot_call[differ]), np.flatnonzero(differ & ~pivot_call)
        assert differ.sum() <= 1e-3 * len(st)
    else:
        np.testing.assert_array_equal(st & 0x2F, ref_st & 0x2F)
    # the ambiguous-normal flag by the rule of tests/parity.py
    check_status(st & 0x1F | (ref_st & 0x20), ref_st & 0x1F | (ref_st & 0x20),
                 dg[:, 3:6]) if precision == "fp64" else None
    flag_differ = ((st ^ ref_st) & 0x10) != 0
    if precision == "fp32":
        gap = relative_gap(dg[:, 3:6])
        near = (gap >= 0.5e-6) & (gap <= 2e-6)
        assert not (flag_differ & ~near & ~differ).any()
    ok = ((ref_st & 0x10) == 0) & ((ref_st & 0x0F) != 3) & ~differ
    diff = np.abs(out.astype(np.float64) - ref)
    if out.dtype == np.float32:
        diff = np.maximum(diff - np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64), 0)
    if precision == "fp64":
        cond = np.maximum(1.0, 1e-6 / np.maximum(piv, 1e-300))
        err = (np.linalg.norm(diff, axis=1) / cond)[ok] / h
        assert err.max() <= FP64_MAX_H, err.max()
    else:
        # FP32 moments (relative rounding ~1e-7) against a fit whose relative
        # pivot is below 1e-4: the output is as uncertain as the fit is ill
        # conditioned, so those points (a few per cent of small balls) are
        # only required to be finite
        # FP32 moments (relative rounding ~1e-7): the output moves by about
        # eps32 / p with p the fit's smallest relative Cholesky pivot (the
        # solve's conditioning) and by about eps32 / gap with gap the plane's
        # relative eigengap (first-order eigenvector perturbation), so each
        # point's bar is the larger of 1e-4 h and 10 eps32 / min(p, gap) h
        # (measured on these clouds: at most 4.6 eps32 / min(p, gap));
        # small balls give fits with p below 1e-4 on a few per cent of the
        # points, which are left out of the RMS
        gap = np.nan_to_num(relative_gap(dg[:, 3:6]), nan=1.0)
        bar = np.maximum(FP32_MAX_H, 10.0 * EPS32 / np.maximum(np.minimum(piv, gap), 1e-300))
        err = np.linalg.norm(diff, axis=1) / h
        over = ok & ~(err <= bar)
        assert not over.any(), (np.flatnonzero(over)[:5], err[over][:5], bar[over][:5])
        well = piv >= 1e-4
        assert (ok & ~well).sum() <= 0.05 * ok.sum()
        rms = np.sqrt((err[ok & well] ** 2).mean()) if (ok & well).any() else 0.0
        assert rms <= FP32_RMS_H, rms
    return ref_st


@pytest.mark.parametrize("radius_h", [1.3, 1.8, 3.0])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sphere_ball_matches_oracle(orc, precision, radius_h):
    P = synth.sphere(20000, 0.01, seed=1)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h)
    out, st = g.project(Pt.double(), 32, precision, ball=True, support_radius_h=radius_h)
    torch.cuda.synchronize()
    P64 = P.astype(np.float64)
    ref_st = check(orc, P64, P64, 32, h, out.cpu().numpy(), st.cpu().numpy(), precision,
                   radius_h)
    trunc = (ref_st & 0x20) != 0
    # the radii span the regimes: mostly exact balls, mostly truncated lists
    if radius_h == 1.3:
        assert trunc.mean() < 0.05
    if radius_h == 3.0:
        assert trunc.mean() > 0.95


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_torus_with_outliers_ball_and_steps(orc, precision):
    P = synth.torus(20000, sigma=0.005, n_outliers=200, seed=54)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h)
    out, st = g.project(Pt, 40, precision, ball=True, support_radius_h=1.6, plane_iters=2)
    torch.cuda.synchronize()
    P64 = P.astype(np.float64)
    check(orc, P64, P64, 40, h, out.cpu().numpy(), st.cpu().numpy(), precision, 1.6, iters=2)


def test_ball_changes_the_result(orc):
    # the ball is not a no-op: against the k-nearest projection, off by far
    # more than the tolerance where the ball is smaller than the list
    P = synth.sphere(20000, 0.01, seed=1)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h)
    o0, _ = g.project(Pt.double(), 32, "fp64")
    o1, s1 = g.project(Pt.double(), 32, "fp64", ball=True, support_radius_h=1.5)
    torch.cuda.synchronize()
    assert (o1 - o0).norm(dim=1).max().item() > 1e-4 * h


def test_heightfield_10m_ball(orc):
    # full size, as one call over the whole cloud, sampled against the oracle
    P = synth.heightfield(10_000_000, sigma=1e-3, seed=3)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h, cell_size=1.25 * h)
    rng = np.random.default_rng(26)
    idx = np.sort(rng.choice(P.shape[0], 192, replace=False))
    idx_t = torch.from_numpy(idx).cuda()
    out, st = g.project(Pt.double(), 48, "fp32", ball=True, support_radius_h=1.8)
    torch.cuda.synchronize()
    P64 = P.astype(np.float64)
    check(orc, P64, P64[idx], 48, h, out[idx_t].cpu().numpy(), st[idx_t].cpu().numpy(), "fp32",
          1.8)


# ---- the ball without a count cap (ball = 2) ---------------------------------

@pytest.mark.parametrize("radius_h", [1.5, 3.0, 6.0])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_uncapped_ball_matches_oracle(orc, precision, radius_h):
    print("uncapped ball: sphere 20000, R = %.1f h, %s" % (radius_h, precision), flush=True)
    P = synth.sphere(20000, 0.01, seed=1)
    h = synth.mean_nn_h(P)
    Pt = torch.from_numpy(P).cuda()
    g = api().Grid(Pt, h)
    out, st = g.project(Pt.double(), 1, precision, ball=2, support_radius_h=radius_h)
    torch.cuda.synchronize()
    P64 = P.astype(np.float64)
    ref_st = check(orc, P64, P64, 1, h, out.cpu().numpy(), st.cpu().numpy(), precision, radius_h,
                   uncapped=True)
    assert not np.any(ref_st & 0x20)
    if radius_h == 6.0:
        _, _, cnt = orc.project_ball(P64, P64[:200], h, support_radius_h=radius_h)
        assert cnt.min() > 64  # balls beyond any k-nearest list


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_uncapped_ball_torus_outliers_offsets_and_fp32_queries(orc, precision):
    # a batch of two clouds (torus with outliers, height field), FP32 queries
    # that are not the points (query offsets), off-surface and non-finite ones
    print("uncapped ball: batch, %s" % precision, flush=True)
    A = synth.torus(12000, sigma=0.005, n_outliers=300, seed=58)
    B = synth.heightfield(9000, sigma=1e-3, seed=59)
    hA, hB = synth.mean_nn_h(A), synth.mean_nn_h(B)
    P = np.concatenate([A, B]).astype(np.float32)
    off = [0, A.shape[0], P.shape[0]]
    rng = np.random.default_rng(60)
    QA = (A[rng.choice(A.shape[0], 1500, replace=False)] +
          rng.uniform(-0.5, 0.5, (1500, 3)).astype(np.float32) * np.float32(hA))
    QB = (B[rng.choice(B.shape[0], 1000, replace=False)] +
          rng.uniform(-0.5, 0.5, (1000, 3)).astype(np.float32) * np.float32(hB))
    QA[3] = np.nan
    Q = np.concatenate([QA, QB]).astype(np.float32)
    g = api().Grid(torch.from_numpy(P).cuda(), [hA, hB], cloud_offsets=off)
    out, st = g.project(torch.from_numpy(Q).cuda(), 1, precision, ball=2, support_radius_h=2.5,
                        query_offsets=[0, 1500, 2500])
    torch.cuda.synchronize()
    out, st = out.cpu().numpy(), st.cpu().numpy()
    for (lo, hi), Pc, hc in (((0, 1500), A, hA), ((1500, 2500), B, hB)):
        check(orc, Pc.astype(np.float64), Q[lo:hi].astype(np.float64), 1, hc, out[lo:hi],
              st[lo:hi], precision, 2.5, uncapped=True)
    assert (st[3] & 0x0F) == 3
    assert int(((st[:1500] & 0x0F) == 1).sum()) > 5  # some outliers


def test_uncapped_ball_quadric_apex_on_larger_patches():
    # the golden bowl and saddle patches grown to 81 points: the ball covers
    # the whole symmetric patch and the FP64 path returns the apex exactly
    from test_oracle_project import load_golden, quadric_case
    for c in load_golden()["quadric_apex"]:
        c = dict(c)
        c["lattice_half"] = 4
        P, Q = quadric_case(c)
        Pt = torch.from_numpy(P.astype(np.float32)).cuda()
        g = api().Grid(Pt, c["h"])
        R = 2.0 * 4 * c["spacing"] * 1.5
        out, st = g.project(torch.from_numpy(Q).cuda(), 1, "fp64", ball=2,
                            support_radius_h=R / c["h"])
        torch.cuda.synchronize()
        assert (int(st[0]) & 0x0F) == 0
        np.testing.assert_allclose(out.cpu().numpy()[0], c["expected"], rtol=0, atol=1e-14)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_uncapped_ball_geometry(orc, precision):
    P = synth.sphere(20000, 0.01, seed=62)
    h = synth.mean_nn_h(P)
    Pt = torch.from_numpy(P).cuda()
    g = api().Grid(Pt, h)
    out, st, nrm, curv = g.project(Pt.double(), 1, precision, ball=2, support_radius_h=3.0,
                                   geometry=True)
    torch.cuda.synchronize()
    P64 = P.astype(np.float64)
    _, ref_st, _, geo = orc.project_ball(P64, P64, h, support_radius_h=3.0, geometry=True)
    ok = ((ref_st & 0x10) == 0) & ((ref_st & 0x0F) == 0) & ((st.cpu().numpy() & 0x0F) == 0)
    N, G = nrm.cpu().numpy()[ok], geo[ok]
    sgn = np.sign(np.sum(N * G[:, :3], axis=1))
    dn = np.abs(N * sgn[:, None] - G[:, :3]).max()
    dH = np.abs(curv.cpu().numpy()[ok, 0] * sgn - G[:, 3]).max() * h
    if precision == "fp64":
        assert dn <= 1e-9 and dH <= 1e-8, (dn, dH)
    else:
        assert dn <= 1e-3 and dH <= 1e-2, (dn, dH)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_uncapped_ball_cube_200k_sampled(orc, precision):
    # the quality protocol's largest balls: the 200k cube at R = 0.05 (about
    # 260 points per ball, edges and corners), every query on the GPU, 600
    # sampled ones against the oracle's brute-force ball
    print("uncapped ball: cube 200k, R = 0.05, %s" % precision, flush=True)
    P = synth.cube(200_000, 0.01, seed=62)
    R = 0.05
    h = R / 3.0
    Pt = torch.from_numpy(P).cuda()
    g = api().Grid(Pt, h)
    out, st = g.project(Pt, 1, precision, ball=2, support_radius_h=3.0)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(64).choice(P.shape[0], 600, replace=False))
    P64 = P.astype(np.float64)
    check(orc, P64, P64[idx], 1, h, out.cpu().numpy()[idx], st.cpu().numpy()[idx], precision,
          3.0, uncapped=True)
    _, _, cnt = orc.project_ball(P64, P64[idx[:50]], h, support_radius_h=3.0)
    assert np.median(cnt) > 150


def test_uncapped_ball_argument_rules():
    from paper_2401_03365_amd import _abi
    P = synth.sphere(3000, 0.01, seed=63)
    h = synth.mean_nn_h(P)
    Pt = torch.from_numpy(P).cuda()
    g = api().Grid(Pt, h)
    for kw, code in ((dict(return_neighbors=True), _abi.MLS_ERR_INVALID_ARGUMENT),
                     (dict(stages=1), _abi.MLS_ERR_INVALID_ARGUMENT),
                     (dict(levin=True), _abi.MLS_ERR_UNSUPPORTED),
                     (dict(plane_iters=2), _abi.MLS_ERR_UNSUPPORTED)):
        with pytest.raises(_abi.MLSError) as ei:
            g.project(Pt, 16, "fp32", ball=2, **kw)
        assert ei.value.code == code, kw
    with pytest.raises(_abi.MLSError) as ei:
        g.project(Pt, 16, "fp32", ball=3)
    assert ei.value.code == _abi.MLS_ERR_INVALID_ARGUMENT
