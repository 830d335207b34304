"""GPU parity of the self-consistent reference plane (``plane_iters`` steps
with the weights of Eq. (1.1) at the plane's own projection q, Section 1.4)
against the FP64 oracle taking the same steps.

Bars as for the one-step plane: neighbour lists and statuses bit for bit,
FP64 path max |out - oracle| <= 1e-10 h, FP32-moment path RMS <= 1e-5 h and
max <= 1e-4 h (points whose normal is flagged ambiguous left out of the
error; the flag itself compared by the rule of tests/parity.py)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2401_03365_amd import synth
from tests.parity import check_errors, check_projection, check_status, oracle_ref, position_errors

pytestmark = pytest.mark.gpu

FP64_MAX_H = 1e-10
FP32_RMS_H = 1e-5


def api():
    from paper_2401_03365_amd import api as a
    return a


def check(orc, P64, Q, k, h, nbr, out, st, precision, iters):
    ref_nbr, _ = orc.knn(P64, Q, k)
    if nbr is not None:
        np.testing.assert_array_equal(nbr, ref_nbr)
    ref = oracle_ref(orc, P64, Q, k, h, nbr=ref_nbr, plane_iters=iters)[0]
    check_projection(orc, P64, Q, k, h, out, st, precision, nbr=ref_nbr, plane_iters=iters,
                     label="plane steps %d" % iters)
    return ref


@pytest.mark.parametrize("iters", [1, 3, 16])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sphere_steps_match_oracle(orc, iters, precision):
    P = synth.sphere(20000, 0.01, seed=1)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h)
    out, st, nbr = g.project(Pt.double(), 32, precision, return_neighbors=True,
                             plane_iters=iters)
    torch.cuda.synchronize()
    P64 = P.astype(np.float64)
    check(orc, P64, P64, 32, h, nbr.cpu().numpy(), out.cpu().numpy(), st.cpu().numpy(),
          precision, iters)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_torus_with_outliers_and_fp32_queries(orc, precision):
    P = synth.torus(20000, sigma=0.005, n_outliers=200, seed=47)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h)
    out, st = g.project(Pt, 24, precision, plane_iters=4)
    torch.cuda.synchronize()
    P64 = P.astype(np.float64)
    check(orc, P64, P64, 24, h, None, out.cpu().numpy(), st.cpu().numpy(), precision, 4)


def test_iterated_passes_with_steps(orc):
    # every pass against the oracle fed the GPU's own pass input
    P = synth.heightfield(30000, sigma=1e-3, seed=48)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h)
    cur = Pt.double()
    P64 = P.astype(np.float64)
    for it in range(3):
        out, st = g.project(cur, 48, "fp32", plane_iters=3)
        torch.cuda.synchronize()
        check(orc, P64, cur.cpu().numpy(), 48, h, None, out.cpu().numpy(), st.cpu().numpy(),
              "fp32", 3)
        cur = out


@pytest.mark.parametrize("iters", [0, 2])
def test_passes_wrapper_matches_oracle_passes(orc, iters):
    # the convenience call: grid built once, 2 passes over FP32 queries (the
    # cloud's dtype), outliers frozen; the oracle takes the same passes on the
    # FP32-rounded outputs of the previous one
    P = synth.torus(8000, sigma=0.005, n_outliers=80, seed=49)
    h = synth.mean_nn_h(P)
    a = api()
    out, st = a.project(torch.from_numpy(P).cuda(), h, 24, "fp64", passes=2,
                        plane_iters=iters)
    torch.cuda.synchronize()
    P64 = P.astype(np.float64)
    cur, ref_st = P64.copy(), None
    for _ in range(2):
        cur_prev = cur
        ref, st_new = orc.project(P64, cur, 24, h, plane_iters=iters)
        if ref_st is not None:
            frozen = (ref_st & 0x0F) == orc.PT_OUTLIER
            ref[frozen] = cur[frozen]
            st_new = np.where(frozen, ref_st, st_new)
        ref_st = st_new
        cur = ref.astype(np.float32).astype(np.float64)
    st = st.cpu().numpy()
    # the flag of the last pass, by the rule of tests/parity.py
    last_in = cur_prev.astype(np.float64)
    lam = oracle_ref(orc, P64, last_in, 24, h, plane_iters=iters)[2]
    check_status(st, ref_st, lam)
    err = position_errors(out.cpu().numpy(), ref, ref_st, h)
    check_errors(err, "fp64")


def test_steps_move_the_plane(orc):
    # off-surface queries: the stepped plane differs from the t = 0 plane by
    # far more than the tolerance, so the parity above is not vacuous
    P = synth.sphere(20000, 0.01, seed=1)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h)
    Q = (Pt.double() * (1.0 + 0.5 * h))[:2000].contiguous()
    o0, _ = g.project(Q, 32, "fp64")
    o3, _ = g.project(Q, 32, "fp64", plane_iters=3)
    torch.cuda.synchronize()
    assert (o3 - o0).norm(dim=1).max().item() > 1e-6 * h


def test_adjoint_rejects_steps():
    from paper_2401_03365_amd import _abi
    a = api()
    P = synth.sphere(2000, 0.01, seed=2)
    h = synth.mean_nn_h(P)
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h)
    prm = _abi.MlsParams(k=16, precision=_abi.MLS_PREC_FP32_MOMENTS, support_radius_h=3.0,
                         min_support=3, stages=0, search_extra=0, plane_iters=2)
    gq = torch.empty_like(Pt)
    gp = torch.empty_like(Pt)
    ws = g._proj_workspace(16, Pt.shape[0])
    code = _abi.load().mls_project_backward(
        g._handle, ctypes.byref(prm), ctypes.c_void_p(Pt.data_ptr()), _abi.MLS_F32, Pt.shape[0],
        None, None, ctypes.c_void_p(Pt.data_ptr()), ctypes.c_void_p(gq.data_ptr()),
        ctypes.c_void_p(gp.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert code == _abi.MLS_ERR_UNSUPPORTED
    bad = _abi.MlsParams(k=16, precision=_abi.MLS_PREC_FP32_MOMENTS, support_radius_h=3.0,
                         min_support=3, stages=0, search_extra=0,
                         plane_iters=_abi.MLS_MAX_PLANE_ITERS + 1)
    out = torch.empty_like(Pt)
    st = torch.empty((Pt.shape[0],), dtype=torch.uint8, device="cuda")
    code = _abi.load().mls_project(
        g._handle, ctypes.byref(bad), ctypes.c_void_p(Pt.data_ptr()), _abi.MLS_F32, Pt.shape[0],
        None, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.data_ptr()), None,
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert code == _abi.MLS_ERR_INVALID_ARGUMENT
