"""mls_project_noalloc: one whole pass with the library's fixed device scratch
as its workspace. Its results must equal mls_project's on the same inputs
(the same kernels run, so outputs, statuses and lists agree bit for bit), on
two calls in a row, the second with fewer queries (queries that are not the
grid's points, so that the second call sorts them in the scratch the first
call filled with lists); calls beyond the scratch are refused on the host."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2401_03365_amd import synth

pytestmark = pytest.mark.gpu


def api():
    from paper_2401_03365_amd import api as a
    return a


def same(a, b):
    return torch.equal(torch.nan_to_num(a, nan=7.0), torch.nan_to_num(b, nan=7.0))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_matches_project_on_two_calls(precision):
    print("noalloc: sphere 20000, k 32, %s" % precision, flush=True)
    P = synth.sphere(20000, 0.01, seed=91)
    h = synth.mean_nn_h(P)
    g = api().Grid(torch.from_numpy(P).cuda(), h)
    k = 32
    dt = torch.float64 if precision == "fp64" else torch.float32
    # call 1: the cloud's own points (grid order)
    q1 = torch.from_numpy(P).cuda().to(dt)
    ref1, rst1, rnb1 = g.project(q1, k, precision, return_neighbors=True)
    out1 = torch.empty_like(q1)
    st1 = torch.empty(q1.shape[0], dtype=torch.uint8, device="cuda")
    nb1 = torch.empty((q1.shape[0], k), dtype=torch.int32, device="cuda")
    g.project_noalloc(q1, k, precision, out=out1, status=st1, neighbors=nb1)
    torch.cuda.synchronize()
    assert torch.equal(nb1, rnb1)
    assert torch.equal(st1, rst1)
    assert same(out1, ref1)
    # call 2: fewer queries, off the cloud and in no particular order
    rng = np.random.default_rng(92)
    Q = P[rng.permutation(P.shape[0])[:3001]].astype(np.float64)
    Q += rng.uniform(-0.3, 0.3, Q.shape) * h
    Q[5] = np.nan
    q2 = torch.from_numpy(Q).cuda().to(dt)
    out2 = torch.empty_like(q2)
    st2 = torch.empty(q2.shape[0], dtype=torch.uint8, device="cuda")
    nb2 = torch.empty((q2.shape[0], k), dtype=torch.int32, device="cuda")
    g.project_noalloc(q2, k, precision, out=out2, status=st2, neighbors=nb2)
    ref2, rst2, rnb2 = g.project(q2, k, precision, return_neighbors=True)
    torch.cuda.synchronize()
    assert torch.equal(nb2, rnb2)
    assert torch.equal(st2, rst2)
    assert same(out2, ref2)
    assert int(st2[5]) & 0x0F == 3  # the non-finite query
    # and the first input again after the smaller call
    g.project_noalloc(q1, k, precision, out=out1, status=st1, neighbors=nb1)
    torch.cuda.synchronize()
    assert torch.equal(nb1, rnb1) and torch.equal(st1, rst1) and same(out1, ref1)


def test_noalloc_batch_with_query_offsets():
    print("noalloc: batch of 3 clouds with query offsets", flush=True)
    sizes = [4000, 9000, 2500]
    clouds = [synth.sphere(sizes[0], 0.01, seed=93), synth.torus(sizes[1], sigma=0.005, seed=94),
              synth.heightfield(sizes[2], 1e-3, seed=95)]
    P = np.concatenate(clouds).astype(np.float32)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    h = [synth.mean_nn_h(c) for c in clouds]
    g = api().Grid(torch.from_numpy(P).cuda(), h, cloud_offsets=off)
    rng = np.random.default_rng(96)
    qs, qoff = [], [0]
    for c, hc in zip(clouds, h):
        m = c.shape[0] // 3
        Q = c[rng.permutation(c.shape[0])[:m]].astype(np.float64)
        qs.append(Q + rng.uniform(-0.2, 0.2, Q.shape) * hc)
        qoff.append(qoff[-1] + m)
    q = torch.from_numpy(np.concatenate(qs)).cuda()
    ref, rst = g.project(q, 32, "fp32", query_offsets=qoff)
    out, st = g.project_noalloc(q, 32, "fp32", query_offsets=qoff)
    torch.cuda.synchronize()
    assert torch.equal(st, rst) and same(out, ref)


def test_noalloc_refuses_what_does_not_fit():
    from paper_2401_03365_amd import _abi
    P = synth.sphere(5000, 0.01, seed=97)
    h = synth.mean_nn_h(P)
    g = api().Grid(torch.from_numpy(P).cuda(), h)
    lib = _abi.load()
    k = 64
    per_query = lib.mls_project_workspace_bytes(g._handle, k, 100000) / 100000
    n = int(_abi.NOALLOC_SCRATCH_BYTES / per_query) + 1000
    assert lib.mls_project_workspace_bytes(g._handle, k, n) > _abi.NOALLOC_SCRATCH_BYTES
    q = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(_abi.MLSError) as ei:
        g.project_noalloc(q, k, "fp32")
    assert ei.value.code == _abi.MLS_ERR_WORKSPACE_TOO_SMALL
    assert b"scratch" in lib.mls_last_error()
    # stages other than a whole pass are refused before any launch
    params = g._params(32, "fp32", 3.0, 3, stages=_abi.MLS_STAGE_FIT)
    out = torch.empty((10, 3), dtype=torch.float32, device="cuda")
    st = torch.empty(10, dtype=torch.uint8, device="cuda")
    code = lib.mls_project_noalloc(g._handle, ctypes.byref(params), ctypes.c_void_p(q.data_ptr()),
                                   _abi.MLS_F32, 10, None, ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(st.data_ptr()), None, None)
    assert code == _abi.MLS_ERR_INVALID_ARGUMENT
    # an empty call is fine
    e = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    g.project_noalloc(e, 32, "fp32")
    torch.cuda.synchronize()
