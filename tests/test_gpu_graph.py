"""Batches of clouds, HIP-graph capture and the cell-size tuner on the GPU.

A batch of three clouds of different shapes, sizes and h shares one grid
(per-cloud geometry). The forward (search + fit), an elementwise loss
gradient and the adjoint (reusing the search's lists) are captured in one
graph and replayed several times, with eager work in between; every replay
must reproduce the eager results (projection and query gradients bit for
bit: same kernels, same inputs; point gradients to rounding, since their
atomic summation order varies). The same holds for queries that are not
the cloud's points, whose captured search sorts them first."""
import numpy as np
import pytest
import torch

from paper_2401_03365_amd import synth

pytestmark = pytest.mark.gpu


def api():
    from paper_2401_03365_amd import api as a
    return a


def small_batch():
    parts = [synth.sphere(20000, 0.01, seed=31), synth.torus(30000, sigma=0.004, seed=32),
             synth.heightfield(25000, sigma=2e-3, seed=33)]
    off = np.concatenate([[0], np.cumsum([p.shape[0] for p in parts])]).astype(np.int64)
    h = np.array([synth.mean_nn_h(p) for p in parts])
    return np.concatenate(parts), off, h


def test_batch_matches_single_clouds():
    a = api()
    P, off, h = small_batch()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h, cloud_offsets=off)
    out, st = g.project(Pt, 32, "fp64")
    gout = torch.ones_like(Pt)
    gq, gp = g.project_backward(Pt, gout, 32, "fp64")
    torch.cuda.synchronize()
    for c in range(3):
        sl = slice(int(off[c]), int(off[c + 1]))
        gc = a.Grid(Pt[sl].contiguous(), h[c])
        oc, sc = gc.project(Pt[sl].contiguous(), 32, "fp64")
        qc, pc = gc.project_backward(Pt[sl].contiguous(), gout[sl].contiguous(), 32, "fp64")
        torch.cuda.synchronize()
        assert torch.equal(sc, st[sl])
        assert (oc - out[sl]).abs().max().item() <= 1e-12 * h[c]
        assert (qc - gq[sl]).abs().max().item() <= 1e-9 * qc.abs().max().item()
        assert (pc - gp[sl]).abs().max().item() <= 1e-9 * pc.abs().max().item()


def test_graph_replay_matches_eager():
    a = api()
    P, off, h = small_batch()
    pts = torch.from_numpy(P).cuda()
    g = a.Grid(pts, h, cloud_offsets=off)
    k = 32
    out = torch.empty_like(pts)
    status = torch.empty((pts.shape[0],), dtype=torch.uint8, device="cuda")
    q = pts.clone()

    def body():
        g.project(q, k, "fp32", stages=1, out=out, status=status)
        g.project(q, k, "fp32", stages=2, out=out, status=status)
        gout = (out - q) * (2.0 / q.shape[0])  # d/d out of mean |out - q|^2, elementwise
        gq, gp = g.project_backward(q, gout, k, "fp32", reuse_lists=True)
        return gq, gp

    gq_e, gp_e = body()
    torch.cuda.synchronize()
    out_e, st_e = out.clone(), status.clone()

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        body()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gq_g, gp_g = body()
    torch.cuda.synchronize()

    for rep in range(3):
        out.zero_()
        status.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, out_e), rep
        assert torch.equal(status, st_e), rep
        assert torch.equal(gq_g, gq_e), rep
        assert (gp_g - gp_e).norm() <= 1e-5 * gp_e.norm(), rep
        # eager work on the same grid between replays
        o2, s2 = g.project(pts[:1000].contiguous(), k, "fp64", query_offsets=[0, 1000, 1000, 1000])
        torch.cuda.synchronize()


def test_autotune_picks_a_measured_candidate():
    a = api()
    P, off, h = small_batch()
    pts = torch.from_numpy(P).cuda()
    best, ms = a.autotune_cell_factor(pts, h, 32, cloud_offsets=off,
                                      candidates=(0.7, 1.25, 3.0), stride=4)
    assert best in ms and all(t > 0 for t in ms.values())
    assert ms[best] == min(ms.values())
    # the tuned grid gives the same lists as the default one
    g1 = a.Grid(pts, h, cloud_offsets=off)
    g2 = a.Grid(pts, h, cloud_offsets=off, cell_size=best * h)
    n1 = g1.knn(pts, 32)
    n2 = g2.knn(pts, 32)
    torch.cuda.synchronize()
    assert torch.equal(n1, n2)


def test_graph_replay_with_unaligned_queries():
    # queries that are not the cloud's points: the captured search sorts them
    # (kernels only), the fit and the adjoint keep its slots; replays with
    # other queries projected eagerly on the same grid in between
    a = api()
    P = synth.torus(30000, sigma=0.004, seed=34)
    h = synth.mean_nn_h(P)
    pts = torch.from_numpy(P).cuda()
    g = a.Grid(pts, h)
    rng = np.random.default_rng(35)
    Q = np.repeat(P, 2, axis=0) + rng.uniform(-0.3, 0.3, (2 * P.shape[0], 3)).astype(np.float32) * h
    q = torch.from_numpy(Q[rng.permutation(Q.shape[0])]).cuda()
    k = 32
    out = torch.empty_like(q)
    status = torch.empty((q.shape[0],), dtype=torch.uint8, device="cuda")
    gout = torch.from_numpy(rng.normal(size=Q.shape).astype(np.float32)).cuda()

    def body():
        g.project(q, k, "fp32", stages=1, out=out, status=status)
        g.project(q, k, "fp32", stages=2, out=out, status=status)
        return g.project_backward(q, gout, k, "fp32", reuse_lists=True)

    gq_e, gp_e = body()
    torch.cuda.synchronize()
    out_e, st_e = out.clone(), status.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        body()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gq_g, gp_g = body()
    torch.cuda.synchronize()
    for rep in range(3):
        out.zero_()
        status.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, out_e), rep
        assert torch.equal(status, st_e), rep
        assert torch.equal(gq_g, gq_e), rep
        assert (gp_g - gp_e).norm() <= 1e-5 * gp_e.norm(), rep
        o2, s2 = g.project(q[: q.shape[0] // 3].flip(0).contiguous(), k, "fp32")
        torch.cuda.synchronize()
