"""mls_rebuild_grid: a grid re-sorted for new point positions with kernels
only (the first build's geometry and table size kept), so that it can be
captured in a HIP graph.

- Rebuilt on the same points, the grid (sorted points, inverse permutation)
  and every projection are those of the first build, bit for bit.
- Rebuilt on moved points (jitter, points thrown outside the first build's
  box, non-finite points), the neighbour lists equal the oracle's brute force
  on the moved cloud bit for bit and the projections meet the parity bars.
- A first build on a tight cluster gives a small table; rebuilt on a spread
  cloud no level fits it, every lookup finds nothing and the search still
  returns the exact lists (through its exhaustive path).
- Captured in a graph with a search and a fit and replayed after new
  positions were copied into the captured input, each replay's results equal
  the same calls made eagerly, bit for bit, and the rebuilt grid's lists
  equal a fresh build's, replay after replay."""
import numpy as np
import pytest
import torch

from paper_2401_03365_amd import synth
from tests.parity import check_projection
from tests.test_gpu_grid import check_table, grid_keys

pytestmark = pytest.mark.gpu


def api():
    from paper_2401_03365_amd import api as a
    return a


def same(a, b):
    return torch.equal(torch.nan_to_num(a, nan=7.0), torch.nan_to_num(b, nan=7.0))


def test_rebuild_on_the_same_points_is_identical():
    P = synth.torus(30000, sigma=0.005, n_outliers=300, seed=71)
    h = synth.mean_nn_h(P)
    Pt = torch.from_numpy(P).cuda()
    g = api().Grid(Pt, h)
    spts, inv = g.sorted_points()
    s0, i0 = spts.clone(), inv.clone()
    o0, st0, nb0 = g.project(Pt.double(), 32, "fp64", return_neighbors=True)
    g.rebuild(Pt.clone())
    o1, st1, nb1 = g.project(Pt.double(), 32, "fp64", return_neighbors=True)
    torch.cuda.synchronize()
    spts, inv = g.sorted_points()
    assert torch.equal(spts, s0) and torch.equal(inv, i0)
    assert torch.equal(nb0, nb1) and torch.equal(st0, st1) and same(o0, o1)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rebuild_on_moved_points_is_exact(orc, precision):
    P = synth.sphere(30000, 0.01, seed=72)
    h = synth.mean_nn_h(P)
    g = api().Grid(torch.from_numpy(P).cuda(), h)
    rng = np.random.default_rng(73)
    M = (P + rng.uniform(-0.3, 0.3, P.shape).astype(np.float32) * np.float32(h))
    M[:40] *= np.float32(3.0)          # far outside the first build's box
    M[100:103] = np.nan                # non-finite
    Mt = torch.from_numpy(M).cuda()
    g.rebuild(Mt)
    if precision == "fp64":  # the rebuilt order and cell table, from the grid's geometry
        check_table(g, grid_keys(g, M, np.array([0, M.shape[0]]))[0])
    Q = M[rng.choice(M.shape[0], 4000, replace=False)].astype(np.float64)
    Q = Q[np.isfinite(Q).all(axis=1)]
    Qt = torch.from_numpy(Q).cuda()
    nbr = g.knn(Qt, 32)
    out, st = g.project(Qt, 32, precision)
    torch.cuda.synchronize()
    M64 = M.astype(np.float64)
    ref_nbr, _ = orc.knn(M64, Q, 32)
    np.testing.assert_array_equal(nbr.cpu().numpy(), ref_nbr)
    check_projection(orc, M64, Q, 32, h, out.cpu().numpy(), st.cpu().numpy(), precision,
                     nbr=ref_nbr, label="rebuilt")
    # the same lists as a fresh build of the moved cloud
    f = api().Grid(Mt, h)
    assert torch.equal(f.knn(Qt, 32), nbr)


def test_rebuild_with_levels_left_out_stays_exact(orc):
    # first build: two tight clusters at opposite corners of the unit cube
    # (a large grid with few occupied cells, so a small table); rebuilt on
    # points spread over the cube, the level-0 cells alone overfill half of
    # that table, so no level is inserted and every lookup finds nothing
    rng = np.random.default_rng(74)
    tight = np.concatenate([rng.normal(size=(1000, 3)) * 1e-3,
                            1.0 + rng.normal(size=(1000, 3)) * 1e-3]).astype(np.float32)
    spread = rng.uniform(0.0, 1.0, (2000, 3)).astype(np.float32)
    g = api().Grid(torch.from_numpy(tight).cuda(), 2e-3)
    cap = g.info()["hash_capacity"]
    origin, cell, dims = g.cloud_grid(0)
    c = np.clip(np.floor((spread.astype(np.float64) - origin) / cell), 0, np.array(dims) - 1)
    assert len(np.unique(c, axis=0)) > cap // 2
    g.rebuild(torch.from_numpy(spread).cuda())
    check_table(g, grid_keys(g, spread, np.array([0, spread.shape[0]]))[0], levels=0)
    Q = spread[:300].astype(np.float64)
    nbr = g.knn(torch.from_numpy(Q).cuda(), 16)
    torch.cuda.synchronize()
    ref, _ = orc.knn(spread.astype(np.float64), Q, 16)
    np.testing.assert_array_equal(nbr.cpu().numpy(), ref)


def test_rebuild_search_and_fit_in_one_graph():
    k = 32
    P1 = synth.heightfield(40000, sigma=1e-3, seed=75)
    h = synth.mean_nn_h(P1)
    rng = np.random.default_rng(76)
    moves = [P1 + rng.uniform(-0.4, 0.4, P1.shape).astype(np.float32) * np.float32(h)
             for _ in range(3)]
    buf = torch.from_numpy(P1).cuda()
    g = api().Grid(buf.clone(), h)
    q = torch.empty((P1.shape[0], 3), dtype=torch.float64, device="cuda")
    out = torch.empty_like(q)
    st = torch.empty((P1.shape[0],), dtype=torch.uint8, device="cuda")

    def body():
        g.rebuild(buf)
        q.copy_(buf)
        g.project(q, k, "fp32", out=out, status=st)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        body()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        body()
    for M in moves + moves[:1]:
        buf.copy_(torch.from_numpy(M).cuda())
        graph.replay()
        torch.cuda.synchronize()
        got_o, got_s = out.clone(), st.clone()
        # the same calls eagerly, between the replays: bit for bit
        body()
        torch.cuda.synchronize()
        assert torch.equal(got_s, st) and torch.equal(got_o, out)
        # and the rebuilt grid's lists are a fresh build's
        Mt = torch.from_numpy(M).cuda()
        f = api().Grid(Mt, h)
        sample = Mt[::37].double()
        assert torch.equal(g.knn(sample, k), f.knn(sample, k))
        ref_o, ref_s = f.project(Mt.double(), k, "fp64")
        torch.cuda.synchronize()
        err = (got_o - ref_o).norm(dim=1).max().item() / h
        assert err <= 1e-4, err  # the FP32-moment path against the FP64 path
