"""Queries that are not the grid's points are processed in the Morton order
of their cells (a sort at each fresh search); the stages that continue from
a search (fit only, refresh, the adjoint with the search's lists) keep that
search's slots. Checked here: results do not depend on the caller's order
(a permutation of the queries permutes the returned lists, the statuses and,
fitted from lists in that ascending order, the outputs bit for bit), refresh
and fit-only calls on such queries match the oracle, and the adjoint reusing
the lists equals the adjoint with its own search."""
import numpy as np
import pytest
import torch

from paper_2401_03365_amd import synth
from tests.parity import check_projection

pytestmark = pytest.mark.gpu


def api():
    from paper_2401_03365_amd import api as a
    return a


def jittered(P, per, scale_h, h, seed):
    rng = np.random.default_rng(seed)
    Q = np.repeat(P.astype(np.float64), per, axis=0)
    return Q + rng.uniform(-scale_h, scale_h, Q.shape) * h


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_permutation_of_queries_permutes_results(orc, precision):
    P = synth.torus(20000, sigma=0.005, n_outliers=100, seed=81)
    h = synth.mean_nn_h(P)
    Q = jittered(P, 3, 0.4, h, 82)
    Q[7] = np.nan  # a non-finite query sorts last
    perm = np.random.default_rng(83).permutation(Q.shape[0])
    g = api().Grid(torch.from_numpy(P).cuda(), h)
    o1, s1, n1 = g.project(torch.from_numpy(Q).cuda(), 32, precision, return_neighbors=True)
    o2, s2, n2 = g.project(torch.from_numpy(Q[perm]).cuda(), 32, precision,
                           return_neighbors=True)
    torch.cuda.synchronize()
    p = torch.from_numpy(perm).cuda()
    assert torch.equal(n2, n1[p]) and torch.equal(s2, s1[p])
    assert torch.equal(torch.nan_to_num(o2, nan=7.0), torch.nan_to_num(o1[p], nan=7.0))
    ref_nbr, _ = orc.knn(P.astype(np.float64), Q[perm][:4000], 32)
    np.testing.assert_array_equal(n2[:4000].cpu().numpy(), ref_nbr)


def test_refresh_and_fit_only_on_unaligned_queries(orc):
    P = synth.heightfield(30000, sigma=1e-3, seed=84)
    h = synth.mean_nn_h(P)
    P64 = P.astype(np.float64)
    g = api().Grid(torch.from_numpy(P).cuda(), h)
    q0 = jittered(P, 2, 0.4, h, 85)
    rng = np.random.default_rng(86)
    perm = rng.permutation(q0.shape[0])
    q0 = q0[perm]
    # search only, then fit only from its lists
    g.project(torch.from_numpy(q0).cuda(), 32, "fp64", stages=1, search_extra=16)
    out, st = g.project(torch.from_numpy(q0).cuda(), 32, "fp64", stages=2, search_extra=16)
    check_projection(orc, P64, q0, 32, h, out.cpu().numpy(), st.cpu().numpy(), "fp64",
                     surface=False)
    # the queries move a little: the refresh keeps the slots of the search
    q1 = q0 + rng.normal(size=q0.shape) * 0.05 * h
    out, st, nbr = g.project(torch.from_numpy(q1).cuda(), 32, "fp64", return_neighbors=True,
                             search_extra=16, refresh=True)
    ref_nbr, _ = orc.knn(P64, q1, 32)
    np.testing.assert_array_equal(nbr.cpu().numpy(), ref_nbr)
    check_projection(orc, P64, q1, 32, h, out.cpu().numpy(), st.cpu().numpy(), "fp64",
                     nbr=ref_nbr, surface=False)


def test_batch_of_clouds_with_shuffled_query_ranges(orc):
    parts = [synth.sphere(3000, 0.01, seed=87), synth.torus(4000, sigma=0.01, seed=88)]
    offs = np.array([0, 3000, 7000], dtype=np.int64)
    P = np.concatenate(parts)
    hs = [synth.mean_nn_h(p) for p in parts]
    qs = [jittered(p, 2, 0.3, hc, 89 + c)[np.random.default_rng(91 + c).permutation(2 * len(p))]
          for c, (p, hc) in enumerate(zip(parts, hs))]
    qoffs = np.array([0, len(qs[0]), len(qs[0]) + len(qs[1])], dtype=np.int64)
    Q = np.concatenate(qs)
    g = api().Grid(torch.from_numpy(P).cuda(), hs, cloud_offsets=offs)
    nbr, keys = g.knn(torch.from_numpy(Q).cuda(), 24, query_offsets=qoffs, return_keys=True)
    torch.cuda.synchronize()
    nbr, keys = nbr.cpu().numpy(), keys.cpu().numpy()
    for c, p in enumerate(parts):
        sl = slice(qoffs[c], qoffs[c + 1])
        ref_idx, ref_key = orc.knn(p.astype(np.float64), qs[c], 24)
        np.testing.assert_array_equal(nbr[sl] - offs[c], ref_idx)
        np.testing.assert_array_equal(keys[sl], ref_key)


def test_adjoint_reusing_the_search_on_unaligned_queries():
    P = synth.torus(30000, sigma=0.005, seed=92)
    h = synth.mean_nn_h(P)
    Q = jittered(P, 2, 0.3, h, 93).astype(np.float32)
    Q = Q[np.random.default_rng(94).permutation(Q.shape[0])]
    a = api()
    g = a.Grid(torch.from_numpy(P).cuda(), h)
    Qt = torch.from_numpy(Q).cuda()
    gout = torch.from_numpy(np.random.default_rng(95).normal(size=Q.shape).astype(np.float32)).cuda()
    gq_fresh, gp_fresh = g.project_backward(Qt, gout, 32, "fp32")
    g.project(Qt, 32, "fp32")
    gq_reuse, gp_reuse = g.project_backward(Qt, gout, 32, "fp32", reuse_lists=True)
    # a permutation of the queries permutes the query gradients (the lists
    # hold the same sets; without returned lists the order of a list's
    # entries may differ, and the FP32 sums round differently: within the
    # adjoint's parity bar)
    perm = torch.from_numpy(np.random.default_rng(96).permutation(Q.shape[0])).cuda()
    gq_perm, gp_perm = g.project_backward(Qt[perm].contiguous(), gout[perm].contiguous(), 32,
                                          "fp32")
    torch.cuda.synchronize()
    assert torch.equal(gq_fresh, gq_reuse)
    assert (gp_fresh - gp_reuse).norm() <= 1e-5 * gp_fresh.norm()
    assert (gq_perm - gq_fresh[perm]).norm() <= 1e-4 * gq_fresh.norm()
    assert (gp_perm - gp_fresh).norm() <= 1e-4 * gp_fresh.norm()


@pytest.mark.parametrize("n", [1, 2, 63, 65, 129])
def test_small_unaligned_query_counts(orc, n):
    # the sort of a handful of queries (single radix tiles, ragged last
    # search tile), FP32 queries, lists bit for bit and the projection
    P = synth.sphere(5000, 0.01, seed=97)
    h = synth.mean_nn_h(P)
    rng = np.random.default_rng(98 + n)
    Q = (P[rng.choice(P.shape[0], n)].astype(np.float64) +
         rng.uniform(-0.5, 0.5, (n, 3)) * h).astype(np.float32)
    g = api().Grid(torch.from_numpy(P).cuda(), h)
    nbr, keys = g.knn(torch.from_numpy(Q).cuda(), 16, return_keys=True)
    out, st = g.project(torch.from_numpy(Q).cuda(), 16, "fp64")
    torch.cuda.synchronize()
    P64, Q64 = P.astype(np.float64), Q.astype(np.float64)
    ref_idx, ref_key = orc.knn(P64, Q64, 16)
    np.testing.assert_array_equal(nbr.cpu().numpy(), ref_idx)
    np.testing.assert_array_equal(keys.cpu().numpy(), ref_key)
    check_projection(orc, P64, Q64, 16, h, out.cpu().numpy(), st.cpu().numpy(), "fp64",
                     nbr=ref_idx, surface=False)
