"""Every list and every position of full-size calls, in the launch
configuration the benchmark times (queries aligned with the cloud's points,
one call over the whole cloud, search and fit as separate stages):

  height field 10,000,000, k = 48, FP32-moment path, 3 iterated passes (the
      second search keeps 16 more neighbours, the third refreshes them): every
      list of every pass exact (its first 48 entries as a set; the second
      pass's 64 entries too), 20,000 queries per pass by brute force over the
      whole cloud, every position against the oracle fed the exact lists;
  torus 1,010,000 (1 % outliers), k = 32: every list, 20,000 by brute force,
      every position on the FP32-moment and FP64 paths.

The list checks are independent of the library's kernels (tests/fullcheck.py);
position bars and status rules are those of tests/parity.py (FP64 max
<= 1e-10 h; FP32-moment RMS <= 1e-5 h and per point max(1e-4 h,
10 eps32 / eigengap h), ambiguous-normal points left out of the max)."""
import time

import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

from paper_2401_03365_amd import synth
from tests.fullcheck import brute_lists, exact_lists, first_mismatch, same_sets, workspace_lists
from tests.parity import check_errors, check_status, fp32_max_bars, oracle_ref, position_errors

pytestmark = pytest.mark.gpu

N_BRUTE = 20_000


def api():
    from paper_2401_03365_amd import api as a
    return a


def log(*a):
    print(*a, flush=True)


def check_lists(orc, tree, P64, Q64, gpu, k, label, rng, sets=()):
    """gpu: (n, k_list) torch lists in query order. Checks the first k as a
    set against the exact lists, and each (k', label') of `sets` likewise;
    returns the exact first-k lists (numpy int32, (key, index) order)."""
    t = time.time()
    kmax = max([k] + [kk for kk, _ in sets])
    ref, n_brute = exact_lists(orc, tree, P64, Q64, kmax)
    for kk, lab in [(k, label)] + list(sets):
        assert same_sets(gpu[:, :kk], ref[:, :kk]), (
            "%s: lists of %d differ at queries %s" % (lab, kk, first_mismatch(gpu[:, :kk], ref[:, :kk])))
    sample = np.sort(rng.choice(Q64.shape[0], min(N_BRUTE, Q64.shape[0]), replace=False))
    bf = brute_lists(P64, Q64[sample], k, chunk=32)
    bf_t = torch.from_numpy(bf).cuda()
    sidx = torch.from_numpy(sample).cuda()
    assert same_sets(gpu[sidx, :k], bf_t), "%s: brute-force sample differs" % label
    assert torch.equal(ref[sidx, :k], bf_t), "%s: the k-d tree lists differ from brute force" % label
    log("%s: %d lists exact (%d by the oracle's brute force at the margin), %d also by "
        "brute force; %.1f s" % (label, Q64.shape[0], n_brute, sample.size, time.time() - t))
    return ref[:, :k].to(torch.int32).cpu().numpy()


def check_positions(orc, P64, Q64, k, h, nbr, out, st, precision, label):
    t = time.time()
    ref, ref_st, lam = oracle_ref(orc, P64, Q64, k, h, nbr=nbr)
    frac = check_status(st, ref_st, lam)
    assert frac <= 0.01, frac
    err, ok = position_errors(out, ref, ref_st, h, return_mask=True)
    bars = fp32_max_bars(lam[ok])
    rms, mx = check_errors(err, precision, max_bar=bars)
    log("%s %s: every position, rms %.2e h, max %.2e h (%d above 1e-4 h, within their "
        "eigengap bars), flagged %.5f; %.1f s"
        % (label, precision, rms, mx, int((err > 1e-4).sum()), frac, time.time() - t))


def test_heightfield_10m_every_list_and_position(orc):
    log("10M height field, k 48, FP32-moment path, 3 passes as timed")
    P = synth.heightfield(10_000_000, sigma=1e-3, seed=3)
    h = synth.mean_nn_h(P)
    P64 = P.astype(np.float64)
    tree = cKDTree(P64, balanced_tree=False, compact_nodes=False)
    Pt = torch.from_numpy(P).cuda()
    g = api().Grid(Pt, h, cell_size=1.25 * h)
    rng = np.random.default_rng(31)
    n = P.shape[0]
    cur = Pt.double()
    for it in range(3):
        extra = 16 if it > 0 else 0
        out = torch.empty_like(cur)
        st = torch.empty(n, dtype=torch.uint8, device="cuda")
        g.project(cur, 48, "fp32", stages=1, out=out, status=st, search_extra=extra,
                  refresh=it == 2)
        torch.cuda.synchronize()
        gpu = workspace_lists(g, 48 + extra, n)
        Q64 = cur.cpu().numpy()
        sets = [(64, "pass %d (64 kept)" % (it + 1))] if it == 1 else []
        nbr = check_lists(orc, tree, P64, Q64, gpu, 48, "pass %d" % (it + 1), rng, sets)
        del gpu
        g.project(cur, 48, "fp32", stages=2, out=out, status=st, search_extra=extra)
        torch.cuda.synchronize()
        check_positions(orc, P64, Q64, 48, h, nbr, out.cpu().numpy(), st.cpu().numpy(), "fp32",
                        "pass %d" % (it + 1))
        cur = out


def test_torus_1m_every_list_and_position(orc):
    log("1.01M torus with outliers, k 32")
    P = synth.torus(1_000_000, sigma=0.005, n_outliers=10_000, seed=2)
    h = synth.mean_nn_h(P)
    P64 = P.astype(np.float64)
    tree = cKDTree(P64)
    Pt = torch.from_numpy(P).cuda()
    g = api().Grid(Pt, h)
    n = P.shape[0]
    rng = np.random.default_rng(32)
    nbr = None
    for precision in ("fp32", "fp64"):
        q = Pt.double()
        out = torch.empty_like(q)
        st = torch.empty(n, dtype=torch.uint8, device="cuda")
        g.project(q, 32, precision, stages=1, out=out, status=st)
        torch.cuda.synchronize()
        if nbr is None:
            gpu = workspace_lists(g, 32, n)
            nbr = check_lists(orc, tree, P64, P64, gpu, 32, "torus", rng)
            del gpu
        g.project(q, 32, precision, stages=2, out=out, status=st)
        torch.cuda.synchronize()
        check_positions(orc, P64, P64, 32, h, nbr, out.cpu().numpy(), st.cpu().numpy(),
                        precision, "torus")
        assert int(((st[1_000_000:] & 0x0F) == 1).sum()) > 5_000  # most outliers flagged
