"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (queries aligned with the cloud's points, one call over the
whole cloud), on sampled queries that the oracle computes one by one with
brute-force kNN over the whole cloud:

  torus 1,010,000 (1 % outliers), k = 32, FP32-moment and FP64 paths;
  height field 10,000,000, k = 48, 3 iterated passes, FP32-moment and FP64
      paths (each pass checked against the oracle fed the GPU's own pass
      input), one pass
      with 3 frozen-weight steps of the reference plane, one pass with
      Levin's plane (both paths), and 40,000,000
      upsampling queries (positions, lists, geometry);
  bumped sphere 2,000,000, k = 32, FP32 forward and the adjoint (1,000
      queries against central finite differences, by themselves and as the
      only nonzero output gradients of the whole-cloud call);
  batch of 256 clouds, ~30M points, k = 32, FP32.

Bars as in the small-size tests: neighbour lists and statuses bit for bit,
FP64 max error <= 1e-10 h, FP32-moment RMS <= 1e-5 h (points whose normal is
flagged ambiguous excluded from max errors), adjoint <= 1e-4 relative."""
import numpy as np
import pytest
import torch

from paper_2401_03365_amd import synth
from tests.parity import check_projection

pytestmark = pytest.mark.gpu

FP64_MAX_H = 1e-10
FP32_RMS_H = 1e-5


def api():
    from paper_2401_03365_amd import api as a
    return a


def check_sample(orc, P64, Qs, k, h, out, st, nbr, precision, label="", **kw):
    """Qs: the sampled queries of the pass input (FP64); out/st/nbr: the GPU
    results for them."""
    ref_nbr, _ = orc.knn(P64, Qs, k)
    np.testing.assert_array_equal(nbr, ref_nbr)
    return check_projection(orc, P64, Qs, k, h, out, st, precision, nbr=ref_nbr, label=label,
                            **kw)


def run_pass(g, q, k, precision, idx_t, **kw):
    out, st, nbr = g.project(q, k, precision, return_neighbors=True, **kw)
    torch.cuda.synchronize()
    return out, st, nbr[idx_t].cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_torus_1m_with_outliers(orc, precision):
    P, mask = synth.torus(1_000_000, sigma=0.005, n_outliers=10_000, seed=2, return_mask=True)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h)
    rng = np.random.default_rng(21)
    idx = np.concatenate([rng.choice(1_000_000, 400, replace=False),
                          1_000_000 + rng.choice(10_000, 100, replace=False)])
    idx_t = torch.from_numpy(idx).cuda()
    q = Pt.double()
    out, st, nbr = run_pass(g, q, 32, precision, idx_t)
    P64 = P.astype(np.float64)
    check_sample(orc, P64, P64[idx], 32, h, out[idx_t].cpu().numpy(),
                 st[idx_t].cpu().numpy(), nbr, precision)
    assert ((st[idx_t[400:]] & 0x0F) == 1).sum().item() > 50  # most outliers flagged


def sampled_tile_sets(g, k_list, kfit, qidx):
    """Sorted original indices of the first kfit entries of the sampled
    queries' lists in the projection workspace (queries aligned with the
    points; the lists lead the workspace in tiles of 64 slots)."""
    spts, inv = g.sorted_points()
    n = spts.shape[0]
    tiles = (n + 63) // 64
    raw = g._proj_ws[: 4 * tiles * 64 * k_list].view(torch.int32).view(tiles, k_list, 64)
    slots = inv[qidx].long()
    pos = raw[slots >> 6, :kfit, :].gather(2, (slots & 63).view(-1, 1, 1).expand(-1, kfit, 1))
    orig = spts[:, 3].contiguous().view(torch.int32).long()
    return torch.sort(orig[pos.view(-1, kfit).long()], dim=1).values.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_heightfield_10m_three_passes(orc, precision):
    P = synth.heightfield(10_000_000, sigma=1e-3, seed=3)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h, cell_size=1.25 * h)
    rng = np.random.default_rng(22)
    idx = np.sort(rng.choice(P.shape[0], 192, replace=False))
    idx_t = torch.from_numpy(idx).cuda()
    P64 = P.astype(np.float64)
    cur = Pt.double()
    for it in range(3):
        # as timed: the second search keeps 16 more, the third pass refreshes
        extra = 16 if it > 0 else 0
        out, st = g.project(cur, 48, precision, search_extra=extra, refresh=it == 2)
        torch.cuda.synchronize()
        sets = sampled_tile_sets(g, 48 + extra, 48, idx_t)
        qs = cur[idx_t].cpu().numpy()
        ref_nbr, _ = orc.knn(P64, qs, 48)
        np.testing.assert_array_equal(sets, np.sort(ref_nbr, axis=1))
        check_sample(orc, P64, qs, 48, h, out[idx_t].cpu().numpy(), st[idx_t].cpu().numpy(),
                     ref_nbr, precision)
        cur = out


def test_heightfield_10m_plane_steps(orc):
    # the self-consistent reference plane (3 steps), FP32-moment path, one
    # call over the whole cloud as timed
    P = synth.heightfield(10_000_000, sigma=1e-3, seed=3)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h, cell_size=1.25 * h)
    rng = np.random.default_rng(25)
    idx = np.sort(rng.choice(P.shape[0], 192, replace=False))
    idx_t = torch.from_numpy(idx).cuda()
    out, st = g.project(Pt.double(), 48, "fp32", plane_iters=3)
    torch.cuda.synchronize()
    P64 = P.astype(np.float64)
    Qs = P64[idx]
    ref_nbr, _ = orc.knn(P64, Qs, 48)
    check_projection(orc, P64, Qs, 48, h, out[idx_t].cpu().numpy(), st[idx_t].cpu().numpy(),
                     "fp32", nbr=ref_nbr, plane_iters=3, label="plane steps")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_heightfield_10m_levin(orc, precision):
    # Levin's reference plane (Newton on Eq. (1.1) over (n, t)), one call
    # over the whole cloud as timed
    print("10M height field, Levin plane, %s" % precision, flush=True)
    P = synth.heightfield(10_000_000, sigma=1e-3, seed=3)
    h = synth.mean_nn_h(P)
    Pt = torch.from_numpy(P).cuda()
    g = api().Grid(Pt, h, cell_size=1.25 * h)
    rng = np.random.default_rng(26)
    idx = np.sort(rng.choice(P.shape[0], 256, replace=False))
    idx_t = torch.from_numpy(idx).cuda()
    out, st = g.project(Pt.double(), 48, precision, levin=True)
    torch.cuda.synchronize()
    P64 = P.astype(np.float64)
    Qs = P64[idx]
    ref_nbr, _ = orc.knn(P64, Qs, 48)
    check_projection(orc, P64, Qs, 48, h, out[idx_t].cpu().numpy(), st[idx_t].cpu().numpy(),
                     precision, nbr=ref_nbr, levin=True, label="levin 10M")


def test_heightfield_10m_upsampling_40m(orc):
    # 4 queries per sample jittered by up to 0.4 h (not the cloud's points:
    # sorted by cell before the search), one call as timed, then once more
    # with the lists and the geometry returned
    P = synth.heightfield(10_000_000, sigma=1e-3, seed=3)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h, cell_size=1.25 * h)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(71)
    q = Pt.double()
    up = (q.repeat_interleave(4, dim=0) +
          (torch.rand((4 * q.shape[0], 3), generator=gen, device="cuda", dtype=torch.float64)
           - 0.5) * (0.8 * h))
    del q
    rng = np.random.default_rng(27)
    idx = np.sort(rng.choice(up.shape[0], 192, replace=False))
    idx_t = torch.from_numpy(idx).cuda()
    out, st = g.project(up, 48, "fp32")
    torch.cuda.synchronize()
    P64 = P.astype(np.float64)
    Qs = up[idx_t].cpu().numpy()
    ref_nbr, _ = orc.knn(P64, Qs, 48)
    check_sample(orc, P64, Qs, 48, h, out[idx_t].cpu().numpy(), st[idx_t].cpu().numpy(),
                 ref_nbr, "fp32")
    out2, st2, nrm, curv, nbr = g.project(up, 48, "fp32", geometry=True, return_neighbors=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(nbr[idx_t].cpu().numpy(), ref_nbr)
    assert torch.equal(st2, st)
    _, ref_st, geo = orc.project(P64, Qs, 48, h, nbr=ref_nbr, geometry=True)
    ok = ((ref_st & 0x0F) == 0) & ((ref_st & 0x10) == 0)
    n_s = nrm[idx_t].cpu().numpy()[ok]
    sgn = np.sign(np.sum(n_s * geo[ok, :3], axis=1))
    dN = np.linalg.norm(n_s - sgn[:, None] * geo[ok, :3], axis=1)
    dH = np.abs(curv[idx_t].cpu().numpy()[ok, 0] * sgn - geo[ok, 3]) * h
    assert np.sqrt((dN ** 2).mean()) <= 1e-4 and np.sqrt((dH ** 2).mean()) <= 1e-3


def test_bumped_sphere_2m_forward_and_adjoint(orc):
    P = synth.sh_sphere(2_000_000, sigma=0.005, seed=4)
    h = synth.mean_nn_h(P)
    a = api()
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h, cell_size=1.25 * h)
    rng = np.random.default_rng(23)
    idx = np.sort(rng.choice(P.shape[0], 1000, replace=False))
    idx_t = torch.from_numpy(idx).cuda()
    out, st, nbr = run_pass(g, Pt, 32, "fp32", idx_t)
    P64 = P.astype(np.float64)
    check_sample(orc, P64, P64[idx[:300]], 32, h, out[idx_t[:300]].cpu().numpy(),
                 st[idx_t[:300]].cpu().numpy(), nbr[:300], "fp32")
    # adjoint: the full aligned call (as timed) and the 1,000 sampled queries
    gout = torch.from_numpy(rng.normal(size=P.shape).astype(np.float32)).cuda()
    gq_full, _ = g.project_backward(Pt, gout, 32, "fp32")
    Qs = P64[idx]
    ref_nbr, _ = orc.knn(P64, Qs, 32)
    _, ref_st = orc.project(P64, Qs, 32, h, nbr=ref_nbr)
    keep = (ref_st & 0x10) == 0
    Qs, ref_nbr = Qs[keep], ref_nbr[keep]
    go = gout[idx_t].cpu().numpy().astype(np.float64)[keep]
    fq, fp = orc.grad_fd(P64, Qs, 32, h, ref_nbr, go)
    Qt = torch.from_numpy(Qs).cuda()
    gq, gp = g.project_backward(Qt, torch.from_numpy(go).cuda(), 32, "fp32",
                                neighbors=torch.from_numpy(ref_nbr).cuda())
    torch.cuda.synchronize()
    gq, gp = gq.cpu().numpy(), gp.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gq - fq) <= 1e-4 * np.linalg.norm(fq)
    assert np.linalg.norm(gp - fp) <= 1e-4 * np.linalg.norm(fp)
    # the full call's query gradients agree with the sampled call's
    gfull = gq_full[idx_t].cpu().numpy().astype(np.float64)[keep]
    assert np.linalg.norm(gfull - gq) <= 1e-5 * np.linalg.norm(gq)
    # the full aligned call with the output gradient only at the checked
    # queries: its point gradients are summed in the block tables of
    # Morton-consecutive queries (the timed path) and must meet the finite
    # differences too
    gm = torch.zeros_like(gout)
    kidx = idx_t[torch.from_numpy(keep).cuda()]
    gm[kidx] = torch.from_numpy(go.astype(np.float32)).cuda()
    _, gp_m = g.project_backward(Pt, gm, 32, "fp32")
    torch.cuda.synchronize()
    gp_m = gp_m.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gp_m - fp) <= 1e-4 * np.linalg.norm(fp), \
        np.linalg.norm(gp_m - fp) / np.linalg.norm(fp)


def test_batch_256_clouds(orc):
    P, off, sig, shapes = synth.batch()
    a = api()
    sel = [0, 1, 2, 100, 177, 255]  # sphere, torus, height field, ...
    h = np.array([synth.mean_nn_h(P[off[c]:off[c + 1]]) for c in range(len(off) - 1)])
    Pt = torch.from_numpy(P).cuda()
    g = a.Grid(Pt, h, cloud_offsets=off, cell_size=2.0 * h)
    rng = np.random.default_rng(24)
    idx = np.concatenate([off[c] + rng.choice(off[c + 1] - off[c], 48, replace=False)
                          for c in sel])
    idx_t = torch.from_numpy(idx).cuda()
    out, st, nbr = run_pass(g, Pt, 32, "fp32", idx_t)
    out_s, st_s = out[idx_t].cpu().numpy(), st[idx_t].cpu().numpy()
    for j, c in enumerate(sel):
        rows = slice(48 * j, 48 * (j + 1))
        Pc = P[off[c]:off[c + 1]].astype(np.float64)
        local = idx[rows] - off[c]
        check_sample(orc, Pc, Pc[local], 32, h[c], out_s[rows], st_s[rows],
                     nbr[rows] - off[c], "fp32")
