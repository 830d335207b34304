"""Benchmark of the MLS projection hot path on one MI355X.

Workload (the metric's configuration): a 10,000,000-point noisy height field
(8 random sinusoids of amplitude 0.05 and frequency 1..8 over [0,1]^2,
sampling density ramping 10x across x, noise sigma 1e-3 along the normal),
k = 48, three iterated projection passes with the FP32-moment path.

One step = build the grid of the cloud + 3 passes (each pass: exact kNN
search, then moments / plane / quadratic fit / projection), inputs resident
in HBM; the third pass refreshes the second pass's lists (exact, see
MLS_STAGE_REFRESH). value = 3 N / step time. The same steps are also timed with the FP64
path. Kernel durations come from HIP events recorded on the stream the
library launches on; the CPU oracle is timed on a bounded sample of the same
workload.

Prints one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLS projected points/sec @10M pts k=48: FP32 vs FP64 path; fwd+bwd pts/sec"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6

# Algorithmic work per query of the fit kernel (moments, plane, quadratic fit,
# projection): FP32 operations per neighbour (pass 1: 34, pass 2: 74; an
# exponential counted as one operation each pass) plus the FP64 per-point
# algebra (eigen-solve, frame, 6x6 Cholesky and solve: ~1,000 operations).
# List refresh (MLS_STAGE_REFRESH) for the third pass: the second pass's
# search keeps 16 neighbours beyond k, the third re-ranks them for the moved
# queries and searches afresh only where the triangle inequality does not
# certify the list (10 % of the queries on the 10M height field). The first
# pass moves the queries by 0.23 h (median), too far for a refresh of pass 2
# (59 % certified); the second moves them by 0.04 h.
SEARCH_EXTRA = 16
REFRESH_FROM = 2  # 0-based pass index of the first refreshed pass
SLOT_ORDER = True  # iterated passes keep intermediate points in sorted order
FIT_FLOPS_PER_NEIGHBOUR = 108 + 2
FIT_FP64_FLOPS_PER_QUERY = 1000
# one step of the reference plane: the pass-1 moments again with the weights
# centred at q (34 flop per neighbour plus the shift of 3 subtractions)
PLANE_STEP_FLOPS = 34 + 3
# Algorithmic work of the exact search per query: 200 candidate FP64 keys of
# 10 flop (a 3^3 block of cells whose edge is about the k-th neighbour
# distance holds 100-300 points on these surfaces).
SEARCH_FP64_FLOPS_PER_QUERY = 200 * 10
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_knn_heightfield10M_k48.json")
ISSUE_FILE = os.path.join(ROOT, "profiles", "valu_issue_heightfield10M_k48.json")
SEARCH_SOURCES = [os.path.join(ROOT, "paper_2401_03365_amd", "csrc", f)
                  for f in ("knn.hip", "mls_internal.h")]


def search_source_hash():
    import hashlib
    hsh = hashlib.sha256()
    for f in SEARCH_SOURCES:
        with open(f, "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def search_traffic_bytes(args):
    """HBM bytes per search launch from the recorded counter runs (FETCH_SIZE
    and WRITE_SIZE scaled by the copy-kernel factors), or None when the
    kernel's source changed since they were taken or the workload differs."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != search_source_hash() or rec.get("n") != args.n or \
            rec.get("k") != args.k:
        return None
    kib = rec["fetch_kib_per_dispatch"] * rec["fetch_factor"] + \
        rec["write_kib_per_dispatch"] * rec["write_factor"]
    return kib * 1024.0


FIT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fit_heightfield10M_k48.json")
FIT_SOURCES = [os.path.join(ROOT, "paper_2401_03365_amd", "csrc", f)
               for f in ("mls_fwd.hip", "mls_fit.h", "mls_math.h", "mls_levin.h")]


def fit_traffic_bytes(args):
    """HBM bytes per fit launch from the recorded counter runs, or None when
    the fit's sources changed since they were taken or the workload differs."""
    import hashlib
    try:
        with open(FIT_TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    hsh = hashlib.sha256()
    for fn in FIT_SOURCES:
        with open(fn, "rb") as fh:
            hsh.update(fh.read())
    if rec.get("source_sha256") != hsh.hexdigest() or rec.get("n") != args.n or \
            rec.get("k") != args.k:
        return None
    return rec.get("bytes_per_launch")


def search_valu_busy(args):
    """Fraction of the VALU issue capacity the full searches use, from the
    recorded SQ_INSTS_VALU counter runs, or None when the kernel's source
    changed since they were taken or the workload differs."""
    try:
        with open(ISSUE_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != search_source_hash() or rec.get("n") != args.n or \
            rec.get("k") != args.k:
        return None
    return rec.get("valu_busy")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--k", type=int, default=48)
    ap.add_argument("--passes", type=int, default=3)
    ap.add_argument("--search-extra", type=int, default=None,
                    help="extra neighbours kept for the refresh (default: tuned)")
    ap.add_argument("--caller-order", action="store_true",
                    help="keep intermediate points of iterated passes in the caller's order")
    ap.add_argument("--no-tune-check", action="store_true",
                    help="skip timing the whole step for every tuning candidate")
    ap.add_argument("--cell-factor", type=float, default=None,
                    help="cell edge in units of h (default: library tuning table)")
    ap.add_argument("--cpu-sample", type=int, default=12288)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-fwd-bwd", action="store_true")
    ap.add_argument("--c4-n", type=int, default=2_000_000)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-geometry", action="store_true",
                    help="skip the geometry-output and upsampling measurement")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the sphere quality table (radius-R neighbourhoods)")
    ap.add_argument("--plane-iters", type=int, default=3,
                    help="steps of the self-consistent reference plane in the extra "
                         "'plane_steps' measurement (0 skips it)")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the sphere 20k and torus 1.01M one-pass measurements")
    ap.add_argument("--acc-sample", type=int, default=2048,
                    help="queries per workload and pass in the accuracy table")
    ap.add_argument("--no-levin", action="store_true",
                    help="skip the 'levin' measurement (Levin's reference plane per fit)")
    ap.add_argument("--gather-calibration-mb", type=int, default=0,
                    help="only gather one 16-byte row from every 128-byte line of a table of "
                         "this many MiB, in random order (counter calibration)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="only run a device-to-device copy of this many MB (3 times) and "
                         "print its bandwidth: the reference for the HBM traffic counters")
    return ap.parse_args()


class Timer:
    def __init__(self, torch):
        self.torch = torch
        self.acc = {}

    def span(self, name):
        torch = self.torch
        timer = self

        class _S:
            def __enter__(self):
                self.a = torch.cuda.Event(enable_timing=True)
                self.b = torch.cuda.Event(enable_timing=True)
                self.a.record()

            def __exit__(self, *exc):
                self.b.record()
                timer.acc.setdefault(name, []).append((self.a, self.b))
        return _S()

    def ms(self, name):
        ev = self.acc.get(name, [])
        return sum(a.elapsed_time(b) for a, b in ev) / max(1, len(ev))

    def reset(self):
        self.acc = {}


def run_steps(api, torch, pts, h, k, passes, precision, cell, steps, warmup, timer,
              plane_iters=0, levin=False, search_extra=SEARCH_EXTRA, slot_order=None):
    """Returns (ms_per_step, last outputs of pass 1, last final outputs,
    [(input, output, status) of every pass of the last step], all in the
    caller's order). ``plane_iters``: frozen-weight steps of the reference
    plane in every fit; ``levin``: Levin's reference plane in every fit;
    ``slot_order``: the passes between the first and the last keep their
    points in the grid's sorted order (default SLOT_ORDER)."""
    if slot_order is None:
        slot_order = SLOT_ORDER
    q0 = pts.double()
    out = None
    passes_io = []
    grid = None

    def step(record):
        nonlocal out, passes_io, grid
        passes_io = []
        ctx = timer.span if record else (lambda name: _Null())
        with ctx("build"):
            grid = api.Grid(pts, h, cell_size=cell)
        cur = q0
        for p in range(passes):
            nxt = torch.empty_like(cur)
            status = torch.empty((pts.shape[0],), dtype=torch.uint8, device=pts.device)
            # the pass before the first refreshed one keeps SEARCH_EXTRA more
            # neighbours; refreshed passes re-rank the lists of the pass
            # before (exact; a fresh search where not certified)
            refresh = 0 < REFRESH_FROM <= p
            extra = search_extra if 0 < REFRESH_FROM and p >= REFRESH_FROM - 1 else 0
            # intermediate points in sorted order: every pass but the first
            # reads its queries in sequence, every pass but the last writes
            # its results in sequence
            s_in = slot_order and p > 0
            s_out = slot_order and p < passes - 1
            so = (1 if s_in else 0) | (2 if s_out else 0)
            if slot_order and p == 0:
                so |= 4  # the first pass's queries are the grid's own points
            with ctx("refresh" if refresh else "search"):
                grid.project(cur, k, precision, stages=1, out=nxt, status=status,
                             search_extra=extra, refresh=refresh, slot_order=so)
            with ctx("fit"):
                grid.project(cur, k, precision, stages=2, out=nxt, status=status,
                             search_extra=extra, plane_iters=plane_iters, levin=levin,
                             slot_order=so)
            passes_io.append((cur, nxt, status, s_in, s_out))
            cur = nxt
        out = cur
        return grid

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    timer.reset()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # rows of the last step in the caller's order (outside the timed region)
    rows = grid.caller_rows()

    def caller(x, in_slots):
        if not in_slots:
            return x
        y = torch.empty_like(x)
        y[rows] = x
        return y

    passes_io = [(caller(c, si), caller(n, so), caller(st, so)) for c, n, st, si, so in passes_io]
    first = passes_io[0][1] if passes_io else None
    return (t1 - t0) * 1000.0 / steps, first, out, passes_io


class _Null:
    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False


def tuned_cell_factor(api, pts, h, k):
    """The tuner's cell edge factor for one cloud (full searches of every
    candidate grid) and its timings."""
    factors, rep = api.autotune_cells(pts, h, k)
    return float(factors[0]), rep[0][1]


def fwd_bwd(api, torch, P, h, k, loss_grad, steps, warmup, label, precision="fp32",
            keep=None, cell_factor=None):
    """fwd (search + fit) and the adjoint of one pass over the whole cloud,
    queries = the cloud's points (FP32 in and out), on the FP32-moment or the
    FP64 path. The grid is built once (cell edge: ``cell_factor`` x h, else
    the tuner's pick); the loss gradient is torch code between the two and is
    timed apart. value = N / (t_fwd + t_bwd). ``keep``: a dict that receives
    the forward's outputs and statuses."""
    pts = torch.from_numpy(P).cuda()
    if cell_factor is None:
        cell_factor, _ = tuned_cell_factor(api, pts, h, k)
    timer = Timer(torch)
    grid = api.Grid(pts, h, cell_size=cell_factor * h)
    out = torch.empty_like(pts)
    status = torch.empty((pts.shape[0],), dtype=torch.uint8, device=pts.device)

    def step(record):
        ctx = timer.span if record else (lambda name: _Null())
        with ctx("fwd_search"):
            grid.project(pts, k, precision, stages=1, out=out, status=status)
        with ctx("fwd_fit"):
            grid.project(pts, k, precision, stages=2, out=out, status=status)
        with ctx("loss_grad"):
            gy = loss_grad(out)
        with ctx("bwd"):
            gq, gp = grid.project_backward(pts, gy, k, precision, reuse_lists=True)
        return gq, gp

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    for _ in range(steps):
        gq, gp = step(True)
    torch.cuda.synchronize()
    br = {n: timer.ms(n) for n in ("fwd_search", "fwd_fit", "loss_grad", "bwd")}
    t = br["fwd_search"] + br["fwd_fit"] + br["bwd"]
    ok = bool(torch.isfinite(gq).all().item() and torch.isfinite(gp).all().item())
    log("%s %s (cell %.2f h): fwd %.2f + %.2f ms, loss %.2f ms, bwd %.2f ms, finite grads %s" %
        (label, precision, cell_factor, br["fwd_search"], br["fwd_fit"], br["loss_grad"],
         br["bwd"], ok))
    if keep is not None:
        keep["out"], keep["status"] = out, status
    del grid
    return {"value": P.shape[0] / (t / 1000.0), "unit": "pts/s", "n_points": int(P.shape[0]),
            "k": k, "h": h, "precision": precision, "cell_factor": cell_factor,
            "breakdown_ms": br, "ms_fwd_plus_bwd": t, "grads_finite": ok}


def sh_sphere_loss(torch, field, P):
    """L = mean_j (|y_j| - rho_j)^2, rho_j = 1 + bump at the sample's own
    direction (evaluated once on the host)."""
    w = P.astype(np.float64)
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    rho = torch.from_numpy((1.0 + field.bump(w)).astype(np.float32)).cuda()

    def grad(out):
        y = out.detach().requires_grad_(True)
        L = ((y.norm(dim=1) - rho) ** 2).mean()
        return torch.autograd.grad(L, y)[0]
    return grad


def heightfield_loss(torch, field):
    """L = mean_j (z_j - f(x_j, y_j))^2 with the generating height field."""
    fr = torch.tensor(field.freq, dtype=torch.float32, device="cuda")
    ca = torch.tensor(np.cos(field.alpha), dtype=torch.float32, device="cuda")
    sa = torch.tensor(np.sin(field.alpha), dtype=torch.float32, device="cuda")
    ph = torch.tensor(field.phase, dtype=torch.float32, device="cuda")

    def grad(out):
        y = out.detach().requires_grad_(True)
        arg = 2.0 * np.pi * fr * (y[:, :1] * ca + y[:, 1:2] * sa) + ph
        f = field.amp * torch.sin(arg).sum(1)
        L = ((y[:, 2] - f) ** 2).mean()
        return torch.autograd.grad(L, y)[0]
    return grad


def batch_loss_grad(torch, P, off, shapes, n_total):
    """Elementwise gradient of L = mean_j res_j^2 over the batch with the
    closed-form residual of each cloud's surface: sphere |y| - 1, torus
    (R = 1, r = 0.3) sqrt((rho - R)^2 + z^2) - r, height field z - f(x, y)
    with the cloud's own field. No reductions, so it can sit in a graph."""
    from paper_2401_03365_amd import synth
    kind = np.zeros(P.shape[0], dtype=np.int8)
    hf_rows, alpha, phase = [], [], []
    for c, sh in enumerate(shapes):
        sl = slice(int(off[c]), int(off[c + 1]))
        if sh == "torus":
            kind[sl] = 1
        elif sh == "heightfield":
            kind[sl] = 2
            f = synth.HeightField(5000 + c + 1000)
            hf_rows.append(np.arange(off[c], off[c + 1]))
            alpha.append(np.broadcast_to(f.alpha, (int(off[c + 1] - off[c]), 8)))
            phase.append(np.broadcast_to(f.phase, (int(off[c + 1] - off[c]), 8)))
            amp = f.amp
    dev = "cuda"
    kind_t = torch.from_numpy(kind).to(dev)
    rows = torch.from_numpy(np.concatenate(hf_rows)).to(dev)
    ca = torch.from_numpy(np.cos(np.concatenate(alpha)).astype(np.float32)).to(dev)
    sa = torch.from_numpy(np.sin(np.concatenate(alpha)).astype(np.float32)).to(dev)
    ph = torch.from_numpy(np.concatenate(phase).astype(np.float32)).to(dev)
    fr = 2.0 * np.pi * torch.arange(1, 9, dtype=torch.float32, device=dev)
    is_sph = (kind_t == 0)[:, None]
    is_tor = (kind_t == 1)[:, None]
    scale = 2.0 / n_total

    def grad(y):
        nrm = y.norm(dim=1, keepdim=True)
        g_s = (nrm - 1.0) * y / nrm
        rho = y[:, :2].norm(dim=1, keepdim=True)
        dt = torch.sqrt((rho - 1.0) ** 2 + y[:, 2:] ** 2)
        res_t = dt - 0.3
        g_t = torch.cat([res_t * (rho - 1.0) / dt * y[:, :2] / rho, res_t * y[:, 2:] / dt], 1)
        g = torch.where(is_sph, g_s, torch.where(is_tor, g_t, torch.zeros_like(y)))
        yh = y[rows]
        arg = fr * (yh[:, :1] * ca + yh[:, 1:2] * sa) + ph
        res_h = yh[:, 2] - amp * torch.sin(arg).sum(1)
        c = amp * torch.cos(arg) * fr
        g_h = torch.stack([-res_h * (c * ca).sum(1), -res_h * (c * sa).sum(1), res_h], 1)
        g = g.index_copy(0, rows, g_h)
        return g * scale
    return grad


def batch_fwd_bwd(api, torch, steps, warmup, keep=None, tune_check=True):
    """256 clouds (~30M points, sizes log-normal, sphere / torus / height
    field, per-cloud h), k = 32, FP32: the cell edge is tuned, the grid built
    once, then [grid rebuild, search, fit, loss gradient, adjoint] is captured
    in one HIP graph and replayed. value = N / (time of one replay)."""
    from paper_2401_03365_amd import synth
    t = time.perf_counter()
    P, off, sig, shapes = synth.batch()
    h = np.array([synth.mean_nn_h(P[off[c]:off[c + 1]]) for c in range(len(off) - 1)])
    log("batch: %d clouds, %d pts generated (%.1f s)" % (len(h), P.shape[0], time.perf_counter() - t))
    pts = torch.from_numpy(P).cuda()
    k = 32
    t = time.perf_counter()
    factors, rep = api.autotune_cells(pts, h, k, cloud_offsets=off)
    tune_s = time.perf_counter() - t
    log("batch: tuned cell factors per size class %s (%.1f s)" %
        ({c: b for c, (b, _) in rep.items()}, tune_s))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    grid = api.Grid(pts, h, cloud_offsets=off, cell_size=factors * h)
    e1.record()
    torch.cuda.synchronize()
    build_ms = e0.elapsed_time(e1)
    loss_grad = batch_loss_grad(torch, P, off, shapes, P.shape[0])
    out = torch.empty_like(pts)
    status = torch.empty((pts.shape[0],), dtype=torch.uint8, device="cuda")

    def body():
        # the grid re-sorted from the (possibly moved) positions with kernels
        # only, then search, fit, loss gradient and adjoint
        grid.rebuild(pts)
        grid.project(pts, k, "fp32", stages=1, out=out, status=status)
        grid.project(pts, k, "fp32", stages=2, out=out, status=status)
        gy = loss_grad(out)
        return grid.project_backward(pts, gy, k, "fp32", reuse_lists=True)

    for _ in range(warmup):
        body()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        body()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1000.0 / steps
    check = None
    if tune_check:
        # the eager step with one factor for every cloud, for each candidate:
        # where does the per-class choice rank?
        check = {"eager_ms_per_uniform_factor": {}, "eager_ms_tuned": eager_ms}
        out2 = torch.empty_like(pts)
        st2 = torch.empty((pts.shape[0],), dtype=torch.uint8, device="cuda")
        for f in sorted(next(iter(rep.values()))[1]):
            g2 = api.Grid(pts, h, cloud_offsets=off, cell_size=f * h)

            def body2():
                g2.rebuild(pts)
                g2.project(pts, k, "fp32", stages=1, out=out2, status=st2)
                g2.project(pts, k, "fp32", stages=2, out=out2, status=st2)
                gy2 = loss_grad(out2)
                return g2.project_backward(pts, gy2, k, "fp32", reuse_lists=True)
            body2()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                body2()
            torch.cuda.synchronize()
            check["eager_ms_per_uniform_factor"][f] = (time.perf_counter() - t0) * 1000.0 / 2
            g2.close()
        best_u = min(check["eager_ms_per_uniform_factor"].values())
        check["tuned_vs_best_uniform"] = eager_ms / best_u - 1.0
        log("batch tuning check: %s" % json.dumps(check))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        body()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gq, gp = body()
    graph.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / steps
    ok = bool(torch.isfinite(gq).all().item() and torch.isfinite(gp).all().item())
    gq_g, gp_g = gq.clone(), gp.clone()
    gq_e, gp_e = body()
    torch.cuda.synchronize()
    same = bool(torch.equal(gq_g, gq_e)) and \
        float((gp_g - gp_e).norm() / gp_e.norm()) <= 1e-5
    log("batch: graph %.2f ms/step, eager %.2f ms/step, build %.2f ms, finite grads %s" %
        (graph_ms, eager_ms, build_ms, ok))
    if keep is not None:
        keep.update({"P": P, "off": off, "h": h, "out": out, "status": status})
    return {"value": P.shape[0] / (graph_ms / 1000.0), "unit": "pts/s",
            "n_points": int(P.shape[0]), "n_clouds": int(len(h)), "k": k,
            "ms_per_step_graph": graph_ms, "ms_per_step_eager": eager_ms, "build_ms": build_ms,
            "cell_factor_per_class": {str(c): b for c, (b, _) in rep.items()},
            "autotune_search_ms": {str(c): m for c, (_, m) in rep.items()},
            "autotune_s": tune_s, "grads_finite": ok,
            "graph_matches_eager": same, "tuning_check": check,
            "step": "grid rebuild + search + fit + loss gradient + adjoint, one graph replay"}


def geometry_and_upsampling(api, torch, pts, h, cell, k, reps=3):
    """Fit with the surface geometry (normal, mean and Gaussian curvature at
    each output) on the headline cloud, and upsampling: 4 queries per sample
    jittered by up to 0.4 h, projected (search + fit) onto the cloud's
    surface. Times from HIP events, inputs resident."""
    n = pts.shape[0]
    grid = api.Grid(pts, h, cell_size=cell)
    q = pts.double()
    out = torch.empty_like(q)
    st = torch.empty((n,), dtype=torch.uint8, device=pts.device)
    grid.project(q, k, "fp32", stages=1, out=out, status=st)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(f):
        f()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    fit = timed(lambda: grid.project(q, k, "fp32", stages=2, out=out, status=st))
    fit_geo = timed(lambda: grid.project(q, k, "fp32", stages=2, out=out, status=st,
                                         geometry=True))
    gen = torch.Generator(device=pts.device)
    gen.manual_seed(71)
    up = (q.repeat_interleave(4, dim=0) +
          (torch.rand((4 * n, 3), generator=gen, device=pts.device, dtype=torch.float64) - 0.5)
          * (0.8 * h))
    up_ms = timed(lambda: grid.project(up, k, "fp32"))
    grid.close()
    return {"fit_ms": fit, "fit_geometry_ms": fit_geo,
            "upsample_4x": {"n_queries": int(up.shape[0]), "ms": up_ms,
                            "value": up.shape[0] / (up_ms / 1000.0), "unit": "pts/s",
                            "step": "search + fit of 4 jittered queries per sample"}}


def one_pass(api, torch, P, h, k, precision, reps=5, cell_factor=1.25):
    """One projection pass (search + fit) of the cloud's own points, grid
    built once; mean ms over ``reps`` after a warm-up. Returns (result dict,
    outputs, statuses)."""
    pts = torch.from_numpy(P).cuda()
    g = api.Grid(pts, h, cell_size=cell_factor * h)
    q = pts.double()
    out = torch.empty_like(q)
    st = torch.empty((pts.shape[0],), dtype=torch.uint8, device="cuda")
    g.project(q, k, precision, out=out, status=st)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        g.project(q, k, precision, out=out, status=st)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    g.close()
    return ({"precision": precision, "ms_per_pass": ms,
             "value": P.shape[0] / (ms / 1000.0), "unit": "pts/s"}, out, st)


def small_configs(api, torch, keep):
    """The sphere (20k, k = 32, FP64 path; FP32 beside it) and the torus
    with outliers (1.01M, k = 32, both paths): one pass each."""
    from paper_2401_03365_amd import synth
    res = {}
    P1 = synth.sphere(20000, 0.01, seed=1)
    h1 = synth.mean_nn_h(P1)
    P2 = synth.torus(1_000_000, sigma=0.005, n_outliers=10_000, seed=2)
    h2 = synth.mean_nn_h(P2)
    for name, P, hh in (("sphere_20k_k32", P1, h1), ("torus_1.01M_k32", P2, h2)):
        cf, cf_ms = tuned_cell_factor(api, torch.from_numpy(P).cuda(), hh, 32)
        res[name] = {"n_points": int(P.shape[0]), "h": hh, "cell_factor": cf,
                     "tuner_search_ms": cf_ms}
        for prec in ("fp64", "fp32"):
            r, out, st = one_pass(api, torch, P, hh, 32, prec, cell_factor=cf)
            res[name][prec] = r
            keep[(name, prec)] = (P, hh, 32, out, st)
            log("%s %s (cell %.2f h): %.3f ms per pass (%.3g pts/s)" %
                (name, prec, cf, r["ms_per_pass"], r["value"]))
    return res


def accuracy_of(oracle, P, Q, k, h, out, st, **kw):
    """max and RMS |GPU - oracle| / h over the sampled queries Q (rows of
    out/st), lists by the oracle's brute force; points flagged ambiguous and
    non-finite queries left out of the error, status mismatches counted."""
    P64 = P.astype(np.float64)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    nbr, _ = oracle.knn(P64, Q, k)
    ref, ref_st = oracle.project(P64, Q, k, h, nbr=nbr, **kw)[:2]
    ok = ((ref_st & 0x10) == 0) & ((ref_st & 0x0F) != 3)
    out = np.asarray(out)
    diff = np.abs(out.astype(np.float64) - ref)
    if out.dtype == np.float32:
        # outputs stored in FP32: their storage rounding (an ulp per
        # coordinate) is not an error of the arithmetic
        diff = np.maximum(diff - np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64), 0)
    e = np.linalg.norm(diff, axis=1)[ok] / h
    return {"rms_over_h": float(np.sqrt((e ** 2).mean())) if e.size else 0.0,
            "max_over_h": float(e.max()) if e.size else 0.0, "n": int(ok.sum()),
            "status_mismatches": int((np.asarray(st) != ref_st).sum()),
            "outputs": "fp32 (storage rounding allowed)" if out.dtype == np.float32 else "fp64"}


def sample_rows(torch, n, m, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, size=min(m, n), replace=False))
    return idx, torch.from_numpy(idx).cuda()


def cpu_info():
    """Model, sockets, threads per core and the cores this process may use."""
    info = {"cores_available": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            key, _, val = line.partition(":")
            key = key.strip()
            if key in ("Socket(s)", "Thread(s) per core", "Core(s) per socket", "CPU(s)"):
                info[key] = val.strip()
    except Exception:
        pass
    return info


def adjoint_check(api, torch, oracle, P, h, m=1000, k=32):
    """The adjoint on m sampled queries of the cloud (lists from the oracle's
    brute force, passed in) against the oracle's central differences:
    relative 2-norm errors of the query and the point gradients."""
    P64 = P.astype(np.float64)
    rng = np.random.default_rng(23)
    idx = np.sort(rng.choice(P.shape[0], m, replace=False))
    Qs = P64[idx]
    nbr, _ = oracle.knn(P64, Qs, k)
    _, st = oracle.project(P64, Qs, k, h, nbr=nbr)
    keepq = (st & 0x10) == 0
    Qs, nbr = Qs[keepq], nbr[keepq]
    go = rng.normal(size=Qs.shape)
    fq, fp = oracle.grad_fd(P64, Qs, k, h, nbr, go)
    g = api.Grid(torch.from_numpy(P).cuda(), h, cell_size=1.25 * h)
    res = {"n_queries": int(Qs.shape[0])}
    for prec in ("fp32", "fp64"):
        gq, gp = g.project_backward(torch.from_numpy(Qs).cuda(), torch.from_numpy(go).cuda(), k,
                                    prec, neighbors=torch.from_numpy(nbr).cuda())
        torch.cuda.synchronize()
        gq, gp = gq.cpu().numpy(), gp.cpu().numpy()
        res[prec] = {"query_grad_rel": float(np.linalg.norm(gq - fq) / np.linalg.norm(fq)),
                     "point_grad_rel": float(np.linalg.norm(gp - fp) / np.linalg.norm(fp))}
    g.close()
    return res


def quality_table(api, torch):
    """The paper's quality protocol (Section 3.3 and its tables) on synthetic
    stand-ins for its meshes: a unit sphere and the unit cube (sharp edges and
    corners), 200,000 points each with Gaussian noise sigma along the normal,
    projected once over the radius-R neighbourhood without a count cap
    (ball = 2; the Gaussian width h = R / 3, so that the ball is the 3h
    support), points with fewer than 3 neighbours within R removed;
    deviation = distance of a kept output to the clean surface. Per shape and
    sigma the best R is chosen among the settings that keep at least 90 % of
    the points (a small R that deletes most of the cloud is data loss, not
    smoothing)."""
    from paper_2401_03365_amd import synth
    shapes = {
        "sphere": (lambda sig: synth.sphere(200_000, sig, seed=61),
                   lambda Y: np.abs(np.linalg.norm(Y, axis=1) - 1.0)),
        "cube": (lambda sig: synth.cube(200_000, sig, seed=62), synth.cube_distance),
    }
    rows, best = [], {}
    for shape, (make, dist) in shapes.items():
        for sigma in (0.005, 0.01, 0.03):
            P = make(sigma)
            Pt = torch.from_numpy(P).cuda()
            dev_in = dist(P.astype(np.float64))
            for R in (0.005, 0.01, 0.02, 0.03, 0.05):
                h = R / 3.0
                g = api.Grid(Pt, h)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                out, st = g.project(Pt, 1, "fp32", ball=2, support_radius_h=3.0)
                e1.record()
                torch.cuda.synchronize()
                out, st = out.cpu().numpy().astype(np.float64), st.cpu().numpy()
                kept = (st & 0x0F) != 1
                dev = dist(out[kept])
                rows.append({"shape": shape, "sigma": sigma, "R": R,
                             "removed": int((~kept).sum()),
                             "kept_fraction": float(kept.mean()),
                             "mean": float(dev.mean()) if dev.size else None,
                             "std": float(dev.std()) if dev.size else None,
                             "min": float(dev.min()) if dev.size else None,
                             "max": float(dev.max()) if dev.size else None,
                             "input_mean": float(dev_in.mean()), "ms": e0.elapsed_time(e1)})
                g.close()
            cand = [r for r in rows if r["shape"] == shape and r["sigma"] == sigma and
                    r["kept_fraction"] >= 0.9 and r["mean"] is not None]
            if cand:
                b = min(cand, key=lambda r: r["mean"])
                best["%s/%g" % (shape, sigma)] = {"R": b["R"], "mean": b["mean"],
                                                  "input_mean": b["input_mean"],
                                                  "kept_fraction": b["kept_fraction"]}
    return {"rows": rows, "best_R_keeping_90pct": best}


def main():
    global SLOT_ORDER
    args = parse()
    SLOT_ORDER = not args.caller_order
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X "
              "(no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2401_03365_amd import api, synth

    if args.copy_calibration_mb:
        nbytes = args.copy_calibration_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(3):
            e0.record()
            dst.copy_(src)
            e1.record()
            torch.cuda.synchronize()
            log("copy %d MiB: %.3f ms, %.1f GB/s (read + write)" %
                (args.copy_calibration_mb, e0.elapsed_time(e1), 2 * nbytes / e0.elapsed_time(e1) / 1e6))
        print(json.dumps({"copy_bytes": nbytes, "ms": e0.elapsed_time(e1)}), flush=True)
        return

    if args.gather_calibration_mb:
        # rows of 16 bytes (float4, as the fit gathers its neighbours), one
        # from each 128-byte line of the table, in random order: every row
        # read touches a line no other read touches
        nbytes = args.gather_calibration_mb << 20
        table = torch.ones((nbytes // 16, 4), dtype=torch.float32, device="cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(7)
        idx = torch.randperm(nbytes // 128, device="cuda", generator=g) * 8
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(3):
            e0.record()
            out = table.index_select(0, idx)
            e1.record()
            torch.cuda.synchronize()
            log("gather of %d rows of 16 B from a %d MiB table: %.3f ms" %
                (idx.numel(), args.gather_calibration_mb, e0.elapsed_time(e1)))
        del out
        print(json.dumps({"rows": idx.numel(), "row_bytes": 16, "line_bytes": 128,
                          "index_bytes": 8, "ms": e0.elapsed_time(e1)}), flush=True)
        return

    t = time.perf_counter()
    P, hfield = synth.heightfield(args.n, sigma=1e-3, seed=3, return_field=True)
    h = synth.mean_nn_h(P)
    log("cloud %d pts generated, h = %.6g (%.1f s)" % (args.n, h, time.perf_counter() - t))
    pts = torch.from_numpy(P).cuda()
    torch.cuda.synchronize()
    # the tuner (outside the timed steps): the cell edge from full searches
    # of every candidate grid, then the extra neighbours of the refresh from
    # the two searches of passes 2 and 3
    tuning = {}
    t = time.perf_counter()
    if args.cell_factor is None:
        factors, rep = api.autotune_cells(pts, h, args.k)
        cf = float(factors[0])
        tuning["cell_factor"] = {"pick": cf, "search_ms": rep[0][1]}
    else:
        cf = args.cell_factor
    cell = cf * h
    extra = args.search_extra
    if extra is None:
        gt = api.Grid(pts, h, cell_size=cell)
        q0 = pts.double()
        o1 = torch.empty_like(q0)
        st1 = torch.empty((args.n,), dtype=torch.uint8, device="cuda")
        gt.project(q0, args.k, "fp32", out=o1, status=st1)
        extra, extra_ms = api.autotune_search_extra(gt, o1, args.k)
        tuning["search_extra"] = {"pick": extra, "two_searches_ms": extra_ms}
        del gt, q0, o1, st1
    tuning["tuner_s"] = time.perf_counter() - t
    log("tuned: cell factor %.2f, search extra %d (%.1f s) %s" %
        (cf, extra, tuning["tuner_s"], json.dumps(tuning)))

    timer = Timer(torch)
    ms32, first32, out32, io32 = run_steps(api, torch, pts, h, args.k, args.passes, "fp32",
                                           cell, args.steps, args.warmup, timer,
                                           search_extra=extra)
    br32 = {n: timer.ms(n) for n in ("build", "search", "refresh", "fit")}
    log("fp32: %.2f ms/step  build %.2f  search %.2f  refresh %.2f  fit %.2f (ms per call)" %
        (ms32, br32["build"], br32["search"], br32["refresh"], br32["fit"]))
    value = args.n * args.passes / (ms32 / 1000.0)

    fp64 = None
    first64 = None
    io64 = None
    if not args.no_fp64:
        timer64 = Timer(torch)
        ms64, first64, _, io64 = run_steps(api, torch, pts, h, args.k, args.passes, "fp64",
                                           cell, max(1, args.steps // 2), 1, timer64,
                                           search_extra=extra)
        br64 = {n: timer64.ms(n) for n in ("build", "search", "refresh", "fit")}
        log("fp64: %.2f ms/step  build %.2f  search %.2f  refresh %.2f  fit %.2f" %
            (ms64, br64["build"], br64["search"], br64["refresh"], br64["fit"]))
        fp64 = {"value": args.n * args.passes / (ms64 / 1000.0), "unit": "pts/s",
                "ms_per_step": ms64, "breakdown_ms": br64}

    # roofline of the dominant kernel of the headline step
    nq = args.n
    if br32["fit"] >= br32["search"]:
        flops = nq * (args.k * FIT_FLOPS_PER_NEIGHBOUR + FIT_FP64_FLOPS_PER_QUERY)
        achieved = flops / (br32["fit"] / 1000.0) / 1e12
        roof = {"kernel": "k_mls_forward<fp32>", "bound": "alu", "achieved": achieved,
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                "traffic": None}
    else:
        flops = nq * SEARCH_FP64_FLOPS_PER_QUERY
        achieved = flops / (br32["search"] / 1000.0) / 1e12
        roof = {"kernel": "k_knn (passes 1-2: k_knn<0> plain, k_knn<1> with extra entries)",
                "bound": "alu", "achieved": achieved,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                "traffic": search_traffic_bytes(args)}
        if roof["traffic"] is not None:
            roof["traffic_GBps"] = roof["traffic"] / (br32["search"] / 1000.0) / 1e9
        # the search is bound by instruction issue: the share of the VALU
        # pipes' issue cycles it fills (counters), beside the flop fraction
        roof["valu_issue_busy"] = search_valu_busy(args)

    # the fit of the headline step: ALU-bound (FP32 moments, FP64 solves)
    flops_fit = nq * (args.k * FIT_FLOPS_PER_NEIGHBOUR + FIT_FP64_FLOPS_PER_QUERY)
    ach_fit = flops_fit / (br32["fit"] / 1000.0) / 1e12
    fit_roof = {"kernel": "k_mls_forward<fp32>", "bound": "alu", "achieved": ach_fit,
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach_fit / FP32_PEAK_TFLOPS,
                "traffic": fit_traffic_bytes(args)}

    res = {"metric": METRIC, "value": value, "unit": "pts/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms32, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "heightfield-10M-k48-3pass", "n_points": args.n, "k": args.k,
                      "passes": args.passes, "precision": "fp32-moments+fp64-solves",
                      "h": h, "cell_size": cell, "step": "grid build + %d passes" % args.passes,
                      "intermediate_order": "caller" if args.caller_order else "sorted"},
           "breakdown_ms": br32,
           "value_excl_build": args.n * args.passes /
           ((ms32 - br32["build"]) / 1000.0),
           "fp64_path": fp64,
           "roofline": roof,
           "fit_roofline": fit_roof}

    if not args.no_tune_check and "cell_factor" in tuning:
        # the whole step for every candidate: does the tuner's pick rank as
        # it does in the full runs?
        chk = {"step_ms_per_cell_factor": {}, "step_ms_per_search_extra": {}}
        for f in tuning["cell_factor"]["search_ms"]:
            ms_f = run_steps(api, torch, pts, h, args.k, args.passes, "fp32", f * h, 2, 1,
                             Timer(torch), search_extra=extra)[0]
            chk["step_ms_per_cell_factor"][f] = ms_f
        if "search_extra" in tuning:
            for e in tuning["search_extra"]["two_searches_ms"]:
                ms_e = run_steps(api, torch, pts, h, args.k, args.passes, "fp32", cell, 2, 1,
                                 Timer(torch), search_extra=e)[0]
                chk["step_ms_per_search_extra"][e] = ms_e
        for key, pick in (("step_ms_per_cell_factor", cf), ("step_ms_per_search_extra", extra)):
            d = chk[key]
            if d:
                best = min(d.values())
                chk[key + "_pick_vs_best"] = d[pick] / best - 1.0 if pick in d else None
        # the same step with every pass in the caller's order
        chk["step_ms_caller_order"] = run_steps(api, torch, pts, h, args.k, args.passes, "fp32",
                                                cell, 2, 1, Timer(torch), search_extra=extra,
                                                slot_order=False)[0]
        chk["step_ms_sorted_order"] = run_steps(api, torch, pts, h, args.k, args.passes, "fp32",
                                                cell, 2, 1, Timer(torch), search_extra=extra,
                                                slot_order=True)[0]
        tuning["full_step_check"] = chk
        log("tuning check: %s" % json.dumps(chk))
    res["tuning"] = tuning
    res["config"]["cell_factor_tuned"] = cf
    res["config"]["search_extra_tuned"] = extra

    first_ps = None
    if args.plane_iters > 0:
        # the same step with the reference plane's weights moved to its own
        # projection of the query (Section 1.4), plane_iters steps per fit
        timer_ps = Timer(torch)
        ms_ps, first_ps, _, _ = run_steps(api, torch, pts, h, args.k, args.passes, "fp32",
                                          cell, max(1, args.steps // 2), 1, timer_ps,
                                          plane_iters=args.plane_iters)
        br_ps = {n: timer_ps.ms(n) for n in ("build", "search", "refresh", "fit")}
        log("plane steps %d: %.2f ms/step  fit %.2f ms" % (args.plane_iters, ms_ps, br_ps["fit"]))
        # fit with steps: pass 1 once plus once per step, pass 2 once
        flops = args.n * (args.k * (FIT_FLOPS_PER_NEIGHBOUR + args.plane_iters * PLANE_STEP_FLOPS)
                          + (1 + args.plane_iters) * FIT_FP64_FLOPS_PER_QUERY // 2
                          + FIT_FP64_FLOPS_PER_QUERY // 2)
        ach = flops / (br_ps["fit"] / 1000.0) / 1e12
        res["plane_steps"] = {
            "plane_iters": args.plane_iters, "value": args.n * args.passes / (ms_ps / 1000.0),
            "unit": "pts/s", "ms_per_step": ms_ps, "breakdown_ms": br_ps,
            "fit_roofline": {"kernel": "k_mls_forward<fp32, steps>", "bound": "alu",
                             "achieved": ach, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": ach / FP32_PEAK_TFLOPS, "traffic": None}}

    first_lv = {}
    if not args.no_levin:
        # the same step with Levin's reference plane (Newton on Eq. (1.1)
        # over (n, t), FP64 terms) in every fit, on both precision paths
        res["levin"] = {}
        for prec in ("fp32", "fp64"):
            timer_lv = Timer(torch)
            ms_lv, first_lv[prec], _, _ = run_steps(api, torch, pts, h, args.k, args.passes,
                                                    prec, cell, max(1, args.steps // 2), 1,
                                                    timer_lv, levin=True)
            br_lv = {n: timer_lv.ms(n) for n in ("build", "search", "refresh", "fit")}
            log("levin %s: %.2f ms/step  fit %.2f ms" % (prec, ms_lv, br_lv["fit"]))
            res["levin"][prec] = {"value": args.n * args.passes / (ms_lv / 1000.0),
                                  "unit": "pts/s", "ms_per_step": ms_lv, "breakdown_ms": br_lv}

    if not args.no_geometry:
        res["geometry"] = geometry_and_upsampling(api, torch, pts, h, cell, args.k)
        log("geometry: fit %.2f ms, with normals and curvatures %.2f ms; upsampling 4x: %.1f ms "
            "(%.3g pts/s)" % (res["geometry"]["fit_ms"], res["geometry"]["fit_geometry_ms"],
                              res["geometry"]["upsample_4x"]["ms"],
                              res["geometry"]["upsample_4x"]["value"]))

    if not args.no_quality:
        t = time.perf_counter()
        res["quality_200k"] = quality_table(api, torch)
        log("quality (200k sphere and cube, radius-R ball without cap): best R keeping 90 %%: "
            "%s (%.1f s)" % (json.dumps(res["quality_200k"]["best_R_keeping_90pct"]),
                             time.perf_counter() - t))

    keep = {}
    if not args.no_small:
        res["small_configs"] = small_configs(api, torch, keep)

    if not args.no_fwd_bwd:
        fb = {}
        for prec in ("fp32", "fp64"):
            key = "heightfield_10M_k48" + ("" if prec == "fp32" else "_fp64")
            fb[key] = fwd_bwd(api, torch, P, h, args.k, heightfield_loss(torch, hfield),
                              args.steps, args.warmup, "fwd+bwd heightfield", precision=prec,
                              cell_factor=cf)
        P4, shf = synth.sh_sphere(args.c4_n, sigma=0.005, seed=4, return_field=True)
        h4 = synth.mean_nn_h(P4)
        cf4, _ = tuned_cell_factor(api, torch.from_numpy(P4).cuda(), h4, 32)
        for prec in ("fp32", "fp64"):
            key = "sh_sphere_2M_k32" + ("" if prec == "fp32" else "_fp64")
            kk = {}
            fb[key] = fwd_bwd(api, torch, P4, h4, 32, sh_sphere_loss(torch, shf, P4),
                              args.steps, args.warmup, "fwd+bwd sh sphere", precision=prec,
                              keep=kk, cell_factor=cf4)
            keep[("sh_sphere_2M_k32", prec)] = (P4, h4, 32, kk["out"], kk["status"])
        if not args.no_batch:
            kb = {}
            fb["batch_256_clouds_30M_k32"] = batch_fwd_bwd(api, torch, args.steps, args.warmup,
                                                           keep=kb)
            keep["batch"] = kb
        res["fwd_bwd"] = fb

    if not args.no_cpu_baseline:
        # the CPU leg: the oracle timed on the host's cores, and the GPU's
        # accuracy against it on every workload
        import oracle
        rng = np.random.default_rng(7)
        sample = np.sort(rng.choice(args.n, size=min(args.cpu_sample, args.n), replace=False))
        P64 = P.astype(np.float64)
        Q = P64[sample]
        t = time.perf_counter()
        nbr, _ = oracle.knn(P64, Q, args.k)
        ref, ref_st = oracle.project(P64, Q, args.k, h, nbr=nbr)
        dt = time.perf_counter() - t
        # the fit alone on 1M queries, lists from SciPy's k-d tree (any lists
        # serve for timing); the brute-force search's cost per query; the k-d
        # tree's own k-nearest rate as a third-party CPU reference
        from scipy.spatial import cKDTree
        ci = cpu_info()
        threads = int(os.environ.get("OMP_NUM_THREADS", ci["cores_available"]))
        tree = cKDTree(P64, balanced_tree=False, compact_nodes=False)
        m_fit = min(1_000_000, args.n)
        Qf = P64[:m_fit]
        t3 = time.perf_counter()
        _, nb_f = tree.query(Qf, args.k, workers=threads)
        dt_tree = time.perf_counter() - t3
        nb_f = nb_f.astype(np.int32)
        t2 = time.perf_counter()
        oracle.project(P64, Qf, args.k, h, nbr=nb_f)
        dt_fit = time.perf_counter() - t2
        del nb_f, tree
        res["cpu_baseline"] = {
            "value": len(sample) / dt, "unit": "pts/s", "cores": threads, "kind": "oracle",
            "sample": "%d random queries of pass 1 of the same 10M cloud (brute-force kNN "
                      "over all points + FP64 projection)" % len(sample),
            "cpu": ci,
            "fit_only_pts_s": m_fit / dt_fit,
            "fit_only_sample": "the first %d points of the cloud as queries, lists of %d from "
                               "SciPy cKDTree" % (m_fit, args.k),
            "brute_force_knn_s_per_query": dt / len(sample),
            "ckdtree_knn_pts_s": m_fit / dt_tree}
        log("cpu oracle %.0f pts/s (brute force + fit), fit alone %.3g pts/s, cKDTree %.3g pts/s "
            "on %d threads, %s" % (len(sample) / dt, m_fit / dt_fit, m_fit / dt_tree, threads, ci))
        ok = (ref_st & 0x10) == 0
        acc = {}
        for name, first in (("fp32", first32), ("fp64", first64)):
            if first is None:
                continue
            g = first.cpu().numpy()[sample]
            e = np.linalg.norm(g - ref, axis=1)[ok] / h
            acc[name] = {"rms_over_h": float(np.sqrt((e ** 2).mean())), "max_over_h": float(e.max()),
                         "n": int(ok.sum())}
        res["accuracy_pass1_vs_oracle"] = acc

        # accuracy per workload, path and pass (sampled queries, the oracle's
        # brute-force lists)
        t = time.perf_counter()
        table = {}
        m = args.acc_sample
        for prec, io in (("fp32", io32), ("fp64", io64)):
            if io is None:
                continue
            for p_i, (qin, qout, qst) in enumerate(io):
                idx, idx_t = sample_rows(torch, args.n, m, 100 + p_i)
                table["heightfield_10M_k48/pass%d/%s" % (p_i + 1, prec)] = accuracy_of(
                    oracle, P, qin[idx_t].cpu().numpy(), args.k, h,
                    qout[idx_t].cpu().numpy(), qst[idx_t].cpu().numpy())
        for key, val in keep.items():
            if key == "batch":
                continue
            name, prec = key
            Pc, hc, kc, outc, stc = val
            idx, idx_t = sample_rows(torch, Pc.shape[0], m, 200)
            table["%s/%s" % (name, prec)] = accuracy_of(
                oracle, Pc, Pc[idx], kc, hc, outc[idx_t].cpu().numpy(), stc[idx_t].cpu().numpy())
        if "batch" in keep:
            kb = keep["batch"]
            off, hb = kb["off"], kb["h"]
            out_b, st_b = kb["out"].cpu().numpy(), kb["status"].cpu().numpy()
            e_all, n_all, mism = [], 0, 0
            per = max(1, m // (len(off) - 1))
            for c in range(len(off) - 1):
                Pc = kb["P"][off[c]:off[c + 1]]
                rng_c = np.random.default_rng(300 + c)
                li = np.sort(rng_c.choice(Pc.shape[0], size=min(per, Pc.shape[0]), replace=False))
                a_c = accuracy_of(oracle, Pc, Pc[li], 32, hb[c], out_b[off[c] + li],
                                  st_b[off[c] + li])
                e_all.append((a_c["rms_over_h"] ** 2 * a_c["n"], a_c["max_over_h"]))
                n_all += a_c["n"]
                mism += a_c["status_mismatches"]
            table["batch_256_clouds_30M_k32/fp32"] = {
                "rms_over_h": float(np.sqrt(sum(x for x, _ in e_all) / max(n_all, 1))),
                "max_over_h": float(max(y for _, y in e_all)), "n": n_all,
                "status_mismatches": mism}
        res["accuracy_vs_oracle"] = table
        log("accuracy table (%.1f s): %s" % (time.perf_counter() - t, json.dumps(table)))

        # the adjoint against the oracle's central differences on 1,000
        # queries of the bumped sphere, both paths
        if ("sh_sphere_2M_k32", "fp32") in keep:
            P4c, h4c = keep[("sh_sphere_2M_k32", "fp32")][:2]
            res["adjoint_vs_fd"] = adjoint_check(api, torch, oracle, P4c, h4c)
            log("adjoint vs central differences: %s" % res["adjoint_vs_fd"])

        if first_ps is not None:
            ref_ps, ref_ps_st = oracle.project(P64, Q, args.k, h, nbr=nbr,
                                               plane_iters=args.plane_iters)
            ok_ps = (ref_ps_st & 0x10) == 0
            e = np.linalg.norm(first_ps.cpu().numpy()[sample] - ref_ps, axis=1)[ok_ps] / h
            res["plane_steps"]["accuracy_pass1_vs_oracle"] = {
                "rms_over_h": float(np.sqrt((e ** 2).mean())), "max_over_h": float(e.max()),
                "n": int(ok_ps.sum())}

        for prec, fl in first_lv.items():
            if fl is None:
                continue
            ref_lv, ref_lv_st = oracle.project(P64, Q, args.k, h, nbr=nbr, levin=True)
            ok_lv = (ref_lv_st & 0x10) == 0
            e = np.linalg.norm(fl.cpu().numpy()[sample] - ref_lv, axis=1)[ok_lv] / h
            res["levin"][prec]["accuracy_pass1_vs_oracle"] = {
                "rms_over_h": float(np.sqrt((e ** 2).mean())), "max_over_h": float(e.max()),
                "n": int(ok_lv.sum())}

    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
