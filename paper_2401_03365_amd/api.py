"""PyTorch-facing binding of libmls.so.

PyTorch provides device memory (tensors, workspaces) and the current HIP
stream; every step of the projection runs in the library's kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _abi

PRECISIONS = {"fp64": _abi.MLS_PREC_FP64, "fp32": _abi.MLS_PREC_FP32_MOMENTS}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _host_i64(a):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def _check_points(t: torch.Tensor, name: str, dtypes=(torch.float32,)):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype not in dtypes or t.dim() != 2 or t.shape[1] != 3 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous (n, 3) tensor of %s" % (name, dtypes))


def _dtype_code(t: torch.Tensor):
    return _abi.MLS_F64 if t.dtype == torch.float64 else _abi.MLS_F32


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Grid:
    """Morton-sorted uniform-grid index of one cloud or a batch of clouds.

    ``h`` is the Gaussian width per cloud; ``cell_size`` (per cloud, or None)
    the finest grid cell edge (default 1.25 h). Calls on the grid can be
    captured in a HIP graph (queries aligned with the points, or one cloud
    without query offsets); the grid and its workspaces must outlive the
    graph."""

    def __init__(self, points: torch.Tensor, h, cloud_offsets=None, cell_size=None):
        lib = _abi.load()
        _check_points(points, "points")
        n = points.shape[0]
        offs, offs_p = _host_i64(cloud_offsets)
        n_clouds = 1 if offs is None else len(offs) - 1
        hh = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (n_clouds,)))
        cs = None
        if cell_size is not None:
            cs = np.ascontiguousarray(np.broadcast_to(np.asarray(cell_size, dtype=np.float64),
                                                      (n_clouds,)))
        nbytes = lib.mls_grid_workspace_bytes(n, n_clouds)
        if nbytes == 0:
            raise ValueError("invalid grid size")
        self.points = points
        self.device = points.device
        self.n_points = n
        self.n_clouds = n_clouds
        self.h = hh
        self.offsets = offs
        self.workspace = _workspace(nbytes, points.device)
        handle = ctypes.c_void_p()
        code = lib.mls_build_grid(_ptr(points), n, offs_p, n_clouds,
                                  hh.ctypes.data_as(ctypes.c_void_p),
                                  cs.ctypes.data_as(ctypes.c_void_p) if cs is not None else None,
                                  _ptr(self.workspace), self.workspace.numel(), _stream(),
                                  ctypes.byref(handle))
        _abi.check(code, "mls_build_grid")
        self._handle = handle
        self._proj_ws = None
        self._retired_ws = []

    def rebuild(self, points: torch.Tensor):
        """Re-sorts the grid for new positions of its points (same shape)
        with kernels only, so it can sit in a captured HIP graph; the grid
        keeps its first build's geometry (see mls_rebuild_grid)."""
        _check_points(points, "points")
        if points.shape[0] != self.n_points:
            raise ValueError("rebuild needs the same number of points")
        code = _abi.load().mls_rebuild_grid(self._handle, _ptr(points), _stream())
        _abi.check(code, "mls_rebuild_grid")
        self.points = points

    # ---- facts ------------------------------------------------------------
    def info(self) -> dict:
        info = _abi.MlsGridInfo()
        _abi.check(_abi.load().mls_get_grid_info(self._handle, ctypes.byref(info)),
                   "mls_get_grid_info")
        return {f: getattr(info, f) for f, _ in info._fields_}

    def cloud_grid(self, c: int = 0):
        origin = (ctypes.c_double * 3)()
        cell = ctypes.c_double()
        dims = (ctypes.c_int32 * 3)()
        _abi.check(_abi.load().mls_get_cloud_grid(self._handle, c, origin, ctypes.byref(cell),
                                                  dims), "mls_get_cloud_grid")
        return list(origin), cell.value, list(dims)

    def sorted_points(self):
        """(xyzw float32 (n,4) view, inverse permutation int32 (n,)) of the grid."""
        xyzw = ctypes.c_void_p()
        inv = ctypes.c_void_p()
        _abi.check(_abi.load().mls_grid_sorted_points(self._handle, ctypes.byref(xyzw),
                                                      ctypes.byref(inv)), "mls_grid_sorted_points")
        base = self.workspace.data_ptr()
        o1 = xyzw.value - base
        o2 = inv.value - base
        pts = self.workspace[o1:o1 + 16 * self.n_points].view(torch.float32).view(-1, 4)
        ip = self.workspace[o2:o2 + 4 * self.n_points].view(torch.int32)
        return pts, ip

    def caller_rows(self) -> torch.Tensor:
        """int64 (n,): the point index of each sorted position, so that
        x_caller[caller_rows()] = x_sorted converts rows in the grid's sorted
        order (slot_order) to the caller's."""
        pts, _ = self.sorted_points()
        return pts[:, 3].contiguous().view(torch.int32).long()

    def cell_table(self):
        """(slots int64 (capacity, 2) view: [tagged key, first | end << 32],
        levels in the table) of the grid's cell hash."""
        tab = ctypes.c_void_p()
        cap = ctypes.c_int64()
        lev = ctypes.c_void_p()
        _abi.check(_abi.load().mls_grid_cell_table(self._handle, ctypes.byref(tab),
                                                   ctypes.byref(cap), ctypes.byref(lev)),
                   "mls_grid_cell_table")
        base = self.workspace.data_ptr()
        o1, o2 = tab.value - base, lev.value - base
        slots = self.workspace[o1:o1 + 16 * cap.value].view(torch.int64).view(-1, 2)
        levels = int(self.workspace[o2:o2 + 4].view(torch.int32).item())
        return slots, levels

    # ---- workspace --------------------------------------------------------
    def _proj_workspace(self, k: int, n: int) -> torch.Tensor:
        """One cached workspace for search, fit and adjoint (sized for the
        adjoint, so that it can reuse the lists of the preceding search)."""
        lib = _abi.load()
        nbytes = max(lib.mls_project_workspace_bytes(self._handle, k, n),
                     lib.mls_project_backward_workspace_bytes(self._handle, k, n,
                                                              _abi.MLS_PREC_FP64))
        if nbytes == 0:
            raise ValueError("invalid k or query count")
        if self._proj_ws is None or self._proj_ws.numel() < nbytes:
            if self._proj_ws is not None:
                # a captured graph may still launch kernels on the old buffer
                self._retired_ws.append(self._proj_ws)
            self._proj_ws = _workspace(nbytes, self.device)
        return self._proj_ws

    # ---- calls ------------------------------------------------------------
    def knn(self, queries: torch.Tensor, k: int, query_offsets=None, return_keys=False):
        _check_points(queries, "queries", (torch.float32, torch.float64))
        n = queries.shape[0]
        nbr = torch.empty((n, k), dtype=torch.int32, device=self.device)
        keys = torch.empty((n, k), dtype=torch.float64, device=self.device) if return_keys else None
        ws = self._proj_workspace(k, n)
        qo, qo_p = _host_i64(query_offsets)
        code = _abi.load().mls_knn(self._handle, k, _ptr(queries), _dtype_code(queries), n, qo_p,
                                   _ptr(nbr), _ptr(keys), _ptr(ws), ws.numel(), _stream())
        _abi.check(code, "mls_knn")
        return (nbr, keys) if return_keys else nbr

    def _params(self, k, precision, support_radius_h, min_support, stages=0, search_extra=0,
                plane_iters=0, ball=False, levin=False, slot_order=0):
        if precision not in PRECISIONS:
            raise ValueError("precision must be 'fp32' or 'fp64'")
        return _abi.MlsParams(k=int(k), precision=PRECISIONS[precision],
                              support_radius_h=float(support_radius_h),
                              min_support=int(min_support), stages=int(stages),
                              search_extra=int(search_extra), plane_iters=int(plane_iters),
                              ball=int(ball), levin=int(bool(levin)),
                              slot_order=int(slot_order))

    def project(self, queries: torch.Tensor, k: int, precision: str = "fp32",
                query_offsets=None, return_neighbors=False, out: Optional[torch.Tensor] = None,
                support_radius_h: float = 3.0, min_support: int = 3, stages: int = 0,
                status: Optional[torch.Tensor] = None, search_extra: int = 0,
                refresh: bool = False, plane_iters: int = 0, ball: bool = False,
                geometry: bool = False, levin: bool = False, slot_order: int = 0):
        """One MLS projection pass. Returns (out, status[, neighbours]).
        ``stages``: 0 = search and fit, 1 = search only (lists stay in the
        grid's workspace), 2 = fit only from the preceding search.
        ``search_extra``: neighbours kept beyond k for later refreshes;
        ``refresh``: start the search from the lists of the previous search
        of the same queries' slots (exact; see MLS_STAGE_REFRESH);
        ``plane_iters``: steps of the reference plane with the weights at
        the plane's own projection of the query (0: weights at the query);
        ``levin``: Levin's reference plane, the local minimum of Eq. (1.1)
        over (n, t) with the weights at q = r + t n (status 4, NO_MINIMUM,
        where the descent leaves the support radius);
        ``ball``: 1 (or True): the neighbourhood is the list entries within
        support_radius_h * h (the paper's radius R), status flag 0x20 where
        the whole list lies inside it; 2: every cloud point within that
        radius, no count cap (k unused, no lists returned); ``geometry``: also return the surface
        normal (n, 3) and the mean and Gaussian curvature (n, 2) at each
        output, after the status: (out, status, normals, curvatures[, nbr]).
        ``slot_order`` (queries aligned with the points only): bit 1 reads
        the query of sorted position p at row p, bit 2 writes its results at
        row p (``caller_rows`` maps rows in that order to point indices)."""
        _check_points(queries, "queries", (torch.float32, torch.float64))
        n = queries.shape[0]
        if refresh:
            stages = (stages or (_abi.MLS_STAGE_SEARCH | _abi.MLS_STAGE_FIT)) | _abi.MLS_STAGE_REFRESH
        params = self._params(k, precision, support_radius_h, min_support, stages, search_extra,
                              plane_iters, ball, levin, slot_order)
        if out is None:
            out = torch.empty_like(queries)
        if status is None:
            status = torch.empty((n,), dtype=torch.uint8, device=self.device)
        nbr = torch.empty((n, k), dtype=torch.int32, device=self.device) if return_neighbors else None
        ws = self._proj_workspace(k + search_extra, n)
        qo, qo_p = _host_i64(query_offsets)
        if geometry:
            normals = torch.empty((n, 3), dtype=queries.dtype, device=self.device)
            curv = torch.empty((n, 2), dtype=queries.dtype, device=self.device)
            code = _abi.load().mls_project_geometry(
                self._handle, ctypes.byref(params), _ptr(queries), _dtype_code(queries), n, qo_p,
                _ptr(out), _ptr(status), _ptr(nbr), _ptr(normals), _ptr(curv), _ptr(ws),
                ws.numel(), _stream())
            _abi.check(code, "mls_project_geometry")
            res = (out, status, normals, curv)
        else:
            code = _abi.load().mls_project(self._handle, ctypes.byref(params), _ptr(queries),
                                           _dtype_code(queries), n, qo_p, _ptr(out),
                                           _ptr(status), _ptr(nbr), _ptr(ws), ws.numel(),
                                           _stream())
            _abi.check(code, "mls_project")
            res = (out, status)
        return res + (nbr,) if return_neighbors else res

    def project_noalloc(self, queries: torch.Tensor, k: int, precision: str = "fp32",
                        query_offsets=None, out: Optional[torch.Tensor] = None,
                        status: Optional[torch.Tensor] = None,
                        neighbors: Optional[torch.Tensor] = None,
                        support_radius_h: float = 3.0, min_support: int = 3):
        """One whole projection pass through mls_project_noalloc: the
        library's fixed device scratch replaces the workspace, so the call
        allocates nothing when ``out``, ``status`` (and ``neighbors``, (n, k)
        int32, if wanted) are given. Returns (out, status)."""
        _check_points(queries, "queries", (torch.float32, torch.float64))
        n = queries.shape[0]
        params = self._params(k, precision, support_radius_h, min_support)
        if out is None:
            out = torch.empty_like(queries)
        if status is None:
            status = torch.empty((n,), dtype=torch.uint8, device=self.device)
        qo, qo_p = _host_i64(query_offsets)
        code = _abi.load().mls_project_noalloc(self._handle, ctypes.byref(params), _ptr(queries),
                                               _dtype_code(queries), n, qo_p, _ptr(out),
                                               _ptr(status), _ptr(neighbors), _stream())
        _abi.check(code, "mls_project_noalloc")
        return out, status

    def project_backward(self, queries: torch.Tensor, grad_out: torch.Tensor, k: int,
                         precision: str = "fp32", neighbors: Optional[torch.Tensor] = None,
                         query_offsets=None, support_radius_h: float = 3.0, min_support: int = 3,
                         reuse_lists: bool = False, search_extra: int = 0):
        """Adjoint of one pass with lists and statuses fixed: returns
        (grad_queries, grad_points), both in the queries' dtype.
        ``neighbors``: the (n, k) int32 original-index lists of the forward
        pass, or None to recompute them; ``reuse_lists``: take the lists the
        last search on this grid's workspace left there (the immediately
        preceding ``project`` of the same queries)."""
        _check_points(queries, "queries", (torch.float32, torch.float64))
        n = queries.shape[0]
        stages = _abi.MLS_STAGE_FIT if reuse_lists else 0
        params = self._params(k, precision, support_radius_h, min_support, stages, search_extra)
        lib = _abi.load()
        if grad_out.shape != queries.shape:
            raise ValueError("grad_out must have the shape of queries")
        grad_out = grad_out.to(device=self.device, dtype=queries.dtype).contiguous()
        if neighbors is not None:
            if reuse_lists:
                raise ValueError("neighbors and reuse_lists exclude each other")
            if neighbors.shape != (n, k) or neighbors.dtype != torch.int32 or not neighbors.is_cuda:
                raise ValueError("neighbors must be a CUDA (n, k) int32 tensor")
            neighbors = neighbors.contiguous()
        gq = torch.empty_like(queries)
        gp = torch.empty((self.n_points, 3), dtype=queries.dtype, device=self.device)
        ws = self._proj_workspace(k + search_extra, n)
        qo, qo_p = _host_i64(query_offsets)
        code = lib.mls_project_backward(
            self._handle, ctypes.byref(params), _ptr(queries), _dtype_code(queries), n, qo_p,
            _ptr(neighbors), _ptr(grad_out), _ptr(gq), _ptr(gp), _ptr(ws), ws.numel(), _stream())
        _abi.check(code, "mls_project_backward")
        return gq, gp

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            _abi.load().mls_grid_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_cell_factor(points: torch.Tensor, h, k: int, cloud_offsets=None,
                         candidates: Sequence[float] = (0.8, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0),
                         stride: int = 1):
    """Measures the neighbour search for each candidate cell edge (factor x
    h) and returns (best factor, {factor: ms}). ``stride`` 1 (the default)
    times the search over every point (its ranking is that of the full run);
    a larger stride samples 1/stride of them (runs of 256 consecutive points
    of each candidate grid's Morton order)."""
    lib = _abi.load()
    _check_points(points, "points")
    n = points.shape[0]
    offs, offs_p = _host_i64(cloud_offsets)
    n_clouds = 1 if offs is None else len(offs) - 1
    hh = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (n_clouds,)))
    cand = np.ascontiguousarray(np.asarray(candidates, dtype=np.float64))
    ms = np.zeros(len(cand), dtype=np.float32)
    nbytes = lib.mls_autotune_workspace_bytes(n, n_clouds, k, stride)
    if nbytes == 0:
        raise ValueError("invalid autotune arguments")
    ws = _workspace(nbytes, points.device)
    best = ctypes.c_double()
    code = lib.mls_autotune_cell(_ptr(points), n, offs_p, n_clouds,
                                 hh.ctypes.data_as(ctypes.c_void_p), int(k),
                                 cand.ctypes.data_as(ctypes.c_void_p), len(cand), int(stride),
                                 _ptr(ws), ws.numel(), _stream(), ctypes.byref(best),
                                 ms.ctypes.data_as(ctypes.c_void_p))
    _abi.check(code, "mls_autotune_cell")
    return best.value, {float(c): float(t) for c, t in zip(cand, ms)}


SIZE_CLASSES = (20_000, 80_000, 250_000)  # upper bounds of the cloud-size classes


def size_class(n: int) -> int:
    return int(np.searchsorted(np.asarray(SIZE_CLASSES), n, side="right"))


def autotune_cells(points: torch.Tensor, h, k: int, cloud_offsets=None,
                   candidates: Sequence[float] = (0.8, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0)):
    """Cell edge factor per cloud: one factor for a single cloud; for a batch,
    one per cloud-size class (clouds below 20k, 80k, 250k points and above),
    each measured on that class's clouds alone (full searches). Returns
    (per-cloud factors (n_clouds,), {class: (best, {factor: ms})})."""
    if cloud_offsets is None:
        best, ms = autotune_cell_factor(points, h, k, candidates=candidates)
        return np.array([best]), {0: (best, ms)}
    off = np.asarray(cloud_offsets, dtype=np.int64)
    hh = np.broadcast_to(np.asarray(h, dtype=np.float64), (len(off) - 1,))
    sizes = np.diff(off)
    cls = np.array([size_class(int(n)) for n in sizes])
    factors = np.empty(len(sizes))
    report = {}
    for c in np.unique(cls):
        ids = np.nonzero(cls == c)[0]
        parts = [points[off[i]:off[i + 1]] for i in ids]
        sub = torch.cat(parts).contiguous()
        sub_off = np.concatenate([[0], np.cumsum(sizes[ids])])
        best, ms = autotune_cell_factor(sub, hh[ids], k, cloud_offsets=sub_off,
                                        candidates=candidates)
        factors[ids] = best
        report[int(c)] = (best, ms)
        del sub
    return factors, report


def autotune_search_extra(grid: Grid, queries: torch.Tensor, k: int, precision: str = "fp32",
                          candidates: Sequence[int] = (8, 12, 16, 24)):
    """Extra neighbours a search keeps for the refresh of the pass after it
    (iterated passes): for each candidate, one pass on ``queries`` (search
    keeping the extras, fit), then the next pass's refreshed search from its
    outputs; the time of the two searches is measured (HIP events, second of
    two runs). Returns (best, {extra: ms})."""
    n = queries.shape[0]
    out = torch.empty_like(queries)
    nxt = torch.empty_like(queries)
    st = torch.empty((n,), dtype=torch.uint8, device=queries.device)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    res = {}
    for extra in candidates:
        extra = int(min(extra, _abi.MLS_MAX_K - k))
        for _ in range(2):
            e0.record()
            grid.project(queries, k, precision, stages=1, out=out, status=st,
                         search_extra=extra)
            e1.record()
            grid.project(queries, k, precision, stages=2, out=out, status=st,
                         search_extra=extra)
            e2.record()
            grid.project(out, k, precision, stages=1, out=nxt, status=st, search_extra=extra,
                         refresh=True)
            e3 = torch.cuda.Event(enable_timing=True)
            e3.record()
            torch.cuda.synchronize()
        res[extra] = e0.elapsed_time(e1) + e2.elapsed_time(e3)
    best = min(res, key=res.get)
    return best, res


def build_grid(points, h, cloud_offsets=None, cell_size=None) -> Grid:
    return Grid(points, h, cloud_offsets=cloud_offsets, cell_size=cell_size)


def project(points: torch.Tensor, h, k: int, precision: str = "fp32", passes: int = 1,
            cell_size=None, cloud_offsets=None, plane_iters: int = 0, ball: bool = False,
            support_radius_h: float = 3.0):
    """Project a cloud onto its own MLS surface ``passes`` times (queries move,
    the cloud and its grid stay fixed). ``plane_iters``: steps of the
    self-consistent reference plane per pass. From the second pass on, the
    search keeps up to 16 extra neighbours and the passes after it refresh
    those lists (exact; see MLS_STAGE_REFRESH) instead of searching every
    query afresh. Returns (out, status)."""
    grid = Grid(points, h, cloud_offsets=cloud_offsets, cell_size=cell_size)
    extra = min(16, _abi.MLS_MAX_K - k) if passes >= 3 else 0
    cur = points
    st = None
    for it in range(passes):
        out, st_new = grid.project(cur, k, precision, plane_iters=plane_iters, ball=ball,
                                   support_radius_h=support_radius_h,
                                   search_extra=extra if it >= 1 else 0,
                                   refresh=extra > 0 and it >= 2)
        if st is not None:
            frozen = (st & 0x0F) == _abi.PT_OUTLIER
            out[frozen] = cur[frozen]
            st_new = torch.where(frozen, st, st_new)
        cur, st = out, st_new
    return cur, st


class MLSProject(torch.autograd.Function):
    """out = P(queries; cloud) with a backward through the hand-written
    adjoint kernel (lists held fixed, moments recomputed)."""

    @staticmethod
    def forward(ctx, queries, points, grid: Grid, k: int, precision: str):
        # the backward reads the same contiguous copy the forward projected
        q = queries.detach().contiguous()
        out, status, nbr = grid.project(q, k, precision, return_neighbors=True)
        ctx.grid, ctx.k, ctx.precision = grid, k, precision
        ctx.points_dtype = points.dtype
        ctx.save_for_backward(q, nbr)
        ctx.mark_non_differentiable(status)
        return out, status

    @staticmethod
    def backward(ctx, grad_out, grad_status):
        queries, nbr = ctx.saved_tensors
        gq, gp = ctx.grid.project_backward(queries, grad_out, ctx.k, ctx.precision, neighbors=nbr)
        return gq, gp.to(ctx.points_dtype), None, None, None


def mls_project(queries, points, grid: Grid, k: int, precision: str = "fp32"):
    """Differentiable projection; gradients flow to queries and points."""
    return MLSProject.apply(queries, points, grid, k, precision)
