"""Checks of every neighbour list of a full-size call, independent of the
library's kernels.

Lists: for every query a SciPy k-d tree (its own FP64 distances) returns the
k + 8 nearest points; their canonical keys ((dx^2 + dy^2) + dz^2, every
operation rounded, no fused multiply-add: separate torch element-wise
kernels) are ordered by (key, index). A point outside that superset is at
least the superset's largest tree distance d_max away, so when the k-th
canonical key lies below d_max^2 (1 - 1e-12) the first k of the superset are
the exact k nearest. Queries that miss this margin (ties or rounding at the
boundary) take the oracle's brute force. A seeded sample of queries is also
searched by brute force over the whole cloud in plain torch (keys of every
point, the k + 8 smallest by key, then the exact (key, index) order).

Positions: every query against the oracle projection fed the exact lists
(tests/parity.py bars)."""
import numpy as np
import torch


def canonical_keys(P_t, Q_t, idx_t):
    """(m, c) canonical FP64 keys of points idx_t (m, c) to queries Q_t (m, 3)."""
    D = P_t[idx_t] - Q_t[:, None, :]
    sx = D[..., 0] * D[..., 0]
    sy = D[..., 1] * D[..., 1]
    sz = D[..., 2] * D[..., 2]
    return (sx + sy) + sz


def order_by_key_index(key, idx):
    """Rows of (key, idx) ordered ascending by key, ties by index."""
    o = torch.argsort(idx, dim=1, stable=True)
    key, idx = key.gather(1, o), idx.gather(1, o)
    o = torch.argsort(key, dim=1, stable=True)
    return key.gather(1, o), idx.gather(1, o)


def exact_lists(orc, tree, P64, Q64, k, extra=8, chunk=1_000_000, workers=16):
    """(m, k) int64 torch tensor (cuda) of the exact k nearest of each query,
    in (key, index) order, and the number of queries resolved by the
    oracle's brute force."""
    P_t = torch.from_numpy(P64).cuda()
    out = torch.empty((Q64.shape[0], k), dtype=torch.int64, device="cuda")
    n_brute = 0
    for a in range(0, Q64.shape[0], chunk):
        Qc = Q64[a:a + chunk]
        d, idx = tree.query(Qc, k + extra, workers=workers)
        idx_t = torch.from_numpy(idx.astype(np.int64)).cuda()
        Q_t = torch.from_numpy(np.ascontiguousarray(Qc)).cuda()
        key, idx_s = order_by_key_index(canonical_keys(P_t, Q_t, idx_t), idx_t)
        dmax2 = torch.from_numpy(d[:, -1] ** 2).cuda()
        ok = key[:, k - 1] < dmax2 * (1.0 - 1e-12)
        out[a:a + Qc.shape[0]] = idx_s[:, :k]
        bad = torch.nonzero(~ok).flatten().cpu().numpy()
        if bad.size:
            ref, _ = orc.knn(P64, Qc[bad], k)
            out[a + torch.from_numpy(bad).cuda()] = torch.from_numpy(ref.astype(np.int64)).cuda()
            n_brute += int(bad.size)
    return out, n_brute


def brute_lists(P64, Q64, k, chunk=8):
    """(m, k) int64 numpy array: brute force over every point in plain torch
    (the k + 8 smallest canonical keys, then the exact (key, index) order;
    a tie at the (k+8)-th key is reported as an error)."""
    P_t = torch.from_numpy(P64).cuda()
    res = np.empty((Q64.shape[0], k), dtype=np.int64)
    for a in range(0, Q64.shape[0], chunk):
        Q_t = torch.from_numpy(np.ascontiguousarray(Q64[a:a + chunk])).cuda()
        D = P_t[None, :, :] - Q_t[:, None, :]
        key = (D[..., 0] * D[..., 0] + D[..., 1] * D[..., 1]) + D[..., 2] * D[..., 2]
        del D
        kv, ki = torch.topk(key, k + 8, dim=1, largest=False)
        last = kv[:, -1:]
        # no point outside the k + 8 may tie with the k-th key
        kth = torch.sort(kv, dim=1).values[:, k - 1:k]
        assert bool((kth < last).all()), "tie reaches the (k+8)-th key"
        _, idx = order_by_key_index(kv, ki)
        res[a:a + Q_t.shape[0]] = idx[:, :k].cpu().numpy()
    return res


def workspace_lists(g, k_list, n):
    """(n, k_list) int64 original indices of the lists the last search left in
    the grid's projection workspace, in query order (queries aligned with the
    points; the lists lead the workspace in tiles of 64 slots, entry-major)."""
    spts, inv = g.sorted_points()
    tiles = (n + 63) // 64
    raw = g._proj_ws[: 4 * tiles * 64 * k_list].view(torch.int32).view(tiles, k_list, 64)
    slot = raw.permute(0, 2, 1).reshape(tiles * 64, k_list)[:n]
    orig = spts[:, 3].contiguous().view(torch.int32).long()
    lists = orig[slot.long().clamp(0, n - 1)]
    lists[slot < 0] = -1
    return lists[inv.long()]


def same_sets(a, b):
    """Row-wise set equality of two (m, c) integer tensors (cuda)."""
    return torch.equal(torch.sort(a, dim=1).values, torch.sort(b, dim=1).values)


def first_mismatch(a, b):
    d = (torch.sort(a, dim=1).values != torch.sort(b, dim=1).values).any(dim=1)
    return torch.nonzero(d).flatten()[:5].cpu().numpy()
