"""GPU checks of the grid build (bounding boxes, cell keys, Morton sort,
gather, cell hash) against a NumPy recomputation from the grid's own
per-cloud geometry: the sorted copy is a permutation of the finite points
with its inverse, ordered by (cloud, Morton code of the cell) and, within a
cell, by original index (a stable sort); the counts of non-empty cells and
non-finite points agree; the hash holds at least twice the non-empty cells
and stays inside its reservation."""
import numpy as np
import pytest
import torch

from paper_2401_03365_amd import synth

pytestmark = pytest.mark.gpu


def api():
    from paper_2401_03365_amd import api as a
    return a


def spread3(v):
    """Every bit of v (< 2^21) moved to bit 3 i."""
    out = np.zeros_like(v, dtype=np.uint64)
    v = v.astype(np.uint64)
    for b in range(21):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def expected_keys(P, origin, cell, dims, bits, cloud, cloud_bits_shift):
    inv = 1.0 / cell
    c = np.empty((P.shape[0], 3), dtype=np.int64)
    for a in range(3):
        t = np.floor((P[:, a].astype(np.float64) - origin[a]) * inv)
        c[:, a] = np.clip(t, 0, dims[a] - 1).astype(np.int64)
    m = spread3(c[:, 0]) | (spread3(c[:, 1]) << np.uint64(1)) | (spread3(c[:, 2]) << np.uint64(2))
    return (np.uint64(cloud) << np.uint64(cloud_bits_shift)) | m


def grid_keys(g, P, offsets):
    """Checks the sorted copy and its order; returns the sorted finite
    points' cell keys recomputed from the grid's geometry, and the count of
    non-empty cells."""
    info = g.info()
    C = len(offsets) - 1
    finite = np.isfinite(P).all(axis=1)
    xyzw, inv = g.sorted_points()
    torch.cuda.synchronize()
    xyzw = xyzw.cpu().numpy()
    inv = inv.cpu().numpy()
    nf = int(finite.sum())
    orig = xyzw[:nf, 3].view(np.int32).astype(np.int64)
    # a permutation of the finite points, coordinates copied exactly
    np.testing.assert_array_equal(np.sort(orig), np.flatnonzero(finite))
    np.testing.assert_array_equal(xyzw[:nf, :3], P[orig])
    np.testing.assert_array_equal(inv[orig], np.arange(nf))
    # order: (cloud, Morton code) ascending, original index within a cell
    cloud_bits = 0
    while (1 << cloud_bits) < C:
        cloud_bits += 1
    bits = (info["key_bits"] - 1 - cloud_bits) // 3
    keys = np.empty(nf, dtype=np.uint64)
    cl = np.searchsorted(offsets, orig, side="right") - 1
    cells = 0
    for c in range(C):
        origin, cell, dims = g.cloud_grid(c)
        sel = cl == c
        keys[sel] = expected_keys(P[orig[sel]], origin, cell, dims, bits, c, 3 * bits)
        cells += np.unique(keys[sel]).size
    assert np.all(keys[1:] >= keys[:-1])
    same = keys[1:] == keys[:-1]
    assert np.all(orig[1:][same] > orig[:-1][same])
    return keys, cells


def check_grid(g, P, offsets):
    info = g.info()
    n = P.shape[0]
    finite = np.isfinite(P).all(axis=1)
    assert info["n_nonfinite"] == int((~finite).sum())
    keys, cells = grid_keys(g, P, offsets)
    assert info["n_cells"] == cells
    cap = info["hash_capacity"]
    assert cap & (cap - 1) == 0 and cap >= 2 * cells
    assert cap <= 1 << int(np.ceil(np.log2(max(4 * n, 64))))
    check_table(g, keys)
    return info


PHI = np.uint64(0x9E3779B97F4A7C15)


def check_table(g, keys, levels=None):
    """The cell table holds exactly the cells of its levels, each as
    {tagged key, first, end} of its run of sorted keys, every key reachable
    by linear probing from its home slot."""
    slots, lev = g.cell_table()
    torch.cuda.synchronize()
    if levels is not None:
        assert lev == levels
    slots = slots.cpu().numpy().view(np.uint64)
    cap = slots.shape[0]
    occ = slots[:, 0] != np.uint64(0xFFFFFFFFFFFFFFFF)
    got = np.stack([slots[occ, 0], slots[occ, 1] & np.uint64(0xFFFFFFFF),
                    slots[occ, 1] >> np.uint64(32)], axis=1)
    exp = []
    nf = keys.size
    for l in range(lev):
        kl = keys >> np.uint64(3 * l)
        st = np.flatnonzero(np.concatenate([[True], kl[1:] != kl[:-1]])) if nf else np.array([], int)
        en = np.append(st[1:], nf)
        tag = kl[st] | (np.uint64(l) << np.uint64(60))
        exp.append(np.stack([tag, st.astype(np.uint64), en.astype(np.uint64)], axis=1))
    exp = np.concatenate(exp) if exp else np.zeros((0, 3), np.uint64)
    np.testing.assert_array_equal(got[np.argsort(got[:, 0])], exp[np.argsort(exp[:, 0])])
    shift = np.uint64(64 - int(np.log2(cap)))
    home = (slots[occ, 0] * PHI) >> shift
    at = np.flatnonzero(occ).astype(np.uint64)
    empties = np.concatenate([[0], np.cumsum(~occ)])
    h, i = home.astype(np.int64), at.astype(np.int64)
    between = np.where(i >= h, empties[i] - empties[h], empties[cap] - empties[h] + empties[i])
    assert not between.any(), "a key sits past an empty slot of its probe sequence"


def test_grid_of_a_height_field():
    P = synth.heightfield(1_000_000, sigma=1e-3, seed=3)
    h = synth.mean_nn_h(P)
    g = api().Grid(torch.from_numpy(P).cuda(), h, cell_size=1.25 * h)
    check_grid(g, P, np.array([0, P.shape[0]]))


@pytest.mark.parametrize("n", [256, 4096, 65536, 64 * 1001, 100_003])
def test_grid_table_at_block_multiples(n):
    # the last cell's run ends at n, which a multiple of the insertion's
    # 256-position blocks puts outside every block holding a point
    P = synth.sphere(n, 0.01, seed=105)
    g = api().Grid(torch.from_numpy(P).cuda(), synth.mean_nn_h(P))
    check_grid(g, P, np.array([0, n]))


def test_grid_of_clouds_with_nonfinite_points():
    parts = [synth.sphere(20000, 0.01, seed=101), synth.torus(30000, sigma=0.01, seed=102),
             synth.heightfield(25000, sigma=1e-3, seed=103)]
    P = np.concatenate(parts)
    rng = np.random.default_rng(104)
    bad = rng.choice(P.shape[0], 50, replace=False)
    P[bad[:20], 0] = np.nan
    P[bad[20:], 2] = np.inf
    offs = np.concatenate([[0], np.cumsum([p.shape[0] for p in parts])]).astype(np.int64)
    hs = [synth.mean_nn_h(p) for p in parts]
    g = api().Grid(torch.from_numpy(P).cuda(), hs, cloud_offsets=offs)
    info = check_grid(g, P, offs)
    assert info["n_clouds"] == 3
