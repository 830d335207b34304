"""Pins of the oracle's brute-force kNN (canonical FP64 keys, ties to the
smaller original index) against NumPy's lexsort over all pairs."""
import numpy as np
import pytest

from paper_2401_03365_amd import synth


def lexsort_knn(P, Q, k):
    """k smallest (key, index) pairs per query from a full sort. The key is
    formed by separate NumPy ufuncs, so no fused multiply-add can occur."""
    P = np.asarray(P, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    idx = np.empty((Q.shape[0], k), dtype=np.int64)
    keys = np.empty((Q.shape[0], k))
    ar = np.arange(P.shape[0])
    for j, r in enumerate(Q):
        d = P - r
        key = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        order = np.lexsort((ar, key))[:k]
        idx[j] = order
        keys[j] = key[order]
    return idx, keys


CLOUDS = {
    "random": lambda: synth.sphere(300, 0.05, seed=7),
    "lattice": lambda: synth.lattice(7, 6, 3, spacing=0.25),
    "duplicates": lambda: np.repeat(synth.sphere(40, 0.0, seed=8), 4, axis=0),
    "collinear": lambda: synth.lattice(64, 1, 1, spacing=0.5),
    "planar_lattice": lambda: synth.lattice(12, 12, 1, spacing=1.0, origin=(-5.5, -5.5, 0.0)),
}


@pytest.mark.parametrize("name", sorted(CLOUDS))
@pytest.mark.parametrize("k", [6, 32])
def test_knn_matches_lexsort(orc, name, k):
    P = CLOUDS[name]().astype(np.float64)
    k = min(k, P.shape[0])
    idx, key = orc.knn(P, P, k)
    ref_idx, ref_key = lexsort_knn(P, P, k)
    np.testing.assert_array_equal(idx, ref_idx)
    np.testing.assert_array_equal(key, ref_key)


def test_knn_off_cloud_queries_and_n_equals_k(orc):
    P = synth.lattice(4, 4, 2, spacing=0.5).astype(np.float64)  # 32 points
    rng = np.random.default_rng(3)
    Q = rng.uniform(-1, 3, (50, 3))
    idx, key = orc.knn(P, Q, 32)  # N == k: every list is a permutation of all points
    ref_idx, ref_key = lexsort_knn(P, Q, 32)
    np.testing.assert_array_equal(idx, ref_idx)
    assert all(sorted(row) == list(range(32)) for row in idx.tolist())


def test_knn_self_included_and_sorted(orc):
    P = synth.sphere(500, 0.01, seed=9).astype(np.float64)
    idx, key = orc.knn(P, P, 16)
    assert np.all(key[:, 0] == 0.0)
    assert np.all(idx[:, 0] == np.arange(500))  # no duplicates in this cloud
    assert np.all(np.diff(key, axis=1) >= 0)


def test_knn_nonfinite(orc):
    P = synth.sphere(50, 0.01, seed=10).astype(np.float64)
    P[3] = np.nan
    Q = np.vstack([P[:2], [[np.inf, 0, 0]]])
    idx, key = orc.knn(P, Q, 8)
    assert not np.any(idx[:2] == 3)
    assert np.all(idx[2] == -1)
