"""Pins of the oracle's radius-R neighbourhood (``ball``: the list entries
within R = support_radius_h * h, the paper's neighbourhood of Section 1.4;
TRUNCATED when the whole k-nearest list lies inside R).

- A ball larger than every list reproduces the k-nearest projection exactly
  and flags every query.
- Otherwise the ball is the first m entries of the sorted k-nearest list, so
  the result equals the k-nearest projection with k = m for that query, bit
  for bit; m equals the number of cloud points within R counted by brute
  force over the whole cloud (numpy), which checks that no point of the ball
  is missing.
- Planes are reproduced exactly."""
import numpy as np
import pytest

from paper_2401_03365_amd import synth

from test_oracle_project import load_golden, plane_case


def test_large_ball_is_the_knn_projection(orc):
    P = synth.sphere(3000, 0.01, seed=51).astype(np.float64)
    h = synth.mean_nn_h(P.astype(np.float32))
    a, sa = orc.project(P, P[:300], 24, h)
    b, sb = orc.project(P, P[:300], 24, h, ball=True, support_radius_h=1e3)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(sa, sb & ~np.uint8(orc.PT_FLAG_TRUNCATED))
    assert np.all(sb & orc.PT_FLAG_TRUNCATED)


@pytest.mark.parametrize("radius_h", [1.2, 1.6, 2.2])
def test_ball_equals_knn_with_the_ball_count(orc, radius_h):
    P = synth.torus(6000, sigma=0.005, n_outliers=60, seed=52).astype(np.float64)
    h = synth.mean_nn_h(P.astype(np.float32))
    k = 40
    rng = np.random.default_rng(53)
    Q = P[rng.choice(P.shape[0], 300, replace=False)]
    nbr, key = orc.knn(P, Q, k)
    out, st, dg = orc.project(P, Q, k, h, nbr=nbr, ball=True, support_radius_h=radius_h,
                              diag=True)
    m = dg[:, 21].astype(int)
    R2 = (radius_h * h) ** 2
    for j in range(Q.shape[0]):
        # brute force over the whole cloud, same canonical key
        d = P - Q[j]
        kk = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        count = int((kk <= R2).sum())
        if st[j] & orc.PT_FLAG_TRUNCATED:
            assert m[j] == k and count >= k
            continue
        assert m[j] == count
        if (st[j] & 0x0F) == orc.PT_OUTLIER:
            continue
        ref, ref_st = orc.project(P, Q[j:j + 1], m[j], h, nbr=nbr[j:j + 1, :m[j]],
                                  support_radius_h=radius_h)
        np.testing.assert_array_equal(out[j:j + 1], ref)
        assert (st[j] & 0x0F) == (ref_st[0] & 0x0F)


def test_ball_reproduces_planes(orc):
    c = load_golden()["planes"][0]
    P, Q, feet, n = plane_case(c)
    out, st = orc.project(P, Q, c["k"], c["h"], ball=True, support_radius_h=2.0)
    fit = (st & 0x0F) == orc.PT_OK
    assert fit.sum() > 0.9 * len(st)
    assert np.abs(out[fit] - feet[fit]).max() < 1e-13


# ---- the radius-R ball without a count cap (project_ball, O3c) -------------

def numpy_ball_counts(P, Q, R):
    counts = np.empty(Q.shape[0], dtype=np.int64)
    for j in range(Q.shape[0]):
        d = P - Q[j]
        kk = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        counts[j] = int((kk <= R * R).sum())
    return counts


@pytest.mark.parametrize("radius_h", [1.0, 2.5, 6.0])
def test_uncapped_ball_counts_match_numpy(orc, radius_h):
    P = synth.torus(5000, sigma=0.005, n_outliers=50, seed=54).astype(np.float64)
    h = synth.mean_nn_h(P.astype(np.float32))
    Q = P[np.random.default_rng(55).choice(P.shape[0], 200, replace=False)]
    out, st, cnt = orc.project_ball(P, Q, h, support_radius_h=radius_h)
    np.testing.assert_array_equal(cnt, numpy_ball_counts(P, Q, radius_h * h))
    # outliers are exactly the queries with fewer than 3 points in the ball
    np.testing.assert_array_equal((st & 0x0F) == orc.PT_OUTLIER, cnt < 3)
    if radius_h == 6.0:
        assert cnt.max() > 64  # beyond any k-nearest list


@pytest.mark.parametrize("radius_h", [1.6, 2.4])
def test_uncapped_ball_is_the_knn_projection_with_the_ball_count(orc, radius_h):
    # the ball holds the same points as the k-nearest list with k = its count,
    # only summed in another order (index order against key order)
    P = synth.sphere(4000, 0.01, seed=56).astype(np.float64)
    h = synth.mean_nn_h(P.astype(np.float32))
    Q = P[np.random.default_rng(57).choice(P.shape[0], 150, replace=False)]
    out, st, cnt = orc.project_ball(P, Q, h, support_radius_h=radius_h)
    checked = 0
    for j in range(Q.shape[0]):
        c = int(cnt[j])
        if c < 3 or c > 64:
            continue
        ref, ref_st = orc.project(P, Q[j:j + 1], c, h, support_radius_h=radius_h)
        assert (ref_st[0] & 0x0F) == (st[j] & 0x0F)
        assert np.abs(ref[0] - out[j]).max() <= 1e-12 * h  # summation order only
        checked += 1
    assert checked > 100


def test_uncapped_ball_reproduces_planes_with_large_balls(orc):
    c = load_golden()["planes"][1]
    P, Q, feet, n = plane_case(c)
    out, st, cnt = orc.project_ball(P, Q, c["h"], support_radius_h=6.0)
    fit = (st & 0x0F) == orc.PT_OK
    assert fit.sum() > 0.9 * len(st) and np.median(cnt) > 64
    assert np.abs(out[fit] - feet[fit]).max() < 1e-13


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_uncapped_ball_quadric_apex_on_larger_patches(orc, idx):
    # the golden patches grown to 9 x 9 = 81 lattice points (more than a
    # k-nearest list can hold): with the ball covering the whole symmetric
    # patch the fit is still exact and the output is the apex (0, 0, c0)
    c = dict(load_golden()["quadric_apex"][idx])
    c["lattice_half"] = 4
    from test_oracle_project import quadric_case
    P, Q = quadric_case(c)
    assert P.shape[0] == 81
    R = 2.0 * 4 * c["spacing"] * 1.5
    out, st, cnt = orc.project_ball(P, Q, c["h"], support_radius_h=R / c["h"])
    assert cnt[0] == 81 and (st[0] & 0x0F) == orc.PT_OK
    np.testing.assert_allclose(out[0], c["expected"], rtol=0, atol=1e-14)
