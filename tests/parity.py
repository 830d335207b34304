"""Shared parity rules of the GPU tests against the FP64 oracle.

Statuses: the whole status byte must match. The low nibble (OK, OUTLIER,
PLANE_ONLY, NONFINITE) and the TRUNCATED flag (0x20) exactly; the
NORMAL_AMBIGUOUS flag (0x10, set when lambda2 - lambda1 < 1e-6 lambda3 of
the plane's weighted covariance) may differ only where the oracle's own
relative gap (lambda2 - lambda1) / lambda3 lies within [0.5, 2] x 1e-6, where
the rounding of either side can move it across the threshold.

Positions, in units of h, over the points whose oracle status carries no
ambiguous-normal flag and is not NONFINITE (reading A17: flagged points have
several correct normals and are left out of max errors):
  FP64 path          max <= 1e-10 h;
  FP32-moment path   RMS <= 1e-5 h, and per point at most the larger of
                     1e-4 h and 10 eps32 / gap h (capped at 1e-2 h), gap =
                     (lambda2 - lambda1) / lambda3 of the oracle's plane
                     covariance, eps32 = 2^-24. The unit normal moves by
                     about dC / (lambda2 - lambda1) under a perturbation dC
                     of the covariance (first-order eigenvector
                     perturbation), and FP32 moments perturb C by about
                     eps32 lambda3, so the FP32 error of a point grows as
                     eps32 / gap; at the gaps of smooth clouds (above 1e-2)
                     the bar is the flat 1e-4 h.
Outputs stored in FP32 are allowed their storage rounding (an FP32 ulp per
coordinate) on top.

Flagged fraction: on clouds sampled from a smooth surface at most 1 % of the
queries may carry the ambiguous flag (the flag removes a point from the max
bars, so a spurious flag would silently shrink the checked set)."""
import numpy as np

FP64_MAX_H = 1e-10
FP32_RMS_H = 1e-5
FP32_MAX_H = 1e-4
FP32_MAX_CAP_H = 1e-2
EPS32 = 2.0 ** -24
GAP = 1e-6
FLAG_FRACTION_SURFACE = 0.01


def oracle_ref(orc, P64, Q64, k, h, nbr=None, **kw):
    """Oracle outputs, statuses and eigenvalues (ascending, NaN where no
    plane was fitted) for the queries."""
    res = orc.project(P64, Q64, k, h, nbr=nbr, diag=True, **kw)
    out, st, dg = res[0], res[1], res[2]
    return (out, st, dg[:, 3:6]) + tuple(res[3:])


def relative_gap(lam):
    with np.errstate(invalid="ignore", divide="ignore"):
        return (lam[:, 1] - lam[:, 0]) / lam[:, 2]


def check_status(st, ref_st, ref_lam):
    """Asserts the status rule above; returns the oracle's flagged fraction."""
    st = np.asarray(st).astype(np.uint8)
    ref_st = np.asarray(ref_st).astype(np.uint8)
    np.testing.assert_array_equal(st & 0x0F, ref_st & 0x0F)
    np.testing.assert_array_equal(st & 0x20, ref_st & 0x20)
    differ = (st & 0x10) != (ref_st & 0x10)
    if differ.any():
        gap = relative_gap(np.asarray(ref_lam))
        near = (gap >= 0.5 * GAP) & (gap <= 2.0 * GAP)
        bad = differ & ~near
        assert not bad.any(), (
            "ambiguous-normal flag differs from the oracle's away from the threshold at "
            "%d queries (first %s, oracle gap %s)" % (bad.sum(), np.nonzero(bad)[0][:5],
                                                     gap[bad][:5]))
    return float(((ref_st & 0x10) != 0).mean()) if ref_st.size else 0.0


def position_errors(out, ref, ref_st, h, return_mask=False):
    """|out - ref| / h per checked query (see the module text)."""
    out = np.asarray(out)
    diff = np.abs(out.astype(np.float64) - ref)
    if out.dtype == np.float32:
        diff = np.maximum(diff - np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64), 0)
    ok = ((ref_st & 0x10) == 0) & ((ref_st & 0x0F) != 3)
    err = np.linalg.norm(diff, axis=1)[ok] / h
    return (err, ok) if return_mask else err


def fp32_max_bars(lam):
    """Per-point FP32 max bar (units of h) from the oracle's eigenvalues."""
    with np.errstate(invalid="ignore", divide="ignore"):
        gap = relative_gap(np.asarray(lam))
        bar = np.where(gap > 0, 10.0 * EPS32 / gap, np.inf)
    return np.clip(np.nan_to_num(bar, nan=FP32_MAX_H), FP32_MAX_H, FP32_MAX_CAP_H)


def check_errors(err, precision, rms_bar=FP32_RMS_H, max_bar=FP32_MAX_H):
    """``max_bar``: a number, or one bar per entry of err (FP32 path)."""
    if err.size == 0:
        return 0.0, 0.0
    mx = float(err.max())
    rms = float(np.sqrt((err ** 2).mean()))
    if precision == "fp64":
        assert mx <= FP64_MAX_H, mx
    else:
        assert rms <= rms_bar, rms
        over = err > max_bar
        assert not np.any(over), (mx, np.nonzero(over)[0][:5])
    return rms, mx


def check_projection(orc, P64, Q64, k, h, out, st, precision, nbr=None, surface=True,
                     label="", **kw):
    """Full parity of one projection call: statuses by the rule above,
    position bars, flagged fraction (surface clouds). Returns
    (rms, max, flagged fraction)."""
    ref, ref_st, lam = oracle_ref(orc, P64, Q64, k, h, nbr=nbr, **kw)[:3]
    frac = check_status(st, ref_st, lam)
    if surface:
        assert frac <= FLAG_FRACTION_SURFACE, frac
    err, ok = position_errors(out, ref, ref_st, h, return_mask=True)
    rms, mx = check_errors(err, precision, max_bar=fp32_max_bars(lam[ok]))
    print("%s %s: rms %.2e h, max %.2e h, flagged %.4f of %d" % (label, precision, rms, mx, frac,
                                                              len(ref_st)))
    return rms, mx, frac
