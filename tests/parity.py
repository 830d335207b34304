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
  FP32-moment path   RMS <= 1e-5 h and max <= 1e-4 h.
Outputs stored in FP32 are allowed their storage rounding (an FP32 ulp per
coordinate) on top.

Flagged fraction: on clouds sampled from a smooth surface at most 1 % of the
queries may carry the ambiguous flag (the flag removes a point from the max
bars, so a spurious flag would silently shrink the checked set)."""
import numpy as np

FP64_MAX_H = 1e-10
FP32_RMS_H = 1e-5
FP32_MAX_H = 1e-4
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


def position_errors(out, ref, ref_st, h):
    """|out - ref| / h per checked query (see the module text)."""
    out = np.asarray(out)
    diff = np.abs(out.astype(np.float64) - ref)
    if out.dtype == np.float32:
        diff = np.maximum(diff - np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64), 0)
    ok = ((ref_st & 0x10) == 0) & ((ref_st & 0x0F) != 3)
    return np.linalg.norm(diff, axis=1)[ok] / h


def check_errors(err, precision, rms_bar=FP32_RMS_H, max_bar=FP32_MAX_H):
    if err.size == 0:
        return 0.0, 0.0
    mx = float(err.max())
    rms = float(np.sqrt((err ** 2).mean()))
    if precision == "fp64":
        assert mx <= FP64_MAX_H, mx
    else:
        assert rms <= rms_bar, rms
        assert mx <= max_bar, mx
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
    err = position_errors(out, ref, ref_st, h)
    rms, mx = check_errors(err, precision)
    print("%s %s: rms %.2e h, max %.2e h, flagged %.4f of %d" % (label, precision, rms, mx, frac,
                                                              len(ref_st)))
    return rms, mx, frac
