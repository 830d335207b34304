"""Plain FP64 CPU oracle of the MLS projection (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product library never imports,
links or executes anything here, and nothing here imports the product.

The arithmetic lives in ``mls_oracle.c`` (compiled with gcc,
``-ffp-contract=off``, no fast-math); this module only builds it and marshals
NumPy arrays. Every function follows the paper's MLS projection:

* ``knn``       -- brute-force k nearest neighbours on canonical FP64 keys,
                   ties to the smaller index (neighbourhood search of
                   Section 2 / Section 2.2, here with k neighbours).
* ``project``   -- reference plane (Section 1.4, Eq. (1.1) at t = 0, or
                   ``plane_iters`` frozen-weight steps that move the weights
                   to the plane's own projection q = r + t n, or Levin's
                   smallest-|t| local minimum over (n, t)), local frame, weighted
                   quadratic height fit and projection (Section 2.1,
                   Algorithm 1), outlier rule (Section 3.3).
* ``project_ball`` -- the same steps over the radius-R ball without a count
                   cap (brute force over the cloud, Section 1.4 / Section 3.3).
* ``grad_fd``   -- J^T g by central finite differences with lists fixed.

Parity pins for each function are in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mls_oracle.c")
# MLS_ORACLE_SANITIZE=1 builds and loads an AddressSanitizer +
# UndefinedBehaviorSanitizer build instead (the Python process must preload
# the sanitizer runtimes)
_SANITIZE = os.environ.get("MLS_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "libmls_oracle_san.so" if _SANITIZE else "libmls_oracle.so")

PT_OK, PT_OUTLIER, PT_PLANE_ONLY, PT_NONFINITE, PT_NO_MINIMUM = 0, 1, 2, 3, 4
PT_FLAG_AMBIGUOUS = 0x10
PT_FLAG_TRUNCATED = 0x20
DIAG_FIELDS = {
    "n": slice(0, 3), "lam": slice(3, 6), "q": slice(6, 9), "u": slice(9, 12),
    "v": slice(12, 15), "a": slice(15, 21), "support": 21, "S0": 22,
    "min_pivot": 23,
}

_lib = None


def build(force: bool = False) -> str:
    """Compile mls_oracle.c into libmls_oracle.so next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC, "-lm"]
        if _SANITIZE:
            cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                        "-fno-omit-frame-pointer", "-g"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.orc_knn.argtypes = [P, i64, P, i64, i32, P, P]
        lib.orc_knn.restype = ctypes.c_int
        lib.orc_project.argtypes = [P, i64, P, i64, i32, f64, P, f64, i32, i32, i32, i32, P, P, P,
                                    P]
        lib.orc_project.restype = ctypes.c_int
        lib.orc_project_ball.argtypes = [P, i64, P, i64, f64, f64, i32, i32, i32, P, P, P, P, P]
        lib.orc_project_ball.restype = ctypes.c_int
        lib.orc_grad_fd.argtypes = [P, i64, P, i64, i32, f64, P, f64, i32, P, f64, P, P]
        lib.orc_grad_fd.restype = ctypes.c_int
        lib.orc_diag_stride.restype = ctypes.c_int
        _lib = lib
    return _lib


def _c64(a, cols=3):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] != cols:
        raise ValueError("expected an (n, %d) array" % cols)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def knn(P, Q, k):
    """Brute-force kNN. Returns (idx int32 (m,k), key float64 (m,k))."""
    lib = _load()
    P, Q = _c64(P), _c64(Q)
    m = Q.shape[0]
    idx = np.empty((m, k), dtype=np.int32)
    key = np.empty((m, k), dtype=np.float64)
    rc = lib.orc_knn(_ptr(P), P.shape[0], _ptr(Q), m, int(k), _ptr(idx), _ptr(key))
    if rc:
        raise ValueError("orc_knn failed (%d)" % rc)
    return idx, key


def project(P, Q, k, h, nbr=None, support_radius_h=3.0, min_support=3, diag=False,
            plane_iters=0, ball=False, geometry=False, levin=False):
    """One MLS projection pass. Returns (out (m,3) float64, status uint8 (m,)
    [, diag (m, 24)]). ``nbr`` are original indices (m, k); computed by brute
    force when omitted. ``plane_iters``: steps of the reference plane with the
    weights at the plane's own projection of the query (0: weights at r).
    ``ball``: the neighbourhood is the list entries within support_radius_h
    * h (the paper's radius R); TRUNCATED flags a list wholly inside it.
    ``geometry``: also return (m, 5) = unit surface normal at the output
    (sign that of the plane normal), mean and Gaussian curvature (after
    ``diag`` when both are asked). ``levin``: the reference plane is the
    local minimum of Eq. (1.1) over (n, t) with the smallest |t| (O5c);
    status NO_MINIMUM (4) where none lies within support_radius_h * h."""
    lib = _load()
    P, Q = _c64(P), _c64(Q)
    m = Q.shape[0]
    if nbr is None:
        nbr, _ = knn(P, Q, k)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    if nbr.shape != (m, k):
        raise ValueError("nbr must be (m, k)")
    out = np.empty((m, 3), dtype=np.float64)
    st = np.empty(m, dtype=np.uint8)
    dg = np.empty((m, lib.orc_diag_stride()), dtype=np.float64) if diag else None
    geo = np.empty((m, 5), dtype=np.float64) if geometry else None
    rc = lib.orc_project(_ptr(P), P.shape[0], _ptr(Q), m, int(k), float(h), _ptr(nbr),
                         float(support_radius_h), int(min_support), int(plane_iters),
                         int(bool(ball)), int(bool(levin)), _ptr(out), _ptr(st), _ptr(dg),
                         _ptr(geo))
    if rc:
        raise ValueError("orc_project failed (%d)" % rc)
    res = (out, st) + ((dg,) if diag else ()) + ((geo,) if geometry else ())
    return res


def project_ball(P, Q, h, support_radius_h=3.0, min_support=3, diag=False, geometry=False,
                 plane_iters=0, levin=False):
    """One projection pass over the paper's radius-R neighbourhood without a
    count cap (O3c): every cloud point within R = support_radius_h * h of the
    query (canonical keys, brute force). Returns (out, status, counts
    [, diag] [, geometry])."""
    lib = _load()
    P, Q = _c64(P), _c64(Q)
    m = Q.shape[0]
    out = np.empty((m, 3), dtype=np.float64)
    st = np.empty(m, dtype=np.uint8)
    cnt = np.empty(m, dtype=np.int64)
    dg = np.empty((m, lib.orc_diag_stride()), dtype=np.float64) if diag else None
    geo = np.empty((m, 5), dtype=np.float64) if geometry else None
    rc = lib.orc_project_ball(_ptr(P), P.shape[0], _ptr(Q), m, float(h), float(support_radius_h),
                              int(min_support), int(plane_iters), int(bool(levin)), _ptr(out),
                              _ptr(st), _ptr(dg), _ptr(geo), _ptr(cnt))
    if rc:
        raise ValueError("orc_project_ball failed (%d)" % rc)
    return (out, st, cnt) + ((dg,) if diag else ()) + ((geo,) if geometry else ())


def grad_fd(P, Q, k, h, nbr, gout, rel_step=1e-6, support_radius_h=3.0, min_support=3):
    """J^T gout by central differences with lists fixed.
    Returns (gq (m,3), gp (n,3))."""
    lib = _load()
    P, Q, gout = _c64(P), _c64(Q), _c64(gout)
    m = Q.shape[0]
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    gq = np.empty((m, 3), dtype=np.float64)
    gp = np.empty_like(P)
    rc = lib.orc_grad_fd(_ptr(P), P.shape[0], _ptr(Q), m, int(k), float(h), _ptr(nbr),
                         float(support_radius_h), int(min_support), _ptr(gout),
                         float(rel_step), _ptr(gq), _ptr(gp))
    if rc:
        raise ValueError("orc_grad_fd failed (%d)" % rc)
    return gq, gp


def project_passes(P, Q, k, h, passes, support_radius_h=3.0, min_support=3, plane_iters=0,
                   levin=False):
    """Iterated passes (queries move, cloud fixed): pass t+1 projects the
    outputs of pass t; a query that was an OUTLIER stays where it is."""
    cur = _c64(Q).copy()
    frozen = np.zeros(cur.shape[0], dtype=bool)
    st = None
    for _ in range(passes):
        out, st_new = project(P, cur, k, h, support_radius_h=support_radius_h,
                              min_support=min_support, plane_iters=plane_iters, levin=levin)
        out[frozen] = cur[frozen]
        st_new = np.where(frozen, np.uint8(PT_OUTLIER), st_new)
        frozen |= (st_new & 0x0F) == PT_OUTLIER
        cur, st = out, st_new
    return cur, st
