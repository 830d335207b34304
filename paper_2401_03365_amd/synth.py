"""Seeded synthetic point clouds shaped like the paper's workloads.

This module only draws inputs; it holds none of the MLS arithmetic, so both
the HIP path and the CPU oracle are fed from it. Every cloud is generated in
FP64 with ``numpy.random.default_rng(seed)`` (PCG64) and rounded once to
FP32; that FP32 array is what every consumer sees. The Gaussian width ``h``
is computed here once per cloud from the FP32 values (twice the mean
distance to the nearest other point, duplicates counting as distance 0) and
handed to both sides as a double.

The paper's own inputs (normalised meshes sampled at 200,000 points with
additive Gaussian noise, Section 3.2, and a 25M-point scan, Section 3.3) are
not available; these recipes stand in for them.
"""
from __future__ import annotations

import math

import numpy as np


def _f32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))


def mean_nn_h(P32, factor=2.0, workers=-1):
    """h = factor * mean distance to the nearest other point (exact, k-d tree)."""
    from scipy.spatial import cKDTree

    P = np.asarray(P32, dtype=np.float64)
    if P.shape[0] < 2:
        raise ValueError("need at least two points")
    tree = cKDTree(P)
    d, _ = tree.query(P, k=2, workers=workers)
    return float(factor * d[:, 1].mean())


def sphere(n, sigma=0.01, seed=1):
    """Unit sphere, noise sigma along the normal: p = (1 + sigma z) n_hat."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    nh = g / np.linalg.norm(g, axis=1, keepdims=True)
    z = rng.standard_normal(n)
    return _f32((1.0 + sigma * z)[:, None] * nh)


def cube(n, sigma=0.01, seed=1, half=0.5):
    """Surface of the cube [-half, half]^3 (a shape with sharp edges and
    corners), area-uniform (each of the 6 faces equally likely), noise sigma
    along the face normal."""
    rng = np.random.default_rng(seed)
    face = rng.integers(0, 6, n)
    axis, side = face // 2, np.where(face % 2 == 0, -1.0, 1.0)
    P = rng.uniform(-half, half, (n, 3))
    P[np.arange(n), axis] = side * (half + sigma * rng.standard_normal(n))
    return _f32(P)


def cube_distance(Y, half=0.5):
    """Distance from each row of Y to the surface of the cube [-half, half]^3."""
    q = np.abs(np.asarray(Y, dtype=np.float64)) - half
    outside = np.linalg.norm(np.maximum(q, 0.0), axis=1)
    inside = np.minimum(q.max(axis=1), 0.0)
    return outside + np.abs(inside)


def sphere_cap(n, cap_angle, seed=0, radius=1.0):
    """Noise-free samples of a spherical cap around +z (area-uniform)."""
    rng = np.random.default_rng(seed)
    cz = rng.uniform(math.cos(cap_angle), 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return _f32(radius * np.stack([s * np.cos(phi), s * np.sin(phi), cz], axis=1))


def torus(n, R=1.0, r=0.3, sigma=0.005, n_outliers=0, seed=2, return_mask=False):
    """Area-uniform torus samples with normal noise, followed by n_outliers
    uniform points in [-1.3,1.3]^2 x [-0.3,0.3]."""
    rng = np.random.default_rng(seed)
    us, vs = [], []
    need = n
    while need > 0:
        m = int(need * 1.6) + 64
        u = rng.uniform(0.0, 2.0 * math.pi, m)
        v = rng.uniform(0.0, 2.0 * math.pi, m)
        acc = rng.uniform(0.0, 1.0, m) < (R + r * np.cos(v)) / (R + r)
        us.append(u[acc][:need])
        vs.append(v[acc][:need])
        need -= us[-1].shape[0]
    u = np.concatenate(us)
    v = np.concatenate(vs)
    nrm = np.stack([np.cos(v) * np.cos(u), np.cos(v) * np.sin(u), np.sin(v)], axis=1)
    ring = (R + r * np.cos(v))
    p = np.stack([ring * np.cos(u), ring * np.sin(u), r * np.sin(v)], axis=1)
    p = p + (sigma * rng.standard_normal(n))[:, None] * nrm
    if n_outliers:
        o = np.stack([rng.uniform(-1.3, 1.3, n_outliers), rng.uniform(-1.3, 1.3, n_outliers),
                      rng.uniform(-0.3, 0.3, n_outliers)], axis=1)
        p = np.concatenate([p, o], axis=0)
    mask = np.zeros(p.shape[0], dtype=bool)
    mask[n:] = True
    return (_f32(p), mask) if return_mask else _f32(p)


class HeightField:
    """z(x, y) = sum_m amp * sin(2 pi m (cos a_m x + sin a_m y) + phi_m),
    m = 1..n_waves, a_m and phi_m uniform in [0, 2 pi)."""

    def __init__(self, seed, n_waves=8, amp=0.05):
        rng = np.random.default_rng(seed)
        self.freq = np.arange(1, n_waves + 1, dtype=np.float64)
        self.alpha = rng.uniform(0.0, 2.0 * math.pi, n_waves)
        self.phase = rng.uniform(0.0, 2.0 * math.pi, n_waves)
        self.amp = amp

    def _arg(self, x, y, m):
        return 2.0 * math.pi * self.freq[m] * (math.cos(self.alpha[m]) * x +
                                               math.sin(self.alpha[m]) * y) + self.phase[m]

    def z(self, x, y):
        out = np.zeros_like(x)
        for m in range(self.freq.shape[0]):
            out += self.amp * np.sin(self._arg(x, y, m))
        return out

    def grad(self, x, y):
        gx = np.zeros_like(x)
        gy = np.zeros_like(x)
        for m in range(self.freq.shape[0]):
            c = self.amp * np.cos(self._arg(x, y, m)) * 2.0 * math.pi * self.freq[m]
            gx += c * math.cos(self.alpha[m])
            gy += c * math.sin(self.alpha[m])
        return gx, gy


def heightfield(n, sigma=1e-3, seed=3, ramp=10.0, return_field=False, chunk=2_000_000):
    """Height field over [0,1]^2 with x-density proportional to 1 + (ramp-1) x
    (a ramp-fold density change across the domain) and noise sigma along the
    analytic unit normal."""
    rng = np.random.default_rng(seed)
    field = HeightField(seed + 1000)
    out = np.empty((n, 3), dtype=np.float32)
    a = ramp - 1.0
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        y = rng.uniform(0.0, 1.0, m)
        U = rng.uniform(0.0, 1.0, m)
        # inverse CDF of density (1 + a x) / (1 + a/2) on [0, 1]
        x = (-1.0 + np.sqrt(1.0 + a * (2.0 + a) * U)) / a
        z = field.z(x, y)
        gx, gy = field.grad(x, y)
        nn = np.sqrt(gx * gx + gy * gy + 1.0)
        e = sigma * rng.standard_normal(m) / nn
        out[s:s + m, 0] = x - e * gx
        out[s:s + m, 1] = y - e * gy
        out[s:s + m, 2] = z + e
    return (out, field) if return_field else out


def _real_sh_matrix(lmax, theta, phi):
    """Real spherical harmonics of degree 1..lmax at polar angle theta and
    azimuth phi, one column per (l, m)."""
    from scipy.special import sph_harm_y

    cols = []
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            if m < 0:
                cols.append(math.sqrt(2.0) * (-1) ** m * Y.imag)
            elif m == 0:
                cols.append(Y.real)
            else:
                cols.append(math.sqrt(2.0) * (-1) ** m * Y.real)
    return np.stack(cols, axis=1)


class SHBumps:
    """Random real spherical-harmonic bump field of degree 1..lmax scaled so
    that max |bump| over a 100k-point Fibonacci sphere equals max_amp."""

    def __init__(self, seed, lmax=8, max_amp=0.02, n_fib=100_000):
        rng = np.random.default_rng(seed)
        self.lmax = lmax
        self.coef = rng.standard_normal((lmax + 1) ** 2 - 1)
        i = np.arange(n_fib) + 0.5
        th = np.arccos(1.0 - 2.0 * i / n_fib)
        ph = (math.pi * (1.0 + math.sqrt(5.0)) * i) % (2.0 * math.pi)
        b = _real_sh_matrix(lmax, th, ph) @ self.coef
        self.coef *= max_amp / np.abs(b).max()

    def bump(self, w):
        w = np.asarray(w, dtype=np.float64)
        th = np.arccos(np.clip(w[:, 2], -1.0, 1.0))
        ph = np.arctan2(w[:, 1], w[:, 0]) % (2.0 * math.pi)
        return _real_sh_matrix(self.lmax, th, ph) @ self.coef


def sh_sphere(n, sigma=0.005, seed=4, return_field=False, chunk=500_000):
    """p = (1 + bump(w) + sigma z) w, w uniform on the unit sphere."""
    rng = np.random.default_rng(seed)
    field = SHBumps(seed + 1000)
    out = np.empty((n, 3), dtype=np.float32)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        g = rng.standard_normal((m, 3))
        w = g / np.linalg.norm(g, axis=1, keepdims=True)
        z = rng.standard_normal(m)
        rad = 1.0 + field.bump(w) + sigma * z
        out[s:s + m] = (rad[:, None] * w).astype(np.float32)
    return (out, field) if return_field else out


def plane_patch(n, normal, seed=0, extent=1.0, jitter=True):
    """Points exactly on the plane through the origin with the given normal
    (exact up to the single FP32 rounding)."""
    rng = np.random.default_rng(seed)
    nrm = np.asarray(normal, dtype=np.float64)
    nrm = nrm / np.linalg.norm(nrm)
    a = np.eye(3)[np.argmin(np.abs(nrm))]
    u = np.cross(a, nrm)
    u /= np.linalg.norm(u)
    v = np.cross(nrm, u)
    s = rng.uniform(-extent, extent, (n, 2))
    return _f32(s[:, :1] * u + s[:, 1:] * v)


def lattice(nx, ny, nz=1, spacing=1.0, origin=(0.0, 0.0, 0.0)):
    """Regular lattice: many exactly equal distances (tie-breaking cases)."""
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    return _f32(g.reshape(-1, 3) * spacing + np.asarray(origin))


def batch(total=30_000_000, n_clouds=256, seed=5, lo=5_000, hi=500_000):
    """Sizes log-normal (sigma 1) clipped to [lo, hi] with the mean solved so the
    sum is close to ``total``; shapes cycle sphere / torus / height field;
    noise log-uniform in [1e-3, 1e-2]. Returns (points float32, offsets int64,
    sigmas, shapes)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(n_clouds)

    def sizes_for(mu):
        return np.clip(np.round(np.exp(mu + z)), lo, hi).astype(np.int64)

    a, b = 0.0, 20.0
    for _ in range(100):
        mid = 0.5 * (a + b)
        if sizes_for(mid).sum() < total:
            a = mid
        else:
            b = mid
    sizes = sizes_for(0.5 * (a + b))
    sig = np.exp(rng.uniform(math.log(1e-3), math.log(1e-2), n_clouds))
    parts, shapes = [], []
    for c in range(n_clouds):
        s = 5000 + c
        kind = c % 3
        if kind == 0:
            parts.append(sphere(int(sizes[c]), float(sig[c]), s))
            shapes.append("sphere")
        elif kind == 1:
            parts.append(torus(int(sizes[c]), sigma=float(sig[c]), seed=s))
            shapes.append("torus")
        else:
            parts.append(heightfield(int(sizes[c]), sigma=float(sig[c]), seed=s))
            shapes.append("heightfield")
    offsets = np.zeros(n_clouds + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    return np.concatenate(parts, axis=0), offsets, sig, shapes
