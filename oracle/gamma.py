"""Gamma-index oracle (test infrastructure only; FP64 numpy, brute force).

Only the test-suite may import this module; it shares nothing with the GPU
library.

The agreement test of Sec. 3.1 (after Low et al. 1998): for every reference
voxel r with D_ref(r) > region_min,

    gamma(r) = min over r' of sqrt((D_ref(r) - D_eval(r'))^2 / dD^2
                                   + |r - r'|^2 / dr^2),

and r passes when gamma(r) < 1.  The paper leaves the set of r' open; the
reading taken here: r' runs over the lattice r + h (i, j, k), h = dr/substeps,
within |r' - r| <= cap * dr, and D_eval(r') is the trilinear interpolant of
D_eval between voxel centres, clamped to the outermost centres.  Minima above
cap^2 are reported as cap.  Every lattice point is visited (no ordering or
early exit).
"""
from __future__ import annotations

import math

import numpy as np


def lattice(dta_cm: float, gamma_cap: float, substeps: int):
    """Integer lattice offsets (i, j, k) with i^2 + j^2 + k^2 <= (cap s)^2."""
    rmax = gamma_cap * substeps
    L = int(math.ceil(rmax))
    r = np.arange(-L, L + 1)
    K, J, I = np.meshgrid(r, r, r, indexing="ij")
    keep = (I * I + J * J + K * K) <= rmax * rmax
    return np.stack([I[keep], J[keep], K[keep]], 1)


def _axis(u, n):
    u = np.clip(u, 0.0, n - 1.0)
    i0 = np.minimum(np.floor(u).astype(np.int64), max(n - 2, 0))
    f = u - i0
    i1 = np.minimum(i0 + 1, n - 1)
    return i0, i1, f


def trilinear(D, x, y, z):
    """D[nz][ny][nx] interpolated at voxel-centre coordinates (x, y, z)."""
    nz, ny, nx = D.shape
    x0, x1, fx = _axis(x, nx)
    y0, y1, fy = _axis(y, ny)
    z0, z1, fz = _axis(z, nz)

    def lerp(a, b, f):
        return a + f * (b - a)

    c00 = lerp(D[z0, y0, x0], D[z0, y0, x1], fx)
    c01 = lerp(D[z0, y1, x0], D[z0, y1, x1], fx)
    c10 = lerp(D[z1, y0, x0], D[z1, y0, x1], fx)
    c11 = lerp(D[z1, y1, x0], D[z1, y1, x1], fx)
    return lerp(lerp(c00, c01, fy), lerp(c10, c11, fy), fz)


def gamma_index(ref, ev, spacing, dose_tol: float, dta_cm: float, region_min: float,
                gamma_cap: float = 2.0, substeps: int = 5):
    """(gamma [nz][ny][nx] with -1 outside the region, n_region, n_pass).
    ref, ev: [nz][ny][nx]; spacing = (dx, dy, dz) in cm."""
    R = np.asarray(ref, dtype=np.float32).astype(np.float64)
    E = np.asarray(ev, dtype=np.float32).astype(np.float64)
    dx, dy, dz = spacing
    iz, iy, ix = np.nonzero(R > region_min)
    dr = R[iz, iy, ix]
    h = dta_cm / substeps
    best = np.full(dr.shape, gamma_cap * gamma_cap)
    for i, j, k in lattice(dta_cm, gamma_cap, substeps):
        dist2 = ((i * h) ** 2 + (j * h) ** 2 + (k * h) ** 2) / (dta_cm * dta_cm)
        de = trilinear(E, ix + i * h / dx, iy + j * h / dy, iz + k * h / dz)
        best = np.minimum(best, dist2 + (dr - de) ** 2 / (dose_tol * dose_tol))
    out = np.full(R.shape, -1.0)
    out[iz, iy, ix] = np.sqrt(best)
    return out, int(dr.size), int(np.count_nonzero(best < 1.0))
