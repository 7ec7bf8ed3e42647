"""Dose report tools on the host: line profiles (depth-dose along the beam,
lateral profiles at a depth, as in Fig. 6) and the gamma pass rate of Sec.
3.1 through the library's gamma kernel.  Numpy only; no transport here."""
from __future__ import annotations

import numpy as np

from . import ctd as L


def _centres(grid: dict):
    return (np.asarray([grid["ox"], grid["oy"], grid["oz"]], dtype=np.float64),
            np.asarray([grid["dx"], grid["dy"], grid["dz"]], dtype=np.float64),
            np.asarray([grid["nx"], grid["ny"], grid["nz"]]))


def sample(values: np.ndarray, grid: dict, points: np.ndarray) -> np.ndarray:
    """Trilinear interpolation of a [nz][ny][nx] array between voxel centres
    at points [..., 3] (cm), clamped to the outermost centres."""
    o, d, n = _centres(grid)
    v = np.asarray(values, dtype=np.float64).reshape(n[2], n[1], n[0])
    u = (np.asarray(points, dtype=np.float64) - o) / d - 0.5
    idx, w = [], []
    for a in range(3):
        ua = np.clip(u[..., a], 0.0, n[a] - 1.0)
        i0 = np.minimum(np.floor(ua).astype(np.int64), max(int(n[a]) - 2, 0))
        idx.append((i0, np.minimum(i0 + 1, n[a] - 1)))
        w.append(ua - i0)
    out = 0.0
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                wt = ((w[2] if cz else 1 - w[2]) * (w[1] if cy else 1 - w[1]) *
                      (w[0] if cx else 1 - w[0]))
                out = out + wt * v[idx[2][cz], idx[1][cy], idx[0][cx]]
    return out


def line_profile(values, grid: dict, start, direction, length: float, step: float | None = None):
    """(t [cm], values) along start + t * direction, t in [0, length]."""
    dvec = np.asarray(direction, dtype=np.float64)
    dvec = dvec / np.linalg.norm(dvec)
    if step is None:
        step = float(min(grid["dx"], grid["dy"], grid["dz"]))
    t = np.arange(0.0, length + 0.5 * step, step)
    pts = np.asarray(start, dtype=np.float64)[None, :] + t[:, None] * dvec[None, :]
    return t, sample(values, grid, pts)


def beam_frame(geometry: dict):
    """Source point, beam axis (unit, towards the isocentre) and the two
    field directions (e_lat, e_z) of a cone source at its first angle."""
    phi = np.radians(geometry["phi0_deg"])
    iso = np.asarray(geometry["iso"], dtype=np.float64)
    src = iso + geometry["sad"] * np.array([np.sin(phi), np.cos(phi), 0.0])
    axis = (iso - src) / np.linalg.norm(iso - src)
    return src, axis, np.array([np.cos(phi), -np.sin(phi), 0.0]), np.array([0.0, 0.0, 1.0])


def entry_depth_point(grid: dict, src, axis):
    """Where the beam axis enters the voxel box (slab method)."""
    o, d, n = _centres(grid)
    lo, hi = o, o + d * n
    with np.errstate(divide="ignore", invalid="ignore"):
        t1, t2 = (lo - src) / axis, (hi - src) / axis
    tn = np.nanmax(np.where(np.isfinite(t1), np.minimum(t1, t2), -np.inf))
    return src + tn * axis


def fig6_profiles(dose, sigma, grid: dict, geometry: dict, depth_cm: float = 3.0):
    """Depth dose along the central axis and lateral profiles along the two
    field directions at depth_cm below the entrance surface, all normalised to
    the maximum dose, with 2-sigma bands (the presentation of Fig. 6)."""
    src, axis, e_a, e_b = beam_frame(geometry)
    entry = entry_depth_point(grid, src, axis)
    dmax = float(np.max(dose))
    o, d, n = _centres(grid)
    extent = float(np.linalg.norm(d * n))
    step = float(min(d))
    out = {}
    t, v = line_profile(dose, grid, entry + 0.5 * step * axis, axis, extent, step)
    _, s = line_profile(sigma, grid, entry + 0.5 * step * axis, axis, extent, step)
    out["depth"] = (t + 0.5 * step, v / dmax, 2 * s / dmax)
    centre = entry + depth_cm * axis
    K = int(0.5 * extent / step)
    for name, e in (("lateral_a", e_a), ("lateral_b", e_b)):
        t = step * np.arange(-K, K + 1)          # symmetric about the beam axis
        pts = centre[None, :] + t[:, None] * e[None, :]
        out[name] = (t, sample(dose, grid, pts) / dmax, 2 * sample(sigma, grid, pts) / dmax)
    return out


def gamma_pass_rate(ctx, grid: dict, ref, ev, dose_frac: float = 0.02, dta_cm: float = 0.2,
                    region_frac: float = 0.2, **kw):
    """P_gamma of ev against ref with dD = dose_frac * max(ref), dr = dta_cm,
    over voxels with ref > region_frac * max(ref) (Sec. 3.1)."""
    g = L.ctd_grid()
    g.nx, g.ny, g.nz = grid["nx"], grid["ny"], grid["nz"]
    g.dx, g.dy, g.dz = grid["dx"], grid["dy"], grid["dz"]
    dmax = float(np.max(ref))
    _, nr, npass = L.ctd_gamma(ctx, g, ref, ev, dose_frac * dmax, dta_cm, region_frac * dmax,
                               want_gamma=False, **kw)
    return npass / nr if nr else float("nan"), nr
