"""Marshalling helpers: hand a workload description to the C ABI.

A workload is any object with the attributes used below (grid dict, mat and
rho arrays, material names, mu_rho(), compton_pdf(), rayleigh_pdf(m),
spectrum_lo/width/w, geometry dict, seed, n_batches, e_cut, rayleigh, e0, de,
ne, n_zeta).  Inverse-CDF surfaces are built by the library's own FP64
routine (ctd_surface_build); nothing here computes a step of the transport.
"""
from __future__ import annotations

import numpy as np

from . import ctd as L

_surface_cache: dict = {}


def _grid(g: dict) -> L.ctd_grid:
    out = L.ctd_grid()
    out.nx, out.ny, out.nz = g["nx"], g["ny"], g["nz"]
    out.dx, out.dy, out.dz = g["dx"], g["dy"], g["dz"]
    out.origin[:] = (g["ox"], g["oy"], g["oz"])
    return out


def _geom(geo: dict) -> L.ctd_geom:
    """ctd_geom for a geometry dict; a fluence map [nb][na] (key "fluence")
    is referenced by pointer, so the dict must outlive ctd_geometry_set."""
    g = L.ctd_geom()
    if geo["kind"] == "pencil":
        g.kind = L.CTD_GEOM_PENCIL
        g.src[:] = geo["src"]
        g.dir[:] = geo["dir"]
    else:
        g.kind = L.CTD_GEOM_CONE
        g.n_proj = geo["nproj"]
        g.sad = geo["sad"]
        g.iso[:] = geo["iso"]
        g.a0, g.a1, g.b0, g.b1 = geo["a0"], geo["a1"], geo["b0"], geo["b1"]
        g.phi0_deg, g.arc_deg = geo["phi0_deg"], geo["arc_deg"]
        g.z_feed = geo.get("feed", 0.0)
        f = geo.get("fluence")
        if f is not None:
            f = np.ascontiguousarray(f, dtype=np.float32)
            g.fluence_nb, g.fluence_na = f.shape
            g.fluence = f.ctypes.data
            g.fluence_chains = int(geo.get("fluence_chains", 0))
            g._keep = f
    return g


def surfaces(wl):
    """(Compton surface [ne][nz], Rayleigh surfaces [M][ne][nz] or None),
    cached by material and grid."""
    if getattr(wl, "compton_per_material", False):
        rows = []
        for m, name in enumerate(wl.materials):
            key = ("compton-wh", name, wl.e0, wl.de, wl.ne, wl.n_mu_c, wl.n_zeta)
            if key not in _surface_cache:
                _surface_cache[key] = L.ctd_surface_build(wl.compton_pdf(m), wl.n_zeta)
            rows.append(_surface_cache[key])
        comp = np.stack(rows)
    else:
        key_c = ("compton", wl.e0, wl.de, wl.ne, wl.n_mu_c, wl.n_zeta)
        if key_c not in _surface_cache:
            _surface_cache[key_c] = L.ctd_surface_build(wl.compton_pdf(), wl.n_zeta)
        comp = _surface_cache[key_c]
    rayl = None
    if wl.rayleigh:
        rows = []
        for m, name in enumerate(wl.materials):
            key = ("rayleigh", name, wl.e0, wl.de, wl.ne, wl.n_mu_r, wl.n_zeta)
            if key not in _surface_cache:
                _surface_cache[key] = L.ctd_surface_build(wl.rayleigh_pdf(m), wl.n_zeta)
            rows.append(_surface_cache[key])
        rayl = np.stack(rows)
    return comp, rayl


class Inputs:
    """Material set, spectrum and geometry of a workload bound in a context
    (without a phantom or case), e.g. for server requests."""

    def __init__(self, ctx, wl, mu_rho=None):
        self.ctx = ctx
        self.ms = self.sp = self.geo = None
        try:
            eg = L.ctd_egrid()
            eg.e0, eg.de, eg.ne = wl.e0, wl.de, wl.ne
            comp, rayl = surfaces(wl)
            self.ms = L.ctd_materials_load(ctx, eg, wl.mu_rho() if mu_rho is None else mu_rho,
                                           comp, int(comp.ndim == 3), rayl)
            self.sp = L.ctd_spectrum_set(ctx, wl.spectrum_lo, wl.spectrum_width, wl.spectrum_w)
            self.geo = L.ctd_geometry_set(ctx, _geom(wl.geometry))
        except BaseException:
            self.close()
            raise

    def close(self):
        for release, name in [(L.ctd_geometry_release, "geo"), (L.ctd_spectrum_release, "sp"),
                              (L.ctd_materials_release, "ms")]:
            h = getattr(self, name)
            if h is not None:
                release(self.ctx, h)
                setattr(self, name, None)


def params(wl, seed=None, n_batches=None, rho_min=0.05, tracking=None,
           macro_cell=0) -> L.ctd_params:
    """ctd_params of a workload; tracking defaults to the workload's own
    (attribute ``tracking``, else the paper's global majorant)."""
    p = L.ctd_params()
    p.e_cut_kev = wl.e_cut
    p.seed = wl.seed if seed is None else seed
    p.n_batches = wl.n_batches if n_batches is None else n_batches
    p.rayleigh = int(wl.rayleigh)
    p.sigma_rho_min = rho_min
    p.tracking = getattr(wl, "tracking", L.CTD_TRACK_GLOBAL) if tracking is None else tracking
    p.macro_cell = getattr(wl, "macro_cell", 0) if not macro_cell else macro_cell
    return p


def grid(wl) -> L.ctd_grid:
    return _grid(wl.grid)


class Case:
    """One dose problem bound in the library (phantom, tables, spectrum,
    geometry, case).  ``close()`` releases everything."""

    def __init__(self, ctx, wl, mu_rho=None, seed=None, n_batches=None, rho_min=0.05,
                 mat=None, rho=None, mem=L.CTD_MEM_HOST, tracking=None, macro_cell=0):
        self.ctx = ctx
        self.wl = wl
        self.V = int(wl.grid["nx"] * wl.grid["ny"] * wl.grid["nz"])
        # device arrays (CTD_MEM_DEVICE: torch tensors or raw pointers) pass as they are
        m = wl.mat if mat is None else mat
        r = wl.rho if rho is None else rho
        if mem == L.CTD_MEM_HOST:
            m = np.ascontiguousarray(m, dtype=np.uint8)
            r = np.ascontiguousarray(r, dtype=np.float32)
        self.cs = self.ph = self.ms = self.sp = self.geo = None
        try:
            self.ph = L.ctd_phantom_load(ctx, _grid(wl.grid), m, r, mem)
            eg = L.ctd_egrid()
            eg.e0, eg.de, eg.ne = wl.e0, wl.de, wl.ne
            comp, rayl = surfaces(wl)
            mu = wl.mu_rho() if mu_rho is None else mu_rho
            self.ms = L.ctd_materials_load(ctx, eg, mu, comp, int(comp.ndim == 3), rayl)
            self.sp = L.ctd_spectrum_set(ctx, wl.spectrum_lo, wl.spectrum_width, wl.spectrum_w)
            self.geo = L.ctd_geometry_set(ctx, _geom(wl.geometry))
            p = params(wl, seed, n_batches, rho_min, tracking, macro_cell)
            self.params = p
            self.cs = L.ctd_case_create(ctx, self.ph, self.ms, self.sp, self.geo, p)
        except BaseException:
            self._release_inputs()   # what was created before the failing call
            raise

    # convenience pass-throughs
    def run(self, n):
        L.ctd_run(self.ctx, self.cs, n)

    def tally(self):
        return L.ctd_read_tally(self.ctx, self.cs, self.V)

    def dose(self):
        return L.ctd_read_dose(self.ctx, self.cs, self.V)

    def balance(self):
        return L.ctd_read_balance(self.ctx, self.cs)

    def stats(self):
        return L.ctd_read_stats(self.ctx, self.cs)

    def _release_inputs(self):
        for release, name in [(L.ctd_geometry_release, "geo"), (L.ctd_spectrum_release, "sp"),
                              (L.ctd_materials_release, "ms"), (L.ctd_phantom_release, "ph")]:
            h = getattr(self, name)
            if h is not None:
                release(self.ctx, h)
                setattr(self, name, None)

    def close(self):
        if self.cs is not None:
            L.ctd_case_destroy(self.ctx, self.cs)
            self.cs = None
            self._release_inputs()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
