"""Seeded synthetic workloads: voxel phantoms, material lists, interaction
tables, spectra, scan geometries and run parameters.

Every generator here is a pure function of its seed.  The oracle and the GPU
library both consume these inputs; nothing here performs a step of the
transport method.  The shapes, sizes and structures follow the paper's two
studies (a water phantom at a few-mm voxel size under a cone beam at 100 cm
source distance, Sec. 3.1; a heterogeneous head phantom with air, tissue and
bone, Sec. 3.2), at the scales of the five benchmark workloads:

* ``tiny``      32^3 water, 0.5 cm voxels, 60 keV pencil beam, 1e5 histories.
* ``water_cbct`` 128x128x100 water cylinder (r 15 cm, 20 cm long) in air,
  0.25x0.25x0.2 cm voxels; full-fan 26x20 cm cone beam at SAD 100 cm,
  360 projections over 360 deg; 120 kVp Kramers + 2 mm Al; Rayleigh on.
* ``head``      256x256x160 at 0.1 cm, nested ellipsoids (tissue, bone shell,
  brain, air sinuses, lung-like insert), +-2 % Gaussian density noise;
  half-fan 100 kVp, 200 projections.
* ``batched``   48 cases of uneven size drawn from seed 4004.
* ``serving``   Poisson arrival trace (2 req/s, seed 5005) over the batched
  distribution.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import physics as ph

E0_KEV = 1.0
DE_KEV = 1.0
N_E = 150
N_ZETA = 256
N_MU_COMPTON = 2049
N_MU_RAYLEIGH = 65537   # the forward peak at 150 keV is ~1/c = 0.005 wide in mu


def e_nodes(e0=E0_KEV, de=DE_KEV, ne=N_E) -> np.ndarray:
    return e0 + de * np.arange(ne, dtype=np.float64)


@dataclass
class Workload:
    name: str
    # grid: nx, ny, nz [voxels]; dx, dy, dz [cm]; ox, oy, oz corner [cm]
    grid: dict
    mat: np.ndarray            # uint8 [nz][ny][nx]
    rho: np.ndarray            # float32 [nz][ny][nx]  g/cm^3
    materials: list
    rayleigh: bool
    spectrum_lo: np.ndarray    # float64 [nbins] keV
    spectrum_width: float      # keV (0 = monoenergetic)
    spectrum_w: np.ndarray     # float64 [nbins] relative weights
    geometry: dict
    seed: int
    n_histories: int
    n_batches: int = 10
    e_cut: float = 1.0
    e0: float = E0_KEV
    de: float = DE_KEV
    ne: int = N_E
    n_zeta: int = N_ZETA
    n_mu_c: int = N_MU_COMPTON
    n_mu_r: int = N_MU_RAYLEIGH
    compton: str = "kn"        # "kn" free electron, "wh" Waller-Hartree (Eq. 2 with S)
    extra: dict = field(default_factory=dict)

    # --- physics data for this workload's material list ---
    def mu_rho(self) -> np.ndarray:
        """float32 [M][N_E][3] (pe, Compton, Rayleigh) cm^2/g."""
        t = ph.mu_rho_table(self.materials, e_nodes(self.e0, self.de, self.ne),
                            rayleigh=self.rayleigh, compton=self.compton)
        return t.astype(np.float32)

    @property
    def compton_per_material(self) -> bool:
        return self.compton == "wh"

    def compton_pdf(self, m: int = 0) -> np.ndarray:
        """Compton angular pdf [N_E][n_mu_c]: one shared K-N table, or the
        bound-electron table of material m."""
        en = e_nodes(self.e0, self.de, self.ne)
        if self.compton == "wh":
            return ph.wh_compton_pdf_table(self.materials[m], en, self.n_mu_c)
        return ph.kn_pdf_table(en, self.n_mu_c)

    def rayleigh_pdf(self, m: int) -> np.ndarray:
        """Rayleigh angular pdf of material m, [N_E][n_mu_r] (one material at
        a time: the fine mu grid makes each table ~80 MB)."""
        en = e_nodes(self.e0, self.de, self.ne)
        return ph.rayleigh_pdf_table(self.materials[m], en, self.n_mu_r)

    @property
    def n_voxels(self) -> int:
        g = self.grid
        return g["nx"] * g["ny"] * g["nz"]

    def voxel_volume(self) -> float:
        g = self.grid
        return g["dx"] * g["dy"] * g["dz"]


def _centered_grid(nx, ny, nz, dx, dy, dz) -> dict:
    return dict(nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz,
                ox=-nx * dx / 2.0, oy=-ny * dy / 2.0, oz=-nz * dz / 2.0)


def _centres(g):
    x = g["ox"] + (np.arange(g["nx"]) + 0.5) * g["dx"]
    y = g["oy"] + (np.arange(g["ny"]) + 0.5) * g["dy"]
    z = g["oz"] + (np.arange(g["nz"]) + 0.5) * g["dz"]
    return np.meshgrid(z, y, x, indexing="ij")   # Z, Y, X each [nz][ny][nx]


def _cone(sad, a0, a1, b0, b1, nproj, arc_deg=360.0, phi0_deg=0.0):
    return dict(kind="cone", sad=sad, iso=(0.0, 0.0, 0.0), a0=a0, a1=a1, b0=b0, b1=b1,
                nproj=nproj, arc_deg=arc_deg, phi0_deg=phi0_deg)


def _ellipsoid(X, Y, Z, c, s):
    return ((X - c[0]) / s[0]) ** 2 + ((Y - c[1]) / s[1]) ** 2 + ((Z - c[2]) / s[2]) ** 2 <= 1.0


def tiny(n_histories: int = 100_000, seed: int = 1) -> Workload:
    g = dict(nx=32, ny=32, nz=32, dx=0.5, dy=0.5, dz=0.5, ox=0.0, oy=0.0, oz=0.0)
    mat = np.zeros((32, 32, 32), np.uint8)
    rho = np.ones((32, 32, 32), np.float32)
    geo = dict(kind="pencil", src=(8.0, 8.0, 0.0), dir=(0.0, 0.0, 1.0))
    return Workload("tiny", g, mat, rho, ["water"], False,
                    np.array([60.0]), 0.0, np.array([1.0]), geo, seed, n_histories)


def water_cbct(n_histories: int = 1_000_000_000, seed: int = 2, scale: int = 1) -> Workload:
    """Water cylinder in air under a full-fan CBCT orbit.  ``scale`` > 1
    coarsens the grid by that factor per axis (same physical phantom) for
    oracle-sized parity cases."""
    nx, ny, nz = 128 // scale, 128 // scale, 100 // scale
    g = _centered_grid(nx, ny, nz, 0.25 * scale, 0.25 * scale, 0.2 * scale)
    Z, Y, X = _centres(g)
    inside = X * X + Y * Y <= 15.0 ** 2
    mats = ["water", "air"]
    mat = np.where(inside, 0, 1).astype(np.uint8)
    rho = np.where(inside, 1.0, ph.MATERIALS["air"][0]).astype(np.float32)
    lo, w = ph.kramers_spectrum(120, 2.0)
    geo = _cone(100.0, -13.0, 13.0, -10.0, 10.0, 360)
    return Workload("water_cbct", g, mat, rho, mats, True, lo, 1.0, w, geo, seed, n_histories)


def head(n_histories: int = 2_000_000_000, seed: int = 3, gen_seed: int = 3003,
         scale: int = 1) -> Workload:
    """Synthetic head of nested ellipsoids with +-2 % density noise (clipped
    at 3 sigma), half-fan 100 kVp, 200 projections over 360 deg."""
    rng = np.random.default_rng(gen_seed)
    nx, ny, nz = 256 // scale, 256 // scale, 160 // scale
    g = _centered_grid(nx, ny, nz, 0.1 * scale, 0.1 * scale, 0.1 * scale)
    Z, Y, X = _centres(g)
    mats = ["air", "soft_tissue", "brain", "cortical_bone", "lung"]
    outer = np.array([8.0, 10.0, 7.5]) * rng.uniform(0.95, 1.05, 3)
    mat = np.zeros(X.shape, np.uint8)
    mat[_ellipsoid(X, Y, Z, (0, 0, 0), outer)] = 1
    mat[_ellipsoid(X, Y, Z, (0, 0, 0), outer - 0.5)] = 3
    mat[_ellipsoid(X, Y, Z, (0, 0, 0), outer - 1.2)] = 2
    for k in range(3):
        c = (-1.8 + 1.8 * k, 5.0 + rng.uniform(-0.5, 0.5), 1.0 + rng.uniform(-0.5, 0.5))
        mat[_ellipsoid(X, Y, Z, c, rng.uniform(0.8, 1.5, 3))] = 0
    c = (rng.uniform(-1, 1), rng.uniform(-1, 1), -4.0 + rng.uniform(-0.5, 0.5))
    mat[_ellipsoid(X, Y, Z, c, rng.uniform(1.0, 2.0, 3))] = 4
    dens = np.array([ph.MATERIALS[m][0] for m in mats])
    noise = np.clip(rng.standard_normal(X.shape), -3.0, 3.0)
    rho = (dens[mat] * (1.0 + 0.02 * noise)).astype(np.float32)
    lo, w = ph.kramers_spectrum(100, 2.0)
    geo = _cone(100.0, -1.0, 14.0, -10.0, 10.0, 200)
    return Workload("head", g, mat, rho, mats, True, lo, 1.0, w, geo, seed, n_histories)


def head_helical(n_histories: int = 1_000_000_000, seed: int = 6, gen_seed: int = 3003,
                 scale: int = 1) -> Workload:
    """The synthetic head under a helical CT scan: 120 kVp fan beam of 2 cm
    collimation at the isocentre (60 cm source-axis distance), pitch 1
    (2 cm feed per turn), 6 turns from z = -6 cm, 180 projections per turn."""
    wl = head(n_histories, seed, gen_seed, scale)
    wl.name = "head_helical"
    wl.spectrum_lo, wl.spectrum_w = ph.kramers_spectrum(120, 2.0)
    geo = _cone(60.0, -12.0, 12.0, -1.0, 1.0, 6 * 180, arc_deg=6 * 360.0)
    geo["iso"] = (0.0, 0.0, -6.0)
    geo["feed"] = 2.0
    wl.geometry = geo
    return wl


def bowtie_fluence(na: int, nb: int, half_a: float, half_b: float, gen_seed: int = 7007,
                   noise: float = 0.01) -> np.ndarray:
    """Synthetic air-scan fluence [nb][na] behind a full-fan aluminium bow-tie
    filter: transmission exp(-mu t(a)) with t rising from 0.5 mm at the centre
    to 12 mm at |a| >= 0.9 half_a (quadratic), mu of Al at 50 keV; a 10 %
    heel-effect slope along b; +-noise multiplicative seeded noise (an air
    scan is measured).  Strictly positive."""
    rng = np.random.default_rng(gen_seed)
    a = (np.arange(na) + 0.5) / na * 2.0 - 1.0          # in units of half_a
    b = (np.arange(nb) + 0.5) / nb * 2.0 - 1.0
    t_cm = 0.05 + (1.2 - 0.05) * np.minimum(1.0, (a / 0.9) ** 2)
    mu_al = float(ph.mu_rho_total("aluminium", 50.0).item()) * ph.MATERIALS["aluminium"][0]
    fa = np.exp(-mu_al * t_cm)
    fb = 1.0 - 0.05 * b
    f = fb[:, None] * fa[None, :] * (1.0 + noise * np.clip(rng.standard_normal((nb, na)), -3, 3))
    return f.astype(np.float32)


def water_box_bowtie(n_histories: int = 250_000_000, seed: int = 7, scale: int = 1,
                     na: int = 128, nb: int = 96) -> Workload:
    """Water cube 20 cm on 0.4 cm voxels under a static cone beam at normal
    incidence (100 cm source-isocentre distance, 26.7 x 20 cm field at the
    isocentre), 125 kVp with 2 mm Al, bow-tie fluence map of na x nb
    beamlets; 10 batches, 1 keV cutoff (the shape of the paper's Sec. 3
    validation case, synthetic fluence)."""
    n = 50 // scale
    g = _centered_grid(n, n, n, 0.4 * scale, 0.4 * scale, 0.4 * scale)
    mat = np.zeros((n, n, n), np.uint8)
    rho = np.ones((n, n, n), np.float32)
    lo, w = ph.kramers_spectrum(125, 2.0)
    geo = _cone(100.0, -13.35, 13.35, -10.0, 10.0, 1, arc_deg=0.0)
    geo["fluence"] = bowtie_fluence(na, nb, 13.35, 10.0)
    return Workload("water_box_bowtie", g, mat, rho, ["water"], True, lo, 1.0, w, geo, seed,
                    n_histories)


_C4_EXTRA = ["water", "brain", "lung", "cortical_bone"]


def batched_case(rng: np.random.Generator, seed: int, name: str = "case",
                 size_scale: float = 1.0, hist_scale: float = 1.0) -> Workload:
    """One case of the uneven multi-phantom distribution.  ``size_scale`` < 1
    shrinks voxel counts (same distribution shape) for oracle-sized tests."""
    t = rng.uniform(0.0, 1.0)
    nx = max(4, int(round(64 * 4.0 ** t * size_scale)))
    nz = max(4, int(round(64 * 2.5 ** t * size_scale)))
    d = rng.uniform(0.1, 0.5)
    d = min(d, 40.0 / nx, 30.0 / nz)
    g = _centered_grid(nx, nx, nz, d, d, d)
    Z, Y, X = _centres(g)
    n_m = int(rng.integers(2, 7))
    extra = list(rng.permutation(_C4_EXTRA))[: max(0, n_m - 2)]
    mats = ["air", "soft_tissue"] + [str(m) for m in extra]
    ext = np.array([nx * d, nx * d, nz * d]) / 2.0
    body = ext * rng.uniform(0.75, 0.92, 3)
    mat = np.zeros(X.shape, np.uint8)
    mat[_ellipsoid(X, Y, Z, (0, 0, 0), body)] = 1
    for k in range(2, n_m):
        f = 0.75 - 0.15 * (k - 2)
        c = rng.uniform(-0.1, 0.1, 3) * body
        mat[_ellipsoid(X, Y, Z, c, body * f)] = k
    dens = np.array([ph.MATERIALS[m][0] for m in mats])
    rho = dens[mat].astype(np.float32)
    kvp = int(rng.integers(80, 141))
    lo, w = ph.kramers_spectrum(kvp, 2.0)
    half = bool(rng.integers(0, 2))
    nproj = int(rng.integers(100, 401))
    geo = _cone(100.0, -1.0 if half else -13.0, 14.0 if half else 13.0, -10.0, 10.0, nproj)
    nh = int(round(10 ** rng.uniform(8.0, 9.0) * hist_scale))
    wl = Workload(name, g, mat, rho, mats, True, lo, 1.0, w, geo, seed, nh)
    wl.extra = dict(kvp=kvp, half_fan=half)
    return wl


def batched(n_cases: int = 48, gen_seed: int = 4004, size_scale: float = 1.0,
            hist_scale: float = 1.0) -> list:
    rng = np.random.default_rng(gen_seed)
    return [batched_case(rng, 4000 + c, f"case{c:02d}", size_scale, hist_scale)
            for c in range(n_cases)]


def serving_trace(n_requests: int = 200, rate_hz: float = 2.0, seed: int = 5005):
    """Poisson arrival times [s] and one request-generator seed per request."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    return np.cumsum(gaps) - gaps[0], rng.integers(0, 2**31, n_requests)


def serving_request(req_seed: int, idx: int, size_scale: float = 1.0) -> Workload:
    rng = np.random.default_rng(int(req_seed))
    return batched_case(rng, 5000 + idx, f"req{idx:03d}", size_scale)


def by_name(name: str, **kw) -> Workload:
    return {"tiny": tiny, "water_cbct": water_cbct, "head": head,
            "head_helical": head_helical, "water_box_bowtie": water_box_bowtie}[name](**kw)


def geometry_turns(geo: dict) -> dict:
    """Angles in turns (1 turn = 360 deg) for code that works in revolutions."""
    out = dict(geo)
    if geo["kind"] == "cone":
        out["phi0_turns"] = geo["phi0_deg"] / 360.0
        out["arc_turns"] = geo["arc_deg"] / 360.0
    return out


def field_area(geo: dict) -> float:
    return (geo["a1"] - geo["a0"]) * (geo["b1"] - geo["b0"])
