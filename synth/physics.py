"""Synthetic photon interaction data (FP64): the stand-in for the tabulated
cross-section databases the paper loads (PENELOPE form factors and scattering
functions, Sec. 2.2.2-2.2.3), which are not available here.

This module is *input data*, shared by the oracle and the GPU library through
the seeded workload generators.  It holds physics models only -- no step of the
transport method, no inverse-CDF construction, no majorant, no sampling.

Models (all per material, cm^2/g unless stated):

* Photoelectric:  mu_pe/rho = (Z/A) N_A * A_PE * Z_eff^3.8 / E^3, E in keV,
  with the free normalisation A_PE fixed so that water's photoelectric and
  free-electron Compton attenuation cross at 26 keV.
* Compton, free electron: mu_C/rho = (Z/A) N_A sigma_KN(E); sigma_KN by
  Gauss-Legendre quadrature of the Klein-Nishina differential cross section
  (the K-N factor of Eq. 2 with S = 1), which stays accurate at small E where
  the closed form cancels.
* Rayleigh: molecule of Z_eff-electron pseudo-atoms with the screened form
  factor F(x) = Z_eff / (1 + x^2/x_s^2)^2, x = (E/hc) sin(theta/2),
  x_s = 0.6 A^-1 (Z_eff/7.4)^(1/3).  Eq. 1 then integrates in closed form.
* Compton, bound electron (Waller-Hartree, Eq. 2 with S): synthetic
  incoherent scattering function S(x) = Z_eff (1 - 1/(1 + x^2/x_b^2)^2),
  x_b = 0.5 A^-1 (Z_eff/7.4)^(1/3), which lowers water's Compton attenuation
  to ~0.7 of the free-electron value at 10 keV and ~0.98 at 60 keV.  Used by
  workloads that ask for per-material C surfaces.
"""
from __future__ import annotations

import math

import numpy as np

ME_C2_KEV = 510.99895            # electron rest energy [keV]
R_E_CM = 2.8179403262e-13        # classical electron radius [cm]
N_A = 6.02214076e23              # Avogadro [1/mol]
HC_KEV_A = 12.3984198            # h*c [keV * Angstrom]
KEV_TO_J = 1.602176634e-16

# name -> (density g/cm^3, Z_eff, Z/A)
MATERIALS = {
    "water":         (1.0,    7.4,  0.5551),
    "soft_tissue":   (1.05,   7.4,  0.5495),
    "brain":         (1.04,   7.4,  0.5523),
    "lung":          (0.3,    7.4,  0.5497),
    "cortical_bone": (1.85,   13.8, 0.5148),
    "air":           (0.0012, 7.6,  0.4992),
    "aluminium":     (2.699,  13.0, 0.4818),
}

_GL_X, _GL_W = np.polynomial.legendre.leggauss(96)


def kn_dsigma_dmu(E, mu):
    """Klein-Nishina d(sigma)/d(mu) per free electron [cm^2], Eq. 2 with S=1
    integrated over azimuth: pi r_e^2 eps^2 (eps + 1/eps - 1 + mu^2)."""
    E = np.asarray(E, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    eps = 1.0 / (1.0 + (E / ME_C2_KEV) * (1.0 - mu))
    return math.pi * R_E_CM**2 * eps * eps * (eps + 1.0 / eps - 1.0 + mu * mu)


def sigma_kn(E):
    """Total Klein-Nishina cross section per electron [cm^2] by 96-point
    Gauss-Legendre quadrature over mu in [-1, 1] (smooth integrand)."""
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    vals = kn_dsigma_dmu(E[:, None], _GL_X[None, :])
    return vals @ _GL_W


def sigma_kn_closed(E):
    """Textbook closed form of the Klein-Nishina total cross section; loses
    accuracy to cancellation at small E, so only used as a cross-check."""
    k = np.asarray(E, dtype=np.float64) / ME_C2_KEV
    l = np.log1p(2.0 * k)
    return 2.0 * math.pi * R_E_CM**2 * (
        (1.0 + k) / k**2 * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k)
        + l / (2.0 * k) - (1.0 + 3.0 * k) / (1.0 + 2.0 * k) ** 2)


def _pe_norm() -> float:
    zwater = MATERIALS["water"][1]
    return float(sigma_kn(26.0)[0]) * 26.0**3 / zwater**3.8


A_PE = _pe_norm()   # cm^2 keV^3, ~5.3e-24


def electrons_per_gram(name: str) -> float:
    return MATERIALS[name][2] * N_A


def mu_rho_pe(name: str, E):
    _, z, _ = MATERIALS[name]
    E = np.asarray(E, dtype=np.float64)
    return electrons_per_gram(name) * A_PE * z**3.8 / E**3


def mu_rho_compton(name: str, E):
    return electrons_per_gram(name) * sigma_kn(E)


def form_factor_xs(name: str) -> float:
    """Screening momentum x_s [1/Angstrom] of the synthetic form factor."""
    z = MATERIALS[name][1]
    return 0.6 * (z / 7.4) ** (1.0 / 3.0)


def rayleigh_c(name: str, E):
    """c = (E/hc)^2 / (2 x_s^2): F^2 = Z^2 / (1 + c (1 - mu))^4."""
    xs = form_factor_xs(name)
    E = np.asarray(E, dtype=np.float64)
    return (E / HC_KEV_A) ** 2 / (2.0 * xs * xs)


def rayleigh_angular_integral(c):
    """Closed form of int_{-1}^{1} (1+mu^2) / (1 + c(1-mu))^4 dmu."""
    c = np.asarray(c, dtype=np.float64)
    return 8.0 * (2.0 * c * c + 2.0 * c + 1.0) / (3.0 * (1.0 + 2.0 * c) ** 3)


def sigma_rayleigh(name: str, E):
    """Rayleigh cross section per pseudo-atom [cm^2], Eq. 1 integrated:
    pi r_e^2 Z^2 * int (1+mu^2) F^2/Z^2 dmu."""
    z = MATERIALS[name][1]
    return math.pi * R_E_CM**2 * z * z * rayleigh_angular_integral(rayleigh_c(name, E))


def mu_rho_rayleigh(name: str, E):
    z = MATERIALS[name][1]
    return electrons_per_gram(name) / z * sigma_rayleigh(name, E)


def mu_rho_total(name: str, E, rayleigh: bool = True):
    t = mu_rho_pe(name, E) + mu_rho_compton(name, E)
    if rayleigh:
        t = t + mu_rho_rayleigh(name, E)
    return t


# --- angular pdfs on a mu grid (input to the inverse-CDF surface build) ---

def mu_grid(n_mu: int) -> np.ndarray:
    return -1.0 + 2.0 * np.arange(n_mu, dtype=np.float64) / (n_mu - 1)


def kn_pdf_table(e_nodes, n_mu: int) -> np.ndarray:
    """Un-normalised Klein-Nishina angular pdf [n_E][n_mu]."""
    mu = mu_grid(n_mu)
    return kn_dsigma_dmu(np.asarray(e_nodes)[:, None], mu[None, :]) / (math.pi * R_E_CM**2)


def rayleigh_pdf_table(name: str, e_nodes, n_mu: int) -> np.ndarray:
    """Un-normalised Rayleigh angular pdf (1+mu^2) F^2 / Z^2 [n_E][n_mu]."""
    mu = mu_grid(n_mu)
    c = rayleigh_c(name, np.asarray(e_nodes))[:, None]
    return (1.0 + mu[None, :] ** 2) / (1.0 + c * (1.0 - mu[None, :])) ** 4


def incoherent_sf(name: str, E, mu):
    """Synthetic Waller-Hartree incoherent scattering function S per molecule
    (pseudo-atom of Z_eff electrons): S -> 0 forward, S -> Z_eff backward."""
    z = MATERIALS[name][1]
    xb = 0.5 * (z / 7.4) ** (1.0 / 3.0)
    x2 = (np.asarray(E) / HC_KEV_A) ** 2 * (1.0 - np.asarray(mu)) / 2.0
    return z * (1.0 - 1.0 / (1.0 + x2 / (xb * xb)) ** 2)


def wh_compton_pdf_table(name: str, e_nodes, n_mu: int) -> np.ndarray:
    """Un-normalised bound-electron Compton pdf (Eq. 2 with S) [n_E][n_mu]."""
    mu = mu_grid(n_mu)
    e = np.asarray(e_nodes)[:, None]
    return kn_pdf_table(e_nodes, n_mu) * incoherent_sf(name, e, mu[None, :])


def sigma_compton_wh(name: str, E):
    """Bound-electron Compton cross section per electron [cm^2]: the K-N
    differential cross section weighted by S/Z_eff, 192-point Gauss-Legendre
    in mu (both factors are smooth in mu)."""
    z = MATERIALS[name][1]
    x, w = np.polynomial.legendre.leggauss(192)
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    vals = kn_dsigma_dmu(E[:, None], x[None, :]) * incoherent_sf(name, E[:, None], x[None, :]) / z
    return vals @ w


def mu_rho_compton_wh(name: str, E):
    return electrons_per_gram(name) * sigma_compton_wh(name, E)


def mu_rho_table(names, e_nodes, rayleigh: bool = True, compton: str = "kn") -> np.ndarray:
    """[M][n_E][3] float64 table of (photoelectric, Compton, Rayleigh) mass
    attenuation coefficients; the Rayleigh column is 0 when disabled.
    compton: "kn" free electron, "wh" bound electron (Waller-Hartree)."""
    e = np.asarray(e_nodes, dtype=np.float64)
    out = np.zeros((len(names), e.size, 3), dtype=np.float64)
    for m, name in enumerate(names):
        out[m, :, 0] = mu_rho_pe(name, e)
        out[m, :, 1] = (mu_rho_compton(name, e) if compton == "kn"
                        else mu_rho_compton_wh(name, e))
        if rayleigh:
            out[m, :, 2] = mu_rho_rayleigh(name, e)
    return out


def kramers_spectrum(kvp: int, al_mm: float = 2.0, e_min: int = 20):
    """Photon-number Kramers spectrum (kVp - E)/E filtered by al_mm of Al,
    sampled at the centre of 1 keV bins [e_min, kVp - 1].  Returns
    (bin_lo [keV], weight)."""
    lo = np.arange(e_min, kvp, dtype=np.float64)
    ec = lo + 0.5
    rho_al = MATERIALS["aluminium"][0]
    att = np.exp(-mu_rho_total("aluminium", ec, rayleigh=True) * rho_al * al_mm / 10.0)
    w = (kvp - ec) / ec * att
    return lo, w
