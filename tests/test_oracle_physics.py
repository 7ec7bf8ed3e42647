"""Pins of the physics input data (closed forms vs quadrature) and of the
oracle's inverse-CDF surfaces (Sec. 2.2.2-2.2.3): against the exact inverse
of the analytic CDF, and by chi-square of sampled angles against the exact
pdf, the paper's own validation procedure for Figs. 3 and 4."""
import math

import numpy as np
import pytest
from scipy import integrate, optimize, stats

from oracle import oracle as O
from synth import physics as ph
from synth import workloads as W

SIGMA_T = 8.0 * math.pi / 3.0 * ph.R_E_CM ** 2


def test_sigma_kn_quadrature_vs_closed_form():
    E = np.linspace(10.0, 250.0, 49)
    q = ph.sigma_kn(E)
    c = ph.sigma_kn_closed(E)
    assert np.max(np.abs(q / c - 1.0)) < 1e-11
    # 60 keV: 0.5456198 barn
    assert abs(ph.sigma_kn(60.0)[0] * 1e24 - 0.5456198) < 5e-7


def test_sigma_kn_low_energy_series():
    # sigma/sigma_T = 1 - 2k + 26/5 k^2 - 133/10 k^3 + ...  (Thomson limit)
    for E in [0.5, 1.0, 2.0]:
        k = E / ph.ME_C2_KEV
        series = 1 - 2 * k + 26 / 5 * k**2 - 133 / 10 * k**3 + 1144 / 35 * k**4
        assert abs(ph.sigma_kn(E)[0] / SIGMA_T - series) < 1e-10


def test_rayleigh_closed_form_vs_quadrature():
    for name in ["water", "cortical_bone", "air"]:
        for E in [5.0, 20.0, 60.0, 140.0]:
            c = float(ph.rayleigh_c(name, E))
            f = lambda mu: (1 + mu * mu) / (1 + c * (1 - mu)) ** 4
            pts = [1 - 1 / c] if c > 1 else None
            v, _ = integrate.quad(f, -1, 1, epsabs=0, epsrel=1e-13, limit=400, points=pts)
            assert abs(v / ph.rayleigh_angular_integral(c) - 1) < 1e-10
    assert ph.rayleigh_angular_integral(0.0) == pytest.approx(8.0 / 3.0, rel=1e-15)
    # water at 60 keV: mu_R/rho = 0.012460 cm^2/g
    assert ph.mu_rho_rayleigh("water", 60.0) == pytest.approx(0.012460, abs=2e-6)


def test_photoelectric_normalisation():
    # water: photoelectric = Compton (free electron) at 26 keV
    assert ph.mu_rho_pe("water", 26.0) == pytest.approx(ph.mu_rho_compton("water", 26.0)[0],
                                                         rel=1e-12)
    assert ph.mu_rho_pe("water", 60.0) == pytest.approx(0.016470, abs=2e-5)


def _kn_pdf(E):
    return lambda mu: float(ph.kn_dsigma_dmu(E, mu))


def _ray_pdf(name, E):
    c = float(ph.rayleigh_c(name, E))
    return lambda mu: (1 + mu * mu) / (1 + c * (1 - mu)) ** 4


def _exact_quantile(pdf, zetas, peak=None):
    pts = None if peak is None else [peak]
    Z, _ = integrate.quad(pdf, -1, 1, epsabs=0, epsrel=1e-13, limit=400, points=pts)

    def cdf(m):
        if m <= -1:
            return 0.0
        pp = None if (peak is None or not (-1 < peak < m)) else [peak]
        v, _ = integrate.quad(pdf, -1, m, epsabs=0, epsrel=1e-13, limit=400, points=pp)
        return v / Z

    return np.array([optimize.brentq(lambda m: cdf(m) - z, -1, 1, xtol=1e-14)
                     for z in zetas])


@pytest.mark.parametrize("E", [10.0, 60.0, 120.0])
def test_kn_surface_vs_exact_inverse_cdf(E):
    wl = W.tiny()
    S = O.build_surface(wl.compton_pdf(), wl.n_zeta)
    j = int(round((E - wl.e0) / wl.de))
    zetas = np.arange(1, wl.n_zeta - 1, 5) / (wl.n_zeta - 1)
    exact = _exact_quantile(_kn_pdf(E), zetas)
    got = S[j, np.arange(1, wl.n_zeta - 1, 5)].astype(np.float64)
    # trapezoid CDF on h = 2/2048 plus linear inversion: error O(h^2)
    assert np.max(np.abs(got - exact)) < 2e-6
    assert S[j, 0] == -1.0 and S[j, -1] == 1.0
    assert np.all(np.diff(S[j]) >= 0)


@pytest.mark.parametrize("E", [10.0, 60.0, 120.0])
def test_rayleigh_surface_vs_exact_inverse_cdf(E, water_rayleigh_surface):
    S = water_rayleigh_surface
    j = int(round(E - W.E0_KEV))
    c = float(ph.rayleigh_c("water", E))
    idx = np.arange(1, W.N_ZETA - 1, 7)
    exact = _exact_quantile(_ray_pdf("water", E), idx / (W.N_ZETA - 1),
                            peak=1 - 1 / c if c > 1 else None)
    assert np.max(np.abs(S[j, idx] - exact)) < 1e-6
    assert np.all(np.diff(S) >= 0)


def _chi2_sampled(mu, pdf, nbins=100, peak=None):
    """Chi-square of sampled mu against the exact pdf over nbins equiprobable
    bins (edges at exact quantiles k/nbins)."""
    edges = _exact_quantile(pdf, np.arange(1, nbins) / nbins, peak)
    n, _ = np.histogram(mu, bins=np.concatenate([[-1.0], edges, [1.0]]))
    e = mu.size / nbins
    return stats.chi2.sf(((n - e) ** 2 / e).sum(), nbins - 1)


@pytest.mark.parametrize("E", [10.0, 60.0, 120.0, 60.5])
def test_kn_sampling_chi2(E):
    """Fig. 4 procedure: 1e6 samples from the C surface vs the K-N pdf."""
    wl = W.tiny()
    S = O.build_surface(wl.compton_pdf(), wl.n_zeta)
    zeta = np.random.default_rng(int(E * 10)).random(1_000_000)
    mu = O.sample_surface(S, E, zeta)
    assert O.sample_surface(S, E, np.array([0.0]))[0] == -1.0
    assert mu.min() >= -1 and mu.max() <= 1
    assert _chi2_sampled(mu, _kn_pdf(E)) > 1e-3


@pytest.fixture(scope="module")
def water_rayleigh_surface():
    return O.build_surface(ph.rayleigh_pdf_table("water", W.e_nodes(), W.N_MU_RAYLEIGH),
                           W.N_ZETA)


@pytest.mark.parametrize("E", [10.0, 60.0, 120.0, 60.5])
def test_rayleigh_sampling_chi2(E, water_rayleigh_surface):
    """Fig. 3 procedure: 1e6 samples from the R surface vs (1+mu^2) F^2."""
    S = water_rayleigh_surface
    zeta = np.random.default_rng(int(E)).random(1_000_000)
    mu = O.sample_surface(S, E, zeta)
    c = float(ph.rayleigh_c("water", E))
    assert _chi2_sampled(mu, _ray_pdf("water", E), peak=1 - 1 / c if c > 1 else None) > 1e-3


def test_mean_energy_transfer_fraction_60kev():
    # mean K-N energy-transfer fraction at 60 keV, used by the kerma check
    E = 60.0
    k = E / ph.ME_C2_KEV
    f = lambda mu: float(ph.kn_dsigma_dmu(E, mu)) * (1 - 1 / (1 + k * (1 - mu)))
    num, _ = integrate.quad(f, -1, 1, epsrel=1e-13)
    den, _ = integrate.quad(_kn_pdf(E), -1, 1, epsrel=1e-13)
    assert num / den == pytest.approx(0.093629, abs=2e-6)


# ---------------- bound-electron Compton (Eq. 2 with S) ----------------

def _wh_pdf(name, E):
    return lambda mu: float(ph.kn_dsigma_dmu(E, mu) * ph.incoherent_sf(name, E, mu))


def test_wh_cross_section_quadrature_and_limits():
    for name in ["water", "cortical_bone"]:
        z = ph.MATERIALS[name][1]
        for E in [10.0, 35.0, 90.0]:
            exact, _ = integrate.quad(lambda m: _wh_pdf(name, E)(m) / z, -1, 1,
                                      epsabs=0, epsrel=1e-13, limit=400)
            assert ph.sigma_compton_wh(name, E)[0] == pytest.approx(exact, rel=1e-11)
        E = np.linspace(5.0, 250.0, 50)
        ratio = ph.sigma_compton_wh(name, E) / ph.sigma_kn(E)
        # S <= Z suppresses scattering, less so as the momentum transfer grows
        assert np.all(ratio < 1.0) and np.all(np.diff(ratio) > 0)
        assert ratio[-1] > 0.99
    # S -> Z at large momentum transfer: backscatter matches K-N exactly in the limit
    assert ph.incoherent_sf("water", 1e5, -1.0) == pytest.approx(7.4, rel=1e-9)
    assert ph.incoherent_sf("water", 60.0, 1.0) == 0.0


@pytest.mark.parametrize("name,E", [("water", 10.0), ("cortical_bone", 30.0),
                                    ("cortical_bone", 120.0)])
def test_wh_surface_vs_exact_inverse_cdf(name, E):
    """S rises from 0 to Z_eff within 1 - mu ~ 2 x_b^2 (hc/E)^2 of the forward
    direction, a few mu cells at high E, so the trapezoid CDF error is larger
    than for K-N; it must still fall as h^2 when the mu grid is refined."""
    j = int(round(E - W.E0_KEV))
    idx = np.arange(1, W.N_ZETA - 1, 5)
    exact = _exact_quantile(_wh_pdf(name, E), idx / (W.N_ZETA - 1))
    errs = []
    for n_mu in [W.N_MU_COMPTON, 2 * W.N_MU_COMPTON - 1]:
        S = O.build_surface(ph.wh_compton_pdf_table(name, W.e_nodes(), n_mu), W.N_ZETA)
        assert np.all(np.diff(S[j]) >= 0)
        errs.append(np.max(np.abs(S[j, idx] - exact)))
    assert errs[0] < 5e-5
    assert errs[1] < errs[0] / 3.0 or errs[0] < 2e-6


@pytest.mark.parametrize("name,E", [("water", 20.0), ("cortical_bone", 60.0),
                                    ("cortical_bone", 45.5)])
def test_wh_sampling_chi2(name, E):
    """1e6 samples from a per-material C surface vs K-N x S, and a check that
    the test separates it from the free-electron law at the same energy."""
    S = O.build_surface(ph.wh_compton_pdf_table(name, W.e_nodes(), W.N_MU_COMPTON), W.N_ZETA)
    mu = O.sample_surface(S, E, np.random.default_rng(int(E * 7)).random(1_000_000))
    assert _chi2_sampled(mu, _wh_pdf(name, E)) > 1e-3
    assert _chi2_sampled(mu, _kn_pdf(E)) < 1e-6
