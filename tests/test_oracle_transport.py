"""Pins of the oracle's transport (Sec. 2.1 Woodcock tracking and interaction
sampling; Sec. 2.2.1 batches; Sec. 2.2.5 spectrum stratification; Sec. 2.2.6
source trajectory) against closed forms, invariances and brute force."""
from dataclasses import replace as dataclass_replace
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import oracle as O
from synth import physics as ph
from synth import workloads as W
from tests._helpers import frac_within, random_phantom, slab_workload

THREADS = 8


def _mu_node(name, rho, E, rayleigh):
    return rho * float(ph.mu_rho_total(name, E, rayleigh))


# ---------------- P1: narrow-beam primary transmission ----------------

def test_narrow_beam_transmission_water():
    wl = W.tiny(n_histories=1_000_000)
    c = O.OracleCase(wl)
    r = O.run(c, threads=THREADS)
    t = c.mu_rho[0, 59].astype(np.float64)
    mu = t[0] + t[1]                       # tables as stored, 60 keV node
    assert mu == pytest.approx(0.198864, abs=2e-6)
    p = np.exp(-mu * 16.0)
    n = r["n_hist"]
    z = (r["n_unscattered"] - n * p) / np.sqrt(n * p * (1 - p))
    assert abs(z) < 4.0, z


def test_layered_slab_transmission_exp_integral():
    """Woodcock is exact in heterogeneous media: T = exp(-sum mu_i l_i)."""
    layers = [("water", 1.0, 4), ("cortical_bone", 1.85, 2), ("lung", 0.3, 6),
              ("air", 0.0012, 4), ("soft_tissue", 1.05, 4)]
    wl = slab_workload(layers, e_kev=60.0, n_hist=1_000_000, dz=0.5)
    c = O.OracleCase(wl)
    r = O.run(c, threads=THREADS)
    tab = c.mu_rho.astype(np.float64)
    mats = wl.materials
    line = sum(rho * tab[mats.index(m), 59].sum() * n * 0.5 for m, rho, n in layers)
    # the stored rho is float32
    line = sum(float(np.float32(rho)) * tab[mats.index(m), 59].sum() * n * 0.5
               for m, rho, n in layers)
    p = np.exp(-line)
    n = r["n_hist"]
    z = (r["n_unscattered"] - n * p) / np.sqrt(n * p * (1 - p))
    assert abs(z) < 4.0, (z, p)
    # majorant is set by bone
    assert c.mu_max[59] >= np.float32(1.85) * np.float32(tab[mats.index("cortical_bone"), 59].sum())


# ---------------- P4: energy conservation ----------------

@pytest.mark.parametrize("name", ["water_cbct", "head"])
def test_energy_conservation(name):
    wl = W.by_name(name, n_histories=20_000, scale=8)
    c = O.OracleCase(wl)
    r = O.run(c, threads=THREADS)
    assert r["n_hist"] == 20_000
    assert abs(r["e_inc"] - r["e_dep"] - r["e_esc"]) <= 1e-12 * r["e_inc"]
    n_q = r["n_hist"] + r["n_deposits"] + r["n_escapes"]
    assert abs(r["q_inc"] - r["q_dep"] - r["q_esc"]) <= 0.5 * n_q
    assert r["s1"].sum() == r["q_dep"]
    assert r["shadow"].sum() == pytest.approx(r["e_dep"], rel=1e-12)


# ---------------- P5: brute force on tiny phantoms ----------------

@pytest.mark.parametrize("shape", [(2, 2, 2), (4, 4, 4)])
def test_tally_equals_event_log(shape):
    wl = random_phantom(shape, 3, seed=sum(shape), n_hist=10_000)
    c = O.OracleCase(wl)
    r = O.run(c, batches=[10_000], threads=3, log_range=(0, 10_000), log_cap=400_000)
    ev = r["log"]
    dep = ev[np.isin(ev["type"], [O.EV_PHOTO, O.EV_COMPTON, O.EV_CUTOFF])]
    V = c.n_voxels
    T = np.zeros(V, np.int64)
    np.add.at(T, dep["vox"], np.rint(dep["e"] * O.Q_SCALE).astype(np.int64))
    assert np.array_equal(T, r["s1"])
    D = np.zeros(V)
    np.add.at(D, dep["vox"], dep["e"])
    assert np.allclose(D, r["shadow"], rtol=1e-12, atol=0)
    # every history has one source event and ends exactly once
    ends = ev[np.isin(ev["type"], [O.EV_PHOTO, O.EV_CUTOFF, O.EV_ESCAPE, O.EV_MISS])]
    assert np.array_equal(np.sort(ends["h"]), np.arange(10_000))
    # per-history balance: source E = deposits + escape
    src = ev[ev["type"] == O.EV_SOURCE]
    tot = np.zeros(10_000)
    np.add.at(tot, dep["h"], dep["e"])
    esc = ev[np.isin(ev["type"], [O.EV_ESCAPE, O.EV_MISS])]
    np.add.at(tot, esc["h"], esc["e"])
    assert np.allclose(tot, src["e"], rtol=1e-13)


# ---------------- P7: special media ----------------

def _table_only(wl, keep):
    t = wl.mu_rho().copy()
    for k in range(3):
        if k not in keep:
            t[..., k] = 0.0
    return t


def test_photoelectric_only_medium_exponential_law():
    wl = W.tiny(n_histories=400_000)
    c = O.OracleCase(wl, mu_rho=_table_only(wl, [0]))
    r = O.run(c, batches=[400_000], threads=1, log_range=(0, 400_000), log_cap=900_000)
    mu = float(c.mu_rho[0, 59, 0])
    E = 60.0
    n = r["n_hist"]
    assert r["n_compton"] == 0 and r["n_rayleigh"] == 0
    assert r["e_dep"] == pytest.approx(n * E - r["n_unscattered"] * E, rel=1e-14)
    ev = r["log"]
    pe = ev[ev["type"] == O.EV_PHOTO]
    iz = pe["vox"] // (32 * 32)
    assert np.all(pe["vox"] % (32 * 32) == 16 * 32 + 16)   # on the beam axis
    obs = np.bincount(iz, minlength=32)
    zc = np.arange(33) * 0.5
    exp = n * (np.exp(-mu * zc[:-1]) - np.exp(-mu * zc[1:]))
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, 31) > 1e-3


def test_rayleigh_only_medium_zero_dose():
    wl = W.tiny(n_histories=20_000)
    wl.rayleigh = True
    c = O.OracleCase(wl, mu_rho=_table_only(wl, [2]))
    r = O.run(c, threads=THREADS)
    assert r["n_rayleigh"] > 0
    assert np.all(r["s1"] == 0) and r["e_dep"] == 0.0
    assert r["n_escapes"] == r["n_hist"]


def test_compton_only_with_cutoff_at_source_energy():
    wl = W.tiny(n_histories=50_000)
    wl.e_cut = 60.0 + 1e-9
    c = O.OracleCase(wl, mu_rho=_table_only(wl, [1]))
    r = O.run(c, threads=THREADS)
    n_int = r["n_hist"] - r["n_unscattered"]
    assert r["n_compton"] == n_int == r["n_cutoff"]
    assert r["n_deposits"] == 2 * n_int
    assert r["e_dep"] == pytest.approx(60.0 * n_int, rel=1e-13)


# ---------------- P8: Woodcock invariances ----------------

def test_majorant_scaling_invariance():
    wl = W.head(n_histories=300_000, scale=8)
    res = []
    for f in [1.0, 2.0, 4.0]:
        c = O.OracleCase(wl, majorant_scale=f)
        r = O.run(c, threads=THREADS)
        d, s = O.dose_and_sigma(r, c, wl.n_histories)
        res.append((d, s, r))
    steps = [x[2]["n_steps"] for x in res]
    assert steps[0] < steps[1] < steps[2]
    d0, s0, r0 = res[0]
    mask = d0 > 0.1 * d0.max()
    for d, s, r in res[1:]:
        assert frac_within(d0, s0, d, s, mask) >= 0.99
        # mean deposited energy per history: |diff| within 4 sigma (E_max bound)
        tol = 4 * 100.0 / np.sqrt(wl.n_histories) * np.sqrt(2)
        assert abs(r["e_dep"] - r0["e_dep"]) / wl.n_histories < tol


def test_voxel_split_invariance():
    """Splitting every voxel into 2x2x2 identical voxels leaves every
    trajectory unchanged; the re-binned tally equals the coarse one."""
    coarse = random_phantom((6, 8, 8), 4, seed=5, n_hist=40_000, dxyz=1.0)
    fine = random_phantom((6, 8, 8), 4, seed=5, n_hist=40_000, dxyz=1.0)
    fine.mat = np.repeat(np.repeat(np.repeat(coarse.mat, 2, 0), 2, 1), 2, 2)
    fine.rho = np.repeat(np.repeat(np.repeat(coarse.rho, 2, 0), 2, 1), 2, 2)
    g = dict(coarse.grid)
    g.update(nx=16, ny=16, nz=12, dx=0.5, dy=0.5, dz=0.5)
    fine.grid = g
    rc = O.run(O.OracleCase(coarse), threads=THREADS)
    rf = O.run(O.OracleCase(fine), threads=THREADS)
    binned = rf["s1"].reshape(6, 2, 8, 2, 8, 2).sum(axis=(1, 3, 5)).reshape(-1)
    same = np.mean(binned == rc["s1"])
    assert same >= 0.999
    assert rf["n_steps"] == rc["n_steps"] or abs(rf["n_steps"] - rc["n_steps"]) < 1e-4 * rc["n_steps"]
    assert rf["e_dep"] == pytest.approx(rc["e_dep"], rel=1e-4)


# ---------------- P9: source sampling ----------------

def _hamilton_exact(n, w):
    fw = [Fraction(x) for x in w]
    W_ = sum(fw)
    q = [Fraction(n) * x / W_ for x in fw]
    base = [int(x) for x in q]
    rem = n - sum(base)
    order = sorted(range(len(w)), key=lambda j: (-(q[j] - base[j]), j))
    for j in order[:rem]:
        base[j] += 1
    return base


@pytest.mark.parametrize("n", [1, 7, 1000, 99_991, 10**9 + 7])
def test_bin_allocation_largest_remainder(n):
    lo, w = ph.kramers_spectrum(120)
    got = O.alloc_bins(n, w)
    assert int(got.sum()) == n
    assert list(map(int, got)) == _hamilton_exact(n, w)


def test_source_sampling_uniformity():
    wl = W.water_cbct(scale=8)
    c = O.OracleCase(wl)
    geo = wl.geometry
    N = 20_000
    S = np.array([O.sample_source(c, h, 7) for h in range(N)])
    iso = np.array(geo["iso"])
    # source on the orbit of radius SAD at one of nproj angles
    r = np.hypot(S[:, 0] - iso[0], S[:, 1] - iso[1])
    assert np.allclose(r, geo["sad"], rtol=1e-12)
    phi = np.degrees(np.arctan2(S[:, 0], S[:, 1])) % 360.0
    p = np.rint(phi * geo["nproj"] / geo["arc_deg"]).astype(int) % geo["nproj"]
    assert np.allclose(phi, p * geo["arc_deg"] / geo["nproj"], atol=1e-9)
    cnt = np.bincount(p, minlength=geo["nproj"])
    assert stats.chisquare(cnt).pvalue > 1e-3
    # energy uniform within bin 7
    e = S[:, 6] - wl.spectrum_lo[7]
    assert stats.kstest(e, "uniform").pvalue > 1e-3
    # hit point on the isocentre plane uniform on the field rectangle
    ph_ = np.radians(p * geo["arc_deg"] / geo["nproj"])
    axis = -np.stack([np.sin(ph_), np.cos(ph_), 0 * ph_], 1)
    t = -np.einsum("ij,ij->i", S[:, :3] - iso, axis) / np.einsum("ij,ij->i", S[:, 3:6], axis)
    P = S[:, :3] + t[:, None] * S[:, 3:6] - iso
    elat = np.stack([np.cos(ph_), -np.sin(ph_), 0 * ph_], 1)
    a = np.einsum("ij,ij->i", P, elat)
    b = P[:, 2]
    assert stats.kstest((a - geo["a0"]) / (geo["a1"] - geo["a0"]), "uniform").pvalue > 1e-3
    assert stats.kstest((b - geo["b0"]) / (geo["b1"] - geo["b0"]), "uniform").pvalue > 1e-3


def test_continuous_source_trajectory():
    """n_proj = 0 is the paper's own form of Sec. 2.2.6: the source angle is
    t uniform over the arc (phi0 + u1 * arc), not one of a set of projection
    angles.  The source stays on the orbit, covers exactly the arc (a 200 deg
    arc from 30 deg, as in the paper's head scan), is uniform over it, takes
    its uniform from the second word of the history's source block, and the
    field crossing at the isocentre stays uniform."""
    wl = W.water_cbct(scale=8)
    geo = dict(wl.geometry, nproj=0, phi0_deg=30.0, arc_deg=200.0)
    wl.geometry = geo
    c = O.OracleCase(wl)
    N = 20_000
    S = np.array([O.sample_source(c, h, 3) for h in range(N)])
    iso = np.array(geo["iso"])
    r = np.hypot(S[:, 0] - iso[0], S[:, 1] - iso[1])
    assert np.allclose(r, geo["sad"], rtol=1e-12)
    assert np.allclose(S[:, 2], iso[2], atol=1e-12)
    phi = np.degrees(np.arctan2(S[:, 0] - iso[0], S[:, 1] - iso[1])) % 360.0
    assert phi.min() >= 30.0 and phi.max() <= 230.0
    assert stats.kstest((phi - 30.0) / 200.0, "uniform").pvalue > 1e-3
    # no projection lattice: 20000 draws give ~20000 distinct angles
    assert len(np.unique(np.round(phi, 9))) > 0.99 * N
    key = [wl.seed & 0xFFFFFFFF, wl.seed >> 32]
    for h in range(0, N, 997):
        u1 = O.uniform(int(O.philox([0, h, 0, 0], key)[1]))
        assert phi[h] == pytest.approx(30.0 + 200.0 * u1, abs=1e-9)
    ph_ = np.radians(phi)
    axis = -np.stack([np.sin(ph_), np.cos(ph_), 0 * ph_], 1)
    t = -np.einsum("ij,ij->i", S[:, :3] - iso, axis) / np.einsum("ij,ij->i", S[:, 3:6], axis)
    P = S[:, :3] + t[:, None] * S[:, 3:6] - iso
    elat = np.stack([np.cos(ph_), -np.sin(ph_), 0 * ph_], 1)
    a = np.einsum("ij,ij->i", P, elat)
    assert stats.kstest((a - geo["a0"]) / (geo["a1"] - geo["a0"]), "uniform").pvalue > 1e-3
    assert stats.kstest((P[:, 2] - geo["b0"]) / (geo["b1"] - geo["b0"]),
                        "uniform").pvalue > 1e-3


def test_history_layout_bin_major():
    wl = W.water_cbct(scale=8, n_histories=1000)
    c = O.OracleCase(wl)
    batches = O.batch_sizes(1000, 10)
    cnt = O.alloc_bins(100, c.bin_w)
    pref = np.concatenate([[0], np.cumsum(cnt)])
    for h in [0, 1, 57, 99, 100, 250, 999]:
        j = O.bin_of_history(c, h, batches)
        assert pref[j] <= h % 100 < pref[j + 1]
        e = O.sample_source(c, h, j)[6]
        assert wl.spectrum_lo[j] <= e < wl.spectrum_lo[j] + 1.0


# ---------------- P10: symmetry ----------------

def test_pencil_mirror_symmetry():
    """Beam through the centre of the middle voxel of a 31x31 cross-section:
    the geometry is symmetric under x- and y-mirrors and the x<->y swap."""
    wl = W.tiny(n_histories=1_000_000)
    wl.grid = dict(wl.grid, nx=31, ny=31)
    wl.mat = np.zeros((32, 31, 31), np.uint8)
    wl.rho = np.ones((32, 31, 31), np.float32)
    wl.geometry = dict(kind="pencil", src=(7.75, 7.75, 0.0), dir=(0.0, 0.0, 1.0))
    c = O.OracleCase(wl)
    r = O.run(c, threads=THREADS)
    d, s = O.dose_and_sigma(r, c, wl.n_histories)
    d, s = d.reshape(32, 31, 31), s.reshape(32, 31, 31)
    mask = d > 0.01 * d.max()
    for op in [lambda a: np.flip(a, 2), lambda a: np.flip(a, 1),
               lambda a: np.swapaxes(a, 1, 2)]:
        assert frac_within(d, s, op(d), op(s), mask & op(mask)) >= 0.99


def test_cylinder_rotational_symmetry():
    """360-deg orbit around a centred cylinder: the energy deposited in each
    ring is the same in the four azimuthal quadrants (chi-square over the
    batch-to-batch spread)."""
    wl = W.water_cbct(scale=4, n_histories=400_000)
    c = O.OracleCase(wl)
    g = wl.grid
    x = g["ox"] + (np.arange(32) + 0.5) * g["dx"]
    X, Y = np.meshgrid(x, x)
    R, A = np.hypot(X, Y), np.arctan2(Y, X)
    masks = [((A >= -np.pi + q * np.pi / 2) & (A < -np.pi / 2 + q * np.pi / 2)
              & (R >= r0) & (R < r0 + 3)) for r0 in range(0, 15, 3) for q in range(4)]
    n = 40_000
    per_batch = []
    for b in range(10):
        r = O.run(c, batches=[n], h0=b * n, threads=THREADS)
        e = r["shadow"].reshape(25, 32, 32)[8:17].sum(0)
        per_batch.append([e[m].sum() for m in masks])
    pb = np.array(per_batch).reshape(10, 5, 4)
    mean = pb.mean(0)
    se2 = pb.var(0, ddof=1) / 10
    ring = (mean / se2).sum(1) / (1 / se2).sum(1)
    chi2 = (((mean - ring[:, None]) ** 2) / se2).sum()
    assert stats.chi2.sf(chi2, 15) > 1e-3, chi2


# ---------------- P11 / resume / threads ----------------

def test_batch_stats_exact_vs_two_pass():
    wl = random_phantom((4, 6, 6), 3, seed=9, n_hist=5000, dxyz=1.0)
    c = O.OracleCase(wl)
    n = 500
    Tb = []
    for b in range(10):
        rb = O.run(c, batches=[n], h0=b * n, threads=2)
        Tb.append(rb["s1"].copy())
    Tb = np.array(Tb)
    r = O.run(c, batches=[n] * 10, threads=4)
    assert np.array_equal(Tb.sum(0), r["s1"])
    s2 = [sum(int(t) ** 2 for t in Tb[:, v]) for v in range(Tb.shape[1])]
    got = [(int(h) << 64) | int(l) for h, l in zip(r["s2_hi"], r["s2_lo"])]
    assert got == s2
    mean, var = O.batch_stats(r["s1"], r["s2_hi"], r["s2_lo"], 10)
    Tf = Tb.astype(np.float64)
    assert np.allclose(mean, Tf.mean(0), rtol=1e-15)
    ref = Tf.var(0, ddof=1) / 10
    assert np.allclose(var, ref, rtol=1e-9, atol=1e-6)


def test_thread_count_invariance_and_resume():
    wl = W.water_cbct(scale=8, n_histories=30_000)
    c = O.OracleCase(wl)
    r1 = O.run(c, threads=1)
    r8 = O.run(c, threads=8)
    for k in ["s1", "s2_hi", "s2_lo"]:
        assert np.array_equal(r1[k], r8[k])
    assert r1["q_dep"] == r8["q_dep"] and r1["n_steps"] == r8["n_steps"]
    bs = O.batch_sizes(30_000, 10)
    ra = O.run(c, batches=bs[:4], h0=0, threads=3)
    rb = O.run(c, batches=bs[4:], h0=sum(bs[:4]), threads=5)
    assert np.array_equal(ra["s1"] + rb["s1"], r1["s1"])


# ---------------- P6: first-collision kerma along the pencil axis ----------------

def test_first_collision_kerma_along_axis():
    wl = W.tiny(n_histories=300_000)
    c = O.OracleCase(wl)
    r = O.run(c, batches=[300_000], threads=1, log_range=(0, 300_000), log_cap=1_500_000)
    ev = r["log"]
    real = ev[np.isin(ev["type"], [O.EV_PHOTO, O.EV_COMPTON])]
    first = real[np.r_[True, real["h"][1:] != real["h"][:-1]]]
    iz = first["vox"] // (32 * 32)
    E = 60.0
    t = c.mu_rho[0, 59].astype(np.float64)
    mu = t[0] + t[1]
    k = E / ph.ME_C2_KEV
    f = lambda m: float(ph.kn_dsigma_dmu(E, m)) * (1 - 1 / (1 + k * (1 - m)))
    ftr = integrate.quad(f, -1, 1, epsrel=1e-13)[0] / integrate.quad(
        lambda m: float(ph.kn_dsigma_dmu(E, m)), -1, 1, epsrel=1e-13)[0]
    z = np.arange(33) * 0.5
    n = r["n_hist"]
    expect = n * E * (t[0] + t[1] * ftr) / mu * (np.exp(-mu * z[:-1]) - np.exp(-mu * z[1:]))
    got = np.bincount(iz, weights=first["e"], minlength=32)
    var = np.bincount(iz, weights=first["e"] ** 2, minlength=32)
    zs = (got - expect) / np.sqrt(var)
    assert np.sum(zs ** 2) < stats.chi2.ppf(1 - 1e-3, 32)


# ---------------- direction update after a scatter ----------------

@pytest.mark.parametrize("d", [(0.0, 0.0, 1.0), (0.0, 0.0, -1.0), (0.6, 0.0, 0.8),
                               (0.3, -0.5, 0.1), (1e-4, 2e-4, 0.99999998)])
def test_rotation_deflection_and_azimuth(d):
    d = np.array(d) / np.linalg.norm(d)
    rng = np.random.default_rng(3)
    mus = rng.uniform(-1, 1, 2000)
    phis = rng.uniform(0, 2 * np.pi, 2000)
    out = np.array([O.rotate(d, m, p) for m, p in zip(mus, phis)])
    assert np.allclose(np.linalg.norm(out, axis=1), 1.0, atol=1e-14)
    # exact off the pole; inside |w| >= 1 - 1e-5 the frame takes d = (0, 0, +-1)
    tol = 1e-12 if abs(d[2]) < 1 - 1e-5 else 2 * np.sqrt(1 - d[2] ** 2) + 1e-12
    assert np.allclose(out @ d, mus, atol=tol)
    # azimuth of the new direction around d is uniform
    ref = np.array([1.0, 0, 0]) if abs(d[0]) < 0.9 else np.array([0, 1.0, 0])
    e1 = ref - (ref @ d) * d
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    az = np.arctan2(out @ e2, out @ e1) % (2 * np.pi)
    ok = np.abs(mus) < 0.999
    assert stats.kstest(az[ok] / (2 * np.pi), "uniform").pvalue > 1e-3
    # a fixed phi gives a fixed azimuth offset (rotation is rigid in phi)
    a1 = O.rotate(d, 0.3, 0.4)
    a2 = O.rotate(d, 0.3, 0.4 + np.pi / 2)
    assert abs(((a1 - (a1 @ d) * d) @ (a2 - (a2 @ d) * d))) < max(tol, 1e-12)


# ---------------- P9: per-material Compton surfaces ----------------

def test_per_material_compton_surface_selects_voxel_material():
    """A stack of C surfaces is indexed by the material of the interaction
    voxel: a phantom made only of material 1 with the stack [K-N, bone] must
    reproduce, bit for bit, the run with the bone surface shared by all."""
    wl = random_phantom((4, 5, 6), 2, seed=21, n_hist=20_000)
    wl.mat[:] = 1
    wl.compton = "wh"
    kn = O.build_surface(ph.kn_pdf_table(W.e_nodes(), W.N_MU_COMPTON), W.N_ZETA)
    bone = O.build_surface(ph.wh_compton_pdf_table("cortical_bone", W.e_nodes(),
                                                   W.N_MU_COMPTON), W.N_ZETA)
    mu_rho = wl.mu_rho()
    r_stack = O.run(O.OracleCase(wl, comp_surf=np.stack([kn, bone]), mu_rho=mu_rho),
                    threads=THREADS)
    wl.compton = "kn"         # shared-surface mode, same attenuation table
    r_shared = O.run(O.OracleCase(wl, comp_surf=bone, mu_rho=mu_rho), threads=THREADS)
    r_wrong = O.run(O.OracleCase(wl, comp_surf=kn, mu_rho=mu_rho), threads=THREADS)
    assert np.array_equal(r_stack["s1"], r_shared["s1"])
    assert r_stack["n_compton"] == r_shared["n_compton"]
    assert not np.array_equal(r_stack["s1"], r_wrong["s1"])


def test_bound_electron_compton_angles_in_transport():
    """Compton-only slab of bone then water, pencil beam at 60 keV: the
    scattering cosine recovered from each first Compton event's energy
    transfer follows K-N x S of the material of that voxel."""
    wl = slab_workload([("cortical_bone", 1.85, 6), ("water", 1.0, 12)], e_kev=60.0,
                       n_hist=300_000, seed=23, nxy=8, dz=0.25)
    wl.compton = "wh"
    c = O.OracleCase(wl, mu_rho=_table_only(wl, [1]))
    r = O.run(c, batches=[wl.n_histories], threads=1, log_range=(0, wl.n_histories),
              log_cap=4_000_000)
    ev = r["log"]
    ev = ev[np.lexsort((ev["seq"], ev["h"]))]
    first = ev[ev["type"] == O.EV_COMPTON]
    first = first[np.r_[True, first["h"][1:] != first["h"][:-1]]]
    E0 = first["e"] + first["E"]
    assert np.allclose(E0, 60.0, rtol=0, atol=1e-9)
    mu = 1.0 - (E0 / first["E"] - 1.0) * ph.ME_C2_KEV / E0
    iz = first["vox"] // 64
    for name, sel in [("cortical_bone", iz < 6), ("water", iz >= 6)]:
        m = np.clip(mu[sel], -1.0, 1.0)
        assert m.size > 50_000
        p_right = _chi2_mu(m, lambda x: float(ph.kn_dsigma_dmu(60.0, x)
                                              * ph.incoherent_sf(name, 60.0, x)))
        p_kn = _chi2_mu(m, lambda x: float(ph.kn_dsigma_dmu(60.0, x)))
        assert p_right > 1e-3 and p_kn < 1e-6, (name, p_right, p_kn)


def _chi2_mu(mu, pdf, nbins=50):
    from scipy import integrate, optimize
    Z, _ = integrate.quad(pdf, -1, 1, epsrel=1e-12, limit=400)
    cdf = lambda m: integrate.quad(pdf, -1, m, epsrel=1e-12, limit=400)[0] / Z
    edges = [optimize.brentq(lambda m: cdf(m) - z, -1, 1, xtol=1e-13)
             for z in np.arange(1, nbins) / nbins]
    n, _ = np.histogram(mu, bins=np.concatenate([[-1.0], edges, [1.0]]))
    e = mu.size / nbins
    return stats.chi2.sf(((n - e) ** 2 / e).sum(), nbins - 1)


# ---------------- P11: helical CT trajectory ----------------

def test_helical_source_on_helix():
    """Source points lie on the helix iso + R(sin phi, cos phi, 0) +
    (0, 0, feed (phi - phi0)/360) at one of nproj uniformly drawn angles over
    several turns, and each ray crosses the field rectangle centred on the
    axis at the source's height uniformly."""
    wl = W.head_helical(scale=8)
    geo = wl.geometry
    c = O.OracleCase(wl)
    N = 20_000
    S = np.array([O.sample_source(c, h, 3) for h in range(N)])
    iso = np.array(geo["iso"])
    r = np.hypot(S[:, 0] - iso[0], S[:, 1] - iso[1])
    assert np.allclose(r, geo["sad"], rtol=1e-12)
    swept = (S[:, 2] - iso[2]) * 360.0 / geo["feed"]       # degrees since phi0
    p = np.rint(swept * geo["nproj"] / geo["arc_deg"]).astype(int)
    assert p.min() >= 0 and p.max() < geo["nproj"]
    assert np.allclose(swept, p * geo["arc_deg"] / geo["nproj"], atol=1e-9)
    phi = np.degrees(np.arctan2(S[:, 0] - iso[0], S[:, 1] - iso[1]))
    dphi = (phi - geo["phi0_deg"] - swept + 180.0) % 360.0 - 180.0
    assert np.max(np.abs(dphi)) < 1e-9, "angle and height on the same helix"
    assert stats.chisquare(np.bincount(p, minlength=geo["nproj"])).pvalue > 1e-3
    ph_ = np.radians(geo["phi0_deg"] + swept)
    axis = -np.stack([np.sin(ph_), np.cos(ph_), 0 * ph_], 1)
    centre = np.stack([np.full(N, iso[0]), np.full(N, iso[1]), S[:, 2]], 1)
    t = -np.einsum("ij,ij->i", S[:, :3] - centre, axis) / np.einsum("ij,ij->i", S[:, 3:6], axis)
    P = S[:, :3] + t[:, None] * S[:, 3:6] - centre
    elat = np.stack([np.cos(ph_), -np.sin(ph_), 0 * ph_], 1)
    a = np.einsum("ij,ij->i", P, elat)
    assert stats.kstest((a - geo["a0"]) / (geo["a1"] - geo["a0"]), "uniform").pvalue > 1e-3
    assert stats.kstest((P[:, 2] - geo["b0"]) / (geo["b1"] - geo["b0"]),
                        "uniform").pvalue > 1e-3


def test_helical_history_equals_circular_with_shifted_isocentre():
    """A helical history whose projection is p is the history of a circular
    scan whose isocentre sits at the helix height of p: identical events."""
    wl = W.head_helical(scale=8, n_histories=1000)
    geo = dict(wl.geometry)
    hel = O.OracleCase(wl)
    nproj, arc, feed = geo["nproj"], geo["arc_deg"], geo["feed"]
    checked = 0
    for h in range(0, 400, 7):
        x = O.sample_source(hel, h, 5)
        swept = (x[2] - geo["iso"][2]) * 360.0 / feed
        p = int(round(swept * nproj / arc))
        sw = p * arc / nproj
        circ = dict(geo, feed=0.0, iso=(geo["iso"][0], geo["iso"][1],
                                        geo["iso"][2] + feed * sw / 360.0))
        wl.geometry = circ
        cc = O.OracleCase(wl)
        wl.geometry = geo
        a = O.history(hel, h, 5)
        b = O.history(cc, h, 5)
        assert np.array_equal(O.sample_source(cc, h, 5), x)
        assert a.tobytes() == b.tobytes()
        checked += len(a)
    assert checked > 100


# ---------------- P12: fluence-map source (Sec. 2.2.4) ----------------

def _field_coords(S, geo):
    """(a, b) where each source ray crosses the field rectangle (static cone
    source at phi0, circular orbit)."""
    phi = np.radians(geo["phi0_deg"])
    iso = np.array(geo["iso"])
    axis = -np.array([np.sin(phi), np.cos(phi), 0.0])
    t = -((S[:, :3] - iso) @ axis) / (S[:, 3:6] @ axis)
    P = S[:, :3] + t[:, None] * S[:, 3:6] - iso
    return P @ np.array([np.cos(phi), -np.sin(phi), 0.0]), P[:, 2]


def test_fluence_map_beamlet_probabilities_and_positions():
    """Beamlets are drawn with probability f_I / sum f (chi-square), the
    logged beamlet is the one that contains the ray's crossing of the field,
    and the crossing is uniform inside its beamlet."""
    wl = W.water_box_bowtie(scale=5, na=16, nb=12)
    geo = wl.geometry
    f = geo["fluence"].astype(np.float64)
    c = O.OracleCase(wl)
    N = 120_000
    S = np.array([O.sample_source(c, h, 0) for h in range(N)])
    I = S[:, 8].astype(int)
    cnt = np.bincount(I, minlength=f.size)
    exp = N * f.reshape(-1) / f.sum()
    assert stats.chisquare(cnt, exp).pvalue > 1e-3
    a, b = _field_coords(S, geo)
    na, nb = f.shape[1], f.shape[0]
    fa = (a - geo["a0"]) / (geo["a1"] - geo["a0"]) * na
    fb = (b - geo["b0"]) / (geo["b1"] - geo["b0"]) * nb
    ia, ib = np.floor(fa + 1e-9).astype(int), np.floor(fb + 1e-9).astype(int)
    inside = (np.abs(fa - np.rint(fa)) > 1e-7) & (np.abs(fb - np.rint(fb)) > 1e-7)
    assert np.array_equal((ib * na + ia)[inside], I[inside])
    assert stats.kstest((fa - ia)[inside], "uniform").pvalue > 1e-3
    assert stats.kstest((fb - ib)[inside], "uniform").pvalue > 1e-3


def test_fluence_map_zero_beamlets_and_brute_force_tiny_map():
    """A 3 x 2 map with two empty beamlets: exact multinomial frequencies,
    and an empty beamlet is never drawn."""
    wl = W.water_box_bowtie(scale=10)
    f = np.array([[1.0, 0.0, 2.0], [5.0, 0.5, 0.0]], np.float32)
    wl.geometry["fluence"] = f
    c = O.OracleCase(wl)
    N = 60_000
    I = np.array([O.sample_source(c, h, 0)[8] for h in range(N)]).astype(int)
    cnt = np.bincount(I, minlength=6)
    assert cnt[1] == 0 and cnt[5] == 0
    p = f.reshape(-1).astype(np.float64) / float(f.sum())
    nz = p > 0
    assert stats.chisquare(cnt[nz], N * p[nz] / p[nz].sum()).pvalue > 1e-3


def test_fluence_map_error_decreases_like_fig5c():
    """Fig. 5c: e = ||p_f - p_f*|| over beamlets falls as the photon count
    grows; for exact sampling E[e^2] = sum p (1 - p) / N."""
    wl = W.water_box_bowtie(scale=10, na=32, nb=24)
    f = wl.geometry["fluence"].astype(np.float64).reshape(-1)
    p = f / f.sum()
    c = O.OracleCase(wl)
    I = np.array([O.sample_source(c, h, 0)[8] for h in range(200_000)]).astype(int)
    es = []
    for n in [2_000, 20_000, 200_000]:
        q = np.bincount(I[:n], minlength=p.size) / n
        es.append(np.linalg.norm(q - p))
        expect = np.sqrt((p * (1 - p)).sum() / n)
        assert 0.8 * expect < es[-1] < 1.2 * expect, (n, es[-1], expect)
    assert es[0] > es[1] > es[2]


def test_single_beamlet_map_equals_uniform_field():
    """A 1 x 1 map is the uniform field: identical transport events (the
    beamlet draw uses its own counter block and perturbs no other draw)."""
    wl = W.water_box_bowtie(scale=10, n_histories=400)
    geo = dict(wl.geometry)
    geo.pop("fluence")
    plain = O.OracleCase(dataclass_replace(wl, geometry=geo))
    wl.geometry["fluence"] = np.array([[3.0]], np.float32)
    one = O.OracleCase(wl)
    for h in range(0, 400, 13):
        a, b = O.history(one, h, 0), O.history(plain, h, 0)
        assert a[0]["vox"] == 0 and b[0]["vox"] == -1
        a["vox"][0] = -1
        assert a.tobytes() == b.tobytes()


def _mh_case(f, chains, scale=10):
    wl = W.water_box_bowtie(scale=scale)
    wl.geometry["fluence"] = np.asarray(f, np.float32)
    wl.geometry["fluence_chains"] = chains
    return O.OracleCase(wl)


def test_metropolis_hastings_two_beamlet_chain():
    """Alg. A1 on a 2-beamlet map f = (1, 3): the chain moves 0 -> 1 with
    probability 1/2 (trial J = 1, always accepted) and 1 -> 0 with 1/2 x 1/3,
    so its stationary law is (1/4, 3/4) = f / sum f."""
    c = _mh_case([[1.0, 3.0]], chains=1)
    I = O.mh_advance(c, 300_000).astype(int)
    a, b = I[:-1], I[1:]
    p01 = np.mean(b[a == 0] == 1)
    p10 = np.mean(b[a == 1] == 0)
    assert abs(p01 - 0.5) < 5 * math.sqrt(0.25 / np.sum(a == 0))
    assert abs(p10 - 1 / 6) < 5 * math.sqrt((1 / 6) * (5 / 6) / np.sum(a == 1))
    # second eigenvalue 1/3: asymptotic variance factor (1 + 1/3) / (1 - 1/3) = 2
    assert abs(np.mean(I == 1) - 0.75) < 5 * math.sqrt(0.75 * 0.25 * 2 / I.size)


def test_metropolis_hastings_chains_and_fig5c():
    """64 logical chains over the bow-tie map: e = ||p_f - p_f*|| falls with
    the photon count (Fig. 5c), within a few times the independent-sampling
    value; resuming the chains in pieces gives the same beamlets."""
    wl = W.water_box_bowtie(scale=10, na=32, nb=24)
    wl.geometry["fluence_chains"] = 64
    f = wl.geometry["fluence"].astype(np.float64).reshape(-1)
    p = f / f.sum()
    I = O.mh_advance(O.OracleCase(wl), 200_000).astype(int)
    es = []
    for n in [2_000, 20_000, 200_000]:
        q = np.bincount(I[:n], minlength=p.size) / n
        es.append(np.linalg.norm(q - p))
        assert es[-1] < 3.0 * np.sqrt((p * (1 - p)).sum() / n)
    assert es[0] > es[1] > es[2]
    c2 = O.OracleCase(wl)
    parts = np.concatenate([O.mh_advance(c2, k) for k in (1, 63, 1000, 198_936)])
    assert np.array_equal(parts, I)


def test_metropolis_hastings_transport_and_guards():
    wl = W.water_box_bowtie(scale=10, n_histories=20_000)
    wl.geometry["fluence_chains"] = 16
    c = O.OracleCase(wl)
    r = O.run(c, threads=THREADS)
    assert r["e_inc"] == pytest.approx(r["e_dep"] + r["e_esc"], rel=1e-12)
    with pytest.raises(ValueError):
        O.run(c, threads=THREADS)               # chains are past history 0
    r2 = O.run(c, h0=20_000, threads=THREADS, n_histories=1000)
    assert r2["n_hist"] == 1000
    with pytest.raises(ValueError):
        O.sample_source(O.OracleCase(wl), 0, 0)  # chains not advanced
    with pytest.raises(ValueError):
        _mh_case([[1.0, 0.0]], chains=4)


# ---------------- P13: readout (dose units, sigma-bar) ----------------

def test_dose_units_and_standard_error_by_hand():
    """One voxel of 1 g receiving 3, 5, 4, 8 keV in four batches of 10
    histories each: dose per history = (20 keV / 40) in J/kg, and its standard
    error = sd of the four batch means / sqrt(4)."""
    wl = slab_workload([("water", 1.0, 1)], nxy=1, dz=1.0, dxy=1.0, n_hist=40)
    c = O.OracleCase(wl)
    q = 2 ** 24
    batches = np.array([3, 5, 4, 8])
    tallies = batches * q
    res = dict(n_batches=4, s1=np.array([tallies.sum()], np.int64),
               s2_hi=np.array([0], np.uint64),
               s2_lo=np.array([int((tallies.astype(object) ** 2).sum())], np.uint64))
    dose, sd = O.dose_and_sigma(res, c, 40)
    kev = 1.602176634e-16
    assert dose[0] == pytest.approx(20.0 / 40 * kev / 1e-3, rel=1e-14)
    per_hist = batches / 10.0                     # keV per history in each batch
    assert sd[0] == pytest.approx(np.std(per_hist, ddof=1) / 2 * kev / 1e-3, rel=1e-12)


def test_sigma_bar_definitions_by_hand():
    dose = np.array([10.0, 6.0, 1.0, 4.0, 12.0])
    sd = np.array([1.0, 1.5, 0.5, 1.0, 3.0])
    rho = np.array([1.0, 1.0, 1.0, 1.0, 0.01])      # the last voxel is air: not inside
    # inside: D_max = 10; paper: D > 2 -> {10, 6, 4}: mean(1, 1.5, 1) / 10
    assert O.sigma_bar(dose, sd, rho, "paper") == pytest.approx((1 + 1.5 + 1) / 3 / 10)
    # local: D > 5 -> {10, 6}: mean(1/10, 1.5/6)
    assert O.sigma_bar(dose, sd, rho, "local") == pytest.approx((0.1 + 0.25) / 2)


# ---------------- P9: the transport's random words (reading 7) ----------------

def _pair(seed: int, h: int, P: int):
    """Uniforms of pair P of history h, straight from Philox4x32-10: words
    2 (P mod 2) and 2 (P mod 2) + 1 of block P // 2 + 1."""
    key = [seed & 0xFFFFFFFF, seed >> 32]
    w = O.philox([P // 2 + 1, h & 0xFFFFFFFF, h >> 32, 0], key)
    return O.uniform(int(w[2 * (P % 2)])), O.uniform(int(w[2 * (P % 2) + 1]))


def test_random_pairs_fictitious_steps_share_a_block():
    """A photoelectric-only cube (water's table at density 20, so that a
    photon takes several steps inside) under a doubled majorant: a tentative
    collision is real when u1 mu_max < mu (probability about 1/2), so
    histories take one, two, three ... steps.  Walking the pencil beam's axis
    with the pairs read off the raw Philox blocks (free path -ln(u0)/mu_max)
    must give, history by history, the step and voxel of the absorption or
    the step of the escape that the oracle logs: this pins which words a step
    takes, including a block's second pair after a fictitious step."""
    wl = W.tiny(n_histories=1)
    wl.rho = np.full_like(wl.rho, 20.0)
    c = O.OracleCase(wl, mu_rho=_table_only(wl, [0]), majorant_scale=2.0)
    je = int(round((60.0 - wl.e0) / wl.de))       # 60 keV is a node: weight 0
    mumax = float(c.mu_max[je])
    mu = 20.0 * float(c.mu_rho[0, je, 0])
    assert 0.45 < mu / mumax < 0.55
    steps = []
    for h in range(400):
        z, P = 0.0, 0                              # the beam enters at z = 0
        while True:
            u0, u1 = _pair(wl.seed, h, P)
            P += 1
            z += -math.log(u0) / mumax
            if not (0.0 <= z / 0.5 < 32):
                want = (O.EV_ESCAPE, P, -1)
                break
            if u1 * mumax < mu:
                want = (O.EV_PHOTO, P, (int(math.floor(z / 0.5)) * 32 + 16) * 32 + 16)
                break
        ev = O.history(c, h, 0)
        end = ev[np.isin(ev["type"], [O.EV_PHOTO, O.EV_ESCAPE])]
        assert len(end) == 1
        got = (int(end["type"][0]), int(end["k"][0]),
               int(end["vox"][0]) if end["type"][0] == O.EV_PHOTO else -1)
        assert got == want, f"history {h}"
        steps.append(P)
    steps = np.array(steps)
    assert (steps >= 2).sum() > 100 and (steps >= 3).sum() > 40 and (steps >= 4).sum() > 15


def test_random_pairs_scatter_takes_the_pair_after_its_step():
    """A Compton-only water cube under a doubled majorant: walking the axis
    with the pairs read off the raw Philox blocks, the first real collision
    takes place at the predicted step and voxel, and its scatter takes the
    next pair -- the same block's second pair after a step at a first pair,
    the next block's first pair after a step at a second pair -- whose first
    uniform is the surface sample: the logged energy of that Compton event
    must be E - E' with E' the Compton relation at the angle the surface
    gives for it."""
    wl = W.tiny(n_histories=1)
    c = O.OracleCase(wl, mu_rho=_table_only(wl, [1]), majorant_scale=2.0)
    je = int(round((60.0 - wl.e0) / wl.de))
    mumax = float(c.mu_max[je])
    mu = float(c.mu_rho[0, je, 1])
    parity = [0, 0]
    for h in range(400):
        z, P = 0.0, 0
        while True:
            u0, u1 = _pair(wl.seed, h, P)
            P += 1
            z += -math.log(u0) / mumax
            if not (z / 0.5 < 32) or u1 * mumax < mu:
                break
        if not (z / 0.5 < 32):
            continue                                # escaped before any collision
        zeta, _ = _pair(wl.seed, h, P)             # the pair after the step
        mu_c = float(O.sample_surface(c.comp, 60.0, [zeta], wl.e0, wl.de)[0])
        Ep = 60.0 / (1.0 + (60.0 / O.ME_C2_KEV) * (1.0 - mu_c))
        ev = O.history(c, h, 0)
        first = ev[ev["type"] == O.EV_COMPTON][0]
        assert int(first["k"]) == P, f"history {h}"
        assert int(first["vox"]) == (int(math.floor(z / 0.5)) * 32 + 16) * 32 + 16
        assert first["e"] == pytest.approx(60.0 - Ep, rel=1e-9, abs=1e-7), f"history {h}"
        assert first["E"] == pytest.approx(Ep, rel=1e-12)
        parity[(P - 1) % 2] += 1                   # the step's pair: first or second
    assert parity[0] > 80 and parity[1] > 60
