"""Python side of the FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It never imports the GPU library, and the GPU library
never imports it.

* ``build_surface`` -- the inverse-CDF "R/C surface" construction of
  Sec. 2.2.2: pdf on equally spaced mu, cumulative distribution by the
  trapezoid rule, normalised, then inverted at equally spaced zeta by linear
  interpolation between the (P_k, mu_k) pairs.
* the transport, tallies and batch statistics live in ``ctd_oracle.c``; this
  module compiles it (gcc) and marshals arguments with ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ctd_oracle.c")
_LIB = os.path.join(_HERE, "libctd_oracle.so")

EV_SOURCE, EV_PHOTO, EV_COMPTON, EV_RAYLEIGH, EV_CUTOFF, EV_ESCAPE, EV_MISS = range(7)
Q_SCALE = 2.0 ** 24
ME_C2_KEV = 510.99895


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-Wall",
               "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Case(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nmat", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
        ("ox", C.c_double), ("oy", C.c_double), ("oz", C.c_double),
        ("mat", C.c_void_p), ("rho", C.c_void_p),
        ("ne", C.c_int32), ("nzeta", C.c_int32), ("rayleigh", C.c_int32), ("kind", C.c_int32),
        ("e0", C.c_double), ("de", C.c_double),
        ("mu_rho", C.c_void_p), ("comp_surf", C.c_void_p), ("rayl_surf", C.c_void_p),
        ("mu_max", C.c_void_p),
        ("nbins", C.c_int32), ("nproj", C.c_int32),
        ("bin_lo", C.c_void_p), ("bin_w", C.c_void_p), ("bin_width", C.c_double),
        ("src", C.c_double * 3), ("dir", C.c_double * 3),
        ("sad", C.c_double), ("iso", C.c_double * 3),
        ("a0", C.c_double), ("a1", C.c_double), ("b0", C.c_double), ("b1", C.c_double),
        ("phi0_deg", C.c_double), ("arc_deg", C.c_double),
        ("e_cut", C.c_double), ("seed", C.c_uint64),
        ("comp_per_mat", C.c_int32), ("pad_c", C.c_int32),
        ("z_feed", C.c_double),
        ("fl_na", C.c_int32), ("fl_nb", C.c_int32), ("fl_cdf", C.c_void_p),
        ("fl_chains", C.c_int32), ("pad_f", C.c_int32), ("fl_f", C.c_void_p),
        ("fl_beam", C.c_void_p), ("fl_h0", C.c_uint64), ("fl_nbeam", C.c_uint64),
    ]


class Event(C.Structure):
    _fields_ = [("h", C.c_uint64), ("seq", C.c_uint32), ("k", C.c_uint32),
                ("type", C.c_int32), ("pad", C.c_int32), ("vox", C.c_int64),
                ("e", C.c_double), ("E", C.c_double)]


EVENT_DTYPE = np.dtype([("h", "<u8"), ("seq", "<u4"), ("k", "<u4"), ("type", "<i4"),
                        ("pad", "<i4"), ("vox", "<i8"), ("e", "<f8"), ("E", "<f8")])


class Result(C.Structure):
    _fields_ = [
        ("s1", C.c_void_p), ("s2_hi", C.c_void_p), ("s2_lo", C.c_void_p),
        ("shadow", C.c_void_p), ("shadow_sq", C.c_void_p),
        ("e_inc", C.c_double), ("e_dep", C.c_double), ("e_esc", C.c_double),
        ("q_inc", C.c_int64), ("q_dep", C.c_int64), ("q_esc", C.c_int64),
        ("n_hist", C.c_uint64), ("n_steps", C.c_uint64), ("n_real", C.c_uint64),
        ("n_pe", C.c_uint64), ("n_compton", C.c_uint64), ("n_rayleigh", C.c_uint64),
        ("n_deposits", C.c_uint64), ("n_escapes", C.c_uint64), ("n_miss", C.c_uint64),
        ("n_cutoff", C.c_uint64), ("n_unscattered", C.c_uint64),
        ("e_unscattered", C.c_double),
        ("n_batches", C.c_uint32),
        ("log", C.c_void_p), ("log_cap", C.c_uint64), ("log_n", C.c_uint64),
        ("log_h0", C.c_uint64), ("log_h1", C.c_uint64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.or_run.argtypes = [C.POINTER(Case), C.c_uint64, C.c_void_p, C.c_int, C.c_int,
                                C.POINTER(Result)]
        _lib.or_majorant.argtypes = [C.POINTER(Case), C.c_void_p]
        _lib.or_alloc_bins.argtypes = [C.c_uint64, C.c_int, C.c_void_p, C.c_void_p]
        _lib.or_philox.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.or_philox.restype = None
        _lib.or_uniform.argtypes = [C.c_uint32]
        _lib.or_uniform.restype = C.c_double
        _lib.or_history.argtypes = [C.POINTER(Case), C.c_uint64, C.c_int, C.c_void_p,
                                    C.c_uint64, C.POINTER(C.c_uint64)]
        _lib.or_tally_replay.argtypes = [C.c_uint64, C.c_void_p, C.c_void_p, C.c_int64,
                                         C.c_void_p]
        _lib.or_sample_surface.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double,
                                           C.c_double, C.c_double, C.c_void_p, C.c_int64,
                                           C.c_void_p]
        _lib.or_sample_source.argtypes = [C.POINTER(Case), C.c_uint64, C.c_int, C.c_void_p]
        _lib.or_mh_fill.argtypes = [C.POINTER(Case), C.c_uint64, C.c_uint64, C.c_void_p,
                                    C.c_void_p]
        _lib.or_rotate.argtypes = [C.c_void_p, C.c_double, C.c_double]
        _lib.or_rotate.restype = None
        _lib.or_batch_stats.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_uint32, C.c_void_p, C.c_void_p]
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---------------- inverse-CDF surfaces (Sec. 2.2.2 / 2.2.3) ----------------

def build_surface(pdf: np.ndarray, n_zeta: int) -> np.ndarray:
    """R/C surface from a pdf tabulated on equally spaced mu in [-1, 1].

    For each energy row: P_0 = 0, P_k = P_{k-1} + h (p_{k-1} + p_k)/2, divide
    by P_last; at zeta_i = i/(n_zeta-1) take the largest k <= n_mu-2 with
    P_k <= zeta_i and interpolate mu = mu_k + h (zeta_i - P_k)/(P_{k+1} - P_k).
    Returned as float32 [n_E][n_zeta]."""
    pdf = np.asarray(pdf, dtype=np.float64)
    n_e, n_mu = pdf.shape
    h = 2.0 / (n_mu - 1)
    mu = -1.0 + 2.0 * np.arange(n_mu, dtype=np.float64) / (n_mu - 1)
    zeta = np.arange(n_zeta, dtype=np.float64) / (n_zeta - 1)
    out = np.empty((n_e, n_zeta), dtype=np.float64)
    for j in range(n_e):
        inc = 0.5 * (pdf[j, :-1] + pdf[j, 1:]) * h
        P = np.concatenate([[0.0], np.cumsum(inc)])
        P = P / P[-1]
        k = np.searchsorted(P, zeta, side="right") - 1
        k = np.clip(k, 0, n_mu - 2)
        out[j] = mu[k] + h * (zeta - P[k]) / (P[k + 1] - P[k])
    return out.astype(np.float32)


# ---------------- case assembly ----------------

class OracleCase:
    """Holds the numpy buffers a ``Case`` struct points into."""

    def __init__(self, wl, majorant_scale: float = 1.0, comp_surf=None, rayl_surf=None,
                 mu_rho=None):
        self.wl = wl
        g = wl.grid
        self.mat = np.ascontiguousarray(wl.mat, dtype=np.uint8)
        self.rho = np.ascontiguousarray(wl.rho, dtype=np.float32)
        self.mu_rho = np.ascontiguousarray(wl.mu_rho() if mu_rho is None else mu_rho,
                                           dtype=np.float32)
        per_mat = getattr(wl, "compton_per_material", False)
        if comp_surf is not None:
            self.comp = np.ascontiguousarray(comp_surf, dtype=np.float32)
        elif per_mat:
            self.comp = np.stack([build_surface(wl.compton_pdf(m), wl.n_zeta)
                                  for m in range(len(wl.materials))])
        else:
            self.comp = build_surface(wl.compton_pdf(), wl.n_zeta)
        want = ((len(wl.materials),) if per_mat else ()) + (wl.ne, wl.n_zeta)
        if self.comp.shape != want:
            raise ValueError(f"Compton surface shape {self.comp.shape}, expected {want}")
        if wl.rayleigh:
            self.rayl = (np.ascontiguousarray(rayl_surf, dtype=np.float32)
                         if rayl_surf is not None
                         else np.stack([build_surface(wl.rayleigh_pdf(m), wl.n_zeta)
                                        for m in range(len(wl.materials))]))
        else:
            self.rayl = None
        self.bin_lo = np.ascontiguousarray(wl.spectrum_lo, dtype=np.float64)
        self.bin_w = np.ascontiguousarray(wl.spectrum_w, dtype=np.float64)
        self.mu_max = np.zeros(wl.ne, dtype=np.float32)
        c = Case()
        c.nx, c.ny, c.nz = g["nx"], g["ny"], g["nz"]
        c.nmat = len(wl.materials)
        c.dx, c.dy, c.dz = g["dx"], g["dy"], g["dz"]
        c.ox, c.oy, c.oz = g["ox"], g["oy"], g["oz"]
        c.mat, c.rho = _p(self.mat), _p(self.rho)
        c.ne, c.nzeta, c.rayleigh = wl.ne, wl.n_zeta, int(wl.rayleigh)
        c.e0, c.de = wl.e0, wl.de
        c.mu_rho, c.comp_surf = _p(self.mu_rho), _p(self.comp)
        c.rayl_surf = _p(self.rayl) if self.rayl is not None else None
        c.mu_max = _p(self.mu_max)
        c.nbins = len(self.bin_lo)
        c.bin_lo, c.bin_w, c.bin_width = _p(self.bin_lo), _p(self.bin_w), wl.spectrum_width
        geo = wl.geometry
        if geo["kind"] == "pencil":
            c.kind = 0
            c.src[:] = geo["src"]
            c.dir[:] = geo["dir"]
            c.nproj = 0
        else:
            c.kind = 1
            c.sad = geo["sad"]
            c.iso[:] = geo["iso"]
            c.a0, c.a1, c.b0, c.b1 = geo["a0"], geo["a1"], geo["b0"], geo["b1"]
            c.phi0_deg, c.arc_deg = geo["phi0_deg"], geo["arc_deg"]
            c.z_feed = geo.get("feed", 0.0)
            f = geo.get("fluence")
            if f is not None:
                f = np.asarray(f, dtype=np.float32)
                if f.ndim != 2 or np.any(~np.isfinite(f)) or np.any(f < 0) or f.sum() <= 0:
                    raise ValueError("fluence map must be [nb][na], finite, >= 0, nonzero")
                # running sums in beamlet order I = ib * na + ia, FP64 (Sec. 2.2.4)
                self.fl_cdf = np.cumsum(f.reshape(-1).astype(np.float64))
                c.fl_nb, c.fl_na = f.shape
                c.fl_cdf = _p(self.fl_cdf)
                chains = int(geo.get("fluence_chains", 0))
                if chains > 0:
                    # Alg. A1 (Metropolis-Hastings) needs f_I > 0 for every beamlet
                    if np.any(f <= 0):
                        raise ValueError("Metropolis-Hastings sampling needs f_I > 0")
                    self.fl_f = np.ascontiguousarray(f.reshape(-1))
                    self.mh_state = np.zeros(chains, np.int32)
                    self.mh_next = 0
                    c.fl_chains = chains
                    c.fl_f = _p(self.fl_f)
            c.nproj = geo["nproj"]
        c.e_cut = wl.e_cut
        c.seed = wl.seed
        c.comp_per_mat = int(per_mat)
        self.c = c
        rc = lib().or_majorant(C.byref(c), _p(self.mu_max))
        if rc != 0:
            raise ValueError(f"or_majorant failed: {rc}")
        if majorant_scale != 1.0:
            self.mu_max *= np.float32(majorant_scale)

    @property
    def n_voxels(self):
        return int(self.mat.size)


def alloc_bins(n: int, weights) -> np.ndarray:
    w = np.ascontiguousarray(weights, dtype=np.float64)
    out = np.zeros(len(w), dtype=np.uint64)
    rc = lib().or_alloc_bins(int(n), len(w), _p(w), _p(out))
    if rc != 0:
        raise ValueError(f"or_alloc_bins failed: {rc}")
    return out


def batch_sizes(n: int, n_batches: int) -> list:
    """N histories split into n_batches equal batches, the first N mod n_b
    batches one larger (Sec. 2.2.1: histories divided evenly)."""
    base, rem = divmod(int(n), int(n_batches))
    return [base + (1 if b < rem else 0) for b in range(n_batches)]


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox(_p(c), _p(k), _p(out))
    return out


def uniform(r: int) -> float:
    return lib().or_uniform(int(r))


def run(case: OracleCase, n_histories: int | None = None, n_batches: int | None = None,
        batches=None, h0: int = 0, threads: int = 1, log_range=None, log_cap: int = 0,
        shadow_sq: bool = False) -> dict:
    """Transport the given batches; returns tallies, balance and counters."""
    wl = case.wl
    if batches is None:
        batches = batch_sizes(n_histories if n_histories is not None else wl.n_histories,
                              n_batches if n_batches is not None else wl.n_batches)
    bs = np.ascontiguousarray(batches, dtype=np.uint64)
    if case.c.fl_chains > 0:
        if h0 != case.mh_next:
            raise ValueError(f"Metropolis-Hastings chains are at history {case.mh_next}, "
                             f"not {h0}: runs must follow each other in history order")
        mh_advance(case, int(bs.sum()))
    V = case.n_voxels
    s1 = np.zeros(V, np.int64)
    s2h = np.zeros(V, np.uint64)
    s2l = np.zeros(V, np.uint64)
    sh = np.zeros(V, np.float64)
    shq = np.zeros(V, np.float64) if shadow_sq else None
    r = Result()
    r.s1, r.s2_hi, r.s2_lo, r.shadow = _p(s1), _p(s2h), _p(s2l), _p(sh)
    r.shadow_sq = _p(shq) if shq is not None else None
    log = None
    if log_range is not None:
        log = np.zeros(max(1, log_cap), dtype=EVENT_DTYPE)
        r.log, r.log_cap = _p(log), log_cap
        r.log_h0, r.log_h1 = log_range
    rc = lib().or_run(C.byref(case.c), int(h0), _p(bs), len(bs), int(threads), C.byref(r))
    if rc != 0:
        raise RuntimeError(f"or_run failed: {rc}")
    out = {f[0]: getattr(r, f[0]) for f in Result._fields_
           if f[0] not in ("s1", "s2_hi", "s2_lo", "shadow", "shadow_sq", "log")}
    out.update(s1=s1, s2_hi=s2h, s2_lo=s2l, shadow=sh, shadow_sq=shq)
    if log is not None:
        n = min(r.log_n, log_cap)
        if r.log_n > log_cap:
            raise RuntimeError("event log overflow")
        ev = log[:n]
        out["log"] = ev[np.lexsort((ev["seq"], ev["h"]))]
    return out


def mh_advance(case: OracleCase, n: int) -> np.ndarray:
    """Alg. A1: advance the logical chains over the next n histories (in id
    order) and make their beamlets the ones the source uses; returns them."""
    out = np.zeros(max(n, 1), np.int32)
    rc = lib().or_mh_fill(C.byref(case.c), int(case.mh_next), int(n), _p(case.mh_state),
                          _p(out))
    if rc != 0:
        raise RuntimeError(f"or_mh_fill failed: {rc}")
    case.mh_beam = out
    case.c.fl_beam, case.c.fl_h0, case.c.fl_nbeam = _p(out), case.mh_next, n
    case.mh_next += n
    return out[:n]


def history(case: OracleCase, h: int, j: int, cap: int = 100000) -> np.ndarray:
    buf = np.zeros(cap, dtype=EVENT_DTYPE)
    n = C.c_uint64(0)
    rc = lib().or_history(C.byref(case.c), int(h), int(j), _p(buf), cap, C.byref(n))
    if rc != 0:
        raise RuntimeError(f"or_history failed: {rc}")
    return buf[: min(n.value, cap)]


def bin_of_history(case: OracleCase, h: int, batches, h0: int = 0) -> int:
    """Spectrum bin of history id h under the bin-major batch layout."""
    base = h0
    for n in batches:
        if h < base + n:
            cnt = alloc_bins(n, case.bin_w)
            pref = np.concatenate([[0], np.cumsum(cnt.astype(np.int64))])
            return int(np.searchsorted(pref, h - base, side="right") - 1)
        base += n
    raise ValueError("history id beyond the batches")


def sample_surface(S, E: float, zeta, e0: float = 1.0, de: float = 1.0) -> np.ndarray:
    """mu = surface(zeta, E) through the transport's bilinear lookup."""
    S = np.ascontiguousarray(S, dtype=np.float32)
    z = np.ascontiguousarray(zeta, dtype=np.float64)
    out = np.zeros(z.size)
    lib().or_sample_surface(_p(S), S.shape[0], S.shape[1], e0, de, float(E), _p(z), z.size,
                            _p(out))
    return out


def sample_source(case: OracleCase, h: int, j: int) -> np.ndarray:
    """(x, y, z, u, v, w, E, hit, beamlet) of the source photon of history h
    (beamlet -1 without a fluence map)."""
    out = np.zeros(9)
    if lib().or_sample_source(C.byref(case.c), int(h), int(j), _p(out)) != 0:
        raise ValueError(f"no source for history {h} (Metropolis-Hastings beamlets "
                         "not advanced that far)")
    return out


def rotate(d, mu: float, phi: float) -> np.ndarray:
    v = np.ascontiguousarray(d, dtype=np.float64).copy()
    lib().or_rotate(_p(v), float(mu), float(phi))
    return v


def tally_replay(vox, e, V: int) -> np.ndarray:
    v = np.ascontiguousarray(vox, dtype=np.int64)
    ee = np.ascontiguousarray(e, dtype=np.float32)
    T = np.zeros(V, np.int64)
    rc = lib().or_tally_replay(len(v), _p(v), _p(ee), int(V), _p(T))
    if rc != 0:
        raise ValueError("bad voxel index in deposit list")
    return T


def batch_stats(s1, s2_hi, s2_lo, nb: int):
    """(mean batch tally, variance of that mean) per voxel, in q units."""
    s1 = np.ascontiguousarray(s1, dtype=np.int64)
    V = s1.size
    mean = np.zeros(V)
    var = np.zeros(V)
    rc = lib().or_batch_stats(V, _p(s1), _p(np.ascontiguousarray(s2_hi, dtype=np.uint64)),
                              _p(np.ascontiguousarray(s2_lo, dtype=np.uint64)), int(nb),
                              _p(mean), _p(var))
    if rc != 0:
        raise ValueError("or_batch_stats failed")
    return mean, var


def dose_and_sigma(res: dict, case: OracleCase, n_hist: int):
    """Dose [Gy/history] and its standard error from the exact integer sums."""
    wl = case.wl
    nb = res["n_batches"]
    mean, var = batch_stats(res["s1"], res["s2_hi"], res["s2_lo"], nb)
    kev_to_j = 1.602176634e-16
    mass_kg = case.rho.reshape(-1).astype(np.float64) * wl.voxel_volume() * 1e-3
    scale = np.where(mass_kg > 0, kev_to_j / (Q_SCALE * mass_kg), 0.0)
    # per-history dose: (S1/N) q-units; batch-size n = N/nb
    n_per_batch = n_hist / nb
    dose = mean / n_per_batch * scale
    sd = np.sqrt(var) / n_per_batch * scale
    return dose, sd


def sigma_bar(dose, sd, rho, kind: str = "local", frac: float | None = None,
              rho_min: float = 0.05):
    """Mean relative uncertainty over the high-dose region inside the phantom
    (rho >= rho_min).  kind='paper': mean of s/D_max over D > 0.2 D_max
    (Sec. 3.1); kind='local': mean of s/D over D > 0.5 D_max."""
    inside = rho.reshape(-1) >= rho_min
    d = np.where(inside, dose, 0.0)
    dmax = d.max()
    if dmax <= 0:
        return float("inf")
    if kind == "paper":
        f = 0.2 if frac is None else frac
        m = d > f * dmax
        return float(np.mean(sd[m] / dmax))
    f = 0.5 if frac is None else frac
    m = d > f * dmax
    return float(np.mean(sd[m] / d[m]))


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
