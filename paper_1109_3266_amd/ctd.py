"""ctypes binding of libctd.so: the C ABI declared in include/ctd.h, with the
same function names.  Argument marshalling only -- every step of the
transport runs in the library's HIP kernels.  Raises if the library has not
been built (``python -m paper_1109_3266_amd.build``)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CTD_LIB_PATH selects another build of the same library (e.g. an
# instrumented variant); by default the in-tree libctd.so is loaded.
LIB_PATH = os.environ.get("CTD_LIB_PATH") or os.path.join(_HERE, "libctd.so")

CTD_OK = 0
CTD_EINVAL = -1
CTD_ENOMEM = -2
CTD_EDEVICE = -3
CTD_EOVERFLOW = -4
CTD_EBUSY = -5
CTD_ENOTFOUND = -6
CTD_ECANCELLED = -7
CTD_ESTEPS = -8
CTD_MEM_HOST = 0
CTD_MEM_DEVICE = 1
CTD_GEOM_PENCIL = 0
CTD_GEOM_CONE = 1
CTD_TRACK_GLOBAL = 0
CTD_TRACK_MACRO = 1
CTD_TRACK_AUTO = 2
CTD_SIGMA_LOCAL = 0
CTD_SIGMA_PAPER = 1

_NAMES = {v: k for k, v in dict(
    CTD_OK=0, CTD_EINVAL=-1, CTD_ENOMEM=-2, CTD_EDEVICE=-3, CTD_EOVERFLOW=-4, CTD_EBUSY=-5,
    CTD_ENOTFOUND=-6, CTD_ECANCELLED=-7, CTD_ESTEPS=-8).items()}


class ctd_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("reserved", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("dz", C.c_double), ("origin", C.c_double * 3)]


class ctd_egrid(C.Structure):
    _fields_ = [("e0", C.c_double), ("de", C.c_double), ("ne", C.c_int32),
                ("reserved", C.c_int32)]


class ctd_geom(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_proj", C.c_int32), ("src", C.c_double * 3),
                ("dir", C.c_double * 3), ("sad", C.c_double), ("iso", C.c_double * 3),
                ("a0", C.c_double), ("a1", C.c_double), ("b0", C.c_double), ("b1", C.c_double),
                ("phi0_deg", C.c_double), ("arc_deg", C.c_double), ("z_feed", C.c_double),
                ("fluence_na", C.c_int32), ("fluence_nb", C.c_int32), ("fluence", C.c_void_p),
                ("fluence_chains", C.c_int32), ("reserved_f", C.c_int32)]


class ctd_params(C.Structure):
    _fields_ = [("e_cut_kev", C.c_double), ("seed", C.c_uint64), ("n_batches", C.c_int32),
                ("rayleigh", C.c_int32), ("sigma_rho_min", C.c_double), ("tracking", C.c_int32),
                ("macro_cell", C.c_int32)]


class ctd_balance(C.Structure):
    _fields_ = [("q_incident_lo", C.c_uint64), ("q_deposited_lo", C.c_uint64),
                ("q_escaped_lo", C.c_uint64), ("q_incident_hi", C.c_uint64),
                ("q_deposited_hi", C.c_uint64), ("q_escaped_hi", C.c_uint64),
                ("n_histories", C.c_uint64), ("n_missed", C.c_uint64),
                ("n_unscattered", C.c_uint64), ("n_cutoff", C.c_uint64)]

    # exact 128-bit sums as Python ints
    @property
    def q_incident(self):
        return (self.q_incident_hi << 64) | self.q_incident_lo

    @property
    def q_deposited(self):
        return (self.q_deposited_hi << 64) | self.q_deposited_lo

    @property
    def q_escaped(self):
        return (self.q_escaped_hi << 64) | self.q_escaped_lo


class ctd_stats(C.Structure):
    _fields_ = [("sigma_local", C.c_double), ("sigma_paper", C.c_double),
                ("n_steps", C.c_uint64), ("n_real", C.c_uint64), ("n_photo", C.c_uint64),
                ("n_compton", C.c_uint64), ("n_rayleigh", C.c_uint64),
                ("n_deposits", C.c_uint64), ("n_escapes", C.c_uint64), ("n_refills", C.c_uint64),
                ("transport_ms", C.c_double), ("fold_ms", C.c_double),
                ("n_batches", C.c_uint32), ("tracking", C.c_int32),
                ("n_histories", C.c_uint64), ("n_crossings", C.c_uint64),
                ("max_s1", C.c_uint64), ("max_s2_hi", C.c_uint64)]


class ctd_tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("waves_per_simd", C.c_int32),
                ("refill_min", C.c_int32), ("chunk", C.c_int32), ("tally_mode", C.c_int32),
                ("bound_block", C.c_int32), ("defer_min", C.c_int32)]


class ctd_gamma_params(C.Structure):
    _fields_ = [("dose_tol", C.c_double), ("dta_cm", C.c_double), ("region_min", C.c_double),
                ("gamma_cap", C.c_double), ("substeps", C.c_int32), ("reserved", C.c_int32)]


class ctd_event(C.Structure):
    _fields_ = [("h", C.c_uint64), ("seq", C.c_uint32), ("k", C.c_uint32), ("type", C.c_int32),
                ("reserved", C.c_int32), ("vox", C.c_int64), ("e", C.c_float), ("E", C.c_float)]


class ctd_server_config(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("batch_histories", C.c_uint64),
                ("max_histories", C.c_uint64), ("dose_frac", C.c_double),
                ("sigma_kind", C.c_int32), ("max_active", C.c_int32), ("tuning", ctd_tuning)]


class ctd_request_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("sigma", C.c_double),
                ("histories", C.c_uint64), ("batches", C.c_uint32), ("reserved", C.c_uint32),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


class ctd_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("rounds", C.c_uint64),
                ("histories", C.c_uint64), ("phantom_loads", C.c_uint64),
                ("phantom_hits", C.c_uint64), ("evictions", C.c_uint64),
                ("resident_bytes", C.c_uint64), ("queued", C.c_uint32), ("active", C.c_uint32)]


EVENT_DTYPE = np.dtype([("h", "<u8"), ("seq", "<u4"), ("k", "<u4"), ("type", "<i4"),
                        ("reserved", "<i4"), ("vox", "<i8"), ("e", "<f4"), ("E", "<f4")])

P = C.c_void_p
PP = C.POINTER(C.c_void_p)
I32, U32, U64, F64 = C.c_int32, C.c_uint32, C.c_uint64, C.c_double

# name -> (restype, argtypes)
_SIGS = {
    "ctd_create": (I32, [PP, I32]),
    "ctd_destroy": (I32, [P]),
    "ctd_last_error": (C.c_char_p, [P]),
    "ctd_set_stream": (I32, [P, P]),
    "ctd_surface_build": (I32, [I32, I32, P, I32, P]),
    "ctd_phantom_load": (I32, [P, C.POINTER(ctd_grid), P, P, I32, PP]),
    "ctd_phantom_release": (I32, [P, P]),
    "ctd_materials_load": (I32, [P, C.POINTER(ctd_egrid), I32, P, P, I32, I32, P, I32, PP]),
    "ctd_materials_release": (I32, [P, P]),
    "ctd_spectrum_set": (I32, [P, I32, P, F64, P, PP]),
    "ctd_spectrum_release": (I32, [P, P]),
    "ctd_geometry_set": (I32, [P, C.POINTER(ctd_geom), PP]),
    "ctd_geometry_release": (I32, [P, P]),
    "ctd_case_create": (I32, [P, P, P, P, P, C.POINTER(ctd_params), PP]),
    "ctd_case_destroy": (I32, [P, P]),
    "ctd_case_reset": (I32, [P, P]),
    "ctd_set_tuning": (I32, [P, P, C.POINTER(ctd_tuning)]),
    "ctd_get_tuning": (I32, [P, P, C.POINTER(ctd_tuning)]),
    "ctd_autotune": (I32, [P, P, U64, C.POINTER(ctd_tuning)]),
    "ctd_run": (I32, [P, P, U64]),
    "ctd_run_batches": (I32, [P, P, U64, U64]),
    "ctd_run_batches_static": (I32, [P, P, U64, U64]),
    "ctd_run_to_sigma": (I32, [P, P, F64, F64, I32, U64, U64, C.POINTER(F64)]),
    "ctd_run_many": (I32, [P, P, P, I32]),
    "ctd_sync": (I32, [P, P]),
    "ctd_sigma": (I32, [P, P, I32, F64, C.POINTER(F64)]),
    "ctd_read_tally": (I32, [P, P, P, P, P, C.POINTER(U32)]),
    "ctd_read_dose": (I32, [P, P, P, P]),
    "ctd_tally_device": (I32, [P, P, PP, PP]),
    "ctd_read_balance": (I32, [P, P, C.POINTER(ctd_balance)]),
    "ctd_read_stats": (I32, [P, P, C.POINTER(ctd_stats)]),
    "ctd_read_majorant": (I32, [P, P, P]),
    "ctd_microbench": (I32, [P, I32, U64, U64, C.POINTER(F64), C.POINTER(F64)]),
    "ctd_gamma": (I32, [P, C.POINTER(ctd_grid), P, P, I32, C.POINTER(ctd_gamma_params), P,
                        C.POINTER(U64), C.POINTER(U64)]),
    "ctd_debug_deposit_log": (I32, [P, P, U64, U64, U64]),
    "ctd_debug_fail_next_round": (I32, [P]),
    "ctd_server_start": (I32, [I32, C.POINTER(ctd_server_config), PP]),
    "ctd_server_last_error": (C.c_char_p, [P]),
    "ctd_server_now": (F64, [P]),
    "ctd_server_add_phantom": (I32, [P, U64, C.POINTER(ctd_grid), P, P]),
    "ctd_server_submit": (I32, [P, U64, P, P, P, C.POINTER(ctd_params), F64, C.POINTER(U64)]),
    "ctd_server_poll": (I32, [P, U64, C.POINTER(ctd_request_info)]),
    "ctd_server_wait": (I32, [P, U64, C.POINTER(ctd_request_info)]),
    "ctd_server_read_tally": (I32, [P, U64, U64, P, P, P, C.POINTER(U32)]),
    "ctd_server_release": (I32, [P, U64]),
    "ctd_server_cancel": (I32, [P, U64]),
    "ctd_server_read_stats": (I32, [P, C.POINTER(ctd_server_stats)]),
    "ctd_server_stop": (I32, [P]),
    "ctd_read_event_log": (I32, [P, P, P, U64, C.POINTER(U64)]),
}

_lib = None


def lib():
    """The loaded libctd.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1109_3266_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class CtdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(rc: int, ctx=None) -> None:
    if rc != CTD_OK:
        msg = ctd_last_error(ctx) if ctx else ""
        raise CtdError(rc, msg)


def ptr(a) -> C.c_void_p:
    """Host numpy array or device tensor (``data_ptr``) as a void pointer."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    if a is None:
        return None
    return C.c_void_p(int(a))


# ---- thin wrappers, one per C entry point (same names) ----

def ctd_create(device: int = 0):
    h = C.c_void_p()
    check(lib().ctd_create(C.byref(h), device))
    return h


def ctd_destroy(ctx):
    return lib().ctd_destroy(ctx)


def ctd_last_error(ctx) -> str:
    s = lib().ctd_last_error(ctx)
    return s.decode() if s else ""


def ctd_set_stream(ctx, stream_ptr: int | None):
    check(lib().ctd_set_stream(ctx, C.c_void_p(stream_ptr) if stream_ptr else None), ctx)


def ctd_surface_build(pdf: np.ndarray, n_zeta: int) -> np.ndarray:
    pdf = np.ascontiguousarray(pdf, dtype=np.float64)
    out = np.zeros((pdf.shape[0], n_zeta), dtype=np.float32)
    check(lib().ctd_surface_build(pdf.shape[0], pdf.shape[1], ptr(pdf), n_zeta, ptr(out)))
    return out


def ctd_phantom_load(ctx, grid: ctd_grid, mat, rho, mem: int = CTD_MEM_HOST):
    h = C.c_void_p()
    check(lib().ctd_phantom_load(ctx, C.byref(grid), ptr(mat), ptr(rho), mem, C.byref(h)), ctx)
    return h


def ctd_phantom_release(ctx, ph):
    check(lib().ctd_phantom_release(ctx, ph), ctx)


def ctd_materials_load(ctx, eg: ctd_egrid, mu_rho, comp, comp_per_mat, rayl):
    mu = np.ascontiguousarray(mu_rho, dtype=np.float32)
    cp = np.ascontiguousarray(comp, dtype=np.float32)
    rl = None if rayl is None else np.ascontiguousarray(rayl, dtype=np.float32)
    h = C.c_void_p()
    check(lib().ctd_materials_load(ctx, C.byref(eg), mu.shape[0], ptr(mu), ptr(cp),
                                   int(comp_per_mat), cp.shape[-1], ptr(rl) if rl is not None
                                   else None, 0 if rl is None else rl.shape[-1], C.byref(h)), ctx)
    return h


def ctd_materials_release(ctx, ms):
    check(lib().ctd_materials_release(ctx, ms), ctx)


def ctd_spectrum_set(ctx, e_lo, width, weight):
    lo = np.ascontiguousarray(e_lo, dtype=np.float64)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    h = C.c_void_p()
    check(lib().ctd_spectrum_set(ctx, len(lo), ptr(lo), float(width), ptr(w), C.byref(h)), ctx)
    return h


def ctd_spectrum_release(ctx, sp):
    check(lib().ctd_spectrum_release(ctx, sp), ctx)


def ctd_geometry_set(ctx, g: ctd_geom):
    h = C.c_void_p()
    check(lib().ctd_geometry_set(ctx, C.byref(g), C.byref(h)), ctx)
    return h


def ctd_geometry_release(ctx, geo):
    check(lib().ctd_geometry_release(ctx, geo), ctx)


def ctd_case_create(ctx, ph, ms, sp, geo, p: ctd_params):
    h = C.c_void_p()
    check(lib().ctd_case_create(ctx, ph, ms, sp, geo, C.byref(p), C.byref(h)), ctx)
    return h


def ctd_case_destroy(ctx, cs):
    check(lib().ctd_case_destroy(ctx, cs), ctx)


def ctd_case_reset(ctx, cs):
    check(lib().ctd_case_reset(ctx, cs), ctx)


def ctd_set_tuning(ctx, cs, t: ctd_tuning):
    check(lib().ctd_set_tuning(ctx, cs, C.byref(t)), ctx)


def ctd_get_tuning(ctx, cs) -> ctd_tuning:
    t = ctd_tuning()
    check(lib().ctd_get_tuning(ctx, cs, C.byref(t)), ctx)
    return t


def ctd_autotune(ctx, cs, trial_histories: int) -> ctd_tuning:
    t = ctd_tuning()
    check(lib().ctd_autotune(ctx, cs, int(trial_histories), C.byref(t)), ctx)
    return t


def ctd_run(ctx, cs, n: int):
    check(lib().ctd_run(ctx, cs, int(n)), ctx)


def ctd_run_batches(ctx, cs, batch_histories: int, count: int):
    check(lib().ctd_run_batches(ctx, cs, int(batch_histories), int(count)), ctx)


def ctd_run_batches_static(ctx, cs, batch_histories: int, count: int):
    check(lib().ctd_run_batches_static(ctx, cs, batch_histories, count), ctx)


def ctd_run_to_sigma(ctx, cs, target, dose_frac, kind, batch_histories, max_histories) -> float:
    out = C.c_double()
    check(lib().ctd_run_to_sigma(ctx, cs, float(target), float(dose_frac), int(kind),
                                 int(batch_histories), int(max_histories), C.byref(out)), ctx)
    return out.value


def ctd_run_many(ctx, cases, ns):
    arr = (C.c_void_p * len(cases))(*[c.value if isinstance(c, C.c_void_p) else c
                                       for c in cases])
    n = np.ascontiguousarray(ns, dtype=np.uint64)
    check(lib().ctd_run_many(ctx, arr, ptr(n), len(cases)), ctx)


def ctd_sync(ctx, cs=None):
    check(lib().ctd_sync(ctx, cs), ctx)


def ctd_sigma(ctx, cs, kind=CTD_SIGMA_LOCAL, dose_frac=0.5) -> float:
    out = C.c_double()
    check(lib().ctd_sigma(ctx, cs, int(kind), float(dose_frac), C.byref(out)), ctx)
    return out.value


def ctd_read_tally(ctx, cs, V: int):
    s1 = np.zeros(V, np.int64)
    hi = np.zeros(V, np.uint64)
    lo = np.zeros(V, np.uint64)
    nb = C.c_uint32()
    check(lib().ctd_read_tally(ctx, cs, ptr(s1), ptr(hi), ptr(lo), C.byref(nb)), ctx)
    return s1, hi, lo, nb.value


def ctd_read_dose(ctx, cs, V: int):
    d = np.zeros(V)
    v = np.zeros(V)
    check(lib().ctd_read_dose(ctx, cs, ptr(d), ptr(v)), ctx)
    return d, v


def ctd_tally_device(ctx, cs):
    a, b = C.c_void_p(), C.c_void_p()
    check(lib().ctd_tally_device(ctx, cs, C.byref(a), C.byref(b)), ctx)
    return a.value, b.value


def ctd_read_balance(ctx, cs) -> ctd_balance:
    b = ctd_balance()
    check(lib().ctd_read_balance(ctx, cs, C.byref(b)), ctx)
    return b


def ctd_read_stats(ctx, cs) -> ctd_stats:
    s = ctd_stats()
    check(lib().ctd_read_stats(ctx, cs, C.byref(s)), ctx)
    return s


def ctd_read_majorant(ctx, cs, ne: int) -> np.ndarray:
    out = np.zeros(ne, np.float32)
    check(lib().ctd_read_majorant(ctx, cs, ptr(out)), ctx)
    return out


def ctd_microbench(ctx, kind: int, nbytes: int, ops: int = 0):
    """(rate, ms): kind 0 copy GB/s, 1 random atomics/s, 2 hot-spot
    atomics/s, 3 random 8-byte gathers/s."""
    r, t = C.c_double(), C.c_double()
    check(lib().ctd_microbench(ctx, int(kind), int(nbytes), int(ops), C.byref(r), C.byref(t)),
          ctx)
    return r.value, t.value


def ctd_gamma(ctx, grid: ctd_grid, ref, ev, dose_tol: float, dta_cm: float, region_min: float,
              gamma_cap: float = 2.0, substeps: int = 5, want_gamma: bool = True):
    """Gamma index of host dose arrays ev against ref on grid: returns
    (gamma [V] float32 or None, n_region, n_pass)."""
    r = np.ascontiguousarray(ref, dtype=np.float32)
    e = np.ascontiguousarray(ev, dtype=np.float32)
    V = grid.nx * grid.ny * grid.nz
    if r.size != V or e.size != V:
        raise ValueError(f"dose arrays must hold {V} voxels")
    p = ctd_gamma_params(float(dose_tol), float(dta_cm), float(region_min), float(gamma_cap),
                         int(substeps), 0)
    g = np.empty(V, np.float32) if want_gamma else None
    nr, npass = C.c_uint64(), C.c_uint64()
    check(lib().ctd_gamma(ctx, C.byref(grid), ptr(r), ptr(e), CTD_MEM_HOST, C.byref(p),
                          ptr(g) if g is not None else None, C.byref(nr), C.byref(npass)), ctx)
    return g, nr.value, npass.value


def ctd_debug_fail_next_round(ctx):
    check(lib().ctd_debug_fail_next_round(ctx), ctx)


def ctd_debug_deposit_log(ctx, cs, h0: int, nh: int, capacity: int):
    check(lib().ctd_debug_deposit_log(ctx, cs, int(h0), int(nh), int(capacity)), ctx)


def ctd_read_event_log(ctx, cs, capacity: int) -> np.ndarray:
    buf = np.zeros(max(1, capacity), dtype=EVENT_DTYPE)
    n = C.c_uint64()
    check(lib().ctd_read_event_log(ctx, cs, ptr(buf), capacity, C.byref(n)), ctx)
    if n.value > capacity:
        raise RuntimeError(f"event log overflow: {n.value} > {capacity}")
    return buf[: n.value]


# ---- serving ----

def _scheck(rc: int, sv) -> None:
    if rc != CTD_OK:
        s = lib().ctd_server_last_error(sv)
        raise CtdError(rc, s.decode() if s else "")


def ctd_server_start(device: int, cfg: ctd_server_config):
    h = C.c_void_p()
    _scheck(lib().ctd_server_start(device, C.byref(cfg), C.byref(h)), None)
    return h


def ctd_server_now(sv) -> float:
    return lib().ctd_server_now(sv)


def ctd_server_add_phantom(sv, key: int, grid: ctd_grid, mat, rho):
    m = np.ascontiguousarray(mat, dtype=np.uint8)
    r = np.ascontiguousarray(rho, dtype=np.float32)
    _scheck(lib().ctd_server_add_phantom(sv, int(key), C.byref(grid), ptr(m), ptr(r)), sv)


def ctd_server_submit(sv, key: int, ms, sp, geo, p: ctd_params, target: float) -> int:
    t = C.c_uint64()
    _scheck(lib().ctd_server_submit(sv, int(key), ms, sp, geo, C.byref(p), float(target),
                                    C.byref(t)), sv)
    return t.value


def ctd_server_poll(sv, ticket: int) -> ctd_request_info:
    info = ctd_request_info()
    _scheck(lib().ctd_server_poll(sv, int(ticket), C.byref(info)), sv)
    return info


def ctd_server_wait(sv, ticket: int):
    """(status, info): status CTD_OK, CTD_ECANCELLED or an error code."""
    info = ctd_request_info()
    rc = lib().ctd_server_wait(sv, int(ticket), C.byref(info))
    return rc, info


def ctd_server_read_tally(sv, ticket: int, V: int):
    s1 = np.zeros(V, np.int64)
    hi = np.zeros(V, np.uint64)
    lo = np.zeros(V, np.uint64)
    nb = C.c_uint32()
    _scheck(lib().ctd_server_read_tally(sv, int(ticket), int(V), ptr(s1), ptr(hi), ptr(lo),
                                        C.byref(nb)), sv)
    return s1, hi, lo, nb.value


def ctd_server_release(sv, ticket: int):
    _scheck(lib().ctd_server_release(sv, int(ticket)), sv)


def ctd_server_cancel(sv, ticket: int):
    _scheck(lib().ctd_server_cancel(sv, int(ticket)), sv)


def ctd_server_read_stats(sv) -> ctd_server_stats:
    st = ctd_server_stats()
    _scheck(lib().ctd_server_read_stats(sv, C.byref(st)), sv)
    return st


def ctd_server_stop(sv):
    return lib().ctd_server_stop(sv)


def declared_symbols(header: str | None = None) -> list:
    """Function names declared in include/ctd.h."""
    import re
    if header is None:
        header = os.path.join(os.path.dirname(_HERE), "include", "ctd.h")
    txt = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:int32_t|const char \*|double)\s*\*?\s*(ctd_\w+)\(",
                                 txt, flags=re.M)))
