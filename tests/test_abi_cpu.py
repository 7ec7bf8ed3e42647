"""The C-ABI library loads, exports every symbol include/ctd.h declares, and
its host-side FP64 surface builder agrees with the oracle's (no GPU needed)."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_1109_3266_amd import ctd as L
from synth import physics as ph
from synth import workloads as W


def test_library_exports_declared_symbols():
    syms = L.declared_symbols()
    assert len(syms) >= 30
    lib = L.lib()
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing
    # the binding wraps exactly the declared entry points
    assert set(L._SIGS) == set(syms)


def test_create_without_device_reports_edevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert L.lib().ctd_create(ctypes.byref(h), 0) == L.CTD_EDEVICE
    assert L.lib().ctd_create(None, 0) == L.CTD_EINVAL


def test_surface_builder_matches_oracle_kn():
    wl = W.tiny()
    pdf = wl.compton_pdf()
    a = L.ctd_surface_build(pdf, wl.n_zeta)
    b = O.build_surface(pdf, wl.n_zeta)
    diff = np.abs(a.astype(np.float64) - b)
    ulp = np.spacing(np.abs(b).astype(np.float32)).astype(np.float64)
    assert np.all(diff <= ulp)
    assert np.mean(a == b) > 0.999


def test_surface_builder_matches_oracle_rayleigh():
    pdf = ph.rayleigh_pdf_table("cortical_bone", W.e_nodes(), W.N_MU_RAYLEIGH)
    a = L.ctd_surface_build(pdf, W.N_ZETA)
    b = O.build_surface(pdf, W.N_ZETA)
    ulp = np.spacing(np.abs(b).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(a.astype(np.float64) - b) <= ulp)


def test_surface_builder_rejects_bad_input():
    lib = L.lib()
    pdf = np.ones((2, 5))
    out = np.zeros((2, 4), np.float32)
    assert lib.ctd_surface_build(2, 1, L.ptr(pdf), 4, L.ptr(out)) == L.CTD_EINVAL
    assert lib.ctd_surface_build(2, 5, L.ptr(pdf), 1, L.ptr(out)) == L.CTD_EINVAL
    neg = -np.ones((2, 5))
    assert lib.ctd_surface_build(2, 5, L.ptr(neg), 4, L.ptr(out)) == L.CTD_EINVAL
    zero = np.zeros((2, 5))
    assert lib.ctd_surface_build(2, 5, L.ptr(zero), 4, L.ptr(out)) == L.CTD_EINVAL
    assert lib.ctd_surface_build(2, 5, L.ptr(pdf), 4, L.ptr(out)) == L.CTD_OK
    # uniform pdf: the inverse CDF is the identity map zeta -> 2 zeta - 1
    assert np.allclose(out, np.linspace(-1, 1, 4)[None, :], atol=1e-7)


def test_server_start_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cfg = L.ctd_server_config()
    cfg.hbm_budget_bytes = 1 << 30
    cfg.batch_histories = 1000
    cfg.max_histories = 10**6
    cfg.dose_frac = 0.5
    cfg.max_active = 4
    with pytest.raises(L.CtdError) as e:
        L.ctd_server_start(0, cfg)
    assert e.value.code == L.CTD_EDEVICE
    bad = L.ctd_server_config()   # zero batch size
    h = ctypes.c_void_p()
    assert L.lib().ctd_server_start(0, ctypes.byref(bad), ctypes.byref(h)) == L.CTD_EINVAL


def test_ctypes_structs_match_the_c_layout(tmp_path):
    """Every ctypes mirror has the size and field offsets gcc gives the C
    struct of include/ctd.h (a drifted mirror would corrupt calls silently)."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = tmp_path / "abi_layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "include"),
                    os.path.join(root, "tests", "native", "abi_layout.c"), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    n = 0
    for line in out.splitlines():
        name, val = line.rsplit(" ", 1)
        if name.endswith(" size"):
            cls = getattr(L, name[:-5])
            assert ctypes.sizeof(cls) == int(val), name
        else:
            struct, field = name.split(".")
            assert getattr(getattr(L, struct), field).offset == int(val), name
        n += 1
    assert n > 40


def test_headroom_decision_branches(tmp_path):
    """The fixed-point headroom check before a batch (csrc/ctd_headroom.h):
    pessimistic bounds admit batches until S1 could pass 2^62; then the
    recorded per-voxel maxima decide, admitting while S1 + b < 2^63 and
    S2 + b^2 < 2^128 (b = n E_max 2^24, the most one batch can add to a
    voxel), and refusing without touching the bounds otherwise."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = tmp_path / "headroom"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I",
                    os.path.join(root, "paper_1109_3266_amd", "csrc"),
                    os.path.join(root, "tests", "native", "headroom_check.cpp"), "-o", str(exe)],
                   check=True)
    b = 1e8 * 120 * 2.0 ** 24                     # 2.01e17 q per batch
    k = int(2.0 ** 62 // b)                       # batches the bounds admit alone
    lines = [(1e8, 120.0, 0, 0)] * k              # stage one only
    lines += [(1e8, 120.0, 10**15, 0)]            # bounds full: exact maxima admit
    lines += [(1e8, 120.0, 0, 0)]                 # bounds restart from the maxima
    lines += [(3e9, 100.0, 0, 0)]                 # one batch of 5.0e18 > 2^62: refused
    inp = "".join(f"{n!r} {e!r} {m1} {m2}\n" for n, e, m1, m2 in lines)
    out = subprocess.run([str(exe)], input=inp, check=True, capture_output=True,
                         text=True).stdout.split("\n")
    rows = [ln.split() for ln in out if ln]
    assert all(r[0] == "0" for r in rows[:k])
    assert float(rows[k - 1][2]) == k * b and float(rows[k - 1][3]) == k * b * b
    assert rows[k][:2] == ["1", "0"]              # exact stage admitted it
    assert float(rows[k][2]) == 1e15 + b and float(rows[k][3]) == 2.0 ** 64 + b * b
    assert rows[k + 1][:2] == ["0", "-1"] and float(rows[k + 1][2]) == 1e15 + 2 * b
    assert rows[k + 2][:2] == ["2", "-1"]
    assert rows[k + 2][2:] == rows[k + 1][2:]     # a refused batch leaves the bounds
    # exact stage refusals: S1 near 2^63, and S2's high word near 2^64 while S1 is small
    for m1, m2 in [(2**63 - 2**40, 0), (10**6, 2**64 - 2**20)]:
        inp = "".join(f"1e8 120.0 {m1} {m2}\n" for _ in range(k + 1))
        rows = [ln.split() for ln in subprocess.run(
            [str(exe)], input=inp, check=True, capture_output=True, text=True).stdout.split("\n")
            if ln]
        assert rows[k][:2] == ["1", "3"]
        assert float(rows[k][2]) == k * b         # bounds unchanged


def test_round_schedule_covers_every_chunk_once(tmp_path):
    """The chunk schedule of a transport round (csrc/ctd_schedule.h and the
    claim protocol of k_transport, played on the CPU with pseudo-random
    interleavings): every workgroup starts inside its home case's range,
    the home waves add up to the grid, every chunk runs exactly once and
    every workgroup exits -- over single cases, many small cases, cases
    with no home workgroup, grids larger than the round, one-wave groups."""
    import os
    import random
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = tmp_path / "schedule"
    subprocess.run(["g++", "-std=c++17", "-O2", "-I",
                    os.path.join(root, "paper_1109_3266_amd", "csrc"),
                    os.path.join(root, "tests", "native", "schedule_check.cpp"), "-o", str(exe)],
                   check=True)
    r = random.Random(11)
    lines = ["1 1280 4 97656", "2 1280 4 1", "3 5 4 3 1 1 1 2", "4 300 1 10 20 30"]
    for s in range(300):
        nrc = r.randint(1, 48)
        lines.append(" ".join(map(str, [100 + s, r.randint(1, 400), r.choice([1, 2, 4, 8])] +
                                  [r.randint(1, 300) for _ in range(nrc)])))
    out = subprocess.run([str(exe)], input="\n".join(lines) + "\n", check=True,
                         capture_output=True, text=True).stdout.split()
    assert out == ["ok"] * len(lines), [o for o in out if o != "ok"][:3]


def test_bound_test_sums_never_reject_a_collision(tmp_path):
    """The bound grid's per-cell sums (csrc/ctd_bound.h) bound the float32
    selection sum the transport forms, at the block's level and below, for
    random tables with steep columns, edges and zero columns, energies at
    the nodes, inside the cells and at the top of the grid (where the cell
    weight can pass 1).  Also: without the 2^-20 margin, or without the
    top-cell extension, the check finds a violation."""
    import os
    import shutil
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    csrc = os.path.join(root, "paper_1109_3266_amd", "csrc")
    src = os.path.join(root, "tests", "native", "bound_check.cpp")

    def run(include, seed, trials):
        exe = tmp_path / f"bound_{seed}_{os.path.basename(include)}"
        subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-I", include, src,
                        "-o", str(exe)], check=True)
        return subprocess.run([str(exe), str(seed), str(trials)], check=True,
                              capture_output=True, text=True).stdout.split()

    for seed in (1, 7):
        out = run(csrc, seed, 300)
        assert out[0] == "ok", " ".join(out)
        assert 0.99999 < float(out[2]) < 1.0
    header = open(os.path.join(csrc, "ctd_bound.h")).read()
    for old, new in [("sum * (1.0 + 0x1p-20)", "sum"),
                     ("const double w = j + 2 == ne ? w_top : 1.0;", "const double w = 1.0;")]:
        assert old in header
        d = tmp_path / ("planted" + str(len(new)))
        d.mkdir()
        (d / "ctd_bound.h").write_text(header.replace(old, new))
        assert run(str(d), 1, 1000)[0] == "violation:"
