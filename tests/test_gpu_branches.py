"""GPU paths that the workloads of the parity suite do not reach, each
against the FP64 oracle on the same random streams:

* the photon absorption energy (Sec. 3.1) -- a raised cutoff under the
  pencil beam, and the Compton-only medium with the cutoff just above the
  source energy, where every scatter ends in a cutoff deposit;
* the continuous source trajectory of Sec. 2.2.6 (n_proj = 0);
* history ids past 2^32 (the high word of the Philox counter);
* densities of -0.0 in the phantom (the majorant keeps the material);
* the recorded per-voxel maxima behind the fixed-point headroom check;
* the device-memory boundary: a phantom read from torch device tensors, work
  enqueued on a borrowed torch stream, sums read through ctd_tally_device;
* validation of the energy and batch-size rules at the boundary.
"""
import numpy as np
import pytest
import torch   # before the library loads: one HIP runtime for torch's streams and the library's

from oracle import oracle as O
from paper_1109_3266_amd import ctd as L
from paper_1109_3266_amd.session import Case
from synth import workloads as W
from tests._helpers import random_phantom
from tests.test_gpu_parity import (PAIR_MIN, _pair_histories, check_balance, gpu_run,
                                   paired_compare, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    h = L.ctd_create(0)
    yield h
    L.ctd_destroy(h)


def _table_only(wl, keep):
    """The workload's mu/rho table with every process outside `keep`
    (0 photoelectric, 1 Compton, 2 Rayleigh) set to zero."""
    t = wl.mu_rho().copy()
    for k in range(3):
        if k not in keep:
            t[:, :, k] = 0.0
    return t


def _oracle_pairs(oc, g_log, hs, batches, h0=0):
    by_h = {h: O.history(oc, h, O.bin_of_history(oc, h, batches, h0)) for h in hs}
    return _pair_histories(g_log, by_h, hs), by_h


def test_cutoff_raised_pencil_beam(ctx):
    """60 keV pencil beam into water with the absorption energy at 55 keV:
    a Compton scatter past ~80 deg leaves E' < 55 keV and ends in a cutoff
    deposit.  Both sides count the same cutoffs, histories pair event by
    event (cutoff events included), the GPU tally is the exact replay of its
    log and the balance is exact."""
    wl = W.tiny(n_histories=100_000)
    wl.e_cut = 55.0
    say("cutoff at 55 keV, tiny")
    n_log = 5000
    g = gpu_run(ctx, wl, log=(0, n_log, 200_000))
    check_balance(g, wl.n_histories)
    oc = O.OracleCase(wl)
    r = O.run(oc, threads=8, log_range=(0, n_log), log_cap=200_000)
    paired_compare(g, r)
    assert g["bal"].n_cutoff > 0 and r["n_cutoff"] > 0
    assert abs(int(g["bal"].n_cutoff) - int(r["n_cutoff"])) <= 2e-3 * r["n_cutoff"] + 3
    gev = g["log"]
    assert np.any(gev["type"] == O.EV_CUTOFF)
    # the cutoff deposits E' < e_cut, and E' > E/2 > 27.5 keV
    cut = gev[gev["type"] == O.EV_CUTOFF]
    assert np.all((cut["e"] < 55.0) & (cut["e"] > 27.5))
    oev = r["log"]
    by_h = {h: oev[oev["h"] == h] for h in range(n_log)}
    with_cut = [h for h in range(n_log) if np.any(by_h[h]["type"] == O.EV_CUTOFF)]
    assert len(with_cut) > 50
    frac = _pair_histories(gev, by_h, range(n_log))
    frac_cut = _pair_histories(gev, by_h, with_cut)
    say(f"pairing {frac:.4f}, histories with a cutoff {frac_cut:.4f} ({len(with_cut)})")
    assert frac >= PAIR_MIN and frac_cut >= PAIR_MIN
    # the full log replays to the tally of those histories
    wl_small = W.tiny(n_histories=n_log)
    wl_small.e_cut = 55.0
    g2 = gpu_run(ctx, wl_small, n_batches=2, log=(0, n_log, 200_000))
    dep = g2["log"][np.isin(g2["log"]["type"], [1, 2, 4])]
    assert np.array_equal(O.tally_replay(dep["vox"], dep["e"], wl.n_voxels), g2["s1"])


def test_cutoff_compton_only_above_source_energy(ctx):
    """Compton-only medium with the absorption energy just above the 60 keV
    source energy: every real interaction is a Compton scatter followed by a
    cutoff deposit of E', so each interacting history deposits exactly
    60 keV and the counts of scatters and cutoffs agree on both sides."""
    wl = W.tiny(n_histories=200_000)
    wl.e_cut = 60.0 + 1e-3
    mu = _table_only(wl, [1])
    say("Compton-only, cutoff above the source energy")
    with Case(ctx, wl, mu_rho=mu) as c:
        L.ctd_debug_deposit_log(ctx, c.cs, 0, 4000, 40_000)
        c.run(wl.n_histories)
        b = c.balance()
        st = c.stats()
        s1, hi, lo, nb = c.tally()
        gev = L.ctd_read_event_log(ctx, c.cs, 40_000)
    gev = gev[np.lexsort((gev["seq"], gev["h"]))]
    assert b.q_incident == b.q_deposited + b.q_escaped
    n_int = b.n_histories - b.n_unscattered
    assert st.n_compton == st.n_real == b.n_cutoff == n_int > 0
    assert st.n_deposits == 2 * n_int
    assert b.q_deposited == n_int * 60 * 2**24          # exact, in q units
    oc = O.OracleCase(wl, mu_rho=mu)
    r = O.run(oc, threads=8)
    assert r["n_compton"] == r["n_cutoff"] == r["n_hist"] - r["n_unscattered"]
    assert abs(int(b.n_cutoff) - int(r["n_cutoff"])) <= 2e-3 * r["n_cutoff"] + 3
    paired_compare(dict(s1=s1, s2_hi=hi, s2_lo=lo, nb=nb, bal=b), r)
    bs = O.batch_sizes(wl.n_histories, wl.n_batches)
    frac, _ = _oracle_pairs(oc, gev, range(4000), bs)
    assert frac >= PAIR_MIN


def test_continuous_trajectory_paired(ctx):
    """n_proj = 0: the source angle is continuous over a 200 deg arc (the
    GPU evaluates sin/cos of the angle in hardware, the oracle in FP64)."""
    wl = W.water_cbct(scale=4, n_histories=200_000)
    wl.geometry = dict(wl.geometry, nproj=0, phi0_deg=30.0, arc_deg=200.0)
    say("continuous trajectory water_cbct/4")
    g = gpu_run(ctx, wl, log=(0, 4000, 200_000))
    check_balance(g, wl.n_histories)
    oc = O.OracleCase(wl)
    r = O.run(oc, threads=8)
    paired_compare(g, r)
    bs = O.batch_sizes(wl.n_histories, wl.n_batches)
    frac, by_h = _oracle_pairs(oc, g["log"], range(4000), bs)
    say(f"continuous trajectory pairing {frac:.4f}")
    assert frac >= PAIR_MIN
    # source angles: the GPU's first step in the phantom is where the oracle's is
    src = g["log"][g["log"]["type"] == O.EV_SOURCE]
    assert np.array_equal(src["h"], np.arange(4000))


def test_history_ids_past_2_32(ctx):
    """2^32 + 10^6 histories of the pencil beam (per-XCD tallies behind LDS
    sub-tallies, the fastest mode on it): the high counter word reaches the
    source and step streams of the last histories, which pair one by one
    with the oracle; counts and the balance carry past 2^32 exactly."""
    wl = W.tiny()
    n = 2**32 + 1_000_000
    h0, nh = 2**32 + 500_000, 1000
    say(f"{n} histories, logging {nh} from {h0}")
    with Case(ctx, wl) as c:
        L.ctd_set_tuning(ctx, c.cs, L.ctd_tuning(256, 4, 16, 1024, 2))
        L.ctd_debug_deposit_log(ctx, c.cs, h0, nh, 50_000)
        c.run(n)
        b = c.balance()
        s1 = c.tally()[0]
        st = c.stats()
        gev = L.ctd_read_event_log(ctx, c.cs, 50_000)
    gev = gev[np.lexsort((gev["seq"], gev["h"]))]
    assert b.n_histories == n and st.n_histories == n
    assert b.q_incident == n * 60 * 2**24
    assert b.q_incident == b.q_deposited + b.q_escaped
    assert int(s1.sum()) == b.q_deposited
    assert np.array_equal(np.unique(gev["h"]), np.arange(h0, h0 + nh, dtype=np.uint64))
    oc = O.OracleCase(wl)
    bs = O.batch_sizes(n, wl.n_batches)
    frac, _ = _oracle_pairs(oc, gev, range(h0, h0 + nh), bs)
    say(f"pairing past 2^32: {frac:.4f}")
    assert frac >= PAIR_MIN
    # the low id words alone would be other histories: their streams differ
    lo = O.history(oc, h0 - 2**32, 0)
    hi = O.history(oc, h0, 0)
    assert len(lo) != len(hi) or not np.array_equal(lo["vox"], hi["vox"]) or \
        not np.array_equal(lo["e"], hi["e"])


def test_negative_zero_density_keeps_majorant(ctx):
    """A bone voxel of density -0.0 (equal to 0 as a value): bone still sets
    the majorant, as the oracle's maximum by value has it, and the run pairs
    with the oracle."""
    wl = random_phantom((6, 7, 8), 2, seed=21, n_hist=40_000)  # water, bone
    rho = wl.rho.copy()
    z = np.argwhere(wl.mat == 1)[0]
    rho[tuple(z)] = -0.0
    assert np.signbit(rho[tuple(z)])
    wl.rho = rho
    say("-0.0 density")
    g = gpu_run(ctx, wl)
    oc = O.OracleCase(wl)
    assert np.array_equal(g["mu_max"], oc.mu_max)
    check_balance(g, wl.n_histories)
    paired_compare(g, O.run(oc, threads=8))


@pytest.mark.parametrize("tally_mode", [0, 1, 2])
def test_fold_records_exact_maxima(ctx, tally_mode):
    """The folds record the largest S1 and the largest high word of S2 over
    the voxels (the overflow headroom check relies on them); after several
    batches they equal the maxima of the sums read back."""
    wl = random_phantom((4, 5, 6), 3, seed=31, n_hist=60_000)
    say(f"fold maxima, tally mode {tally_mode}")
    with Case(ctx, wl, n_batches=6) as c:
        L.ctd_set_tuning(ctx, c.cs, L.ctd_tuning(256, 4, 16, 256, tally_mode))
        c.run(60_000)
        L.ctd_run_batches(ctx, c.cs, 10_000, 3)
        s1, hi, lo, nb = c.tally()
        st = c.stats()
    assert nb == 9
    assert st.max_s1 == int(s1.max()) > 0
    assert st.max_s2_hi == int(hi.max()) > 0     # T_b above 2^32 q: S2 past 2^64


def test_device_phantom_and_borrowed_stream(ctx):
    """Phantom arrays handed over as torch device tensors (CTD_MEM_DEVICE)
    and every launch enqueued on a borrowed torch stream give the host path's
    sums bit for bit; ctd_tally_device's pointers hold the same sums."""
    wl = W.head(scale=8, n_histories=200_000)
    say("device phantom on a borrowed stream")
    ref = gpu_run(ctx, wl)
    dev = torch.device("cuda:0")
    mat = torch.from_numpy(np.ascontiguousarray(wl.mat).reshape(-1)).to(dev)
    rho = torch.from_numpy(np.ascontiguousarray(wl.rho).reshape(-1)).to(dev)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()           # the uploads above are done before the library reads
    L.ctd_set_stream(ctx, stream.cuda_stream)
    try:
        with Case(ctx, wl, mat=mat, rho=rho, mem=L.CTD_MEM_DEVICE) as c:
            c.run(wl.n_histories)
            L.ctd_sync(ctx, c.cs)
            s1, hi, lo, nb = c.tally()
            p1, p2 = L.ctd_tally_device(ctx, c.cs)
            V = wl.n_voxels

            class _Dev:   # a view of the library's device arrays
                def __init__(self, ptr, shape, typestr):
                    self.__cuda_array_interface__ = dict(shape=shape, typestr=typestr,
                                                         data=(ptr, False), version=2)

            with torch.cuda.stream(stream):
                d1 = torch.as_tensor(_Dev(p1, (V,), "<i8"), device=dev).cpu().numpy()
                d2 = torch.as_tensor(_Dev(p2, (V, 2), "<u8"), device=dev).cpu().numpy()
            b = c.balance()
    finally:
        L.ctd_set_stream(ctx, None)
    assert np.array_equal(s1, ref["s1"]) and np.array_equal(hi, ref["s2_hi"])
    assert np.array_equal(lo, ref["s2_lo"]) and nb == ref["nb"]
    assert b.q_deposited == ref["bal"].q_deposited
    assert np.array_equal(d1, s1)
    assert np.array_equal(d2[:, 0], lo) and np.array_equal(d2[:, 1], hi)


def test_energy_and_batch_rules(ctx):
    """Boundary rules of the exact tally: e_cut and every spectrum bin at or
    above 1 keV (an energy grid that starts lower would otherwise admit
    them); the batch statistics (dose, sigma-bar, run to sigma-bar) refuse
    batches of unequal size."""
    low_cut = W.tiny()
    low_cut.e0, low_cut.e_cut = 0.5, 0.75
    with pytest.raises(L.CtdError) as e:
        Case(ctx, low_cut)
    assert e.value.code == L.CTD_EINVAL and "1 keV" in str(e.value)
    low_bin = W.tiny()
    low_bin.e0 = 0.5
    low_bin.spectrum_lo = np.array([0.75, 60.0])
    low_bin.spectrum_w = np.array([1.0, 1.0])
    with pytest.raises(L.CtdError) as e:
        Case(ctx, low_bin)
    assert e.value.code == L.CTD_EINVAL and "1 keV" in str(e.value)
    ok = W.tiny()
    ok.e0 = 0.5
    with Case(ctx, ok) as c:          # the same grid with a 1 keV cutoff is accepted
        c.run(1000)
        assert c.balance().n_histories == 1000
    with Case(ctx, W.tiny()) as c:
        c.run(1005)                   # 101 x 5 + 100 x 5: equal up to the remainder
        c.dose()
        L.ctd_sigma(ctx, c.cs)
        L.ctd_run_to_sigma(ctx, c.cs, 1e-9, 0.5, L.CTD_SIGMA_LOCAL, 100, 2000)
        with pytest.raises(L.CtdError) as e:
            L.ctd_run_to_sigma(ctx, c.cs, 1e-9, 0.5, L.CTD_SIGMA_LOCAL, 150, 5000)
        assert e.value.code == L.CTD_EINVAL
        c.run(3000)                   # batches of 300 next to those of 100
        for call in (lambda: c.dose(), lambda: L.ctd_sigma(ctx, c.cs)):
            with pytest.raises(L.CtdError) as e:
                call()
            assert e.value.code == L.CTD_EINVAL and "equal batches" in str(e.value)
        c.tally()                     # the exact sums stay readable
