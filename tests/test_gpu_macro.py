"""MACRO tracking (Woodcock tracking with a macro-cell majorant, an exact
variant of the Sec. 2.1 method) on the GPU: closed-form narrow-beam
transmission through a slab stack whose material boundaries cut through
cells, statistical agreement with the oracle's global-majorant dose (the two
consume random numbers differently, so histories are not paired), exact
energy balance and deposit-log replay, bit identity across launch
configurations, and mixed-mode batched rounds equal to solo runs."""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1109_3266_amd import ctd as L
from paper_1109_3266_amd.session import Case
from synth import workloads as W
from tests._helpers import random_phantom, slab_workload

pytestmark = pytest.mark.gpu
MACRO = L.CTD_TRACK_MACRO


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    h = L.ctd_create(0)
    yield h
    L.ctd_destroy(h)


def run(ctx, wl, n, tuning=None, log=None, **kw):
    with Case(ctx, wl, **kw) as c:
        if tuning is not None:
            L.ctd_set_tuning(ctx, c.cs, tuning)
        if log is not None:
            L.ctd_debug_deposit_log(ctx, c.cs, 0, n, log)
        c.run(n)
        s1, hi, lo, nb = c.tally()
        out = dict(s1=s1, s2_hi=hi, s2_lo=lo, nb=nb, bal=c.balance(), st=c.stats())
        if log is not None:
            out["log"] = L.ctd_read_event_log(ctx, c.cs, log)
    return out


@pytest.mark.parametrize("cell", [1, 2, 3, 8])
def test_macro_slab_transmission_closed_form(ctx, cell):
    """Unscattered transmission of a 60 keV pencil through water / bone /
    lung / air / water slabs is exp(-sum mu_i L_i) whatever the cell size."""
    layers = [("water", 1.0, 4), ("cortical_bone", 1.85, 3), ("lung", 0.3, 5),
              ("air", 0.0012, 2), ("water", 1.0, 3)]
    wl = slab_workload(layers, e_kev=60.0, n_hist=10_000_000, seed=31, nxy=4, dz=0.5)
    tab = wl.mu_rho()                     # float32, as the library uses it
    j = int(round(60.0 - wl.e0))
    mu_L = sum(r * float(np.sum(tab[wl.materials.index(m), j, :].astype(np.float64))) * n * 0.5
               for m, r, n in layers)
    p = math.exp(-mu_L)
    g = run(ctx, wl, wl.n_histories, tracking=MACRO, macro_cell=cell)
    b = g["bal"]
    frac = b.n_unscattered / wl.n_histories
    sd = math.sqrt(p * (1 - p) / wl.n_histories)
    say(f"cell {cell}: transmission {frac:.6f} vs {p:.6f} ({(frac - p) / sd:+.2f} sd), "
        f"crossings/history {g['st'].n_crossings / wl.n_histories:.2f}")
    assert abs(frac - p) < 4.5 * sd
    assert b.q_incident == b.q_deposited + b.q_escaped
    assert g["st"].n_crossings > 0


@pytest.mark.parametrize("name,kw,cell", [
    ("head", dict(n_histories=2_000_000, scale=4), 4),
    ("head_helical", dict(n_histories=2_000_000, scale=4), 8),
    ("water_cbct", dict(n_histories=2_000_000, scale=4), 8),
])
def test_macro_dose_matches_oracle(ctx, name, kw, cell):
    wl = W.by_name(name, **kw)
    say(f"macro vs oracle {name} {kw} cell {cell}")
    g = run(ctx, wl, wl.n_histories, tracking=MACRO, macro_cell=cell)
    gg = run(ctx, wl, wl.n_histories)
    r = O.run(O.OracleCase(wl), threads=16)
    m_g, v_g = O.batch_stats(g["s1"], g["s2_hi"], g["s2_lo"], g["nb"])
    m_o, v_o = O.batch_stats(r["s1"], r["s2_hi"], r["s2_lo"], r["n_batches"])
    mask = m_o > 0.1 * m_o.max()
    frac = float(np.mean(np.abs(m_g - m_o)[mask] <= 3.0 * np.sqrt(v_g + v_o)[mask]))
    rel = abs(g["bal"].q_deposited - r["q_dep"]) / r["q_dep"]
    steps_g, steps_m = gg["st"].n_steps, g["st"].n_steps
    say(f"  3-sigma {frac:.4f} over {mask.sum()} voxels, dE/E {rel:.2e}, steps/history "
        f"global {steps_g / wl.n_histories:.2f} macro {steps_m / wl.n_histories:.2f}, "
        f"crossings/history {g['st'].n_crossings / wl.n_histories:.2f}")
    assert frac >= 0.99
    assert rel < 3e-3
    b = g["bal"]
    assert b.q_incident == b.q_deposited + b.q_escaped
    assert steps_m <= steps_g
    # interaction counts agree with the global tracking statistically
    for key in ("n_compton", "n_photo"):
        a, c = getattr(g["st"], key), getattr(gg["st"], key)
        assert abs(a - c) < 5 * math.sqrt(a + c) + 5, key


def test_macro_deposit_log_replay_and_bit_identity(ctx):
    wl = random_phantom((9, 13, 11), 4, seed=12, n_hist=20_000)
    say("macro log replay and tunings")
    g = run(ctx, wl, 20_000, log=400_000, tracking=MACRO, macro_cell=3)
    ev = g["log"]
    dep = ev[np.isin(ev["type"], [1, 2, 4])]
    assert np.array_equal(O.tally_replay(dep["vox"], dep["e"], int(wl.mat.size)), g["s1"])
    ends = ev[np.isin(ev["type"], [1, 4, 5, 6])]
    assert np.array_equal(np.sort(ends["h"]), np.arange(20_000))
    outs = [run(ctx, wl, 20_000, tuning=L.ctd_tuning(*t), tracking=MACRO, macro_cell=3)
            for t in [(256, 4, 16, 256, 0), (512, 2, 64, 4096, 1), (64, 1, 1, 64, 0),
                      (256, 4, 16, 1024, 2), (64, 2, 8, 64, 2)]]
    for o in outs:
        assert np.array_equal(o["s1"], g["s1"])
        assert np.array_equal(o["s2_lo"], g["s2_lo"])
        assert o["st"].n_crossings == g["st"].n_crossings


def test_mixed_tracking_batched_round_matches_solo(ctx):
    cases = W.batched(n_cases=4, size_scale=0.2, hist_scale=1e-3)
    modes = [MACRO, L.CTD_TRACK_GLOBAL, MACRO, L.CTD_TRACK_GLOBAL]
    say("mixed tracking in one batched run")
    solo = [run(ctx, wl, wl.n_histories, tracking=m) for wl, m in zip(cases, modes)]
    objs = [Case(ctx, wl, tracking=m) for wl, m in zip(cases, modes)]
    try:
        L.ctd_run_many(ctx, [o.cs for o in objs], [wl.n_histories for wl in cases])
        for o, s in zip(objs, solo):
            s1, hi, lo, nb = o.tally()
            assert np.array_equal(s1, s["s1"]) and np.array_equal(lo, s["s2_lo"])
    finally:
        for o in objs:
            o.close()


def test_macro_parameter_errors(ctx):
    wl = W.tiny(n_histories=10)
    with pytest.raises(L.CtdError):
        Case(ctx, wl, tracking=7)
    with pytest.raises(L.CtdError):
        Case(ctx, wl, tracking=MACRO, macro_cell=65)


def test_macro_full_size_head_matches_global(ctx):
    """Full head grid, 2e8 histories each: macro-cell and global tracking
    (independent random streams in effect) agree voxel by voxel within 3
    sigma over the high-dose region and in total deposited energy."""
    wl = W.head(n_histories=200_000_000)
    say("full-size head: macro vs global")
    g = run(ctx, wl, wl.n_histories, tracking=MACRO)
    r = run(ctx, wl, wl.n_histories)
    m_g, v_g = O.batch_stats(g["s1"], g["s2_hi"], g["s2_lo"], g["nb"])
    m_r, v_r = O.batch_stats(r["s1"], r["s2_hi"], r["s2_lo"], r["nb"])
    mask = m_r > 0.5 * m_r.max()
    frac = float(np.mean(np.abs(m_g - m_r)[mask] <= 3.0 * np.sqrt(v_g + v_r)[mask]))
    rel = abs(g["bal"].q_deposited - r["bal"].q_deposited) / r["bal"].q_deposited
    say(f"  3-sigma {frac:.4f} over {mask.sum()} voxels, dE/E {rel:.2e}")
    assert frac >= 0.99 and rel < 1e-3


def test_auto_tracking_choice_and_identity(ctx):
    """CTD_TRACK_AUTO picks macro cells where a dense minority material sets
    the majorant (the head's bone, a bone-bearing request phantom) and the
    global majorant otherwise (water cylinder, tissue-only phantom), and then
    runs exactly that mode: tallies equal the explicit mode's bit for bit."""
    say("AUTO tracking")
    arrivals, seeds = W.serving_trace(200, 2.0, 5005)
    req = {i: W.serving_request(seeds[i], i, size_scale=0.3) for i in (2, 8)}
    cases = [("head", W.head(scale=4, n_histories=200_000), MACRO),
             ("water_cbct", W.water_cbct(scale=4, n_histories=200_000), L.CTD_TRACK_GLOBAL),
             ("tissue-only request", req[2], L.CTD_TRACK_GLOBAL),
             ("bone-bearing request", req[8], MACRO)]
    for name, wl, want in cases:
        assert "cortical_bone" in wl.materials or want == L.CTD_TRACK_GLOBAL, name
        a = run(ctx, wl, 200_000, tracking=L.CTD_TRACK_AUTO)
        b = run(ctx, wl, 200_000, tracking=want)
        assert a["st"].tracking == want, name
        assert b["st"].tracking == want, name
        assert np.array_equal(a["s1"], b["s1"]), name
        assert np.array_equal(a["s2_lo"], b["s2_lo"]), name
        assert (a["st"].n_crossings > 0) == (want == MACRO), name
