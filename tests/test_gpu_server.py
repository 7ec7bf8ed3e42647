"""Serving loop (continuous batching) on the GPU: each request's exact sums
equal a solo ctd_run_to_sigma with the same batch size; admission by device
footprint with resident phantoms; cancellation and error codes."""
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_1109_3266_amd import ctd as L
from paper_1109_3266_amd.session import Case, Inputs, grid, params
from synth import workloads as W
from tests.test_gpu_parity import paired_compare

pytestmark = pytest.mark.gpu

BATCH = 50_000
TARGET = 0.08
MAX_H = 20_000_000


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    h = L.ctd_create(0)
    yield h
    L.ctd_destroy(h)


def _cfg(budget=8 << 30, max_active=16, max_h=MAX_H):
    c = L.ctd_server_config()
    c.hbm_budget_bytes = budget
    c.batch_histories = BATCH
    c.max_histories = max_h
    c.dose_frac = 0.5
    c.sigma_kind = L.CTD_SIGMA_LOCAL
    c.max_active = max_active
    return c


def _requests(n, seed=77):
    rng = np.random.default_rng(seed)
    return [W.batched_case(rng, 9000 + i, f"r{i}", size_scale=0.25) for i in range(n)]


def _solo(ctx, wl, max_h=MAX_H):
    with Case(ctx, wl) as c:
        sig = L.ctd_run_to_sigma(ctx, c.cs, TARGET, 0.5, L.CTD_SIGMA_LOCAL, BATCH, max_h)
        s1, hi, lo, nb = c.tally()
    return sig, s1, hi, lo, nb


@pytest.mark.parametrize("tally_mode", [None, 2])
def test_server_results_identical_to_solo(ctx, tally_mode):
    """Each request's sums equal its solo run's; the rounds may use another
    launch configuration (here the LDS sub-tally) than the solo runs."""
    say(f"server vs solo, tally mode {tally_mode}")
    wls = _requests(5)
    # model variants ride the same rounds: macro-cell tracking, an Alg. A1
    # fluence map, bound-electron Compton, the automatic tracking choice
    wls[1].tracking = L.CTD_TRACK_MACRO
    g = wls[2].geometry
    g["fluence"] = W.bowtie_fluence(32, 24, (g["a1"] - g["a0"]) / 2, (g["b1"] - g["b0"]) / 2)
    g["fluence_chains"] = 64
    wls[3].compton = "wh"
    wls[4].tracking = L.CTD_TRACK_AUTO
    solo = [_solo(ctx, wl) for wl in wls]
    cfg = _cfg()
    if tally_mode is not None:
        cfg.tuning = L.ctd_tuning(256, 5, 16, 1024, tally_mode)
    sv = L.ctd_server_start(0, cfg)
    inputs = [Inputs(ctx, wl) for wl in wls]
    try:
        tickets = []
        for i, (wl, inp) in enumerate(zip(wls, inputs)):
            L.ctd_server_add_phantom(sv, i, grid(wl), wl.mat, wl.rho)
            tickets.append(L.ctd_server_submit(sv, i, inp.ms, inp.sp, inp.geo, params(wl),
                                               TARGET))
            time.sleep(0.01 * i)   # staggered arrivals join running rounds
        for i, (t, wl) in enumerate(zip(tickets, wls)):
            rc, info = L.ctd_server_wait(sv, t)
            assert rc == L.CTD_OK and info.state == 2
            s1, hi, lo, nb = L.ctd_server_read_tally(sv, t, wl.n_voxels)
            sig, r1, rhi, rlo, rnb = solo[i]
            assert nb == rnb and info.batches == rnb
            assert info.sigma == pytest.approx(sig, rel=0, abs=0)
            assert np.array_equal(s1, r1) and np.array_equal(hi, rhi) and np.array_equal(lo, rlo)
            assert info.t_submit <= info.t_admit <= info.t_done
            if i in (0, 2, 3):   # the global-majorant requests, against the oracle
                r = O.run(O.OracleCase(wl), batches=[BATCH] * nb, threads=8)
                b = {"s1": s1, "s2_hi": hi, "s2_lo": lo, "nb": nb,
                     "bal": type("B", (), {"q_deposited": int(s1.sum())})}
                paired_compare(b, r)
            L.ctd_server_release(sv, t)
        st = L.ctd_server_read_stats(sv)
        assert st.completed == 5 and st.rounds >= 10 and st.phantom_loads == 5
    finally:
        L.ctd_server_stop(sv)
        for inp in inputs:
            inp.close()


def test_server_admission_budget_and_resident_phantoms(ctx):
    say("server admission")
    wls = _requests(3, seed=5)
    V = max(wl.n_voxels for wl in wls)
    # room for one request on the largest phantom (tallies 32 B/voxel +
    # phantom 9 B/voxel) and little more: the third request on phantom 0
    # must evict an unused phantom to fit.  Evictions happen only when they
    # make enough room for the admission.
    sv = L.ctd_server_start(0, _cfg(budget=V * 41 + (256 << 10)))
    inputs = [Inputs(ctx, wl) for wl in wls]
    try:
        for i, wl in enumerate(wls):
            L.ctd_server_add_phantom(sv, i, grid(wl), wl.mat, wl.rho)
        # the same phantom twice in a row is served from the resident copy
        keys = [0, 0, 1, 2, 0]
        tickets = [L.ctd_server_submit(sv, k, inputs[k].ms, inputs[k].sp, inputs[k].geo,
                                       params(wls[k]), TARGET) for k in keys]
        infos = []
        for t in tickets:
            rc, info = L.ctd_server_wait(sv, t)
            assert rc == L.CTD_OK
            infos.append(info)
        st = L.ctd_server_read_stats(sv)
        assert st.completed == 5
        assert st.phantom_hits >= 1
        assert st.evictions >= 1
        assert st.active == 0 and st.queued == 0
        # identical inputs give identical results
        a = L.ctd_server_read_tally(sv, tickets[0], wls[0].n_voxels)
        b = L.ctd_server_read_tally(sv, tickets[4], wls[0].n_voxels)
        assert np.array_equal(a[0], b[0])
    finally:
        L.ctd_server_stop(sv)
        for inp in inputs:
            inp.close()


def test_server_cancel_and_errors(ctx):
    say("server cancel")
    wl = _requests(1, seed=9)[0]
    sv = L.ctd_server_start(0, _cfg(max_h=10**15))
    inp = Inputs(ctx, wl)
    try:
        L.ctd_server_add_phantom(sv, 1, grid(wl), wl.mat, wl.rho)
        with pytest.raises(L.CtdError) as e:
            L.ctd_server_submit(sv, 99, inp.ms, inp.sp, inp.geo, params(wl), TARGET)
        assert e.value.code == L.CTD_ENOTFOUND
        with pytest.raises(L.CtdError) as e:
            L.ctd_server_add_phantom(sv, 1, grid(wl), wl.mat, wl.rho)
        assert e.value.code == L.CTD_EBUSY
        t = L.ctd_server_submit(sv, 1, inp.ms, inp.sp, inp.geo, params(wl), 1e-9)
        time.sleep(0.2)
        assert L.ctd_server_poll(sv, t).state == 1   # running: the target is out of reach
        # the request holds its inputs until it finishes
        for release, h in [(L.ctd_materials_release, inp.ms), (L.ctd_spectrum_release, inp.sp),
                           (L.ctd_geometry_release, inp.geo)]:
            with pytest.raises(L.CtdError) as e:
                release(ctx, h)
            assert e.value.code == L.CTD_EBUSY
        L.ctd_server_cancel(sv, t)
        rc, info = L.ctd_server_wait(sv, t)
        assert rc == L.CTD_ECANCELLED and info.state == 3
        with pytest.raises(L.CtdError) as e:
            L.ctd_server_poll(sv, 12345)
        assert e.value.code == L.CTD_ENOTFOUND
    finally:
        L.ctd_server_stop(sv)
        inp.close()
    # a request larger than the whole budget fails with ENOMEM
    sv = L.ctd_server_start(0, _cfg(budget=1 << 20))
    inp = Inputs(ctx, wl)
    try:
        L.ctd_server_add_phantom(sv, 1, grid(wl), wl.mat, wl.rho)
        t = L.ctd_server_submit(sv, 1, inp.ms, inp.sp, inp.geo, params(wl), TARGET)
        rc, info = L.ctd_server_wait(sv, t)
        assert rc == L.CTD_ENOMEM and info.state == 4
    finally:
        L.ctd_server_stop(sv)
        inp.close()


def _resident_while_running(ctx, wl, inp):
    """(phantom bytes, phantom + case bytes) the server counts for `wl`: read
    while an out-of-reach request runs, then after cancelling it."""
    sv = L.ctd_server_start(0, _cfg(max_h=10**15))
    try:
        L.ctd_server_add_phantom(sv, 0, grid(wl), wl.mat, wl.rho)
        t = L.ctd_server_submit(sv, 0, inp.ms, inp.sp, inp.geo, params(wl), 1e-9)
        for _ in range(500):
            if L.ctd_server_poll(sv, t).state == 1:
                break
            time.sleep(0.01)
        both = L.ctd_server_read_stats(sv).resident_bytes
        L.ctd_server_cancel(sv, t)
        rc, _ = L.ctd_server_wait(sv, t)
        assert rc == L.CTD_ECANCELLED
        ph = L.ctd_server_read_stats(sv).resident_bytes
    finally:
        L.ctd_server_stop(sv)
    assert 0 < ph < both
    return ph, both


def test_server_admission_keeps_own_phantom(ctx):
    """A resident phantom is never evicted by the admission of a request on it:
    with A and B resident and room for A's tallies only once B is gone, a
    second request on A (the least recently used) evicts B and reuses A."""
    say("server eviction keeps the admitted phantom")
    rng = np.random.default_rng(31)
    wls = [W.batched_case(rng, 9100 + i, f"e{i}", size_scale=0.25) for i in range(6)]
    wls.sort(key=lambda w: w.n_voxels)
    a, b = wls[-1], wls[0]
    assert a.n_voxels > b.n_voxels
    ia, ib = Inputs(ctx, a), Inputs(ctx, b)
    try:
        pa, pca = _resident_while_running(ctx, a, ia)
        pb, pcb = _resident_while_running(ctx, b, ib)
        ca, cb = pca - pa, pcb - pb
        assert ca > cb
        delta = min(pb, ca - cb) // 2
        budget = pa + pb + ca - delta   # A + B + B's case fit; A + B + A's case do not
        assert pa + ca <= budget and pa + pb + cb <= budget < pa + pb + ca
        sv = L.ctd_server_start(0, _cfg(budget=budget))
        try:
            L.ctd_server_add_phantom(sv, 0, grid(a), a.mat, a.rho)
            L.ctd_server_add_phantom(sv, 1, grid(b), b.mat, b.rho)
            out = []
            for key, wl, inp in [(0, a, ia), (1, b, ib), (0, a, ia)]:
                t = L.ctd_server_submit(sv, key, inp.ms, inp.sp, inp.geo, params(wl), TARGET)
                rc, info = L.ctd_server_wait(sv, t)
                assert rc == L.CTD_OK, L.ctd_server_last_error(sv)
                out.append(L.ctd_server_read_tally(sv, t, wl.n_voxels))
                if key == 1:
                    with pytest.raises(L.CtdError) as e:   # arrays of the wrong size
                        L.ctd_server_read_tally(sv, t, wl.n_voxels + 1)
                    assert e.value.code == L.CTD_EINVAL
            st = L.ctd_server_read_stats(sv)
            assert (st.phantom_loads, st.phantom_hits, st.evictions) == (2, 1, 1)
            assert st.resident_bytes == pa   # only A stays resident, counted in full
            for x, y in zip(out[0], out[2]):
                assert np.array_equal(x, y)
        finally:
            L.ctd_server_stop(sv)
    finally:
        ia.close()
        ib.close()


def test_server_many_requests_with_evictions_and_cancels(ctx):
    """Sixteen requests over four phantoms with at most three admitted and a
    budget that holds the largest request with its phantom and one more
    phantom: requests queue,
    resident phantoms are evicted and reloaded, admissions and result copies
    overlap the rounds, and two requests are cancelled (one while queued,
    one while running).  Every other request ends done with the sums of its
    solo run; at the end nothing is queued, running or resident beyond the
    phantoms, and the byte count matches them."""
    say("server: 16 requests, evictions, cancels")
    rng = np.random.default_rng(23)
    base = [W.batched_case(rng, 9300 + i, f"m{i}", size_scale=0.2) for i in range(4)]
    inputs = [Inputs(ctx, wl) for wl in base]
    keys = [int(k) for k in rng.integers(0, 4, 16)]
    solo = {k: _solo(ctx, base[k], max_h=10**15) for k in set(keys)}
    # room for the largest request's tallies and phantom plus one more
    # phantom: switching between phantoms keeps evicting unused ones
    Vs = sorted(wl.n_voxels for wl in base)
    budget = 32 * Vs[-1] + (320 << 10) + 10 * (Vs[-1] + Vs[-2]) + (16 << 10)
    sv = L.ctd_server_start(0, _cfg(budget=budget, max_active=3, max_h=10**15))
    try:
        for k, wl in enumerate(base):
            L.ctd_server_add_phantom(sv, k, grid(wl), wl.mat, wl.rho)
        tickets = []
        for i, k in enumerate(keys):
            tickets.append(L.ctd_server_submit(sv, k, inputs[k].ms, inputs[k].sp,
                                               inputs[k].geo, params(base[k]), TARGET))
            if i == 3:   # out of reach: runs until cancelled
                L.ctd_server_cancel(sv, tickets[-1])
        # a request with an unreachable target, cancelled once running
        long_t = L.ctd_server_submit(sv, keys[0], inputs[keys[0]].ms, inputs[keys[0]].sp,
                                     inputs[keys[0]].geo, params(base[keys[0]]), 1e-9)
        cancel_at = time.time() + 0.5
        for i, (t, k) in enumerate(zip(tickets, keys)):
            if time.time() > cancel_at and long_t is not None:
                L.ctd_server_cancel(sv, long_t)
                long_t_done = long_t
                long_t = None
            rc, info = L.ctd_server_wait(sv, t)
            if i == 3:
                assert rc == L.CTD_ECANCELLED and info.state == 3
                continue
            assert rc == L.CTD_OK and info.state == 2, L.ctd_server_last_error(sv)
            s1, hi, lo, nb = L.ctd_server_read_tally(sv, t, base[k].n_voxels)
            sig, r1, rhi, rlo, rnb = solo[k]
            assert nb == rnb and info.sigma == pytest.approx(sig, rel=0, abs=0)
            assert np.array_equal(s1, r1) and np.array_equal(hi, rhi) and np.array_equal(lo, rlo)
            L.ctd_server_release(sv, t)
        if long_t is not None:
            L.ctd_server_cancel(sv, long_t)
            long_t_done = long_t
        rc, info = L.ctd_server_wait(sv, long_t_done)
        assert rc == L.CTD_ECANCELLED and info.state == 3
        st = L.ctd_server_read_stats(sv)
        assert st.completed == 15 and st.active == 0 and st.queued == 0
        assert st.evictions >= 1 and st.phantom_loads >= 5
        assert 0 < st.resident_bytes <= sum(9 * wl.n_voxels + wl.n_voxels // 8 +
                                            wl.n_voxels // 64 + 8192 for wl in base)
    finally:
        L.ctd_server_stop(sv)
        for inp in inputs:
            inp.close()
