"""The entry point that allocates nothing, ctd_run_batches_static, against
ctd_run_batches: the same batches give the same exact sums, balance and
counters bit for bit, on two calls in a row (the second on a smaller input,
which leaves the static round table holding the first call's contents), and
when a case continues with more batches.  Its limits are refused with
CTD_EINVAL before anything is enqueued."""
import sys

import numpy as np
import pytest

from paper_1109_3266_amd import ctd as L
from paper_1109_3266_amd.session import Case
from synth import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    h = L.ctd_create(0)
    yield h
    L.ctd_destroy(h)


def _state(c):
    s1, hi, lo, nb = c.tally()
    b = c.balance()
    st = c.stats()
    return dict(s1=s1, hi=hi, lo=lo, nb=nb,
                bal=(b.q_incident, b.q_deposited, b.q_escaped, b.n_histories, b.n_missed,
                     b.n_unscattered, b.n_cutoff),
                st=(st.n_steps, st.n_real, st.n_photo, st.n_compton, st.n_rayleigh,
                    st.n_deposits, st.n_escapes, st.n_batches, st.n_histories, st.max_s1,
                    st.max_s2_hi))


def _same(a, b):
    assert a["nb"] == b["nb"]
    assert np.array_equal(a["s1"], b["s1"])
    assert np.array_equal(a["hi"], b["hi"]) and np.array_equal(a["lo"], b["lo"])
    assert a["bal"] == b["bal"]
    assert a["st"] == b["st"]


@pytest.mark.parametrize("order", ["large_then_small"])
def test_static_entry_point_matches_run_batches(ctx, order):
    # call 1: the cone-beam water cylinder (100 spectrum bins), default launch;
    # call 2: the 60 keV pencil beam (1 bin, 4x fewer histories) with LDS
    # sub-tallies in front of per-XCD tallies
    calls = [(W.water_cbct(scale=4), 200_000, 3, None),
             (W.tiny(), 50_000, 2, L.ctd_tuning(256, 4, 16, 256, 2))]
    for wl, batch, count, tuning in calls:
        say(f"static entry point: {wl.name}, {count} x {batch}")
        with Case(ctx, wl) as a, Case(ctx, wl) as b:
            if tuning is not None:
                L.ctd_set_tuning(ctx, a.cs, tuning)
                L.ctd_set_tuning(ctx, b.cs, tuning)
            L.ctd_run_batches(ctx, a.cs, batch, count)
            L.ctd_run_batches_static(ctx, b.cs, batch, count)
            ra, rb = _state(a), _state(b)
            _same(ra, rb)
            assert ra["bal"][0] == ra["bal"][1] + ra["bal"][2]
            assert ra["nb"] == count and int(ra["s1"].sum()) > 0
            # the cases continue: the next batch takes the next history ids
            L.ctd_run_batches(ctx, a.cs, batch, 1)
            L.ctd_run_batches_static(ctx, b.cs, batch, 1)
            _same(_state(a), _state(b))
            assert _state(b)["nb"] == count + 1


def test_static_entry_point_limits(ctx):
    say("static entry point limits")
    wl = W.water_cbct(scale=8, n_histories=1000)
    wl.spectrum_lo = 20.0 + 0.25 * np.arange(300)      # 300 bins of 0.25 keV
    wl.spectrum_width = 0.25
    wl.spectrum_w = np.ones(300)
    with Case(ctx, wl) as c:
        with pytest.raises(L.CtdError) as e:
            L.ctd_run_batches_static(ctx, c.cs, 10_000, 1)
        assert e.value.code == L.CTD_EINVAL and "256" in str(e.value)
        assert c.stats().n_batches == 0
    # Alg. A1 chains: the beamlet buffer must exist at the batch size first
    bow = W.water_box_bowtie(scale=5)
    bow.geometry["fluence_chains"] = 64
    with Case(ctx, bow) as a, Case(ctx, bow) as b:
        with pytest.raises(L.CtdError) as e:
            L.ctd_run_batches_static(ctx, b.cs, 20_000, 1)
        assert e.value.code == L.CTD_EINVAL
        L.ctd_run_batches(ctx, a.cs, 20_000, 3)
        L.ctd_run_batches(ctx, b.cs, 20_000, 1)
        L.ctd_run_batches_static(ctx, b.cs, 20_000, 2)
        _same(_state(a), _state(b))
    # a batch that alone could pass 2^62 q in a voxel: refused, the case unchanged
    with Case(ctx, W.tiny()) as c:
        with pytest.raises(L.CtdError) as e:
            L.ctd_run_batches_static(ctx, c.cs, 5_000_000_000, 1)
        assert e.value.code == L.CTD_EOVERFLOW
        assert c.stats().n_batches == 0 and c.stats().n_histories == 0
