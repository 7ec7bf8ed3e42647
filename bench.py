"""Benchmark: photon histories/s of the transport hot path on one MI355X.

Workload (default, the largest single-GPU configuration): the synthetic head
-- 256x256x160 voxels of 0.1 cm (10.5 M voxels, 8-byte records: the +-2 %
density noise makes every voxel distinct), nested ellipsoids of soft tissue,
cortical bone, brain, air sinuses and a lung-like insert in air; half-fan
cone beam at SAD 100 cm, 200 projections over 360 deg, 100 kVp Kramers
spectrum with 2 mm Al in 1 keV bins, Rayleigh on; Woodcock tracking against
the paper's global majorant; batches of 1e8 histories.  One step = one batch:
transport launch plus the batch fold.  Inputs are resident in device memory
before timing.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-cpu] [--quick]

Prints one JSON line (rank 0).  Extra legs (the cone-beam water cylinder,
time to 1 % sigma, batched engine vs per-case runs, serving, the model
variants and the gamma tool) are included unless --quick.

    python bench.py --summarize-counters [--workload W]

turns the rocprofv3 counter runs listed in the counter summary's "commands"
(written under gpurun_out/) into profiles/k_transport_<W>_pmc.json.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photon histories/s + time-to-1%-σ dose; batched serving p50/p99 latency"
# main-leg workloads (the benchmark is water_cbct; the others serve profiling)
WORKLOADS = {
    "water_cbct": "water_cbct_128x128x100_cyl30cm_120kVp_cbct360",
    "tiny": "water_cube_32cube_0.5cm_60keV_pencil",
    "head": "head_256x256x160_0.1cm_100kVp_halffan200",
    "head_helical": "head_256x256x160_0.1cm_120kVp_helical6turns_pitch1",
    "water_box_bowtie": "water_box_50cube_0.4cm_125kVp_bowtie128x96",
}
BATCH = 100_000_000
PEAK_LANE_OPS = 256 * 64 * 2.4e9      # 256 CUs x 64 lanes/clk x 2.4 GHz (non-packed)

# Algorithmic 32-bit lane operations per unit of work (counted from the kernel's
# arithmetic; the roofline figure divides their sum by the launch time).  A
# Philox4x32-10 block is 100; with the global majorant a step and a scatter
# each take a pair of its four words (half a block), with MACRO tracking a
# flight takes a block whose other words also serve its scatter.
OPS_STEP = 82        # half a Philox block 50, 2 uniforms 6, free path 2, move 3,
                     # inside 6, voxel index 5, two table lerps + cumulative 7,
                     # selection 3
OPS_SCATTER = 96     # half a Philox block 50, 2 uniforms 6, bilinear surface 12,
                     # rotation 28
OPS_FLIGHT_MACRO = 132   # a MACRO flight: a whole block instead of half
OPS_SCATTER_MACRO = 46   # a MACRO scatter: no block of its own
OPS_COMPTON = 13     # kinematics 4, energy-grid update 7, deposit conversion 2
OPS_HISTORY = 170    # source block 100 + 4 uniforms 12, projection/source/field 12,
                     # direction 8, slab entry 30, energy-grid set-up 8


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the transport kernel's source: the part of ctd_kernels.hip
    before the set-up, fold and auxiliary kernels (its helpers, the step
    functions and k_transport).  Comment-only and blank lines and trailing //
    comments do not count as a change of the kernel."""
    p = os.path.join(ROOT, "paper_1109_3266_amd", "csrc", "ctd_kernels.hip")
    code = []
    for line in open(p, encoding="utf-8"):
        if line.startswith("// MACRO tracking set-up"):
            break
        s = line.split("//", 1)[0].rstrip()
        if s:
            code.append(s)
    return hashlib.sha256("\n".join(code).encode()).hexdigest()[:16]


# Launch configuration each workload's main leg times, as (block, waves per
# SIMD, refill_min, chunk, tally mode, bound-grid block, collision deferral);
# the committed counter summaries are taken with the same one.
TUNING_KEYS = ("block", "waves_per_simd", "refill_min", "chunk", "tally_mode", "bound_block",
               "defer_min")
PINNED_TUNING = {
    "head": (256, 5, 16, 1024, 0, 2, 16),
    "head_helical": (256, 5, 16, 1024, 0, 2, 16),
    "water_cbct": (256, 5, 16, 1024, 0, 2, 16),
    "water_box_bowtie": (256, 5, 32, 1024, 1, 2, 16),
    "tiny": (256, 4, 16, 1024, 2, 2, 16),
}


def counter_commands(workload: str) -> list:
    """rocprofv3 runs behind profiles/k_transport_<workload>_pmc.json (one
    counter group per run, repository root, output under gpurun_out/)."""
    b = (f"python -u bench.py --quick --no-cpu --workload {workload} --steps 2 --warmup 0")
    return [
        f"rocprofv3 --pmc FETCH_SIZE -f csv -d gpurun_out/pmc_{workload}_fetch -o f -- {b}",
        f"rocprofv3 --pmc WRITE_SIZE -f csv -d gpurun_out/pmc_{workload}_write -o w -- {b}",
        f"rocprofv3 --pmc VALUBusy VALUUtilization SQ_INSTS_VALU SQ_INSTS_SALU -f csv "
        f"-d gpurun_out/pmc_{workload}_valu -o v -- {b}",
        "rocprofv3 --pmc FETCH_SIZE -f csv -d gpurun_out/pmc_copy_fetch -o cf -- "
        "python -u bench.py --calibrate-copy",
        "rocprofv3 --pmc WRITE_SIZE -f csv -d gpurun_out/pmc_copy_write -o cw -- "
        "python -u bench.py --calibrate-copy",
    ]


def _pmc_rows(d: str):
    """(kernel name, counter, value) of every dispatch in a rocprofv3 csv run."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(ROOT, d, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                rows.append((r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"]),
                             r.get("Dispatch_Id", "")))
    if not rows:
        raise SystemExit(f"no counter rows under {d}")
    return rows


def summarize_counters(workload: str):
    """Write profiles/k_transport_<workload>_pmc.json from the counter runs."""
    import statistics
    # the unlogged global-majorant instances: plain steps (0) and steps
    # with collision passes (1)
    kerns = ("k_transport<false, 0,", "k_transport<false, 1,")

    def per_launch(d, name):
        v = [x for k, n, x, _ in _pmc_rows(d) if any(p in k for p in kerns) and n == name]
        return statistics.mean(v), len(v)

    names = sorted({k.split("(")[0].replace("void ctd::", "")
                    for k, n, x, _ in _pmc_rows(f"gpurun_out/pmc_{workload}_fetch")
                    if any(p in k for p in kerns)})

    def copy_scale(d, name):
        v = sorted((x for k, n, x, _ in _pmc_rows(d) if "copy" in k.lower() and n == name),
                   reverse=True)[:3]
        return float(1 << 20) / statistics.median(v)   # KiB counted per KiB moved

    fetch, n1 = per_launch(f"gpurun_out/pmc_{workload}_fetch", "FETCH_SIZE")
    write, n2 = per_launch(f"gpurun_out/pmc_{workload}_write", "WRITE_SIZE")
    fs = copy_scale("gpurun_out/pmc_copy_fetch", "FETCH_SIZE")
    ws = copy_scale("gpurun_out/pmc_copy_write", "WRITE_SIZE")
    valu = {name: per_launch(f"gpurun_out/pmc_{workload}_valu", name)[0]
            for name in ("VALUBusy", "VALUUtilization", "SQ_INSTS_VALU", "SQ_INSTS_SALU")}
    t = PINNED_TUNING[workload]
    out = dict(kernel=", ".join(names), workload=workload,
               kernel_sha=kernel_source_hash(),
               kernel_sha_covers="ctd_kernels.hip up to the MACRO set-up kernel (transport "
                                 "helpers, steps, k_transport)",
               tuning=dict(zip(TUNING_KEYS, t)),
               histories_per_launch=BATCH, launches=min(n1, n2),
               fetch_kib_per_launch=fetch, write_kib_per_launch=write,
               fetch_scale=fs, write_scale=ws,
               hbm_bytes_per_launch=(fetch * fs + write * ws) * 1024.0,
               valu=dict(valu_busy_pct=valu["VALUBusy"],
                         valu_utilization_pct=valu["VALUUtilization"],
                         sq_insts_valu_per_launch=valu["SQ_INSTS_VALU"],
                         sq_insts_salu_per_launch=valu["SQ_INSTS_SALU"]),
               commands=counter_commands(workload))
    p = os.path.join(ROOT, "profiles", f"k_transport_{workload}_pmc.json")
    with open(p, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def load_counters(workload: str, tuning=None):
    """The committed rocprofv3 counter summary of the transport kernel on
    this workload, if it was taken on the current kernel source and with the
    launch configuration being timed; else None."""
    p = os.path.join(ROOT, "profiles", f"k_transport_{workload}_pmc.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_sha") != kernel_source_hash():
        return None
    if tuning is not None and "tuning" in d:
        if any(getattr(tuning, k) != d["tuning"][k] for k in TUNING_KEYS):
            return None
    return d


def load_traffic(workload: str, launch_histories: int, tuning=None):
    """HBM bytes per transport launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)
    from the committed counter summary, or None."""
    d = load_counters(workload, tuning)
    if d is None:
        return None
    return d["hbm_bytes_per_launch"] / d["histories_per_launch"] * launch_histories


def cpu_baseline(wl, n_hist: int | None, target_s: float = 15.0, n_batches: int = 10):
    """The FP64 CPU oracle on the host's cores; with n_hist None a pilot sizes
    the sample to about target_s seconds.  Large phantoms take few batches:
    every batch costs the oracle a pass over its per-thread tallies."""
    from oracle import oracle as O
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    threads = max(1, min(cores, 16))
    c = O.OracleCase(wl)
    adaptive = n_hist is None
    if adaptive:  # pilot; its per-batch merge makes it underestimate the rate
        n_hist = 1_000_000
    for _ in range(3):
        t0 = time.perf_counter()
        r = O.run(c, n_histories=n_hist, n_batches=n_batches, threads=threads)
        dt = time.perf_counter() - t0
        if not adaptive or dt >= 0.5 * target_s:
            break
        n_hist = int(min(n_hist * target_s / dt, 4e8)) // 10 * 10
    # one thread on a small sample, for the per-core rate
    n1 = max(10, int(r["n_hist"] / dt / threads * 1.0) // 10 * 10)
    t0 = time.perf_counter()
    O.run(O.OracleCase(wl), n_histories=n1, n_batches=n_batches, threads=1)
    rate1 = n1 / (time.perf_counter() - t0)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                         "")
    except OSError:
        pass
    return dict(value=r["n_hist"] / dt, unit="histories/s", cores=threads, kind="oracle",
                sample=f"{n_hist:.1e} histories of the same workload in {n_batches} batches, "
                       f"FP64 CPU oracle, {threads} threads, {dt:.1f} s",
                single_thread_histories_per_s=rate1, host_cpus=os.cpu_count(),
                cpu_model=model), r


def other_oracle_rates(threads: int):
    """Oracle histories/s on the 32^3 pencil-beam cube (1e5 histories in 10
    batches, the whole case) and on 2e7 histories of the cone-beam water
    cylinder in 10 batches."""
    from oracle import oracle as O
    from synth import workloads as W
    out = {}
    for name, wl, n, nb in [("tiny_pencil_beam", W.tiny(n_histories=100_000), 100_000, 10),
                            ("water_cbct", W.water_cbct(n_histories=20_000_000), 20_000_000,
                             10)]:
        c = O.OracleCase(wl)
        t0 = time.perf_counter()
        O.run(c, n_histories=n, n_batches=nb, threads=threads)
        dt = time.perf_counter() - t0
        out[name] = dict(histories=n, batches=nb, seconds=dt, histories_per_s=n / dt)
    return out


def batched_leg(ctx, L, W, Case, tuning, torch, hist_scale, tracking=None):
    """48 uneven cases: each run alone back to back (plain per-case launches)
    vs one batched launch per round over all cases; results must match.
    tracking: None (each case's own, the global majorant) or a CTD_TRACK_*
    mode for every case on both sides."""
    import numpy as np
    log("batched: generating 48 cases")
    cases = W.batched(hist_scale=hist_scale)
    objs = [Case(ctx, wl, tracking=tracking) for wl in cases]
    ns = [wl.n_histories for wl in cases]
    total = float(sum(ns))
    for o in objs:
        L.ctd_set_tuning(ctx, o.cs, tuning)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for o, n in zip(objs, ns):
        L.ctd_run(ctx, o.cs, n)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    ref = [o.tally()[0] for o in objs[:4]]
    for o in objs:
        L.ctd_case_reset(ctx, o.cs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L.ctd_run_many(ctx, [o.cs for o in objs], ns)
    torch.cuda.synchronize()
    t_many = time.perf_counter() - t0
    same = all(np.array_equal(r, o.tally()[0]) for r, o in zip(ref, objs[:4]))
    for o in objs:
        o.close()
    log(f"batched {total / t_many:.4g} vs plain {total / t_plain:.4g} histories/s")
    return dict(cases=len(cases), histories=total, histories_per_s=total / t_many,
                plain_histories_per_s=total / t_plain, speedup=t_plain / t_many,
                identical_to_plain=bool(same))


def extensions_leg(ctx, L, W, Case, torch, tuning, n_hist: int = 200_000_000):
    """Throughput of the variants beside the plain path (macro-cell tracking,
    bound-electron Compton, helical CT, fluence-map source; each autotuned),
    the paper's Table 1 water-box
    case timed end to end as the paper times it (set-up and upload included),
    and the gamma-index kernel on a full head grid."""
    import numpy as np
    from paper_1109_3266_amd.session import grid
    out = {}

    tuned = {}

    def timed_run(key, wl, n, **kw):
        with Case(ctx, wl, **kw) as c:
            # each variant gets its own launch configuration (tally copies pay
            # off where deposits concentrate); tuning never changes results
            t = L.ctd_autotune(ctx, c.cs, 10_000_000)
            tuned[key] = t
            L.ctd_run(ctx, c.cs, 10_000_000)          # warm
            L.ctd_case_reset(ctx, c.cs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L.ctd_run(ctx, c.cs, n)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = L.ctd_read_stats(ctx, c.cs)
            return dict(histories_per_s=n / dt, steps_per_history=st.n_steps / n,
                        tuning={k: getattr(t, k) for k in TUNING_KEYS},
                        deposits_per_history=st.n_deposits / n,
                        crossings_per_history=st.n_crossings / n,
                        sigma_paper=L.ctd_sigma(ctx, c.cs, L.CTD_SIGMA_PAPER, 0.2))

    from dataclasses import replace
    hw = W.head()
    bow = W.water_box_bowtie()
    bow_mh = W.water_box_bowtie()
    bow_mh.geometry["fluence_chains"] = 1 << 18
    macro = dict(tracking=L.CTD_TRACK_MACRO)
    for name, mk, kw in [("head_macro_tracking", lambda: hw, macro),
                         ("head_bound_electron_compton", lambda: replace(hw, compton="wh"), {}),
                         ("head_helical", lambda: W.head_helical(), {}),
                         ("head_helical_macro_tracking", lambda: W.head_helical(), macro),
                         ("water_box_bowtie", lambda: bow, {}),
                         ("water_box_bowtie_metropolis_hastings", lambda: bow_mh, {})]:
        log(f"extensions: {name}")
        out[name] = timed_run(name, mk(), n_hist, **kw)

    # tally contention: the pencil beam into the 32^3 water cube concentrates
    # deposits on the beam axis; one shared tally, one copy per XCD, and the
    # copies behind per-wave LDS sub-tallies
    tw = W.tiny(n_histories=n_hist)
    modes = {}
    for tm in (0, 1, 2):
        with Case(ctx, tw) as c:
            try:
                L.ctd_set_tuning(ctx, c.cs, L.ctd_tuning(256, 4, 16, 1024, tm))
            except L.CtdError:
                continue          # no per-XCD tallies on this device
            L.ctd_run(ctx, c.cs, 10_000_000)
            L.ctd_case_reset(ctx, c.cs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L.ctd_run(ctx, c.cs, n_hist)
            torch.cuda.synchronize()
            modes[f"tally_mode_{tm}"] = n_hist / (time.perf_counter() - t0)
    out["tiny_pencil_beam_histories_per_s"] = modes

    # the head to 1 % sigma (local, D > 0.5 D_max), batches of 1e8, with
    # macro-cell majorants (the global majorant's is the main leg's)
    for name, kw, key in [("head_time_to_1pct_sigma_macro_tracking", macro,
                           "head_macro_tracking")]:
        log(f"extensions: {name}")
        with Case(ctx, hw, **kw) as c:
            L.ctd_set_tuning(ctx, c.cs, tuned.get(key, tuning))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sig = L.ctd_run_to_sigma(ctx, c.cs, 0.01, 0.5, L.CTD_SIGMA_LOCAL, 100_000_000,
                                     200_000_000_000)
            st = L.ctd_read_stats(ctx, c.cs)
            out[name] = dict(seconds=time.perf_counter() - t0, sigma_local=sig,
                             histories=st.n_histories)

    # Table 1 water phantom: 2.5e8 histories in 10 batches, T from host
    # inputs to the dose on the host (the paper includes initialisation)
    wl = W.water_box_bowtie()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with Case(ctx, wl) as c:
        L.ctd_set_tuning(ctx, c.cs, tuned.get("water_box_bowtie", tuning))
        L.ctd_run(ctx, c.cs, wl.n_histories)
        dose, _ = c.dose()
        T = time.perf_counter() - t0
        sig = L.ctd_sigma(ctx, c.cs, L.CTD_SIGMA_PAPER, 0.2)
    out["table1_water_bowtie"] = dict(
        histories=wl.n_histories, seconds_end_to_end=T, sigma_paper=sig,
        efficiency_1_over_sigma2_T=1.0 / (sig * sig * T),
        paper_context="gCTD Table 1 water phantom: 2.5e8 histories, 6.95 s, sigma 0.64 %, "
                      "Tesla C2050 (efficiency 1/(sigma^2 T) = 3.5e3 /s)")

    # gamma index (2 %, 2 mm, D > 20 % D_max) between two independent runs:
    # the head on 0.4 cm voxels with 2.5e8 histories each (the paper's Zubal
    # resolution and history count), and the tool's speed on the full head grid
    def two_doses(wl, n):
        doses = []
        for seed in (3, 13):
            with Case(ctx, wl, seed=seed) as c:
                L.ctd_set_tuning(ctx, c.cs, tuning)
                L.ctd_run(ctx, c.cs, n)
                doses.append(c.dose()[0].astype(np.float32))
        return doses

    def gamma(wl, doses):
        dmax = float(doses[0].max())
        L.ctd_gamma(ctx, grid(wl), doses[0], doses[1], 0.02 * dmax, 0.2, 0.2 * dmax)  # warm
        t0 = time.perf_counter()
        _, nr, npass = L.ctd_gamma(ctx, grid(wl), doses[0], doses[1], 0.02 * dmax, 0.2,
                                   0.2 * dmax, want_gamma=False)
        return dict(voxels=wl.n_voxels, region_voxels=nr, pass_rate=npass / max(nr, 1),
                    seconds=time.perf_counter() - t0)

    log("extensions: gamma index")
    h4 = W.head(scale=4)
    out["gamma_head_0p4cm"] = dict(gamma(h4, two_doses(h4, 250_000_000)),
                                   note="two independent 2.5e8-history runs (seeds 3, 13)")
    out["gamma_head_full_grid"] = dict(gamma(hw, two_doses(hw, 1_000_000_000)),
                                       note="two independent 1e9-history runs; time includes "
                                            "the host-to-device copy of both doses")
    return out


def _wait_all(L, sv, tickets, n: int):
    """Block until all n submitted requests have finished, printing progress."""
    last = time.time()
    while True:
        done = sum(1 for t in tickets if t is not None and L.ctd_server_poll(sv, t).state >= 2)
        if done == n:
            return
        if time.time() - last > 20:
            log(f"serving: {done}/{n} requests finished")
            last = time.time()
        time.sleep(0.2)


def serving_leg(ctx, L, W, torch, n_req: int, rate_hz: float = 2.0,
                batch: int = 10_000_000, max_h: int = 300_000_000_000, tracking=None,
                max_active: int = 64, detail: bool = False, warmup_req: int = 0):
    """Poisson stream of run-to-1%-sigma requests from the batched case
    distribution.  Baseline: the same requests run one at a time in arrival
    order (FIFO), latencies from the measured service times and the trace; a
    service time covers what the server does per request (phantom load from
    host arrays, case creation, the run, the exact sums back to the host,
    freeing), the material set, spectrum and geometry being built beforehand
    in both.  Served: the continuous-batching server fed in real time.
    tracking as in batched_leg, for the solo runs and the served requests.
    Latency percentiles leave out the first warmup_req requests (they still
    run and load the queue)."""
    import threading

    import numpy as np

    from paper_1109_3266_amd.session import Inputs, grid, params

    arrivals, seeds = W.serving_trace(200, rate_hz, 5005)
    arrivals = arrivals[:n_req]
    log(f"serving: generating {n_req} requests")
    wls = [W.serving_request(seeds[i], i) for i in range(n_req)]
    service, hist_plain, ref = [], 0, {}
    inputs = [Inputs(ctx, wl) for wl in wls]
    for i, wl in enumerate(wls):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ph = L.ctd_phantom_load(ctx, grid(wl), wl.mat, wl.rho)
        cs = L.ctd_case_create(ctx, ph, inputs[i].ms, inputs[i].sp, inputs[i].geo,
                               params(wl, tracking=tracking))
        L.ctd_run_to_sigma(ctx, cs, 0.01, 0.5, L.CTD_SIGMA_LOCAL, batch, max_h)
        s1 = L.ctd_read_tally(ctx, cs, wl.n_voxels)[0]
        t1 = time.perf_counter()
        hist_plain += L.ctd_read_stats(ctx, cs).n_histories   # not timed
        t2 = time.perf_counter()
        L.ctd_case_destroy(ctx, cs)
        L.ctd_phantom_release(ctx, ph)
        torch.cuda.synchronize()
        service.append((t1 - t0) + (time.perf_counter() - t2))
        if i < 3:
            ref[i] = s1
        if (i + 1) % 10 == 0:
            log(f"serving: {i + 1}/{n_req} FIFO service times measured")
    end, lat_plain = 0.0, []
    for a, sv_t in zip(arrivals, service):
        end = max(end, a) + sv_t
        lat_plain.append(end - a)
    makespan_plain = end - arrivals[0]
    log(f"serving: FIFO plain p50 {np.percentile(lat_plain, 50):.2f} s")

    cfg = L.ctd_server_config()
    cfg.hbm_budget_bytes = 64 << 30
    cfg.batch_histories = batch
    cfg.max_histories = max_h
    cfg.dose_frac = 0.5
    cfg.sigma_kind = L.CTD_SIGMA_LOCAL
    cfg.max_active = max_active
    sv = L.ctd_server_start(0, cfg)
    try:
        for i, wl in enumerate(wls):
            L.ctd_server_add_phantom(sv, i, grid(wl), wl.mat, wl.rho)
        tickets = [None] * n_req
        t_base = L.ctd_server_now(sv) + 0.05

        def feed():
            for i in range(n_req):
                while L.ctd_server_now(sv) < t_base + arrivals[i]:
                    time.sleep(0.001)
                tickets[i] = L.ctd_server_submit(sv, i, inputs[i].ms, inputs[i].sp,
                                                 inputs[i].geo,
                                                 params(wls[i], tracking=tracking), 0.01)

        th = threading.Thread(target=feed)
        th.start()
        th.join()
        _wait_all(L, sv, tickets, n_req)
        infos = [L.ctd_server_wait(sv, t)[1] for t in tickets]
        same = all(np.array_equal(ref[i], L.ctd_server_read_tally(sv, tickets[i],
                                                                  wls[i].n_voxels)[0])
                   for i in ref)
        st = L.ctd_server_read_stats(sv)
    finally:
        L.ctd_server_stop(sv)
        for inp in inputs:
            inp.close()
    lat = [x.t_done - x.t_submit for x in infos]
    hist = sum(x.histories for x in infos)
    w = min(warmup_req, n_req - 1)
    lat_w, lat_plain_w = lat[w:], lat_plain[w:]
    per_request = dict(arrival_s=[float(a) for a in arrivals], service_s=service,
                       fifo_latency_s=lat_plain, served_latency_s=lat,
                       served_admit_s=[x.t_admit - x.t_submit for x in infos]) if detail else None
    makespan = max(x.t_done for x in infos) - min(x.t_submit for x in infos)
    service_rate = n_req / sum(service)
    log(f"serving: served p50 {np.percentile(lat_w, 50):.2f} s, {hist / makespan:.4g} hist/s")
    return dict(requests=n_req,
                trace=(f"{n_req} of the 200 requests of the Poisson trace" if n_req < 200 else
                       "the 200-request Poisson trace"),
                warmup_requests=w, arrival_rate_hz=rate_hz, sigma_target=0.01,
                batch_histories=batch, max_active=max_active,
                p50_s=float(np.percentile(lat_w, 50)), p99_s=float(np.percentile(lat_w, 99)),
                histories_per_s=hist / makespan,
                plain_fifo_p50_s=float(np.percentile(lat_plain_w, 50)),
                plain_fifo_p99_s=float(np.percentile(lat_plain_w, 99)),
                plain_histories_per_s=hist_plain / makespan_plain,
                mean_service_s=float(np.mean(service)),
                single_gpu_service_rate_hz=service_rate,
                queue_stable=bool(service_rate > rate_hz),
                note=("offered load exceeds one GPU (service rate < arrival rate): the queue "
                      "is unstable; latencies are for this finite trace, not a steady state")
                if service_rate <= rate_hz else "",
                identical_to_plain=bool(same), rounds=st.rounds,
                phantom_loads=st.phantom_loads,
                **({"per_request": per_request} if detail else {}))


def trace_idle(trace_dir: str):
    """GPU idle share of the served phase in a rocprofv3 kernel trace (csv)
    of a run with the serving leg: the server's host threads launch every
    dispatch from the first served round on, so the window runs from the first
    dispatch of a thread other than the one that launched the process's first
    dispatch to the last dispatch; busy time is the union of the dispatch
    intervals inside it."""
    import csv
    import glob
    import statistics
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)[0]
    rows = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Thread_Id"],
                   r["Kernel_Name"]) for r in csv.DictReader(open(f)))
    main_thread = rows[0][2]
    served = [r for r in rows if r[2] != main_thread]
    w0, w1 = served[0][0], max(e for _, e, _, _ in served)
    busy, gaps, cur = 0, [], None
    for s, e, _, _ in rows:
        if e <= w0 or s >= w1:
            continue
        s, e = max(s, w0), min(e, w1)
        if cur is None or s > cur[1]:
            if cur is not None:
                busy += cur[1] - cur[0]
                gaps.append(s - cur[1])
            cur = [s, e]
        else:
            cur[1] = max(cur[1], e)
    busy += cur[1] - cur[0]
    span = w1 - w0
    big = [g for g in gaps if g > 1_000_000]
    kinds = {}
    for _, _, _, n in served:
        k = n.split("(")[0].replace("void ", "")
        kinds[k] = kinds.get(k, 0) + 1
    print(json.dumps(dict(
        trace=f, window_s=span / 1e9, busy_s=busy / 1e9, idle_frac=(span - busy) / span,
        gaps=len(gaps), gap_sum_s=sum(gaps) / 1e9,
        gap_median_us=statistics.median(gaps) / 1e3 if gaps else 0.0,
        gaps_over_1ms=len(big), gaps_over_1ms_s=sum(big) / 1e9,
        dispatches=len(served), dispatches_by_kernel=kinds), indent=1))


def calibrate_copy():
    """A plain device copy of known size, for scaling HBM counters."""
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes_read=n, copy_bytes_written=n, launches=3)))


def transport_leg(ctx, L, W, Case, torch, stream, name: str, steps: int, warmup: int,
                  tracking=None, tune=None, tally_mode=None):
    """One case of workload `name`, timed over `steps` batches of BATCH
    histories after `warmup` untimed ones, bracketed by synchronizations and
    HIP events on the library's stream.  tune: None = the pinned launch
    configuration (the one the committed counters were taken with), "auto" =
    ctd_autotune.  Returns the leg's figures, including the roofline of its
    transport kernel."""
    log(f"building {name} workload")
    wl = W.by_name(name)
    tracking = L.CTD_TRACK_GLOBAL if tracking is None else tracking
    case = Case(ctx, wl, tracking=tracking)
    if tune == "auto":
        tuning = L.ctd_autotune(ctx, case.cs, 20_000_000)
    else:
        tuning = L.ctd_tuning(*PINNED_TUNING[name])
        if tally_mode is not None:
            tuning.tally_mode = tally_mode
        L.ctd_set_tuning(ctx, case.cs, tuning)
    log(f"{name}: block={tuning.block} waves/simd={tuning.waves_per_simd} "
        f"refill_min={tuning.refill_min} chunk={tuning.chunk} tally_mode={tuning.tally_mode} "
        f"bound_block={tuning.bound_block} defer_min={tuning.defer_min}")
    L.ctd_run_batches(ctx, case.cs, BATCH, warmup)
    torch.cuda.synchronize()
    st0 = L.ctd_read_stats(ctx, case.cs)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    L.ctd_run_batches(ctx, case.cs, BATCH, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    assert gpu_ms > 0.5 * wall * 1e3, "timing events do not bracket the library's work"
    st1 = L.ctd_read_stats(ctx, case.cs)
    bal = L.ctd_read_balance(ctx, case.cs)
    assert bal.q_incident == bal.q_deposited + bal.q_escaped, "energy balance broken"
    n_timed = steps * BATCH
    value = n_timed / wall
    log(f"{name}: {value:.4g} histories/s ({wall:.3f} s wall, {gpu_ms:.1f} ms events)")

    # roofline of the dominant kernel (k_transport): one launch = one batch;
    # launch time from the HIP events the library records around each
    # transport launch on its stream
    d_steps = st1.n_steps - st0.n_steps
    d_scat = (st1.n_compton - st0.n_compton) + (st1.n_rayleigh - st0.n_rayleigh)
    d_comp = st1.n_compton - st0.n_compton
    d_dep = st1.n_deposits - st0.n_deposits
    macro = st1.tracking == L.CTD_TRACK_MACRO
    ops = ((OPS_FLIGHT_MACRO if macro else OPS_STEP) * d_steps +
           (OPS_SCATTER_MACRO if macro else OPS_SCATTER) * d_scat + OPS_COMPTON * d_comp +
           OPS_HISTORY * n_timed)
    launch_ms = (st1.transport_ms - st0.transport_ms) / steps
    launch_s = launch_ms * 1e-3
    alu = ops / steps / launch_s
    # algorithmic bytes: a 5 B voxel read (u8 material + f32 density) per
    # Woodcock step and an 8 B tally update per deposit
    alg_bytes = 5.0 * d_steps + 8.0 * d_dep
    hbm = alg_bytes / steps / launch_s
    atom_rate = d_dep / steps / launch_s
    atom_peak, _ = L.ctd_microbench(ctx, 1, wl.n_voxels * 8, 1 << 28)
    counters = load_counters(name, tuning) if tracking == L.CTD_TRACK_GLOBAL else None
    traffic = (counters["hbm_bytes_per_launch"] / counters["histories_per_launch"] * BATCH
               if counters else None)
    valu = None
    if counters is not None and "valu" in counters:
        v = counters["valu"]
        valu = dict(busy_pct=v["valu_busy_pct"], utilization_pct=v["valu_utilization_pct"],
                    insts_per_history=v["sq_insts_valu_per_launch"] / counters["histories_per_launch"],
                    source=f"rocprofv3 VALUBusy, VALUUtilization, SQ_INSTS_VALU "
                           f"(profiles/k_transport_{name}_pmc.json)")
    fracs = dict(alu=alu / PEAK_LANE_OPS, hbm=hbm / 8e12, atomic=atom_rate / atom_peak)
    bound = max(fracs, key=fracs.get)
    unit = dict(alu="T lane-ops/s", hbm="GB/s", atomic="int64 atomics/s")[bound]
    ach = dict(alu=alu / 1e12, hbm=hbm / 1e9, atomic=atom_rate)[bound]
    peak = dict(alu=PEAK_LANE_OPS / 1e12, hbm=8000.0, atomic=atom_peak)[bound]
    roof = dict(bound=bound, achieved=ach, peak=peak, unit=unit, frac=fracs[bound],
                traffic=traffic, kernel="k_transport", launch_ms=launch_ms,
                note="bound = the largest of the ALU, HBM and atomic fractions below",
                ops_per_history=ops / n_timed, steps_per_history=d_steps / n_timed,
                deposits_per_history=d_dep / n_timed,
                alu=dict(achieved=alu / 1e12, peak=PEAK_LANE_OPS / 1e12, unit="T lane-ops/s",
                         frac=fracs["alu"],
                         peak_source="256 CUs x 64 lanes x 2.4 GHz, non-packed FP32 / int32"),
                hbm=dict(achieved=hbm / 1e9, peak=8000.0, unit="GB/s", frac=fracs["hbm"],
                         bytes_per_history=alg_bytes / n_timed,
                         counted_bytes_per_history=(traffic / BATCH if traffic else None)),
                valu=valu,
                atomic=dict(achieved=atom_rate, peak=atom_peak, unit="int64 atomics/s",
                            frac=fracs["atomic"],
                            peak_source="ctd_microbench random 64-bit atomics into a "
                                        "tally-sized array, measured in this run",
                            note="tally updates per second; with tally_mode 2 part of them "
                                 "are LDS atomics" if tuning.tally_mode == 2 else ""))
    out = dict(workload=WORKLOADS[name] + ("" if tracking == L.CTD_TRACK_GLOBAL
                                           else "_macro_tracking"),
               histories_per_s=value, wall_s=wall, ms_per_step=wall * 1e3 / steps,
               voxels=wl.n_voxels,
               tuning={k: getattr(tuning, k) for k in TUNING_KEYS},
               roofline=roof,
               transport_only_histories_per_s=n_timed / ((st1.transport_ms - st0.transport_ms)
                                                         * 1e-3),
               sigma_local=L.ctd_sigma(ctx, case.cs, L.CTD_SIGMA_LOCAL, 0.5),
               sigma_paper=L.ctd_sigma(ctx, case.cs, L.CTD_SIGMA_PAPER, 0.2))
    case.close()
    return out, wl, tuning


def time_to_sigma(ctx, L, Case, torch, wl, tuning, tracking=None):
    """Wall time of ctd_run_to_sigma to 1 % sigma-bar (local, D > 0.5 D_max)
    with batches of BATCH histories, from a fresh case."""
    c = Case(ctx, wl, tracking=tracking)
    L.ctd_set_tuning(ctx, c.cs, tuning)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sig = L.ctd_run_to_sigma(ctx, c.cs, 0.01, 0.5, L.CTD_SIGMA_LOCAL, BATCH, 200_000_000_000)
    tts = time.perf_counter() - t0
    st = L.ctd_read_stats(ctx, c.cs)
    out = dict(seconds=tts, sigma_local=sig, histories=st.n_histories, batches=st.n_batches,
               sigma_paper=L.ctd_sigma(ctx, c.cs, L.CTD_SIGMA_PAPER, 0.2))
    c.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="main leg only")
    ap.add_argument("--autotune", action="store_true",
                    help="time the main leg in the tuner's configuration instead of the pinned one")
    ap.add_argument("--cpu-histories", type=int, default=None)
    ap.add_argument("--batched-scale", type=float, default=1.0)
    ap.add_argument("--serving-requests", type=int, default=12)
    ap.add_argument("--serving-warmup", type=int, default=0,
                    help="leading requests left out of the latency percentiles")
    ap.add_argument("--serving-rate", type=float, default=2.0,
                    help="mean arrival rate of the Poisson trace [requests/s]")
    ap.add_argument("--serving-modes", default="global,auto",
                    help="tracking modes of the serving leg: global, auto or both")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--summarize-counters", action="store_true")
    ap.add_argument("--trace-idle", metavar="DIR",
                    help="GPU idle share of the served phase in a kernel trace, then exit")
    ap.add_argument("--workload", default="head", choices=sorted(WORKLOADS),
                    help="main-leg workload (default: the synthetic head)")
    ap.add_argument("--tracking", default="global", choices=["global", "macro"])
    ap.add_argument("--tally-mode", type=int, default=None, choices=[0, 1, 2],
                    help="force the main leg's tally mode (profiling)")
    ap.add_argument("--legs", default="main,water,sigma,batched,serving,extensions",
                    help="comma-separated legs to run")
    args = ap.parse_args()
    legs = set(args.legs.split(","))
    if args.quick:
        legs = {"main"}
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.summarize_counters:
        summarize_counters(args.workload)
        return
    if args.trace_idle:
        trace_idle(args.trace_idle)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the transport runs on a single MI355X "
              "(histories would shard across GPUs by id range; multi-GPU execution is not "
              "implemented).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1109_3266_amd import ctd as L
    from paper_1109_3266_amd.session import Case
    from synth import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # a dedicated stream (default priority): the library enqueues on it and
    # the timing events below are recorded on it
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    ctx = L.ctd_create(0)
    L.ctd_set_stream(ctx, stream.cuda_stream)
    tracking = L.CTD_TRACK_MACRO if args.tracking == "macro" else L.CTD_TRACK_GLOBAL

    main_leg, wl, tuning = transport_leg(ctx, L, W, Case, torch, stream, args.workload,
                                         args.steps, args.warmup, tracking,
                                         "auto" if args.autotune else None, args.tally_mode)
    value = main_leg["histories_per_s"]
    out = dict(metric=METRIC, value=value, unit="histories/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=main_leg["ms_per_step"], higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=main_leg["workload"], histories_per_step=BATCH,
                           histories_total=(args.steps + args.warmup) * BATCH,
                           voxels=main_leg["voxels"], tally="int64 fixed point 2^-24 keV",
                           tracking="Woodcock, global majorant" if tracking ==
                           L.CTD_TRACK_GLOBAL else "Woodcock, macro-cell majorants",
                           tuning=main_leg["tuning"]),
               roofline=main_leg["roofline"],
               transport_only_histories_per_s=main_leg["transport_only_histories_per_s"],
               sigma_local=main_leg["sigma_local"], sigma_paper=main_leg["sigma_paper"],
               paper_context="gCTD: ~17 s at 0.4 % mean relative sigma (s/D_max over "
                             "D > 20 % D_max), Zubal HN, 2.5e8 histories, Tesla C2050 FP32")

    if "sigma" in legs:
        log("time to 1% sigma")
        out["time_to_1pct_sigma"] = time_to_sigma(ctx, L, Case, torch, wl, tuning, tracking)
        log(f"time to 1% sigma {out['time_to_1pct_sigma']['seconds']:.2f} s")
    if "water" in legs and args.workload != "water_cbct":
        # the cone-beam water cylinder: 1-byte palette phantom, deposits spread
        # over 1.6 M voxels, bound by the memory-side tally atomics
        wleg, wwl, wtun = transport_leg(ctx, L, W, Case, torch, stream, "water_cbct",
                                        args.steps, args.warmup)
        if "sigma" in legs:
            wleg["time_to_1pct_sigma"] = time_to_sigma(ctx, L, Case, torch, wwl, wtun)
        out["water_cbct"] = wleg
    # the batched and serving legs with the paper's global majorant, then the
    # same cases with the library's automatic choice between global and
    # macro-cell majorants (both sides of each comparison use the same mode)
    if "batched" in legs:
        out["batched"] = batched_leg(ctx, L, W, Case, tuning, torch, args.batched_scale)
        out["batched_auto_tracking"] = batched_leg(ctx, L, W, Case, tuning, torch,
                                                   args.batched_scale, L.CTD_TRACK_AUTO)
    if "serving" in legs and args.serving_requests > 0:
        modes = set(args.serving_modes.split(","))
        if "global" in modes:
            out["serving"] = serving_leg(ctx, L, W, torch, args.serving_requests,
                                         rate_hz=args.serving_rate,
                                         warmup_req=args.serving_warmup)
        if "auto" in modes:
            out["serving_auto_tracking"] = serving_leg(ctx, L, W, torch, args.serving_requests,
                                                       rate_hz=args.serving_rate,
                                                       tracking=L.CTD_TRACK_AUTO,
                                                       warmup_req=args.serving_warmup)
    if "extensions" in legs:
        out["extensions"] = extensions_leg(ctx, L, W, Case, torch, tuning)

    if not args.no_cpu:
        log("cpu baseline")
        cb, _ = cpu_baseline(wl, args.cpu_histories,
                             n_batches=2 if wl.n_voxels > 4_000_000 else 10)
        tts = out.get("time_to_1pct_sigma")
        if tts:   # the oracle would need the same histories to reach 1 % sigma
            cb["time_to_1pct_sigma_s_extrapolated"] = tts["histories"] / cb["value"]
        cb["other_workloads"] = other_oracle_rates(cb["cores"])
        out["cpu_baseline"] = cb
    L.ctd_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
