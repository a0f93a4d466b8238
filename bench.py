"""Benchmark of the reacting-species D2Q9 lattice Boltzmann step on one MI355X.

Headline workload: Gray-Scott (u, v), D2Q9 BGK, 4096 x 4096 periodic, FP32
storage (the FP32 run of the 4096^2 workload: 2.4 GB of ping-pong state,
beyond the 256 MB Infinity Cache, so the step streams from HBM), tau = (1.0,
0.75), F = 0.04, k = 0.06, central 64 x 64 square with u = 0.5, v = 0.25 plus
U(-0.01, 0.01) noise (seed 0).  One "step" is one lattice time step of the
whole field (every species, every site): collide, react and stream.

Timing: W untimed warm-up steps, then windows of exactly K = --steps steps,
each bracketed by HIP events on the solver's stream and a device
synchronisation on both sides, repeated until at least five windows and one
second of timed device time; the line reports the median window (and the
spread).  --tune runs the library's autotuner first.

The roofline of the step kernel follows the algorithmic byte count per
species-site-step, 2 x 9 x sizeof(storage) (every population read once and
written once per time step), times the species-site-steps one launch
advances, over the launch duration from the same events, against the 8 TB/s
HBM peak.  A kernel that keeps several time steps on chip moves the state
through HBM once per launch, so this per-step fraction can exceed 1; the
HBM bytes it really moves per launch (hardware counters, from the committed
summary when it was taken on the current kernel sources and launch shape)
and the fraction of VALU issue slots it uses are reported beside it.

Also reported: the FP64 oracle on the host cores (a bounded sample of the
same workload), and extra legs: the 1024^2 workload (cache-resident), the
one-step kernel at 4096^2, 16-bit storage at 4096^2, the batched sweep, the
continuous-batching server at its defined load, the 16-bit storage errors,
the 64^2 FP64 decay, the rescaling study and device copies.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s
VALU_ISSUE_PEAK = 256 * 2.4e9   # wave-instructions per second: 256 CUs x 1 VALU issue per cycle per CU (4 SIMDs x 1/4)
METRIC = "MLUPS per species and % HBM roofline; batched p50/p99 solve latency"

# sources that define the multi-step kernels; a committed counter summary
# records their digest, and its figures are reported only while it matches
STEP_SOURCES = ("paper_1007_3109_amd/csrc/lbrd_device.h", "paper_1007_3109_amd/csrc/lbrd_internal.h",
                "paper_1007_3109_amd/csrc/lbrd_step_launch.h", "paper_1007_3109_amd/csrc/step_f32.hip")
TRAFFIC_SUMMARY = "profiles/pmc_gray_scott_4096_f32.txt"
ISSUE_SUMMARY = "profiles/sq_gray_scott_4096_f32.txt"


def source_digest():
    """SHA-256 of the step kernel's sources with comments and blank space
    removed, so that a change of wording alone keeps the counters valid."""
    h = hashlib.sha256()
    for rel in STEP_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def read_summary(rel):
    """key: value lines of a committed profile summary (not indented, not
    comments)."""
    path = os.path.join(ROOT, rel)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def summary_for(rel, tuning):
    """The summary's key/values when it was taken on the current kernel
    sources and this launch shape, else (None, reason)."""
    kv = read_summary(rel)
    if kv is None:
        return None, "no counter summary"
    if kv.get("source_sha256") != source_digest():
        return None, "kernel sources changed since the counters were taken"
    if kv.get("tuning") != json.dumps(tuning, sort_keys=True):
        return None, "launch shape differs from the one the counters were taken on"
    return kv, rel


def measured_traffic(tuning):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, scaled by the plain
    copy calibration) from the committed counter summary, or None with the
    reason when it was taken on other kernel sources or launch shape."""
    kv, src = summary_for(TRAFFIC_SUMMARY, tuning)
    if kv is None:
        return None, src
    return int(kv["traffic_bytes_per_launch"]), src


def measured_issue(tuning):
    """Fraction of the chip's VALU issue slots the kernel used per launch
    (SQ_ACTIVE_INST_VALU x 4 cycles / 1024 SIMDs over the launch's cycles),
    from the committed instruction-counter summary, or None with the reason."""
    kv, src = summary_for(ISSUE_SUMMARY, tuning)
    if kv is None:
        return None, src
    return float(kv["valu_issue_frac"]), src


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(nspecies, sites, storage_bytes):
    """Bytes of one time step over the lattice: every population read once and
    written once, 2 x 9 x sizeof(storage) per species-site-step."""
    return 2 * 9 * storage_bytes * nspecies * sites


STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


def time_windows(torch, s, steps, warmup, min_total_s=1.0, min_reps=5, max_reps=4000):
    """W warm-up steps, then windows of exactly `steps` steps, each between two
    HIP events on the solver's stream (torch's current stream) with the device
    synchronised on both sides, until at least `min_reps` windows and
    `min_total_s` of timed device time.  Returns the window times (s)."""
    s.step(warmup)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    wins = []
    while len(wins) < max_reps and (len(wins) < min_reps or sum(wins) < min_total_s):
        torch.cuda.synchronize()
        e0.record(st)
        s.step(steps)
        e1.record(st)
        torch.cuda.synchronize()
        wins.append(e0.elapsed_time(e1) / 1e3)
    return wins


def window_stats(wins, steps):
    w = np.array(wins)
    med = float(np.median(w))
    return med, {"windows": len(wins), "steps_per_window": steps, "median_ms": round(med * 1e3, 4),
                 "min_ms": round(float(w.min()) * 1e3, 4), "max_ms": round(float(w.max()) * 1e3, 4),
                 "spread_pct": round(float((w.max() - w.min()) / med * 100), 2),
                 "timed_s": round(float(w.sum()), 3)}


def roofline(nspecies, sites, storage, steps_per_launch, launch_s, kernel, traffic=None, traffic_src=None,
             issue=None, issue_src=None, note=None):
    """Roofline of one launch: algorithmic bytes = 2 x 9 x sizeof(storage) per
    species-site-step x the species-site-steps of one launch (N sites T)."""
    b = STORAGE_BYTES[storage]
    per_launch = algorithmic_bytes(nspecies, sites, b) * steps_per_launch
    achieved = per_launch / launch_s / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "kernel": kernel, "steps_per_launch": steps_per_launch, "launch_us": round(launch_s * 1e6, 3),
           "algorithmic_bytes_per_launch": per_launch,
           "bytes_per_species_site_step": 2 * 9 * b,
           "species_site_steps_per_launch": nspecies * sites * steps_per_launch}
    if traffic is not None:
        out["traffic_unit"] = "HBM bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE, copy-calibrated)"
        out["traffic_source"] = traffic_src
        out["hbm_measured_GBs"] = round(traffic / launch_s / 1e9, 1)
        out["hbm_measured_frac"] = round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
    elif traffic_src:
        out["traffic_null_reason"] = traffic_src
    if issue is not None:
        out["valu_issue_frac"] = issue
        out["valu_issue_source"] = issue_src
    elif issue_src:
        out["valu_issue_null_reason"] = issue_src
    if note:
        out["note"] = note
    return out


def gs_config(lbrd, workloads, n, storage):
    extra = dict(rho_ref=(1.0, 0.0)) if storage in ("f16", "bf16") else {}
    return lbrd.make_config(n, n, 2, tau=workloads.GS_TAU, storage=storage, reaction="gray_scott",
                            F=workloads.GS_F, k=workloads.GS_K, **extra)


def kernel_name(t):
    if t.fused_steps > 1 and t.march_rows > 0:
        return (f"k_stepW ({t.fused_steps} steps per launch, marching wave strips of "
                f"{64 - 2 * (t.fused_steps - 1)} columns x {t.march_rows} rows, {t.waves} waves per workgroup)")
    if t.fused_steps > 1:
        return f"k_stepT ({t.fused_steps} steps per launch, {t.tile_cols} x {t.tile_rows} tiles in LDS)"
    return "k_step (one step per launch)"


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def cpu_baseline(workloads, n, budget_s, max_steps=200):
    """The FP64 oracle on the host cores, on a bounded sample of the headline
    workload: the same n^2 Gray-Scott field, stepped in chunks of 10 until
    max_steps steps or budget_s of wall time."""
    import oracle

    rho0 = workloads.gray_scott_square(n, n, seed=0)
    f = oracle.init(rho0)
    steps = 0
    chunk = 10
    t0 = time.perf_counter()
    while steps < max_steps:
        f = oracle.run(f, chunk, list(workloads.GS_TAU), oracle.REACT_GRAY_SCOTT, F=workloads.GS_F,
                       k=workloads.GS_K)
        steps += chunk
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    del f
    mlups = 2 * n * n * steps / el / 1e6
    return {"value": round(mlups, 2), "unit": "MLUPS per species", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"Gray-Scott {n}x{n} (the headline field), FP64 oracle (C, OpenMP over rows), first {steps} "
                      f"steps from the benchmark's initial state, {el:.1f} s",
            "cpu_model": cpu_info(), "nproc": os.cpu_count(),
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def solver_leg(torch, lbrd, workloads, n, storage, steps, warmup, tune=False, fused=None, shape=None, note=None):
    """One Gray-Scott lattice, the headline timing protocol; the roofline of
    its step kernel.  `shape`: tuning fields set instead of the default."""
    cfg = gs_config(lbrd, workloads, n, storage)
    s = lbrd.Solver(cfg)
    if tune:
        s.autotune(steps=10)
    if fused is not None:
        s.set_tuning(fused_steps=fused)
    if shape is not None:
        s.set_tuning(**shape)
    s.init(workloads.gray_scott_square(n, n, seed=0))
    wins = time_windows(torch, s, steps, warmup)
    med, stats = window_stats(wins, steps)
    t = s.tuning()
    sites = n * n
    per_step = med / steps
    spl = t.fused_steps
    out = {"workload": f"gray_scott {n}x{n} {storage}", "ms_per_step": round(per_step * 1e3, 5),
           "mlups_per_species": round(2 * sites / per_step / 1e6, 1), "timing": stats,
           "roofline": roofline(2, sites, storage, spl, per_step * spl, kernel_name(t), note=note),
           "tuning": t.as_dict()}
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


def batch_cpu_baseline(workloads, insts, steps, sample_every=16, sample_steps=20):
    """The FP64 oracle on a sample of the sweep's instances (every
    `sample_every`-th, `sample_steps` steps each from its initial state),
    extrapolated to the whole sweep at the sampled rate."""
    import oracle

    work, secs = 0, 0.0
    for inst in insts[::sample_every]:
        f = oracle.init(workloads.batch_initial(inst))
        t0 = time.perf_counter()
        f = oracle.run(f, sample_steps, list(workloads.GS_TAU), oracle.REACT_GRAY_SCOTT, F=inst.F, k=inst.k)
        secs += time.perf_counter() - t0
        work += 2 * inst.side * inst.side * sample_steps
        del f
    mlups = work / secs / 1e6
    total = sum(2 * i.side * i.side for i in insts) * steps
    return {"value": round(mlups, 2), "unit": "MLUPS per species", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{len(insts[::sample_every])} of the {len(insts)} instances (every {sample_every}th), "
                      f"{sample_steps} steps each, {secs:.2f} s",
            "extrapolated_s_for_the_timed_steps": round(total / (mlups * 1e6), 1)}


def batch_leg(torch, lbrd, workloads, steps, warmup, seed=0, cpu=True):
    insts = workloads.batch_sweep(seed)
    cfgs = [lbrd.make_config(i.side, i.side, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott",
                             F=i.F, k=i.k) for i in insts]
    b = lbrd.Batch(cfgs)
    t = b.autotune(steps=14)
    for idx, inst in enumerate(insts):
        b.init(idx, workloads.batch_initial(inst))
    b.step(warmup)
    torch.cuda.synchronize()
    ms = b.time_steps(steps)
    species_sites = sum(2 * i.side * i.side for i in insts)
    mlups = species_sites * steps / (ms / 1e3) / 1e6
    spl = t.fused_steps
    launch_s = ms / 1e3 / steps * spl
    # the plain single-lattice kernel on the same instances, one after another
    solo_ms = 0.0
    solo_steps = 20
    for inst in insts:
        s = lbrd.Solver(lbrd.make_config(inst.side, inst.side, 2, tau=workloads.GS_TAU, storage="f32",
                                         reaction="gray_scott", F=inst.F, k=inst.k))
        s.set_tuning(graph_steps=0)
        s.init(workloads.batch_initial(inst))
        s.step(2)
        solo_ms += s.time_steps(solo_steps)
        s.close()
    solo_mlups = species_sites * solo_steps / (solo_ms / 1e3) / 1e6
    kname = (f"k_batch_stepW ({spl} steps per launch, marching strips of {t.march_rows} rows)" if t.march_rows > 0
             else f"k_batch_stepT ({spl} steps per launch, {t.tile_cols} x {t.tile_rows} tiles in LDS)")
    rl = roofline(1, species_sites, "f32", spl, launch_s, kname)
    out = {"workload": f"{len(insts)} Gray-Scott instances, sides {sorted(set(i.side for i in insts))}, FP32",
           "species_sites": species_sites, "steps": steps, "ms_per_step": round(ms / steps, 4),
           "mlups_per_species": round(mlups, 1), "roofline": rl, "tuning": t.as_dict(),
           "plain_kernel_one_by_one_mlups_per_species": round(solo_mlups, 1),
           "vs_plain_kernel": round(mlups / solo_mlups, 3)}
    if cpu:
        out["cpu_baseline"] = batch_cpu_baseline(workloads, insts, steps)
    b.close()
    del b
    torch.cuda.empty_cache()
    return out


def serve_leg(torch, lbrd, workloads, n_requests, pool_gb, steps_range, seed=0, rate=None, occupancy=0.8):
    """Poisson stream of mixed requests into the continuous-batching server at
    the load its configuration defines: the arrival rate keeps the mean
    resident footprint near `occupancy` of the pool.  The starting rate comes
    from a processor-sharing model (the server shares its throughput Theta
    among the resident requests; at load rho = lambda E[work] / Theta the mean
    resident footprint is rho / (1 - rho) x E[footprint x work] / E[work]),
    with the expectations over this stream's own requests and Theta from the
    plain kernel on a sample of them; while requests arrive, the rate is then
    corrected every half second, by at most 5 %, from the arena occupancy the
    server measured over the last two seconds (arrival gaps exponential at
    the current rate: a Poisson stream with a slowly varying rate).  A fixed
    `rate` disables the correction."""
    import threading

    reqs = workloads.request_stream(n_requests, 1.0, seed=seed, steps_range=steps_range)
    cfgs, inits = [], []
    for r in reqs:
        if r.reaction == "linear":
            cfg = lbrd.make_config(r.side, r.side, 1, tau=r.tau, storage=r.storage, reaction="linear", K=[[-r.K]],
                                   rho_ref=(1.0,))
        else:
            cfg = lbrd.make_config(r.side, r.side, 2, tau=r.tau, storage=r.storage, reaction="gray_scott", F=r.F,
                                   k=r.k, rho_ref=(1.0, 0.0))
        cfgs.append(cfg)
        inits.append(workloads.request_initial(r))
    work = np.array([c.nspecies * c.nx * c.ny * r.nsteps for c, r in zip(cfgs, reqs)], np.float64)
    fp = np.array([lbrd.server_footprint(c) for c in cfgs], np.float64)
    # the plain single-lattice kernel on a sample of the same requests
    solo_work, solo_s = 0, 0.0
    for i in range(0, len(reqs), max(1, len(reqs) // 12)):
        s = lbrd.Solver(cfgs[i])
        s.init(inits[i])
        n = min(reqs[i].nsteps, 400)
        s.step(2)
        solo_s += s.time_steps(n) / 1e3
        solo_work += cfgs[i].nspecies * cfgs[i].nx * cfgs[i].ny * n
        s.close()
    plain = solo_work / solo_s
    pool = pool_gb * (1 << 30)
    m = float((fp * work).sum() / work.sum())            # work-weighted mean footprint
    target = occupancy * pool
    rho = target / (target + m)
    controlled = rate is None
    rate0 = rho * plain / float(work.mean()) if controlled else rate
    lam = [rate0]
    srv = lbrd.Server(arena_bytes=int(pool), chunk_steps=500)
    tickets = [None] * len(reqs)
    gaps = np.random.default_rng([seed, 1]).exponential(1.0, size=len(reqs))

    def feeder():
        t0 = time.perf_counter()
        t_next = 0.0
        for i in range(len(reqs)):
            t_next += gaps[i] / lam[0]
            dt = t_next - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets[i] = srv.submit(cfgs[i], inits[i], reqs[i].nsteps)

    th = threading.Thread(target=feeder)
    t0 = time.perf_counter()
    st0 = srv.stats()
    th.start()
    hist = [(st0.clock_s, st0.arena_used_byte_s)]
    samples, rates = [], []
    while th.is_alive():
        th.join(0.5)
        st = srv.stats()
        samples.append((st.resident, st.queued))
        hist.append((st.clock_s, st.arena_used_byte_s))
        if controlled:
            old = [h for h in hist if h[0] <= st.clock_s - 2.0]
            if old:
                c0, b0 = old[-1]
                occ = (st.arena_used_byte_s - b0) / max(st.clock_s - c0, 1e-9) / st.arena_bytes
                # gentle: the occupancy answers a change of rate only after
                # about one residence time (seconds), so fast corrections
                # overshoot
                lam[0] *= float(np.clip((occupancy / max(occ, 0.05)) ** 0.15, 0.95, 1.05))
                rates.append(lam[0])
    st_arr = srv.stats()          # the end of the arrivals: occupancy is averaged over the arrival period
    lat = []
    for i, t in enumerate(tickets):
        srv.wait(t, 900)
        _, _, info = srv.take(t)
        lat.append(info.done_s - info.submit_s)
        if (i + 1) % 50 == 0:
            log(f"bench: serving, {i + 1} of {len(reqs)} requests done")
    makespan = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    del srv
    torch.cuda.empty_cache()
    arrival_period = st_arr.clock_s - st0.clock_s
    mean_occ = (st_arr.arena_used_byte_s - st0.arena_used_byte_s) / max(arrival_period, 1e-9) / st.arena_bytes
    # the second half of the arrival period (the controller settled)
    mid = [h for h in hist if h[0] <= st0.clock_s + arrival_period / 2]
    c_mid, b_mid = mid[-1]
    occ_late = (st_arr.arena_used_byte_s - b_mid) / max(st_arr.clock_s - c_mid, 1e-9) / st.arena_bytes
    mean_occ_all = st.arena_used_byte_s / max(st.clock_s, 1e-9) / st.arena_bytes
    lat = np.array(lat)
    total = float(work.sum())
    return {"workload": f"{len(reqs)} requests, Poisson arrivals at a rate held near {occupancy:.0%} arena occupancy, "
                        f"sides log-uniform [64, 2048], steps U[{steps_range[0]}, {steps_range[1]}], half linear N=1 / "
                        f"half Gray-Scott, FP32 or F16 storage, pool {pool_gb} GiB",
            "rate_start_per_s": round(rate0, 4), "rate_end_per_s": round(lam[0], 4),
            "rate_mean_per_s": round(len(reqs) / arrival_period, 4),
            "target_occupancy": occupancy, "model_load_rho": round(rho, 4),
            "work_weighted_mean_footprint_mb": round(m / 1e6, 1),
            "mean_arena_occupancy_during_arrivals": round(float(mean_occ), 4),
            "mean_arena_occupancy_second_half_of_arrivals": round(float(occ_late), 4),
            "mean_arena_occupancy_whole_run": round(float(mean_occ_all), 4),
            "arena_peak_occupancy": round(st.arena_peak_used / st.arena_bytes, 4),
            "mean_resident_requests": round(float(np.mean([a for a, _ in samples])) if samples else 0.0, 2),
            "mean_queued_requests": round(float(np.mean([q for _, q in samples])) if samples else 0.0, 2),
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
            "mean_latency_s": round(float(lat.mean()), 4), "arrival_period_s": round(arrival_period, 3),
            "makespan_s": round(makespan, 3),
            "aggregate_mlups_per_species": round(total / makespan / 1e6, 1),
            "busy_mlups_per_species": round(total / max(st.busy_s, 1e-9) / 1e6, 1),
            "plain_kernel_sample_mlups_per_species": round(plain / 1e6, 1)}


def rescaling_leg(torch, steps=400000):
    """Section IV length-rescaling study at paper scale (Figs. 11, 12): the
    Turing-regime point of the text, eta = 2.014, tau_GS = 2.733 (D_u / D_v =
    2), on boxes of side 50 .. 500 with diffusivities (L / 100)^2 (0.0625,
    0.03125) from the cos start, 400000 steps (the paper's t), plus control
    boxes of twice the side with unscaled diffusivities; one batch.  Reports
    the stripe count |n| of the dominant mode, the stripes crossed along y / L
    = 0.85, the range of v on that line and the relative gaps between the
    profiles of boxes L and 2L."""
    from paper_1007_3109_amd import studies

    sizes = [50, 100, 200, 400, 500]
    r = studies.rescaling_study(sizes, 100, (0.0625, 0.03125), 2.014, 2.733, steps, start="cos")

    def crossings(row):
        d = np.sign(row - row.mean())
        d[d == 0] = 1
        return int(np.sum(d != np.roll(d, 1))) // 2

    rows = {L: r["sizes"][L]["v"][int(round(0.85 * L)) % L] for L in sizes}
    prof = {L: r["sizes"][L]["profile"] for L in sizes}
    out = {"workload": f"Gray-Scott eta 2.014 tau 2.733, sides {sizes} with D scaled as L^2 (D_u 0.0625 at 100), "
                       f"{steps} steps, controls at twice the side with unscaled D",
           "stripe_count": {str(L): round(r["sizes"][L]["n"], 2) for L in sizes},
           "q_max_L": {str(L): round(r["sizes"][L]["qL"], 2) for L in sizes},
           "stripes_along_y_0.85": {str(L): crossings(rows[L]) for L in sizes},
           "v_range_along_y_0.85": {str(L): [round(float(rows[L].min()), 4), round(float(rows[L].max()), 4)]
                                    for L in sizes},
           "profile_gap_L_vs_2L": {f"{L}->{2 * L}": round(float(np.sqrt(((prof[L] - prof[2 * L]) ** 2).mean() /
                                                                        (prof[2 * L] ** 2).mean())), 4)
                                   for L in sizes if 2 * L in sizes},
           "control_stripe_count": {f"{a}->{b}": round(c["n"], 2) for (a, b), c in r["control_modes"].items()},
           "seconds": round(r["seconds"], 3), "mlups_per_species": round(r["mlups_per_species"], 1)}
    torch.cuda.empty_cache()
    return out


def truncation_leg(torch):
    """Section II.B point-source study (Figs. 1c,d): E_rho against the exact
    Gaussian for kappa = 0.01 and 0.033 over D, at the same diffusive time
    D t = C for every D, for C = 2, 4, 8; one FP64 batch of 100^2 lattices per
    C (per-lattice step counts)."""
    from paper_1007_3109_amd import studies

    Ds = [0.004, 0.006, 0.008, 0.01, 0.012, 0.015, 0.02, 0.025, 0.03, 0.04, 0.05, 0.06]
    kappas = [0.01, 0.033]
    out = {"workload": "point source on 100^2, FP64, t = C / D", "D": Ds, "E_rho": {}, "D_min": {}, "seconds": 0.0}
    for C in (2.0, 4.0, 8.0):
        r = studies.truncation_error_sweep(Ds, kappas, C=C)
        key = f"C={C:g}"
        out["E_rho"][key] = {f"kappa={k}": [round(float(e), 6) for e in r["E"][a]] for a, k in enumerate(kappas)}
        out["D_min"][key] = {f"kappa={k}": float(r["D_min"][a]) for a, k in enumerate(kappas)}
        out["seconds"] = round(out["seconds"] + r["seconds"], 4)
    torch.cuda.empty_cache()
    return out


def precision_leg(torch, lbrd, workloads, n=4096, steps=(1000, 10000), check_n=256):
    """16-bit shifted storage (rho_ref = (1, 0)) against FP32 storage on the
    same n^2 Gray-Scott field (same seed), and every storage form against the
    FP64 oracle on a check_n^2 instance with the same seed, at each checkpoint
    in `steps`.  The pattern dynamics amplify any perturbation, so pointwise
    errors grow with time; the field means (FP64 reductions) are reported
    beside them."""
    import oracle

    out = {"workload": f"gray_scott {n}x{n} and {check_n}x{check_n}, checkpoints {list(steps)}",
           "rho_ref": [1.0, 0.0]}
    rho0 = workloads.gray_scott_square(n, n, seed=0)
    solvers = {st: lbrd.Solver(gs_config(lbrd, workloads, n, st)) for st in ("f32", "f16", "bf16")}
    for s in solvers.values():
        s.init(rho0)
    done = 0
    for cp in steps:
        for s in solvers.values():
            s.step(cp - done)
        done = cp
        ref_rho, m_ref = solvers["f32"].moments(dtype=torch.float32)
        row = {"f32_mean": [float(m) / (n * n) for m in m_ref]}
        for st in ("f16", "bf16"):
            rho, m = solvers[st].moments(dtype=torch.float32)
            row[f"{st}_vs_f32_rel_l2"] = [float(x) for x in solvers[st].rel_l2(ref_rho)]
            row[f"{st}_vs_f32_max_abs"] = [float((rho[k] - ref_rho[k]).abs().max()) for k in range(2)]
            row[f"{st}_mean"] = [float(x) / (n * n) for x in m]
            del rho
        del ref_rho
        out[f"step_{cp}_{n}"] = row
    for s in solvers.values():
        s.close()
    del solvers
    torch.cuda.empty_cache()
    small0 = workloads.gray_scott_square(check_n, check_n, seed=0)
    f = oracle.init(small0)
    done = 0
    small = {st: lbrd.Solver(gs_config(lbrd, workloads, check_n, st)) for st in ("f32", "f16", "bf16")}
    for s in small.values():
        s.init(small0)
    t0 = time.perf_counter()
    for cp in steps:
        f = oracle.run(f, cp - done, list(workloads.GS_TAU), oracle.REACT_GRAY_SCOTT, F=workloads.GS_F,
                       k=workloads.GS_K)
        ref64 = torch.tensor(oracle.moments(f), device="cuda")
        row = {"fp64_mean": [float(x) / check_n ** 2 for x in ref64.sum(dim=(1, 2))]}
        for st, s in small.items():
            s.step(cp - done)
            rho, m = s.moments()
            row[f"{st}_vs_fp64_rel_l2"] = [float(x) for x in s.rel_l2(ref64)]
            row[f"{st}_vs_fp64_max_abs"] = [float((rho[k] - ref64[k]).abs().max()) for k in range(2)]
            row[f"{st}_mean"] = [float(x) / check_n ** 2 for x in m]
            m64 = oracle.mass(oracle.moments(f))
            row[f"{st}_mass_rel_diff_vs_fp64"] = [float(abs(a - b) / abs(b)) for a, b in zip(m, m64)]
        done = cp
        out[f"step_{cp}_{check_n}_vs_oracle"] = row
    out["oracle_seconds"] = round(time.perf_counter() - t0, 2)
    for s in small.values():
        s.close()
    # FP64 mass drift of each storage form without reaction (the update
    # conserves mass exactly in real arithmetic): 1024^2, two species, the
    # Gray-Scott start, 2000 steps
    drift = {}
    start = workloads.gray_scott_square(1024, 1024, seed=0)
    for st in ("f64", "f32", "f16", "bf16"):
        extra = dict(rho_ref=(1.0, 0.0)) if st in ("f16", "bf16") else {}
        s = lbrd.Solver(lbrd.make_config(1024, 1024, 2, tau=workloads.GS_TAU, storage=st, reaction="none", **extra))
        s.init(start)
        _, m0 = s.moments()
        s.step(2000)
        _, m1 = s.moments()
        drift[st] = [float(abs(b - a) / abs(a)) for a, b in zip(m0, m1)]
        s.close()
    out["mass_drift_no_reaction_1024_2000_steps"] = drift
    return out


def config1_leg(torch, lbrd, workloads, steps=1000):
    """64^2 single species, FP64, linear decay k = 1e-3, tau = 1 (the decay
    workload): launch-bound, state in the Infinity Cache; the default launches
    and replayed graphs of one-step launches, each with its roofline."""
    rho0 = workloads.sinusoid(64, 64, 0.1, 1)
    out = {"workload": "linear decay 64x64 f64, tau 1, k 1e-3, 1000-step windows"}
    for name, kw in (("default", {}), ("graphs32_one_step", dict(fused_steps=1, graph_steps=32))):
        s = lbrd.Solver(lbrd.make_config(64, 64, 1, tau=1.0, storage="f64", reaction="linear", K=[[-1e-3]]))
        if kw:
            s.set_tuning(**kw)
        s.init(rho0)
        wins = time_windows(torch, s, steps, 64, min_total_s=0.2)
        med, stats = window_stats(wins, steps)
        t = s.tuning()
        per_step = med / steps
        out[name] = {"us_per_step": round(per_step * 1e6, 3), "mlups": round(64 * 64 / per_step / 1e6, 1),
                     "timing": stats,
                     "roofline": roofline(1, 64 * 64, "f64", t.fused_steps, per_step * t.fused_steps, kernel_name(t),
                                          note="0.6 MB of state: launch-bound and cache-resident, not an HBM "
                                               "measurement"),
                     "tuning": t.as_dict()}
        s.close()
    return out


def copy_leg(torch, nbytes=1 << 30, reps=20):
    """Device-to-device copy of an nbytes tensor: at 1 GiB the achievable HBM
    rate; at the size of one lattice buffer the rate of a plain read + write
    of the same working set (inside the Infinity Cache when it fits)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    out = {"bytes_per_copy": 2 * nbytes, "GBs": round(2 * nbytes / sec / 1e9, 1)}
    del a, b
    torch.cuda.empty_cache()
    return out


ALL_LEGS = ("gs1024_f32,tiles1024_f32,one_step_4096_f32,hbm4096_f16,hbm4096_bf16,batch,serve,precision,rescaling,truncation,config1,"
            "copy")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000, help="steps per timed window (K)")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--size", type=int, default=4096, help="side of the headline lattice")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--cpu-steps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--tune", action="store_true", help="run the library's autotuner before timing")
    ap.add_argument("--extra-steps", type=int, default=300, help="steps per window of the 4096^2 extra legs")
    ap.add_argument("--legs", default=ALL_LEGS, help="extra legs to run (comma list)")
    ap.add_argument("--serve-requests", type=int, default=300)
    ap.add_argument("--serve-pool-gb", type=float, default=4.0, help="device arena of the serving leg (GiB)")
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="Poisson arrival rate of the serving leg (default: from the footprint, ~80%% occupancy)")
    ap.add_argument("--serve-steps", default="1000,50000", help="range of steps per request")
    ap.add_argument("--serve-seed", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the build has no multi-GPU path); "
                                   "--gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_1007_3109_amd import lbrd, workloads

    torch.cuda.set_device(0)
    n = args.size
    cfg = gs_config(lbrd, workloads, n, "f32")
    s = lbrd.Solver(cfg)
    if args.tune:
        s.autotune(steps=20)          # launch shape picked by the library's autotuner
    rho0 = workloads.gray_scott_square(n, n, seed=0)
    # initial state from host memory (FP64 densities over PCIe, then the
    # equilibrium kernel): outside the timed region, reported beside it.  The
    # first call also loads the library's code object; the second is timed.
    init_ms = []
    for _ in range(2):
        torch.cuda.synchronize()
        t_init = time.perf_counter()
        s.init(rho0)
        torch.cuda.synchronize()
        init_ms.append((time.perf_counter() - t_init) * 1e3)
    first_init_ms, init_ms = init_ms
    log(f"bench: Gray-Scott {n}x{n} f32, warmup {args.warmup}, windows of {args.steps} steps, "
        f"tuning {s.tuning().as_dict()}")
    wall0 = time.perf_counter()
    wins = time_windows(torch, s, args.steps, args.warmup)
    wall = time.perf_counter() - wall0
    med, stats = window_stats(wins, args.steps)
    sites = n * n
    per_step = med / args.steps
    value = 2 * sites / per_step / 1e6
    tun = s.tuning()
    spl = tun.fused_steps
    traffic, traffic_src = measured_traffic(tun.as_dict())
    issue, issue_src = measured_issue(tun.as_dict())
    _, mass = s.moments()
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "MLUPS per species",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(per_step * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"gray_scott_{n}x{n}_f32", "lattice": [n, n], "species": 2, "storage": "f32",
                   "tau": list(workloads.GS_TAU), "F": workloads.GS_F, "k": workloads.GS_K, "seed": 0,
                   "initial": "u=1, v=0, central 64x64 square u=0.5 v=0.25, U(-0.01,0.01) noise",
                   "parallelism": "single GPU"},
        "timing": stats,
        "roofline": roofline(2, sites, "f32", spl, per_step * spl, kernel_name(tun), traffic, traffic_src, issue,
                             issue_src,
                             note="achieved counts 72 B per species-site-step (every population read and written "
                                  "once per step) x the steps one launch advances; the launch keeps its "
                                  f"{spl} steps on chip and moves the state through HBM once (hbm_measured_*), so "
                                  "frac above 1 is the gain of temporal blocking over a one-pass kernel"),
        "wall_s": round(wall, 3),
        "init_from_host_ms": round(init_ms, 3),
        "first_init_from_host_ms": round(first_init_ms, 3),
        "host_inclusive_mlups_per_species": round(2 * sites * args.steps / (med + init_ms / 1e3) / 1e6, 1),
        "mass_after": [float(m) for m in mass],
        "tuning": tun.as_dict(),
    }
    s.close()
    del s
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(workloads, n, args.cpu_budget, args.cpu_steps)
    if not args.no_extra:
        extra = {}
        legs = [x for x in args.legs.split(",") if x]
        if "gs1024_f32" in legs:
            log("bench: 1024^2 f32")
            extra["gs_1024_f32"] = solver_leg(torch, lbrd, workloads, 1024, "f32", 5000, 100, tune=args.tune,
                                              note="1024^2 x 2 species x 9 x 2 buffers x 4 B = 151 MB: resident in "
                                                   "the 256 MB Infinity Cache, not an HBM measurement")
        if "tiles1024_f32" in legs:
            log("bench: 1024^2 f32 on LDS tiles")
            extra["tiles_1024_f32"] = solver_leg(
                torch, lbrd, workloads, 1024, "f32", 5000, 100,
                shape=dict(march_rows=0, fused_steps=5, tile_cols=32, tile_rows=10, waves=8, tile_strip=0,
                           nontemporal=0, graph_steps=0),
                note="the LDS-tile kernel (the default inside the Infinity Cache for the 16-bit forms and below "
                     "1024^2 sites) on the 1024^2 lattice, for comparison with its marching default")
        if "one_step_4096_f32" in legs:
            log("bench: 4096^2 f32, one step per launch")
            extra["one_step_4096_f32"] = solver_leg(torch, lbrd, workloads, 4096, "f32", args.extra_steps, 20,
                                                    fused=1,
                                                    note="one step per launch: the fraction of the HBM roofline "
                                                         "of a one-pass kernel")
        for storage in ("f16", "bf16"):
            if f"hbm4096_{storage}" in legs:
                log(f"bench: 4096^2 {storage}")
                extra[f"hbm_4096_{storage}"] = solver_leg(torch, lbrd, workloads, 4096, storage, args.extra_steps, 20,
                                                          tune=args.tune)
        if "batch" in legs:
            log("bench: batched sweep")
            extra["batched"] = batch_leg(torch, lbrd, workloads, 5000, 32, cpu=not args.no_cpu_baseline)
        if "serve" in legs:
            log("bench: serving")
            lo, hi = (int(x) for x in args.serve_steps.split(","))
            extra["serving"] = serve_leg(torch, lbrd, workloads, args.serve_requests, args.serve_pool_gb, (lo, hi),
                                         seed=args.serve_seed, rate=args.serve_rate)
        if "precision" in legs:
            log("bench: precision forms")
            extra["precision"] = precision_leg(torch, lbrd, workloads)
        if "rescaling" in legs:
            log("bench: rescaling study")
            extra["rescaling"] = rescaling_leg(torch)
        if "truncation" in legs:
            log("bench: truncation-error curves")
            extra["truncation"] = truncation_leg(torch)
        if "config1" in legs:
            log("bench: 64^2 f64")
            extra["config1"] = config1_leg(torch, lbrd, workloads)
        if "copy" in legs:
            log("bench: copy")
            extra["copy_1GiB"] = copy_leg(torch)
            copy = extra["copy_1GiB"]["GBs"]
            line["roofline"]["copy_GBs"] = copy
            if "hbm_measured_GBs" in line["roofline"]:
                line["roofline"]["hbm_measured_frac_of_copy"] = round(line["roofline"]["hbm_measured_GBs"] / copy, 4)
        line["extra"] = extra
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
