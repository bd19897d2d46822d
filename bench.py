#!/usr/bin/env python3
"""Throughput of Looking Forward track following on one MI355X.

Workload: the nominal batch -- 1,000 synthetic events, each with 350
particles (p 2-100 GeV, pt > 0.3 GeV), 200 upstream input tracks (170 true,
30 fake) and ~5.4k SciFi hits -- resident in HBM.  One step is one pass of
the whole hot path (windows, triplet seeding, extension, fits, selection,
momentum) over the batch.  ``value`` is events/s of the batched launch (one
wavefront per input track, XCD-ordered); the persistent (resident waves
pulling from per-XCD work queues) and per-event-launch (plain, eager and
graph-captured) modes are reported beside it, with identical output, and so
are the serving loop's rates and latencies.

Roofline: the path is bound by plain VALU arithmetic (binary32 and integer,
no FMA contraction, no packed math, no dense contraction), so the dominant
kernel is reported against the non-packed VALU issue rate of the chip.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Peak VALU lane-operations per second for single (non-FMA, non-packed)
# binary32/int32 operations: 256 CUs x 4 SIMDs x 32 lanes per clock x
# 2.4 GHz = 78.6 T/s, i.e. the fp32 vector peak of 157.3 TFLOP/s counted as
# one operation per lane instead of two per FMA.  (A 16-lane reading, 39.3 T/s,
# is contradicted by the counters: the kernel retires VALU lane-operations
# faster than that.)
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# Algorithmic VALU lane-operations of the method per work unit: every (h0, h2)
# pair of the two seed sets' windows ~15 (doublet slope, charge and magnet
# filters), every doublet ~100 (middle-hit prediction, closest-hit search,
# chi2 cut, ranking), every kept triplet ~1.5k (triplet model, nine extension
# searches, x and y fits, Q), every input track ~1.2k (kick, 24 window bounds
# with their searches, caps).  The method's own work, including the pairs an
# exact bracket lets the kernel skip; units from lf_work_counts.
MODEL_OPS = {"pairs_all": 15, "doublets": 100, "kept": 1500, "tracks": 1200}
# Lane-operations the kernel executes per work unit (the arithmetic and
# compares of the fixed evaluation order on the pairs it actually tests;
# loads, stores and address arithmetic not counted).
OPS_PER_UNIT = {
    "tracks": 1160,        # extrapolation and bounds 12 x 14, 36 searches x 8 probes x 3, caps
    "staged_hits": 2,      # common-z / common-stereo checks
    "seed_items": 45,      # slope bracket of one first-layer hit and its two searches
    "pairs_tested": 17,    # doublet slope, charge and magnet filters
    "doublets": 35,        # middle-hit prediction, sorted closest-hit search, chi2 cut, key
    "triplets": 20,        # rank counting into the top-n list
    "kept": 328,           # triplet model 28, nine closest-hit searches 270, candidate rule 30
    "fitted": 514,         # x and y least squares, residuals, Q
}
# No-UT tuning: two windows per layer, 72 bound searches per track, straight
# extrapolation (the other units cost the same).
NO_UT_TRACK_OPS = 2100
# Paper-form kick per track: the five coefficients of F (42 terms), the sine
# of the input slope, three solves of the kick equation.
PAPER_KICK_OPS = 150
# Algorithmic HBM bytes: 12 B per hit in (x, z, dxdy), 20 B per input track
# in, 78 B per track out, plus the offsets.
BYTES_PER_HIT_IN = 12
BYTES_PER_TRACK_IN = 20
BYTES_PER_TRACK_OUT = 78
# HBM traffic of the batched kernel from rocprofv3 FETCH_SIZE + WRITE_SIZE
# (per launch, scaled by the counters' reading of a known-size copy), valid
# only for the kernel source and the workload it was measured on.
TRAFFIC = {"kernel_sha256": "985bb2886f02f49228c45613d199e605f3c3a98cd426572fa0fcbc2bdcc8e45b",
           "workload": "nominal", "events": 0, "bytes_per_launch": 51952280}
WORKLOADS = {
    "nominal": "nominal: 1000 events x 200 input tracks, ~5.4k SciFi hits/event, toy kick field",
    "uneven": "uneven: 20000 events, Poisson(7.6) x 50 particles, 0-13k hits and 0-600 tracks/event",
    "stress": "stress: 5000 events x 486 input tracks (30% fake), ~41.5k hits/event, p 1.5-10 GeV",
    "single": "single: 1 event, 40 particles, p 5-50 GeV",
}
KERNEL = "k_grid"   # the batched mode's kernel (one wavefront per input track)
KERNEL_SRC = os.path.join(ROOT, "paper_2402_14670_amd", "csrc", "lf_kernels.hip")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=16.0,
                    help="wall time of the oracle baseline, half single-threaded, half on all cores (0 disables it)")
    ap.add_argument("--workload", default="nominal", choices=sorted(WORKLOADS))
    ap.add_argument("--events", type=int, default=0, help="events of the workload (0: its full size)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--persistent-exec", default="",
                    help="W,I,B: wavefronts per block, tracks per claim and blocks per CU of the persistent "
                         "launch (instead of the autotuner's choice)")
    ap.add_argument("--modes", default="batched,persistent,plain",
                    help="comma-separated subset of batched,persistent,plain to time (batched is always timed)")
    ap.add_argument("--serve-requests", type=int, default=200000,
                    help="requests per serving run (0 skips the serving runs)")
    ap.add_argument("--variants", default="no_ut,paper,fp16,general",
                    help="method variants timed after the main modes: no_ut (VELO-only input), paper "
                         "(paper-form field and momentum), fp16 (binary16 triplet seeding), general (per-hit z "
                         "and stereo slopes); 'none' for none")
    ap.add_argument("--scan-window", action="store_true",
                    help="instead of the throughput line: events/s and physics efficiency of the batched mode "
                         "for n_hits_window = 16, 32, 48, 64 (one JSON line)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (a known-size reference for HBM "
                         "byte counters under a profiler)")
    return ap.parse_args()


def algorithmic_bytes(ev) -> int:
    return (BYTES_PER_HIT_IN * ev.n_hits + BYTES_PER_TRACK_IN * ev.n_tracks + BYTES_PER_TRACK_OUT * ev.n_tracks
            + 4 * (24 * ev.n_events + 1) + 4 * (ev.n_events + 1))


def time_mode(lf, ctx, bid, mode, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        lf.lf_find_tracks(ctx, bid, mode, stream.cuda_stream)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        lf.lf_find_tracks(ctx, bid, mode, stream.cuda_stream)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / steps, wall


def pinned_copy_peak(mib=256, reps=5):
    """Host-link copy rates of plain pinned-memory copies (torch, one stream):
    host to device and device to host, best of reps, GB/s."""
    import torch
    n = mib * (1 << 20)
    h = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(n, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    res = {}
    for name, dst, src in (("h2d", d, h), ("d2h", h, d)):
        best = None
        for _ in range(reps):
            st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            st.record(s)
            with torch.cuda.stream(s):
                dst.copy_(src, non_blocking=True)
            en.record(s)
            torch.cuda.synchronize()
            ms = st.elapsed_time(en)
            best = ms if best is None else min(best, ms)
        res[name + "_GBs"] = round(n / (best * 1e-3) / 1e9, 2)
    res["bytes"] = n
    del h, d
    return res


def _serve_runs(lf, ctx, ev, ref, req, cfg, base_rate, fracs, rng, label):
    """One saturated run (every request arrives at t = 0), then open-loop
    Poisson arrivals at the given fractions of base_rate (None: of the
    saturated rate); each request's digest is compared with the batched run's."""
    import numpy as np
    n = len(req)
    dig, lat, st = lf.lf_serve_run(ctx, ev, req, np.zeros(n), cfg)
    ok = bool(np.array_equal(dig, ref[req]))
    sat = st["events_per_s"]
    base = sat if base_rate is None else base_rate
    print(f"bench: serving {label} saturated {sat:12.0f} events/s, mean batch {st['mean_batch_events']:.0f}",
          file=sys.stderr, flush=True)
    link = {"bytes_in_per_event": round(st["bytes_in"] / n, 1), "bytes_out_per_event": round(st["bytes_out"] / n, 1),
            "link_in_GBs": round(st["bytes_in"] / st["wall_s"] / 1e9, 2),
            "link_out_GBs": round(st["bytes_out"] / st["wall_s"] / 1e9, 2)}
    rates = []
    for frac in fracs:
        arr = np.cumsum(rng.exponential(1.0 / (frac * base), size=n))
        dig, lat, s2 = lf.lf_serve_run(ctx, ev, req, arr, cfg)
        ok = ok and bool(np.array_equal(dig, ref[req]))
        rates.append({"frac": frac, "offered_events_per_s": round(frac * base, 1),
                      "events_per_s": round(s2["events_per_s"], 1),
                      "p50_ms": round(s2["lat_p50_s"] * 1e3, 4), "p99_ms": round(s2["lat_p99_s"] * 1e3, 4),
                      "p999_ms": round(s2["lat_p999_s"] * 1e3, 4), "max_ms": round(s2["lat_max_s"] * 1e3, 4),
                      "mean_batch_events": round(s2["mean_batch_events"], 1), "max_queue": s2["max_queue"]})
        print(f"bench: serving {label} {frac:4.2f}  {s2['events_per_s']:12.0f} events/s  p50 "
              f"{s2['lat_p50_s']*1e3:.3f} ms  p99 {s2['lat_p99_s']*1e3:.3f} ms  p99.9 {s2['lat_p999_s']*1e3:.3f} ms"
              f"  mean batch {s2['mean_batch_events']:.0f}", file=sys.stderr, flush=True)
    return {"config": cfg, "saturated_events_per_s": round(sat, 1), "saturated_mean_batch_events":
            round(st["mean_batch_events"], 1), "host_link_at_saturation": link, "rates": rates,
            "results_equal_batched": ok}


# Device pool, results to host memory: four slots, a batch as soon as a slot
# is free.  The downloads (15.6 kB per nominal event) run as copy kernels on
# the GPU beside the hot path; the rate they leave to it varies from run to
# run, which no slot count or batching policy tried here removes.
SERVE_DEVICE_CFG = {"max_batch_events": 1024, "n_slots": 4, "device_budget_bytes": 8 << 30, "pool_on_device": 1}
# Device pool, results kept on the device: four slots, and a batch waits for
# 384 events or until its oldest event has waited 150 us, which keeps
# batches large enough to run near the batched rate at moderate load.
SERVE_KEEP_CFG = {"max_batch_events": 1024, "n_slots": 4, "min_batch_events": 384, "max_wait_us": 150,
                  "device_budget_bytes": 8 << 30, "pool_on_device": 1, "results_on_device": 1}
SERVE_HOST_CFG = {"max_batch_events": 256, "n_slots": 2, "device_budget_bytes": 8 << 30}


def serving(lf, ctx, ev, batched_out, n_requests, batched_eps, seed=40):
    """Serving loop on the workload's events as a request pool.  A pool
    resident on the device (events already in HBM, as upstream GPU stages
    leave them; arrivals at 50%, 80% and 95% of the batched throughput),
    first with every result copied to host memory, then with the results
    kept on the device for later GPU stages (digests to the host); and a
    pool in pinned host memory (every event read over the host link;
    arrivals at fractions of its own saturated rate, with the link's bytes
    and rates).  Every request's result digest is checked against the
    batched run's result."""
    import numpy as np
    ref = lf.result_digests(batched_out, ev.trk_off)
    rng = np.random.default_rng(seed)
    req = rng.integers(0, ev.n_events, size=n_requests).astype(np.uint32)
    fr = (0.5, 0.8, 0.95)
    dev = _serve_runs(lf, ctx, ev, ref, req, SERVE_DEVICE_CFG, batched_eps, fr, rng, "device pool")
    dev_keep = _serve_runs(lf, ctx, ev, ref, req, SERVE_KEEP_CFG, batched_eps, fr, rng,
                           "device pool, results on device")
    host = _serve_runs(lf, ctx, ev, ref, req, SERVE_HOST_CFG, None, fr, rng, "host pool")
    peak = pinned_copy_peak()
    host["pinned_copy_peak"] = peak
    sat_link = host["host_link_at_saturation"]
    host["link_frac_of_h2d_peak"] = round(sat_link["link_in_GBs"] / peak["h2d_GBs"], 3)
    basis = "fractions of the batched throughput (%.1f events/s)" % batched_eps
    return {"requests_per_run": n_requests, "pool_events": ev.n_events,
            "device_pool": dict(dev, rate_basis=basis,
                                latency="arrival to results in host memory (digests and every track slot)"),
            "device_pool_results_on_device": dict(dev_keep, rate_basis=basis,
                                                  latency="arrival to the digest in host memory; the results "
                                                          "stay in device memory"),
            "host_pool": dict(host, rate_basis="fractions of the host-pool saturated rate",
                              latency="arrival to results in host memory (digests and every track slot)")}


def host_cores() -> int:
    """Cores this process may use (capped at 16, the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ev, world, min_seconds, gpu_out):
    """The oracle, as it stands, on the host: single-threaded over a sample,
    then over the whole workload with the events split into one contiguous
    slice per core (threads; the oracle call releases the GIL), repeated
    until min_seconds have elapsed.  The first whole pass is also compared,
    event by event, with the GPU's batched results (digests)."""
    import concurrent.futures as cf
    import numpy as np
    import lfgen
    import oracle
    from paper_2402_14670_amd import lf
    oracle.build(force=False)
    n1 = min(ev.n_events, 250)
    sub = lfgen.select_events(ev, range(n1))
    done, t0 = 0, time.perf_counter()
    while True:
        oracle.run(sub, world)
        done += n1
        el1 = time.perf_counter() - t0
        if el1 >= min_seconds / 2:
            break
    single = done / el1
    W = host_cores()
    bounds = [(ev.n_events * k // W, ev.n_events * (k + 1) // W) for k in range(W)]
    parts = [lfgen.select_events(ev, range(a, b)) for a, b in bounds]
    with cf.ThreadPoolExecutor(max_workers=W) as pool:
        first = None
        passes, t0 = 0, time.perf_counter()
        while True:
            outs = list(pool.map(lambda part: oracle.run(part, world), parts))
            if first is None:
                first = outs
            passes += 1
            el = time.perf_counter() - t0
            if el >= min_seconds / 2:
                break
    multi = passes * ev.n_events / el
    ref = {k: np.concatenate([o[k] for o in first]) for k in first[0]}
    ok = lf.result_digests(ref, ev.trk_off) == lf.result_digests(gpu_out, ev.trk_off)
    return dict(value=round(multi, 1), unit="events/s", cores=W, kind="oracle",
                sample=f"whole workload ({ev.n_events} events) split over {W} threads, {passes} passes in "
                       f"{el:.1f} s; single-threaded on its first {n1} events: {single:.1f} events/s "
                       f"({done} events in {el1:.1f} s)",
                single_core_events_per_s=round(single, 1), cpu_model=cpu_model(),
                events_equal_gpu=int(ok.sum()), events_checked=int(ok.size))


def truth_summary(ev, out) -> dict:
    from lfgen import truth
    ph = truth.physics(ev, out, p_min=5.0)
    return {"efficiency_p_gt_5GeV": ph["efficiency"], "ghost_rate": ph["ghost_rate"],
            "qop_resolution": ph["qop_resolution"], "reconstructible_p_gt_5GeV": ph["n_reconstructible"]}


def model_ops(work) -> int:
    return sum(MODEL_OPS[k] * work[k] for k in MODEL_OPS)


def alu_roofline(lf, ctx, bid, stream, ms, track_ops=None, extra_per_track=0):
    """Algorithmic lane-ops of one launch (the method's work from the counting
    build's units) and their rate against the VALU peak; the executed-work
    figure beside it."""
    work = lf.lf_work_counts(ctx, bid, stream.cuda_stream)
    ops = model_ops(work)
    ex = sum(OPS_PER_UNIT[k] * work[k] for k in OPS_PER_UNIT)
    if track_ops is not None:
        ex += (track_ops - OPS_PER_UNIT["tracks"]) * work["tracks"]
    ex += extra_per_track * work["tracks"]
    achieved = ops / (ms * 1e-3) / 1e12
    ach_ex = ex / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s",
            "frac": round(achieved / VALU_PEAK_TOPS, 4), "ops_per_launch": ops,
            "achieved_executed": round(ach_ex, 3), "frac_executed": round(ach_ex / VALU_PEAK_TOPS, 4),
            "ops_per_launch_executed": ex}


def tune_batched(ctx, bid, stream, tune):
    """Wavefronts per block of the batched mode, autotuned (or the default)."""
    if not tune:
        return None
    from paper_2402_14670_amd import autotune
    return autotune.autotune(ctx, bid, stream, modes=("batched",), steps=3)["best"]["waves_per_block"]


def no_ut_mode(lf, world, ev, stream, steps, warmup, tune=True):
    """The same batch under the paper's no-UT tuning (VELO-only input: two
    windows per layer, 64 hits each, per-side seeding), batched mode."""
    from lfgen import truth
    ctx = lf.lf_create(world, lf.lf_default_params(no_ut=True))
    try:
        bid = lf.lf_upload_events(ctx, ev, stream.cuda_stream)
        wpb = tune_batched(ctx, bid, stream, tune)
        ms, _ = time_mode(lf, ctx, bid, lf.LF_MODE_BATCHED, max(5, steps // 2), warmup, stream)
        roof = alu_roofline(lf, ctx, bid, stream, ms, track_ops=NO_UT_TRACK_OPS)
        out = lf.lf_fetch_tracks(ctx, bid, ev.n_tracks, stream.cuda_stream)
    finally:
        lf.lf_destroy(ctx)
    ph = truth.physics(ev, out, p_min=5.0)
    print(f"bench: no-UT      {ms:8.3f} ms/step  {ev.n_events / ms * 1e3:12.0f} events/s", file=sys.stderr, flush=True)
    return {"ms_per_step": round(ms, 4), "events_per_s": round(ev.n_events / ms * 1e3, 1),
            "waves_per_block": wpb, "found_tracks": ph["n_found"],
            "efficiency_p_gt_5GeV": round(ph["efficiency"], 5), "ghost_rate": round(ph["ghost_rate"], 5),
            "roofline": roof}


def fp16_mode(lf, world, ev, stream, steps, warmup, tune=True):
    """The same batch with the triplet seeding in binary16 (the paper's
    Performance section): packed half-precision doublet filters and
    middle-hit search over every pair of the seed windows; batched mode."""
    from lfgen import truth
    ctx = lf.lf_create(world, {"seed_fp16": 1})
    try:
        bid = lf.lf_upload_events(ctx, ev, stream.cuda_stream)
        wpb = tune_batched(ctx, bid, stream, tune)
        ms, _ = time_mode(lf, ctx, bid, lf.LF_MODE_BATCHED, max(5, steps // 2), warmup, stream)
        roof = alu_roofline(lf, ctx, bid, stream, ms)
        out = lf.lf_fetch_tracks(ctx, bid, ev.n_tracks, stream.cuda_stream)
    finally:
        lf.lf_destroy(ctx)
    ph = truth.physics(ev, out, p_min=5.0)
    print(f"bench: fp16 seeding {ms:7.3f} ms/step  {ev.n_events / ms * 1e3:12.0f} events/s", file=sys.stderr,
          flush=True)
    return {"ms_per_step": round(ms, 4), "events_per_s": round(ev.n_events / ms * 1e3, 1),
            "waves_per_block": wpb, "found_tracks": ph["n_found"],
            "efficiency_p_gt_5GeV": round(ph["efficiency"], 5), "ghost_rate": round(ph["ghost_rate"], 5),
            "qop_resolution": round(ph["qop_resolution"], 5), "roofline": roof}


def paper_field_mode(lf, workload, n_events, stream, steps, warmup, tune=True):
    """The same workload generated in the paper-form field (sqrt-normalised
    pt-kick, an integrated field that depends on the entry slopes and the
    bending, a falling tail) and followed with the kick solved for the
    windows and q/p from the fitted parametrisation F(tx, ty, dSlope);
    batched mode.  The q/p resolution is also given for F replaced by its
    constant term."""
    import lfgen
    from lfgen import truth
    ev = lfgen.generate(workload, field="paper", **({"n_events": n_events} if n_events else {}))
    world = lfgen.world("paper")
    res = {}
    for label, w in (("fitted", world), ("constant", dict(world, F_coef=[lfgen.KICK] + [0.0] * 49))):
        ctx = lf.lf_create(w)
        try:
            bid = lf.lf_upload_events(ctx, ev, stream.cuda_stream)
            if label == "fitted":
                wpb = tune_batched(ctx, bid, stream, tune)
                ms, _ = time_mode(lf, ctx, bid, lf.LF_MODE_BATCHED, max(5, steps // 2), warmup, stream)
                roof = alu_roofline(lf, ctx, bid, stream, ms, extra_per_track=PAPER_KICK_OPS)
            else:
                lf.lf_find_tracks(ctx, bid, lf.LF_MODE_BATCHED, stream.cuda_stream)
            res[label] = lf.lf_fetch_tracks(ctx, bid, ev.n_tracks, stream.cuda_stream)
        finally:
            lf.lf_destroy(ctx)
    ph = truth.physics(ev, res["fitted"], p_min=5.0)
    ph_c = truth.physics(ev, res["constant"], p_min=5.0)
    print(f"bench: paper field {ms:8.3f} ms/step  {ev.n_events / ms * 1e3:12.0f} events/s  "
          f"q/p resolution {ph['qop_resolution']:.4f} (constant F: {ph_c['qop_resolution']:.4f})",
          file=sys.stderr, flush=True)
    return {"ms_per_step": round(ms, 4), "events_per_s": round(ev.n_events / ms * 1e3, 1),
            "waves_per_block": wpb, "events": ev.n_events, "input_tracks": ev.n_tracks, "hits": ev.n_hits,
            "found_tracks": ph["n_found"], "efficiency_p_gt_5GeV": round(ph["efficiency"], 5),
            "ghost_rate": round(ph["ghost_rate"], 5), "qop_resolution": round(ph["qop_resolution"], 5),
            "qop_resolution_constant_F": round(ph_c["qop_resolution"], 5), "roofline": roof}


def general_path(lf, world, ev, stream, steps, warmup, tune=True, z_mm=1.5, slope_rel=0.02, seed=11):
    """The same events with every hit's z and stereo slope jittered (tilted
    or bowed layers: no bucket shares one z or one slope), so the kernel
    stages z and slope per hit, brackets each doublet's third window over
    the z range of its hits, and scans stereo windows; batched mode."""
    import numpy as np
    import lfgen
    rng = np.random.default_rng(seed)
    hz = (ev.hit_z + rng.uniform(-z_mm, z_mm, ev.n_hits)).astype(np.float32)
    hd = (ev.hit_dxdy * (1.0 + rng.uniform(-slope_rel, slope_rel, ev.n_hits))).astype(np.float32)
    gev = lfgen.Events(**{**ev.__dict__, "hit_z": hz, "hit_dxdy": hd})
    ctx = lf.lf_create(world)
    try:
        bid = lf.lf_upload_events(ctx, gev, stream.cuda_stream)
        wpb = tune_batched(ctx, bid, stream, tune)
        ms, _ = time_mode(lf, ctx, bid, lf.LF_MODE_BATCHED, max(5, steps // 2), warmup, stream)
        out = lf.lf_fetch_tracks(ctx, bid, gev.n_tracks, stream.cuda_stream)
    finally:
        lf.lf_destroy(ctx)
    print(f"bench: general path {ms:7.3f} ms/step  {ev.n_events / ms * 1e3:12.0f} events/s", file=sys.stderr,
          flush=True)
    return {"ms_per_step": round(ms, 4), "events_per_s": round(ev.n_events / ms * 1e3, 1),
            "waves_per_block": wpb, "found_tracks": int(out["found"].sum()),
            "inputs": f"the workload's hits with z jittered by +-{z_mm} mm and stereo slopes by +-{slope_rel:.0%} "
                      f"(uniform, seed {seed}): per-hit z and slope on every bucket"}


def end_to_end(lf, ctx, ev, stream, reps=3):
    """The whole batch from host buffers: validation and upload, the hot path,
    and the download of the results (host link included)."""
    import torch
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bid = lf.lf_upload_events(ctx, ev, stream.cuda_stream)
        lf.lf_find_tracks(ctx, bid, lf.LF_MODE_BATCHED, stream.cuda_stream)
        lf.lf_fetch_tracks(ctx, bid, ev.n_tracks, stream.cuda_stream)
        el = time.perf_counter() - t0
        best = el if best is None else min(best, el)
    return {"ms_per_batch": round(best * 1e3, 3), "events_per_s": round(ev.n_events / best, 1),
            "includes": "host validation, upload, hot path, download (best of %d)" % reps}


def scan_window(lf, world, ev, stream, steps, warmup, workload):
    """The paper's tuning experiment on the window cap: throughput and
    efficiency (reconstructible particles with p > 5 GeV, truth matching of
    the generator) for each n_hits_window."""
    from lfgen import truth
    rows = []
    for n in (16, 32, 48, 64):
        ctx = lf.lf_create(world, {"n_hits_window": n})
        try:
            bid = lf.lf_upload_events(ctx, ev, stream.cuda_stream)
            wpb = tune_batched(ctx, bid, stream, True)
            ms, _ = time_mode(lf, ctx, bid, lf.LF_MODE_BATCHED, steps, warmup, stream)
            out = lf.lf_fetch_tracks(ctx, bid, ev.n_tracks, stream.cuda_stream)
        finally:
            lf.lf_destroy(ctx)
        ph = truth.physics(ev, out, p_min=5.0)
        rows.append({"n_hits_window": n, "waves_per_block": wpb, "ms_per_step": round(ms, 4), "events_per_s": round(ev.n_events / ms * 1e3, 1),
                     "efficiency_p_gt_5GeV": round(ph["efficiency"], 5), "ghost_rate": round(ph["ghost_rate"], 5),
                     "found_tracks": ph["n_found"], "qop_resolution": round(ph["qop_resolution"], 6)})
        print(f"bench: n_hits_window {n:3d}  {ms:8.3f} ms/step  efficiency {ph['efficiency']:.4f}  "
              f"ghosts {ph['ghost_rate']:.4f}", file=sys.stderr, flush=True)
    return {"metric": "n_hits_window scan: events/s and efficiency (batched mode)", "n_gpus": 1,
            "config": {"workload": WORKLOADS[workload], "events": ev.n_events, "input_tracks": ev.n_tracks},
            "steps": steps, "warmup": warmup, "data": "synthetic", "scan": rows}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (--gpus {args.gpus} requested); events are "
              f"independent, so N GPUs would each take their own batches of events", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import lfgen
    from paper_2402_14670_amd import lf

    torch.cuda.set_device(0)
    # an explicit stream: the library launches on it and the timing events are recorded on it
    stream = torch.cuda.Stream()
    world = lfgen.world()
    gen = {"n_events": args.events} if args.events else {}
    ev = lfgen.generate(args.workload, **gen)
    print(f"bench: {args.workload}: {ev.n_events} events, {ev.n_tracks} tracks, {ev.n_hits} hits", file=sys.stderr,
          flush=True)

    if args.calib_copy_mb:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        with torch.cuda.stream(stream):
            torch.mul(src, 2.0, out=dst)   # reads and writes exactly n*4 bytes
        torch.cuda.synchronize()
        del src, dst

    if args.scan_window:
        print(json.dumps(scan_window(lf, world, ev, stream, args.steps, args.warmup, args.workload)), flush=True)
        return

    ctx = lf.lf_create(world)
    bid = lf.lf_upload_events(ctx, ev, stream.cuda_stream)
    tuned = None
    if not args.no_autotune:
        from paper_2402_14670_amd import autotune
        tuned = autotune.autotune(ctx, bid, stream, steps=3)
        print(f"bench: autotuned {tuned['per_mode']}", file=sys.stderr, flush=True)
    res = {}
    wanted = set(args.modes.split(",")) | {"batched"}
    for mode, steps, warm in (("batched", args.steps, args.warmup), ("persistent", args.steps, args.warmup),
                              ("plain", args.plain_steps, 1)):
        if mode not in wanted:
            continue
        if mode == "persistent" and args.persistent_exec:
            w, i, b = (int(v) for v in args.persistent_exec.split(","))
            lf.lf_set_exec(ctx, waves_per_block=w)
            lf.lf_set_exec(ctx, items_per_grab=i, blocks_per_cu=b)
        elif tuned and mode in tuned["per_mode"]:
            c = tuned["per_mode"][mode]
            lf.lf_set_exec(ctx, waves_per_block=c["waves_per_block"])
            lf.lf_set_exec(ctx, items_per_grab=c["items_per_grab"], blocks_per_cu=c["blocks_per_cu"])
        ms, wall = time_mode(lf, ctx, bid, mode, steps, warm, stream)
        res[mode] = ms
        print(f"bench: {mode:10s} {ms:8.3f} ms/step  {ev.n_events / ms * 1e3:12.0f} events/s", file=sys.stderr,
              flush=True)
        if mode == "plain":
            # the same per-event launch sequence, captured once in a HIP graph
            g = lf.lf_graph_create(ctx, [bid], "plain")
            try:
                for _ in range(1):
                    lf.lf_graph_launch(ctx, g, stream.cuda_stream)
                torch.cuda.synchronize()
                st_, en_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                st_.record(stream)
                for _ in range(steps):
                    lf.lf_graph_launch(ctx, g, stream.cuda_stream)
                en_.record(stream)
                torch.cuda.synchronize()
                res["plain_graph"] = st_.elapsed_time(en_) / steps
            finally:
                lf.lf_graph_destroy(g)
            print(f"bench: {'plain_graph':10s} {res['plain_graph']:8.3f} ms/step  "
                  f"{ev.n_events / res['plain_graph'] * 1e3:12.0f} events/s", file=sys.stderr, flush=True)
    if tuned:
        c = tuned["per_mode"]["batched"]
        lf.lf_set_exec(ctx, waves_per_block=c["waves_per_block"])
    # the workload as a sequence of 4 resident sub-batches, replayed from one HIP graph
    parts = [lfgen.select_events(ev, range(ev.n_events * k // 4, ev.n_events * (k + 1) // 4)) for k in range(4)]
    sub = [lf.lf_upload_events(ctx, part, stream.cuda_stream) for part in parts if part.n_events]
    g = lf.lf_graph_create(ctx, sub, "batched")
    try:
        lf.lf_graph_launch(ctx, g, stream.cuda_stream)
        torch.cuda.synchronize()
        st_, en_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st_.record(stream)
        for _ in range(args.steps):
            lf.lf_graph_launch(ctx, g, stream.cuda_stream)
        en_.record(stream)
        torch.cuda.synchronize()
        res["batched_graph_4_batches"] = st_.elapsed_time(en_) / args.steps
    finally:
        lf.lf_graph_destroy(g)
        for b in sub:
            lf.lf_release_batch(ctx, b)
    print(f"bench: {'graph x4':10s} {res['batched_graph_4_batches']:8.3f} ms/step  "
          f"{ev.n_events / res['batched_graph_4_batches'] * 1e3:12.0f} events/s", file=sys.stderr, flush=True)
    work = lf.lf_work_counts(ctx, bid, stream.cuda_stream)
    out = lf.lf_fetch_tracks(ctx, bid, ev.n_tracks, stream.cuda_stream)
    e2e = end_to_end(lf, ctx, ev, stream)
    variants = set(args.variants.split(","))
    tune = not args.no_autotune
    no_ut = no_ut_mode(lf, world, ev, stream, args.steps, args.warmup, tune) if "no_ut" in variants else None
    paper = (paper_field_mode(lf, args.workload, args.events, stream, args.steps, args.warmup, tune)
             if "paper" in variants else None)
    fp16 = fp16_mode(lf, world, ev, stream, args.steps, args.warmup, tune) if "fp16" in variants else None
    general = (general_path(lf, world, ev, stream, args.steps, args.warmup, tune)
               if "general" in variants else None)
    print(f"bench: end to end {e2e['ms_per_batch']:8.3f} ms/batch  {e2e['events_per_s']:12.0f} events/s",
          file=sys.stderr, flush=True)
    ms = res["batched"]
    value = ev.n_events / (ms * 1e-3)
    serve = serving(lf, ctx, ev, out, args.serve_requests, value) if args.serve_requests else None
    lf.lf_destroy(ctx)

    ops = model_ops(work)
    achieved = ops / (ms * 1e-3) / 1e12
    ops_ex = sum(OPS_PER_UNIT[k] * work[k] for k in OPS_PER_UNIT)
    achieved_ex = ops_ex / (ms * 1e-3) / 1e12
    import hashlib
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    traffic = (TRAFFIC["bytes_per_launch"] if (TRAFFIC["kernel_sha256"], TRAFFIC["workload"], TRAFFIC["events"]) ==
               (sha, args.workload, args.events) else None)
    nbytes = algorithmic_bytes(ev)
    line = {
        "metric": "events/s on 1 MI355X (plain vs batched vs serving); p50/p99 event latency",
        "value": round(value, 1),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "events": ev.n_events, "input_tracks": ev.n_tracks, "hits": ev.n_hits,
                   "n_hits_window": 32, "n_triplets": 12},
        "modes": {m: {"ms_per_step": round(v, 4), "events_per_s": round(ev.n_events / v * 1e3, 1),
                      "input_tracks_per_s": round(ev.n_tracks / v * 1e3, 1),
                      "hbm_frac": round(nbytes / (v * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)} for m, v in res.items()},
        "batched_over_plain": round(res["plain"] / ms, 2) if "plain" in res else None,
        "autotune": ({m: {k: v for k, v in c.items() if k != "mode"} for m, c in tuned["per_mode"].items()}
                     if tuned else None),
        "found_tracks": int(out["found"].sum()),
        "physics": {k: round(v, 5) if isinstance(v, float) else v
                    for k, v in truth_summary(ev, out).items()},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                     "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": traffic,
                     "kernel": KERNEL, "ops_per_launch": ops,
                     "ops_model": "method work per launch: 15 per window pair of the seed sets + 100 per "
                                  "doublet + 1500 per kept triplet + 1200 per input track (lane-operations)",
                     "achieved_executed": round(achieved_ex, 3),
                     "frac_executed": round(achieved_ex / VALU_PEAK_TOPS, 4), "ops_per_launch_executed": ops_ex,
                     "ops_executed": "arithmetic and compares the kernel executes on the pairs it tests "
                                     "(bracketing skips the rest); loads, stores and addressing not counted",
                     "work_units": {k: v for k, v in work.items() if not k.startswith("cy_")},
                     "phase_cycle_share": {k[3:]: round(v / max(1, sum(x for n, x in work.items()
                                                                          if n.startswith("cy_"))), 4)
                                           for k, v in work.items() if k.startswith("cy_")},
                     "hbm": {"algorithmic_bytes": nbytes, "achieved_GBs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                             "peak_GBs": HBM_PEAK_GBS,
                             "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)}},
        "latency_ms": ({"p50": serve["device_pool_results_on_device"]["rates"][1]["p50_ms"],
                        "p99": serve["device_pool_results_on_device"]["rates"][1]["p99_ms"],
                        "p999": serve["device_pool_results_on_device"]["rates"][1]["p999_ms"],
                        "at": "serving from a device-resident pool at 80% of the batched throughput, results "
                              "kept in device memory for the next GPU stage (digests to the host)",
                        "results_to_host": {k: serve["device_pool"]["rates"][1][k + "_ms"]
                                            for k in ("p50", "p99", "p999")}}
                       if serve else None),
        "serving": serve,
        "end_to_end": e2e,
        "no_ut": no_ut,
        "paper_field": paper,
        "fp16_seeding": fp16,
        "general_path": general,
    }
    if args.cpu_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(ev, world, args.cpu_seconds, out)
        print(f"bench: cpu oracle {line['cpu_baseline']['value']:.0f} events/s on "
              f"{line['cpu_baseline']['cores']} cores; equal to the GPU on "
              f"{line['cpu_baseline']['events_equal_gpu']}/{line['cpu_baseline']['events_checked']} events",
              file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
