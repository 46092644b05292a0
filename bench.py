"""Benchmark of the gfx950 Asp-Clean2016 minor cycle.

A step is one minor-cycle iteration: peak search, stop test, start values,
active-set selection, LM fit, commit and residual update, all on the device.
The default workload is the 4096 x 4096 synthetic EVLA-like field (2000
points, 300 Gaussians with sigma U[2, 120] px, Y-array PSF, active set <= 10,
gain 0.1).  The images are generated on the host and copied to HBM before the
timed region; the timed region runs K iterations after W warm-up iterations.

Besides the throughput the line carries:
  roofline      the dominant kernel (the LM fit), timed with HIP events on the
                context's stream over the timed region; its algorithmic work
                is the FP32 Gram accumulation, (n+1)(n+2) flops per pixel
                evaluation, against the FP32 vector peak
  update_large  the residual update in its own launch on a field of the same
                size holding one extended Gaussian: windows of millions of
                pixels, the update's HBM rate when the work is large
  hbm           achieved HBM rates of the peak search (4 H W bytes per
                launch) and, with --update-launch 1, of the residual update
                (8 bytes per pixel read-modify-written); by default the
                update runs at the end of the fit kernel and is part of its
                launch time
  peak_cold     the peak search on HBM-cold data (a 1 GiB scrub before each
                timed launch) and warm (launches back to back), 4 H W bytes
                per launch against 8 TB/s
  full_run      every iteration of the workload's configuration (20000 at
                4096^2) from the dirty image in one asp_run call, its rate and
                final residual RMS, and the oracle stepped beside the device
                for a few iterations at the end: per-component errors
  learned_vs_plain  time to the full run's final residual RMS with the
                network's start values, from the dirty image, at equal RMS
                (tracked sum of R^2, first iteration at or below it)
  cpu_baseline  the FP64 oracle, single-threaded and pinned to one core,
                continuing the same run from the state at the start of the
                timed region for a bounded number of seconds; the CPU model
                and core counts beside it
  smoothing     the smoothing method of initial values with the 5 % switch
                (init mode 2) on the same field: a full refresh of the
                smoothed images (every tile, both passes, all trial widths)
                against the FP32 vector peak, and the same iterations as the
                timed region run in init mode 2 (throughput, the share of
                fits started from the smoothing method, the incremental
                refresh per iteration, residual RMS against the plain run)
  peak_tiles    the same iterations with the incremental peak search: the
                64 x 64 tiles the updates touched are rescanned and the tile
                maxima reduced; its bytes per iteration (rescanned pixels x 4
                plus the tile keys) against the full scan's 4 H W, and a
                check that the residual equals the full-scan run's
  refresh       the exact-PSF residual refresh (R = I_dirty - B (*) I_model):
                the time of one refresh, and the same iterations run with a
                refresh after every 500th; the true residual (refreshed once
                more at the end) of both runs

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "c4096": ("make_c4096", 4096),
    "c1024": ("make_c1024", 1000),
    "c128": ("make_c128", 0),
    "batch": ("make_batch", 64),
}

PEAK_HBM_GBS = 8000.0            # MI355X HBM3E
PEAK_FP32_VECTOR_TFLOPS = 157.3  # MI355X FP32 vector


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


FIT_SOURCES = ("fit.hip", "cycle.h", "asp_device.h")   # what the fit kernel is built from


def fit_source_digest() -> str:
    """SHA-256 over the fit kernel's sources, in FIT_SOURCES order."""
    h = hashlib.sha256()
    for name in FIT_SOURCES:
        with open(os.path.join(ROOT, "paper_1606_07872_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def fit_traffic(workload: str, warmup: int, steps: int):
    """HBM bytes per fit launch from the committed PMC record of this workload,
    if one was taken over the same timed window (iterations warmup ..
    warmup + steps) on the current fit kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"k_fit_{workload}_traffic.json")
    try:
        with open(path) as fh:
            recs = json.load(fh)
        digest = fit_source_digest()
    except (OSError, ValueError):
        return None
    for rec in recs.get("windows", []):
        if rec.get("warmup") == warmup and rec.get("steps") == steps and \
                rec.get("fit_sources_sha256") == digest:
            return rec.get("bytes_per_launch")
    return None


def cpu_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "cpus_allowed": len(os.sched_getaffinity(0))}


def cpu_baseline(f, R0, comps0, k0, alpha_b, omega_b, seconds):
    """The oracle continuing the run from (R0, comps0, k0) for about `seconds`,
    on one core: the process is pinned to its first allowed CPU meanwhile."""
    import oracle
    info = cpu_info()
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[-1]              # the last allowed CPU: away from CPU 0's system work
    os.sched_setaffinity(0, {core})
    try:
        o = oracle.Oracle(f.dirty, gain=f.gain, threshold=f.threshold, max_iter=f.max_iter,
                          max_active=f.max_active, cap=f.max_iter + 1, alpha_b=alpha_b,
                          omega_b=omega_b)
        o.load_state(R0, comps0, k0)
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            r = o.step()
            if r["status"] in (1, 2) or r["status"] < 0:    # a stop or an error; 3 = fit budget used
                break
            done += 1
        secs = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, set(allowed))
    return {"value": done / secs if secs > 0 else 0.0, "unit": "iterations/s", "cores": 1,
            "kind": "oracle", "pinned_cpu": core, **info,
            "sample": f"{done} iterations ({secs:.1f} s) of the same field continuing from "
                      f"iteration {k0}, the state at the start of the timed region; FP64 C, "
                      "one thread, pinned to one core"}


def device_field(f, torch):
    return torch.from_numpy(f.dirty).cuda(), torch.from_numpy(f.psf).cuda()


def tracked_rms(ctx, npx: int) -> float:
    return math.sqrt(max(ctx.residual_sumsq(tracked=True), 0.0) / npx)


def step_errors(ctx, f, o, peak):
    """One lockstep iteration: the oracle loaded with the context's pre-step
    state steps once beside it; per-member errors of the fit (a and s
    relative, x and y in units of max(1, s)) and the residual's max error
    relative to the dirty image's peak."""
    import numpy as np
    R0, comps0, k0 = ctx.residual(), ctx.components_raw(), ctx.counts()[0]
    rc, idx, val = ctx.find_peak()
    if rc != 0:
        return None
    rc, rep = ctx.fit_active_set(idx)
    ctx.update_residual()
    o.load_state(R0, comps0, k0)
    orep = o.step()
    out = {"k": int(k0), "same_peak": orep["idx"] == idx,
           "same_members": orep["members"] == rep["members"], "members": len(rep["members"]),
           "converged": [bool(rep["converged"]), bool(orep["converged"])],
           "resid_err_over_peak": float(np.abs(ctx.residual().astype(np.float64) - o.R).max()
                                        / peak)}
    if out["same_members"]:
        g, c = np.asarray(rep["theta"]).reshape(-1, 4), np.asarray(orep["theta"]).reshape(-1, 4)
        ea = np.abs(g[:, 0] - c[:, 0]) / np.maximum(np.abs(c[:, 0]), 1e-30)
        es = np.abs(g[:, 3] - c[:, 3]) / c[:, 3]
        ep = np.maximum(np.abs(g[:, 1] - c[:, 1]), np.abs(g[:, 2] - c[:, 2])) / np.maximum(1.0, c[:, 3])
        out["per_member"] = [{"amp_rel": float(a), "width_rel": float(w), "pos_over_scale": float(q)}
                             for a, w, q in zip(ea, es, ep)]
    return out


def full_run_leg(args, f, torch, asp):
    """The workload's whole run, every iteration of its configuration from the
    dirty image (20000 at 4096^2), in one asp_run call; then the oracle steps
    beside the device for a few iterations at the end of the run (lockstep)
    and the per-component errors of those fits are reported."""
    import numpy as np
    import oracle
    n = f.max_iter
    d_dirty, d_psf = device_field(f, torch)
    ctx = asp.Context(d_dirty, d_psf, f.gain, f.threshold, max_iter=n + args.full_samples,
                      max_active=f.max_active, fit_solo_tiles=args.solo_tiles,
                      fit_min_tiles=args.min_tiles, fit_group=args.group)
    del d_dirty, d_psf
    torch.cuda.synchronize()
    prof0 = ctx.fit_profile()
    t0 = time.perf_counter()
    rc, rep = ctx.run(n)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    H, W = f.shape
    rms = tracked_rms(ctx, H * W)
    prof1 = ctx.fit_profile()
    hist = ctx.fit_histogram()
    out = {"iterations": rep["iterations"], "seconds": secs,
           "iterations_per_s": rep["iterations"] / secs if secs > 0 else 0.0,
           "components": rep["components"], "not_added": rep["not_added"],
           "trials_per_fit": rep["lm_trials"] / max(rep["iterations"], 1),
           "not_converged": rep["not_converged"], "rms": rms,
           "rms_dirty": float(np.sqrt(np.mean(f.dirty.astype(np.float64) ** 2))),
           "fit_phases_us": {k: round(prof1[k] - prof0[k], 1) for k in prof1},
           "by_active_set": {int(m): {"fits": int(hist["fits"][m]), "trials": int(hist["trials"][m]),
                                      "ms": round(float(hist["us"][m]) / 1e3, 2)}
                             for m in range(len(hist["fits"])) if hist["fits"][m]}}
    log(f"full run {json.dumps(out)}")
    ab, wb = ctx.psf_gauss()
    o = oracle.Oracle(f.dirty, gain=f.gain, threshold=f.threshold, max_iter=n + args.full_samples,
                      max_active=f.max_active, alpha_b=ab, omega_b=wb, cap=n + args.full_samples + 1)
    peak = float(np.abs(f.dirty).max())
    samples = []
    for _ in range(args.full_samples):
        e = step_errors(ctx, f, o, peak)
        if e is None:
            break
        samples.append(e)
    out["oracle_lockstep_at_end"] = samples
    log(f"full run, lockstep at the end {json.dumps(samples)}")
    ctx.close()
    return out, rms, secs


def learned_equal_rms(args, f, wpath, n_plain, rms_plain, secs_plain, torch, asp):
    """Time to the plain run's final residual RMS with the network's start
    values, both from the dirty image.  A search pass runs the learned context
    in chunks, reading the tracked sum of R^2 after each; in the chunk that
    crosses the plain RMS it goes back to the chunk's start and steps one
    iteration at a time, which gives the first iteration N at or below it.  A
    fresh learned context then runs exactly N iterations in one timed asp_run
    call (the learned path is deterministic, so it ends at the same RMS)."""
    import numpy as np
    w = np.load(wpath)
    H, W = f.shape
    cap = 2 * n_plain
    d_dirty, d_psf = device_field(f, torch)

    def learned_ctx():
        c = asp.Context(d_dirty, d_psf, f.gain, f.threshold, max_iter=cap, max_active=f.max_active)
        c.set_mlp(w)
        c.set_init_mode(1)
        return c

    ctx = learned_ctx()
    N, chunk = None, 512
    while ctx.counts()[0] < cap:
        blob = ctx.save_state()
        k0 = ctx.counts()[0]
        rc, r = ctx.run(min(chunk, cap - k0))
        if tracked_rms(ctx, H * W) <= rms_plain:
            ctx.load_state(blob)
            while ctx.counts()[0] < cap:
                ctx.run(1)
                if tracked_rms(ctx, H * W) <= rms_plain:
                    N = ctx.counts()[0]
                    break
            break
        if r["iterations"] == 0:
            break
    rms_cap = tracked_rms(ctx, H * W)
    ctx.close()
    out = {"weights": os.path.basename(wpath),
           "plain": {"iterations": n_plain, "seconds": secs_plain, "rms": rms_plain},
           "reached_plain_rms": N is not None, "iteration_cap": cap}
    if N is None:
        out["learned"] = {"iterations": cap, "rms": rms_cap}
    else:
        ctx = learned_ctx()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, r = ctx.run(N)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out["learned"] = {"iterations": r["iterations"], "seconds": t,
                          "rms": tracked_rms(ctx, H * W),
                          "trials_per_fit": r["lm_trials"] / max(r["iterations"], 1),
                          "fallbacks": r["fallbacks"],
                          "fallback_rate": r["fallbacks"] / max(r["iterations"], 1),
                          "not_added": r["not_added"], "components": r["components"]}
        out["time_ratio_learned_over_plain"] = t / secs_plain if secs_plain > 0 else None
        ctx.close()
    del d_dirty, d_psf
    log(f"learned vs plain at equal RMS {json.dumps(out)}")
    return out


def cold_peak_leg(args, f, torch, asp, reps: int = 20):
    """The peak search on HBM-cold data: before each timed launch a 1 GiB
    buffer is read and written (four times the 256 MB Infinity Cache and all
    of L2), so the 4 H W bytes of the scan come from HBM.  The same launches
    back to back give the warm (cache-resident) rate.  HIP events on the
    context's stream."""
    H, W = f.shape
    d_dirty, d_psf = device_field(f, torch)
    ctx = asp.Context(d_dirty, d_psf, f.gain, f.threshold, max_iter=f.max_iter,
                      max_active=f.max_active)
    del d_dirty, d_psf
    scrub = torch.zeros(256 << 20, dtype=torch.float32, device="cuda")
    ctx.kernel_timing(True)
    ctx.find_peak()
    m0, n0 = ctx.kernel_times()["peak"]
    for _ in range(reps):
        scrub.add_(1.0)
        torch.cuda.synchronize()
        ctx.find_peak()
    m1, n1 = ctx.kernel_times()["peak"]
    for _ in range(reps):
        ctx.find_peak()
    m2, n2 = ctx.kernel_times()["peak"]
    ctx.close()
    del scrub
    b = 4.0 * H * W
    cold_us = (m1 - m0) / max(n1 - n0, 1) * 1e3
    warm_us = (m2 - m1) / max(n2 - n1, 1) * 1e3
    out = {"bytes_per_launch": b, "launches": n1 - n0, "scrub_bytes": 4 * (256 << 20),
           "cold": {"avg_launch_us": cold_us, "achieved_gbs": b / cold_us / 1e3,
                    "frac": b / cold_us / 1e3 / PEAK_HBM_GBS},
           "warm": {"avg_launch_us": warm_us, "achieved_gbs": b / warm_us / 1e3,
                    "frac": b / warm_us / 1e3 / PEAK_HBM_GBS}}
    log(f"peak search cold/warm {json.dumps(out)}")
    return out


def smoothing_leg(args, f, rep, secs, rms_plain, torch, asp):
    """The smoothing method on the same field (see the module docstring)."""
    d_dirty = torch.from_numpy(f.dirty).cuda()
    d_psf = torch.from_numpy(f.psf).cuda()
    total = args.warmup + args.steps
    ctx = asp.Context(d_dirty, d_psf, f.gain, f.threshold, max_iter=max(f.max_iter, total),
                      max_active=f.max_active, fit_solo_tiles=args.solo_tiles,
                      fit_min_tiles=args.min_tiles, fit_group=args.group)
    del d_dirty, d_psf
    widths = [float(w) for w in ctx.smooth_widths()]
    # full refreshes: every tile stale (entering init mode 2 marks them), then
    # one pick, timed with HIP events on the context's stream
    ctx.kernel_timing(True)
    reps = 3
    px0, fl0 = ctx.smooth_work()
    for _ in range(reps):
        ctx.set_init_mode(2)
        ctx.smooth_peak()
    px1, fl1 = ctx.smooth_work()
    kt = ctx.kernel_times()
    ms, n = kt["smooth_passes"]
    full_s = ms / reps * 1e-3
    flops = (fl1 - fl0) / reps
    achieved = flops / full_s / 1e12 if full_s > 0 else 0.0
    full = {"kernels": "k_smooth_cols + k_smooth_rows", "bound": "alu", "achieved": achieved,
            "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
            "frac_of_unpacked_fp32": achieved / (PEAK_FP32_VECTOR_TFLOPS / 2),
            "ms": full_s * 1e3, "flops": flops, "pixels": (px1 - px0) / reps,
            "pick_us": kt["smooth_pick"][0] / max(kt["smooth_pick"][1], 1) * 1e3}
    log(f"smoothing full refresh {json.dumps(full)}")
    # the timed region's iterations in init mode 2, from iteration 0
    ctx.set_init_mode(2)
    ctx.kernel_timing(False)
    ctx.run(args.warmup)
    ctx.kernel_timing(True)
    px0, fl0 = ctx.smooth_work()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc, r = ctx.run(args.steps)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t1
    px1, fl1 = ctx.smooth_work()
    kt = ctx.kernel_times()
    done = r["iterations"]
    pm, pn = kt["smooth_passes"]
    qm, qn = kt["smooth_pick"]
    out = {"widths": widths, "norm": "peak-1 beams", "switch": "convolved areas",
           "full_refresh": full,
           "run": {"iterations": done, "seconds": t_s,
                   "iterations_per_s": done / t_s if t_s > 0 else 0.0,
                   "plain_iterations_per_s": rep["iterations"] / secs if secs > 0 else 0.0,
                   "smoothed_fits": r["smoothed"],
                   "smoothed_fraction": r["smoothed"] / max(done, 1),
                   "trials_per_fit": r["lm_trials"] / max(done, 1),
                   "plain_trials_per_fit": rep["lm_trials"] / max(rep["iterations"], 1),
                   "rms": ctx.residual_rms(), "plain_rms": rms_plain,
                   "passes_us_per_iteration": pm / max(done, 1) * 1e3,
                   "pick_us_per_smoothed_iteration": qm / max(r["smoothed"], 1) * 1e3,
                   "refresh_pixels_per_smoothed_iteration": (px1 - px0) / max(r["smoothed"], 1),
                   "refresh_flops_per_smoothed_iteration": (fl1 - fl0) / max(r["smoothed"], 1),
                   "fit_ms": kt["fit"][0], "passes_ms": pm, "pick_ms": qm}}
    log(f"smoothing run {json.dumps(out['run'])}")
    ctx.close()
    return out


def peak_tiles_leg(args, f, rep, secs, ctx_full, torch, asp):
    """The timed region's iterations with the incremental peak search."""
    import numpy as np
    d_dirty = torch.from_numpy(f.dirty).cuda()
    d_psf = torch.from_numpy(f.psf).cuda()
    total = args.warmup + args.steps
    ctx = asp.Context(d_dirty, d_psf, f.gain, f.threshold, max_iter=max(f.max_iter, total),
                      max_active=f.max_active, fit_solo_tiles=args.solo_tiles,
                      fit_min_tiles=args.min_tiles, fit_group=args.group, peak_tiles=1)
    del d_dirty, d_psf
    ctx.run(args.warmup)
    ctx.kernel_timing(not args.no_kernel_events)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc, r = ctx.run(args.steps)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t1
    H, W = f.shape
    ntiles = ((H + 63) // 64) * ((W + 63) // 64)
    done = max(r["iterations"], 1)
    tiles = r["peak_tiles_scanned"] / done
    bytes_it = tiles * 64 * 64 * 4 + 8 * (ntiles + tiles)
    out = {"iterations": r["iterations"], "seconds": t_s,
           "iterations_per_s": r["iterations"] / t_s if t_s > 0 else 0.0,
           "full_scan_iterations_per_s": rep["iterations"] / secs if secs > 0 else 0.0,
           "tiles_per_iteration": tiles, "tiles": ntiles,
           "bytes_per_iteration": bytes_it, "full_scan_bytes_per_iteration": 4.0 * H * W,
           "same_residual_as_full_scan": bool(np.array_equal(ctx.residual(), ctx_full.residual()))}
    if not args.no_kernel_events:
        ms, n = ctx.kernel_times()["peak"]
        if n:
            out["peak_us_per_iteration"] = ms / n * 1e3
            out["achieved_gbs"] = bytes_it / (ms / n * 1e-3) / 1e9
    log(f"peak tiles {json.dumps(out)}")
    ctx.close()
    return out


def update_large_leg(args, f, torch, asp):
    """The residual update on large windows: a field of the same size holding one
    extended Gaussian (sigma 200 px, convolved), so that every iteration
    rewrites a window of millions of pixels; the update in its own launch, timed
    with HIP events, at 8 bytes per pixel read-modify-written."""
    import numpy as np
    H, W = f.shape
    sig = 200.0
    y = np.arange(H, dtype=np.float64)[:, None] - H / 2.0
    x = np.arange(W, dtype=np.float64)[None, :] - W / 2.0
    dirty = np.exp(-(x * x + y * y) / (2.0 * sig * sig)).astype(np.float32)
    d_dirty = torch.from_numpy(dirty).cuda()
    d_psf = torch.from_numpy(f.psf).cuda()
    del dirty
    n_iter = 20
    ctx = asp.Context(d_dirty, d_psf, 0.1, 0.0, max_iter=n_iter + 2, max_active=1,
                      update_launch=1)
    del d_dirty, d_psf
    ctx.run(2)
    ctx.kernel_timing(True)
    torch.cuda.synchronize()
    rc, r = ctx.run(n_iter)
    torch.cuda.synchronize()
    ms, n = ctx.kernel_times()["update"]
    ctx.close()
    if not n or ms <= 0.0:
        return None
    b = 8.0 * r["pixels_updated"] / n
    gbs = b / (ms / n * 1e-3) / 1e9
    out = {"field": f"{H}x{W}, one Gaussian of sigma {sig:.0f} px, gain 0.1, active set of 1",
           "launches": n, "pixels_per_launch": r["pixels_updated"] / n,
           "bytes_per_launch": b, "avg_launch_us": ms / n * 1e3, "achieved_gbs": gbs,
           "frac": gbs / PEAK_HBM_GBS}
    log(f"update on large windows {json.dumps(out)}")
    return out


def refresh_leg(args, f, rep, secs, ctx_plain, torch, asp):
    """The exact-PSF refresh: cost and effect on the true residual."""
    total = args.warmup + args.steps
    every = 500
    d_dirty = torch.from_numpy(f.dirty).cuda()
    d_psf = torch.from_numpy(f.psf).cuda()
    ctx = asp.Context(d_dirty, d_psf, f.gain, f.threshold, max_iter=max(f.max_iter, total),
                      max_active=f.max_active, fit_solo_tiles=args.solo_tiles,
                      fit_min_tiles=args.min_tiles, fit_group=args.group, refresh_every=every)
    del d_dirty, d_psf
    ctx.run(args.warmup)
    ctx.kernel_timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc, r = ctx.run(args.steps)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t1
    ms, n = ctx.kernel_times()["refresh"]
    rms_minor = ctx.residual_rms()
    ctx.refresh_residual()
    rms_true = ctx.residual_rms()
    ctx.close()
    # the plain run's residual against its exact one (the plain context is not
    # used after this leg)
    rms_plain_minor = ctx_plain.residual_rms()
    ctx_plain.kernel_timing(True)
    ctx_plain.refresh_residual()
    pms, pn = ctx_plain.kernel_times()["refresh"]
    rms_plain_true = ctx_plain.residual_rms()
    out = {"every": every, "iterations": r["iterations"], "seconds": t_s,
           "iterations_per_s": r["iterations"] / t_s if t_s > 0 else 0.0,
           "plain_iterations_per_s": rep["iterations"] / secs if secs > 0 else 0.0,
           "refreshes": n, "ms_per_refresh": ms / n if n else (pms / pn if pn else None),
           "rms_minor_cycle": rms_minor, "rms_true": rms_true,
           "plain_rms_minor_cycle": rms_plain_minor, "plain_rms_true": rms_plain_true}
    log(f"refresh {json.dumps(out)}")
    return out


def fft_size(n: int) -> int:
    """The smallest size >= n whose prime factors are 2, 3, 5 and 7 (the padded
    grid of the library's FFT convolutions)."""
    m = max(n, 1)
    while True:
        r = m
        for p in (2, 3, 5, 7):
            while r % p == 0:
                r //= p
        if r == 1:
            return m
        m += 1


def eval2004_bytes(H, W, Py, Px):
    """Least HBM bytes of one Asp-Clean2004 evaluation by FFT if the inverse
    transform were a single read-and-write pass: the PSF's half spectrum read
    and the four spectra formed from the factor DFTs written (8 + 32 bytes per
    padded pixel), transformed back (32 read, 32 written), and the image part
    of the four results read with R for the sums."""
    P = float(Py * Px)
    return 40 * P + 64 * P + 36.0 * H * W


def time_2004(f, n, mode, torch, asp):
    """n Asp-Clean2004 iterations from iteration 1 of the field, B (*) g formed
    as mode says ("auto": the cheaper of direct and FFT; "fft"): wall time,
    the per-iteration reports and the kernel timers."""
    # the 2004 iteration takes the smoothing method's matched-filter (L2) norm:
    # with peak-1 beams, and no switch back to the residual's peak, it keeps
    # choosing the widest trial width
    ctx4 = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                       max_active=f.max_active, smooth_norm=1)
    ctx4.set_2004_convolution(mode)
    ctx4.run_2004(1)                         # buffers, plans and the PSF spectrum
    ctx4.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(n):
        rc, r = ctx4.step_2004()
        if rc in (asp.ASP_STOP_THRESHOLD, asp.ASP_STOP_MAXITER):
            break
        reps.append(r)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    kt = ctx4.kernel_times()
    ctx4.close()
    return t, reps, kt


def asp2004_leg(args, f, rep, secs, torch, asp):
    """The paper's comparison (Table 3): Asp-Clean2004 -- Eq. 3 fitted with the
    true PSF convolved in every evaluation -- against Asp-Clean2016, both on
    the GPU.  On this field: the one-iteration time from iteration 1 of each,
    the 2004 iteration with its default convolution (direct where cheaper)
    and with FFTs only; on a 256^2 field with loop gain 0.35 (the size and
    gain of Table 3): both run to the same stop, then the ratios of total
    runtime, one-iteration runtime and iteration count (2004 over 2016)."""
    import numpy as np
    H, W = f.shape
    n = args.iters_2004
    out = {}
    t4, reps4, kt = time_2004(f, n, "auto", torch, asp)
    tf, repsf, ktf = time_2004(f, n, "fft", torch, asp)
    it4 = len(reps4)
    ev_ms, ev_n = kt["eval2004"]
    up_ms, up_n = kt["update2004"]
    evf_ms, evf_n = ktf["eval2004"]
    upf_ms, upf_n = ktf["update2004"]
    n_eval = sum(r["evaluations"] for r in reps4)
    n_direct = sum(r["direct_evals"] for r in reps4)
    ctx6 = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                       max_active=f.max_active)
    ctx6.run(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc6, r6 = ctx6.run(n)
    torch.cuda.synchronize()
    t6 = time.perf_counter() - t0
    ctx6.close()
    Py = fft_size(H + f.psf.shape[0] - 1)
    Px = fft_size(W + f.psf.shape[1] - 1)
    eb = eval2004_bytes(H, W, Py, Px)
    evf_s = evf_ms / evf_n * 1e-3 if evf_n else None
    it6 = r6["iterations"]
    itf = len(repsf)
    out["headline_field"] = {
        "iterations": it4, "from_iteration": 1,
        "ms_per_iteration_2004": 1e3 * t4 / max(it4, 1),
        "ms_per_iteration_2004_fft_only": 1e3 * tf / max(itf, 1),
        "ms_per_iteration_2016_same_iterations": 1e3 * t6 / max(it6, 1),
        "ms_per_iteration_2016_timed_region": 1e3 * secs / max(rep["iterations"], 1),
        "one_iteration_ratio": (t4 / max(it4, 1)) / (t6 / max(it6, 1)) if it6 and t6 > 0 else None,
        "one_iteration_ratio_fft_only":
            (tf / max(itf, 1)) / (t6 / max(it6, 1)) if it6 and t6 > 0 else None,
        "evaluations_per_fit": n_eval / max(it4, 1),
        "direct_evaluations": n_direct, "direct_updates": sum(r["direct_update"] for r in reps4),
        "fitted_omega_px": [float(np.sqrt(max(r["theta"][3], 0.0))) for r in reps4],
        "trials_per_fit_2004": sum(r["trials"] for r in reps4) / max(it4, 1),
        "trials_per_fit_2016": r6["lm_trials"] / max(it6, 1),
        "padded_grid": [Py, Px],
        "evaluation": {"kernels": "per-axis factors + row pass + column pass with the sums + LM "
                                  "(direct), or the FFT route below",
                       "ms": ev_ms / ev_n if ev_n else None,
                       "share_of_iteration": ev_ms / (t4 * 1e3) if t4 > 0 else None},
        "evaluation_fft_only": {
            "kernels": "per-axis factors + their 1-D DFTs + spectra x PSF spectrum + batched Z2D "
                       "+ sums + LM",
            "bound": "hbm", "ms": evf_s * 1e3 if evf_s else None,
            "bytes": eb, "achieved_gbs": eb / evf_s / 1e9 if evf_s else None,
            "frac": eb / evf_s / 1e9 / PEAK_HBM_GBS if evf_s else None},
        "update_ms": up_ms / up_n if up_n else None,
        "update_ms_fft_only": upf_ms / upf_n if upf_n else None}
    log(f"2004 on {f.name}: {json.dumps(out['headline_field'])}")

    import skygen
    g = skygen.make_evla(256, 256, 60, 6, 16.0, args.max_iter_2004, 5, psf_crop=128)
    gain = 0.35
    thr = float(0.02 * np.abs(g.dirty).max())
    # rocFFT compiles its kernels for a new size at first use (seconds): a
    # throwaway context takes that cost before either algorithm is timed
    w = asp.Context(g.dirty, g.psf, gain, thr, max_iter=2, smooth_norm=1)
    w.run_2004(1)
    w.run(1)
    w.close()
    res = {}
    for name in ("2004", "2016", "2016_kmax1"):
        # Asp-Clean2016 with its start-value heuristic (the smoothing method
        # and the 5 % switch), with an active set of up to 5 and of 1 (one
        # component per fit, as the 2004 iteration); the 2004 iteration always
        # smooths; all with the matched-filter (L2) norm of the smoothed images
        c = asp.Context(g.dirty, g.psf, gain, thr, max_iter=args.max_iter_2004,
                        max_active=1 if name == "2016_kmax1" else 5,
                        init_mode=0 if name == "2004" else 2, smooth_norm=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, r = c.run_2004(args.max_iter_2004) if name == "2004" else c.run(args.max_iter_2004)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        rms_minor = c.residual_rms()
        c.refresh_residual()
        res[name] = {"iterations": r["iterations"], "seconds": t,
                     "stop": {0: "iteration cap", 1: "threshold", 2: "max_iter"}.get(rc, str(rc)),
                     "ms_per_iteration": 1e3 * t / max(r["iterations"], 1),
                     "trials_per_fit": r["lm_trials"] / max(r["iterations"], 1),
                     "rms_minor_cycle": rms_minor, "rms_true": c.residual_rms()}
        c.close()
    a, b, b1 = res["2004"], res["2016"], res["2016_kmax1"]
    out["table3_style"] = {
        "field": "256x256 EVLA-like (60 points, 6 Gaussians), gain 0.35, "
                 f"threshold {thr:.4g} (2 % of the dirty peak), at most {args.max_iter_2004} "
                 "iterations, smoothing with the L2 norm",
        "asp2004": a, "asp2016": b, "asp2016_active_set_1": b1,
        "total_runtime_ratio": a["seconds"] / b["seconds"] if b["seconds"] > 0 else None,
        "one_iteration_runtime_ratio": a["ms_per_iteration"] / b["ms_per_iteration"],
        "iteration_number_ratio": a["iterations"] / max(b["iterations"], 1),
        "vs_active_set_1": {
            "total_runtime_ratio": a["seconds"] / b1["seconds"] if b1["seconds"] > 0 else None,
            "one_iteration_runtime_ratio": a["ms_per_iteration"] / b1["ms_per_iteration"],
            "iteration_number_ratio": a["iterations"] / max(b1["iterations"], 1)}}
    log(f"2004 vs 2016, Table 3 style: {json.dumps(out['table3_style'])}")
    return out


def bench_batch(args):
    """64 independent fields of sizes in {256, 512, 1024, 2048}^2, each with its
    own Gaussian PSF: aggregate iterations/s of one graph-captured persistent
    launch (team size and tile thresholds from the autotuner) against the
    same fields run one after another through asp_run, both from iteration 0."""
    import torch

    import paper_1606_07872_amd as asp
    import skygen
    t0 = time.time()
    fields = skygen.make_batch(64, 64)
    log(f"generated {len(fields)} fields, {sum(f.dirty.size for f in fields) / 1e6:.1f} Mpx, "
        f"in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    spec = [(f.dirty, f.psf, f.gain, f.threshold) for f in fields]
    n_iter = args.steps
    # the autotuner works on a batch of its own (its probes advance the fields)
    b = asp.Batch(spec, max_iter=5000, max_active=5)
    t1 = time.perf_counter()
    cfg = b.autotune(args.probe)
    log(f"autotuned {cfg} in {time.perf_counter() - t1:.1f}s")
    b.close()
    b = asp.Batch(spec, max_iter=5000, max_active=5)
    b.config(**cfg)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rep = b.run(n_iter)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t1
    value = rep["iterations"] / secs
    log(f"batched: {rep} in {secs:.3f}s -> {value:.0f} iterations/s")
    b.close()
    seq_secs, seq_iter = 0.0, 0
    for i, f in enumerate(fields):
        ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=5000, max_active=5)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rc, r = ctx.run(n_iter)
        torch.cuda.synchronize()
        seq_secs += time.perf_counter() - t1
        seq_iter += r["iterations"]
        ctx.close()
        if (i + 1) % 8 == 0:
            log(f"sequential: {i + 1} of {len(fields)} fields, {seq_iter} iterations in "
                f"{seq_secs:.1f}s")
    seq = seq_iter / seq_secs
    log(f"sequential: {seq_iter} iterations in {seq_secs:.3f}s -> {seq:.0f} iterations/s")
    line = {
        "metric": "aggregate minor-cycle iterations/s, batched fields",
        "value": value,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": rep["iterations"],
        "warmup": 0,
        "ms_per_step": 1e3 * secs / max(rep["iterations"], 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"64 fields of 256^2..2048^2 ({sum(f.dirty.size for f in fields)} px), "
                               f"Gaussian PSFs FWHM U[2.5, 6], {n_iter} iterations per field from 0, "
                               "one graph-captured persistent launch", "seed": 64,
                   "autotuned": cfg, "device_ms": rep["ms"]},
        "sequential": {"value": seq, "iterations": seq_iter, "seconds": seq_secs,
                       "speedup": value / seq if seq > 0 else None},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="c4096", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="time without the per-launch event pairs")
    ap.add_argument("--solo-tiles", type=int, default=0)
    ap.add_argument("--min-tiles", type=int, default=0)
    ap.add_argument("--group", type=int, default=0, help="work-groups per arrival counter")
    ap.add_argument("--update-launch", type=int, default=0, choices=(0, 1),
                    help="1: the residual update in its own launch instead of at the end "
                         "of the fit kernel")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (reference for HBM counters)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-versus-plain start comparison")
    ap.add_argument("--no-full-run", action="store_true",
                    help="skip the whole-configuration run (and the learned comparison)")
    ap.add_argument("--full-samples", type=int, default=4,
                    help="oracle lockstep iterations at the end of the whole run")
    ap.add_argument("--no-cold-peak", action="store_true",
                    help="skip the cold-cache peak search")
    ap.add_argument("--only", default=None, choices=("cold_peak", "update_large", "full_run"),
                    help="run one auxiliary leg alone (for profiling), no JSON line")
    ap.add_argument("--weights", default=None, help="proposal network weights (.npy)")
    ap.add_argument("--no-smoothing", action="store_true",
                    help="skip the smoothing-method (init mode 2) leg")
    ap.add_argument("--no-peak-tiles", action="store_true",
                    help="skip the incremental peak search leg")
    ap.add_argument("--no-update-large", action="store_true",
                    help="skip the update on large windows")
    ap.add_argument("--no-refresh", action="store_true",
                    help="skip the exact-PSF refresh leg")
    ap.add_argument("--no-2004", action="store_true",
                    help="skip the Asp-Clean2004 comparison leg")
    ap.add_argument("--iters-2004", type=int, default=6,
                    help="Asp-Clean2004 iterations timed on the bench field")
    ap.add_argument("--max-iter-2004", type=int, default=1000,
                    help="iteration cap of the Table 3 style comparison (256^2 field)")
    ap.add_argument("--probe", type=int, default=5,
                    help="iterations per field of each autotuner probe (batch workload)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the minor cycle "
              "here has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.workload == "batch":
        bench_batch(args)
        return
    if args.calibrate_copy:
        n = 64 << 20                        # floats: 256 MiB read and 256 MiB written
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 4 * n, "copies": 3}), flush=True)
        return

    import paper_1606_07872_amd as asp
    import skygen

    gen, seed = WORKLOADS[args.workload]
    t0 = time.time()
    f = getattr(skygen, gen)(seed)
    H, W = f.shape
    log(f"generated {f.name} {f.shape} in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    if args.only:
        fn = {"cold_peak": lambda: cold_peak_leg(args, f, torch, asp),
              "update_large": lambda: update_large_leg(args, f, torch, asp),
              "full_run": lambda: full_run_leg(args, f, torch, asp)[0]}[args.only]
        fn()
        return
    d_dirty = torch.from_numpy(f.dirty).cuda()
    d_psf = torch.from_numpy(f.psf).cuda()
    total = args.warmup + args.steps
    ctx = asp.Context(d_dirty, d_psf, f.gain, f.threshold, max_iter=max(f.max_iter, total),
                      max_active=f.max_active, fit_solo_tiles=args.solo_tiles,
                      fit_min_tiles=args.min_tiles, fit_group=args.group,
                      update_launch=args.update_launch)
    del d_dirty, d_psf
    torch.cuda.synchronize()
    ctx.run(args.warmup)
    torch.cuda.synchronize()
    want_cpu = not args.no_cpu_baseline
    if want_cpu:
        R0 = ctx.residual()
        comps0 = ctx.components_raw()
        k0, _ = ctx.counts()
        alpha_b, omega_b = ctx.psf_gauss()
    prof0 = ctx.fit_profile()
    ctx.kernel_timing(not args.no_kernel_events)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc, rep = ctx.run(args.steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    done = rep["iterations"]
    secs = t2 - t1
    value = done / secs if secs > 0 else 0.0
    log(f"{done} iterations in {secs:.3f}s, trials {rep['lm_trials']}, "
        f"not converged {rep['not_converged']}")
    prof1 = ctx.fit_profile()
    log("fit profile over the timed region " +
        json.dumps({k: round(prof1[k] - prof0[k], 1) for k in prof1}))

    roofline = None
    hbm = None
    if not args.no_kernel_events:
        kt = ctx.kernel_times()
        log(f"kernel times {kt}")
        fit_ms, fit_n = kt["fit"]
        peak_ms, peak_n = kt["peak"]
        upd_ms, upd_n = kt["update"]
        if fit_n and fit_ms > 0:
            avg_s = fit_ms / fit_n * 1e-3
            flops_per_launch = rep["gram_flops"] / fit_n
            achieved = flops_per_launch / avg_s / 1e12
            tr = fit_traffic(args.workload, args.warmup, done)
            roofline = {"kernel": "k_fit", "bound": "alu", "achieved": achieved,
                        "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": tr,
                        "avg_launch_us": avg_s * 1e6, "launches": fit_n,
                        "work_per_launch": flops_per_launch,
                        "includes_update": not args.update_launch,
                        "share_of_step": fit_ms / (secs * 1e3)}
        hbm = {}
        if peak_n and peak_ms > 0:
            b = 4.0 * H * W
            gbs = b / (peak_ms / peak_n * 1e-3) / 1e9
            hbm["k_peak"] = {"achieved_gbs": gbs, "frac": gbs / PEAK_HBM_GBS,
                             "avg_launch_us": peak_ms / peak_n * 1e3, "bytes_per_launch": b}
        if upd_n and upd_ms > 0:
            b = 8.0 * rep["pixels_updated"] / upd_n
            gbs = b / (upd_ms / upd_n * 1e-3) / 1e9
            hbm["k_update"] = {"achieved_gbs": gbs, "frac": gbs / PEAK_HBM_GBS,
                               "avg_launch_us": upd_ms / upd_n * 1e3, "bytes_per_launch": b}
        elif not args.update_launch:
            hbm["k_update"] = {"fused_into": "k_fit",
                               "bytes_per_iteration": 8.0 * rep["pixels_updated"] / max(done, 1)}

    rms_plain = ctx.residual_rms()

    cold_peak = None
    if not args.no_cold_peak and not args.no_kernel_events:
        cold_peak = cold_peak_leg(args, f, torch, asp)

    full_run, learned = None, None
    if not args.no_full_run:
        full_run, rms_full, secs_full = full_run_leg(args, f, torch, asp)
        wpath = args.weights or os.path.join(ROOT, "paper_1606_07872_amd", "proposal_weights.npy")
        if not args.no_learned and os.path.exists(wpath):
            learned = learned_equal_rms(args, f, wpath, full_run["iterations"], rms_full,
                                        secs_full, torch, asp)

    peak_tiles = None
    if not args.no_peak_tiles:
        peak_tiles = peak_tiles_leg(args, f, rep, secs, ctx, torch, asp)

    smoothing = None
    if not args.no_smoothing:
        smoothing = smoothing_leg(args, f, rep, secs, rms_plain, torch, asp)

    refresh = None
    if not args.no_refresh:
        refresh = refresh_leg(args, f, rep, secs, ctx, torch, asp)

    update_large = None
    if not args.no_update_large and not args.no_kernel_events:
        update_large = update_large_leg(args, f, torch, asp)

    asp2004 = None
    if not args.no_2004:
        asp2004 = asp2004_leg(args, f, rep, secs, torch, asp)

    cpu = None
    if want_cpu:
        log(f"oracle baseline for {args.cpu_seconds:.0f}s from iteration {k0}")
        cpu = cpu_baseline(f, R0, comps0, k0, alpha_b, omega_b, args.cpu_seconds)
        log(f"oracle {cpu['value']:.2f} iterations/s")

    line = {
        "metric": "minor-cycle iterations/s",
        "value": value,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": done,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * secs / max(done, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{f.name}: {H}x{W} FP32 EVLA-like field, active set <= "
                               f"{f.max_active}, gain {f.gain}, iterations "
                               f"{args.warmup}..{args.warmup + done}", "seed": f.seed,
                   "kernel_events": not args.no_kernel_events},
        "roofline": roofline,
        "hbm": hbm,
        "peak_cold": cold_peak,
        "full_run": full_run,
        "learned_vs_plain": learned,
        "smoothing": smoothing,
        "peak_tiles": peak_tiles,
        "refresh": refresh,
        "update_large": update_large,
        "asp2004_vs_2016": asp2004,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
