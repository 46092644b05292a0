"""Benchmark of the gfx950 Asp-Clean2016 minor cycle.

A step is one minor-cycle iteration: peak search, stop test, start values,
active-set selection, LM fit, commit and residual update, all on the device.
The workload is the 4096 x 4096 synthetic EVLA-like field (2000 points, 300
Gaussians with sigma U[2, 120] px, Y-array PSF, active set <= 10, gain 0.1).
Inputs are generated on the host, copied to HBM before the timed region, and
the timed region runs K iterations after W warm-up iterations.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "c4096": ("make_c4096", 4096),
    "c1024": ("make_c1024", 1000),
    "c128": ("make_c128", 0),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="c4096", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1606_07872_amd as asp
    import skygen

    gen, seed = WORKLOADS[args.workload]
    t0 = time.time()
    f = getattr(skygen, gen)(seed)
    print(f"[bench] generated {f.name} {f.shape} in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    torch.cuda.set_device(0)
    d_dirty = torch.from_numpy(f.dirty).cuda()
    d_psf = torch.from_numpy(f.psf).cuda()
    total = args.warmup + args.steps
    ctx = asp.Context(d_dirty, d_psf, f.gain, f.threshold, max_iter=max(f.max_iter, total),
                      max_active=f.max_active)
    del d_dirty, d_psf
    torch.cuda.synchronize()
    rc, wrep = ctx.run(args.warmup)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc, rep = ctx.run(args.steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    done = rep["iterations"]
    secs = t2 - t1
    value = done / secs if secs > 0 else 0.0
    print(f"[bench] {done} iterations in {secs:.3f}s, trials {rep['lm_trials']}, "
          f"not converged {rep['not_converged']}", file=sys.stderr, flush=True)
    print(f"[bench] fit profile {ctx.fit_profile()}", file=sys.stderr, flush=True)
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
        "dtype": "f32 pixels, f64 solve",
        "data": "synthetic",
        "config": {"workload": f"{f.name}: {f.shape[0]}x{f.shape[1]} FP32, active set <= "
                               f"{f.max_active}, gain {f.gain}", "seed": f.seed},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
