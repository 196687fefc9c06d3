#!/usr/bin/env python3
"""CRKSPH pair-interaction throughput on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the 64^3 = 262,144-particle Sedov-like jittered lattice (periodic
unit box, u = 1e4 on the 27 sites nearest the centre, 1e-2 elsewhere,
adaptive h for 64 neighbours, cubic spline), inputs resident in HBM.
One step = one pass of the whole hot path: cell list, h solve and volume,
neighbour list, moments + FP64 corrections, density / grad v / EOS, force and
du/dt. value = ordered force pairs (j != i, r_ij < max(h_i, h_j)) per second
of step wall time, FP32 pairs with FP64 solve and accumulators. The same run
reports the plain FP64 GPU form, the error of the timed outputs against the
FP64 oracle, the roofline of the dominant kernel (from the library's HIP-event
pass timers on the launch stream) and the oracle timed on the host cores.
Prints exactly one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CRKSPH pair interactions/s (fwd, fwd+bwd) FP32 vs FP64 at rel err ≤1e-5"
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (published)
PEAK_HBM_GBS = 8000.0

# Algorithmic flops per ordered pair of each pair pass (FMA = 2, add/mul/
# div/sqrt/rsqrt = 1, one branch of the piecewise kernel); see the design doc.
FLOPS_PER_PAIR = {"force": 216, "density": 94, "moments": 109}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(ps, precision, steps, warmup):
    import numpy as np
    import torch

    from paper_2511_21921_amd import Context, Params
    dev = torch.device("cuda:0")
    p = Params(box=ps.box, n_h=ps.n_h, h_mode=ps.h_mode, precision=precision, timing=1)
    ctx = Context(p)
    R = p.real
    t = lambda a, dt=R: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    x, v, m, u, h = t(ps.x, torch.float64), t(ps.v), t(ps.m), t(ps.u), t(ps.h)
    ctx.reserve(ps.n)
    out = ctx.forward(x, v, m, u, h, stats=True)   # sizes workspace and lists
    stats = out["stats"]
    for _ in range(warmup):
        ctx.forward(x, v, m, u, h, out=out)
    torch.cuda.synchronize()
    ctx.pass_times(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.forward(x, v, m, u, h, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    passes = ctx.pass_times(reset=True)
    res = {k: val.cpu().numpy().astype(np.float64) for k, val in out.items()
           if isinstance(val, torch.Tensor)}
    ctx.close()
    ms = (t1 - t0) * 1e3 / steps
    return ms, stats, passes, res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU form")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the CRKSPH passes run on a single MI355X here "
              "(multi-GPU sharding is a design note, not a measured path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import synth
    from paper_2511_21921_amd import FP32, FP64

    ps = synth.sedov64()
    log("workload %s n=%d" % (ps.name, ps.n))
    ms32, st32, passes32, out32 = run_gpu(ps, FP32, args.steps, args.warmup)
    pairs = st32["n_pairs_force"]
    log("fp32: %.3f ms/step, pairs %d, passes %s" % (ms32, pairs, passes32))
    value = pairs / (ms32 * 1e-3)

    def pass_ms(passes, name):
        tot, calls = passes[name]
        return tot / calls if calls else float("nan")

    f_ms = pass_ms(passes32, "force")
    achieved = FLOPS_PER_PAIR["force"] * pairs / (f_ms * 1e-3) / 1e12
    breakdown = {k: round(pass_ms(passes32, k), 4) for k in
                 ("cells", "hsolve", "nlist", "moments", "density", "force")}
    pass_tflops = {
        "moments": FLOPS_PER_PAIR["moments"] * st32["n_pairs_gather"] /
        (pass_ms(passes32, "moments") * 1e-3) / 1e12,
        "density": FLOPS_PER_PAIR["density"] * st32["n_pairs_gather"] /
        (pass_ms(passes32, "density") * 1e-3) / 1e12,
        "force": achieved}

    fp64 = None
    if not args.no_fp64:
        ms64, st64, passes64, _ = run_gpu(ps, FP64, max(3, args.steps // 2), 1)
        log("fp64: %.3f ms/step" % ms64)
        fp64 = {"value": st64["n_pairs_force"] / (ms64 * 1e-3), "ms_per_step": round(ms64, 4),
                "fp32_speedup": round(ms64 / ms32, 3),
                "pass_ms": {k: round(pass_ms(passes64, k), 4) for k in breakdown}}

    cpu = None
    errs = None
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        t0 = time.perf_counter()
        ref = oracle.forward(ps.x, ps.v, ps.m, ps.u, ps.h, oracle.params_for(ps), nbr_mode=1)
        tc = time.perf_counter() - t0
        cpu = {"value": ref["pairs_force"] / tc, "unit": "interactions/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "whole workload once (262144 particles, %d force pairs), FP64 forward "
                         "with grid neighbour search, %.1f s" % (ref["pairs_force"], tc)}
        rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
        errs = {"accel_relL2": rel(out32["accel"], ref["accel"]),
                "dudt_abs_max": float(np.abs(out32["dudt"]).max()),
                "h_relmax": float(np.max(np.abs(out32["h"] / ref["h"] - 1))),
                "rho_relmax": float(np.max(np.abs(out32["rho"] / ref["rho"] - 1))),
                "pairs_oracle": ref["pairs_force"]}
        log("errors", errs)

    line = {
        "metric": METRIC, "value": value, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms32, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sedov64: 64^3=262144-particle jittered lattice, Sedov spike, "
                               "adaptive h (64 neighbours), cubic spline, forward passes",
                   "n": ps.n, "pairs_force": pairs, "pairs_gather": st32["n_pairs_gather"],
                   "step": "forward"},
        "roofline": {"bound": "alu", "kernel": "k_force", "achieved": round(achieved, 3),
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
                     "flops_per_pair": FLOPS_PER_PAIR["force"], "kernel_ms": round(f_ms, 4)},
        "pass_ms": breakdown, "pass_tflops": {k: round(v, 3) for k, v in pass_tflops.items()},
        "fp64": fp64, "errors": errs, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
