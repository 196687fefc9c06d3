#!/usr/bin/env python3
"""CRKSPH pair-interaction throughput on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the 64^3 = 262,144-particle Sedov-like jittered lattice (periodic
unit box, u = 1e4 on the 27 sites nearest the centre, 1e-2 elsewhere,
adaptive h for 64 neighbours, cubic spline) with N(0, 0.1) velocities and
N(0, 1) loss weights, inputs resident in HBM. One step = one pass of the
whole hot path: the forward (cell list, h solve and volume, neighbour list,
moments + FP64 corrections, density / grad v / EOS, force and du/dt) and the
adjoint of L = sum w_a . a + sum w_u du/dt (force, density, correction,
moment and volume adjoints). value = ordered force pairs (j != i,
r_ij < max(h_i, h_j)) per second of step wall time, FP32 pairs with FP64
solve and accumulators. The same run reports the forward alone on the
zero-velocity Sedov set, the same particles at the paper's gas resolution
(Wendland C4, n_h = 4, ~268 neighbours), the plain FP64 GPU form, the error of the
timed outputs against the FP64 oracle (values and one directional
derivative), the roofline of the dominant kernel (from the library's
HIP-event pass timers on the launch stream) and the oracle timed on the host
cores. Prints exactly one JSON line on stdout.
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

# Algorithmic flops per unit of each pair pass (FMA = 2, add/mul/div/sqrt/
# rsqrt = 1, one branch of the piecewise kernel): (flops, unit).
FLOPS_PER_PAIR = {"force": (216, "pairs_force"), "bwd_force": (680, "pairs_force"),
                  "moments": (109, "pairs_gather"), "density": (94, "pairs_gather")}
# Passes timed around exactly one kernel (the others group several).
SINGLE_KERNEL = ("candidates", "hsolve", "nlist", "moments", "density", "force", "bwd_force",
                 "bwd_density", "bwd_corr", "bwd_moments", "bwd_volume")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sedov64_v_fp32_traffic.md")


def kernel_source_hash() -> str:
    """sha256 over the library's kernel sources, as recorded with the traffic counters."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2511_21921_amd", "csrc", "*"))):
        if f.endswith((".hip", ".h")):
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def traffic_bytes(kernel: str):
    """HBM bytes per launch of kernel from the committed FETCH_SIZE / WRITE_SIZE counters,
    each scaled by its plain-copy calibration; None when the kernels changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            line = next(l for l in fh if l.startswith("traffic-json:"))
    except (OSError, StopIteration):
        return None
    t = json.loads(line.split(":", 1)[1])
    k = t["kernels"].get(kernel)
    if k is None or t["source_sha256"] != kernel_source_hash():
        return None
    return 1024.0 * (k["fetch_kib"] * t["fetch_factor"] + k["write_kib"] * t["write_factor"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(ps, precision, steps, warmup, backward, kernel=0):
    import numpy as np
    import torch

    from paper_2511_21921_amd import Context, Params
    dev = torch.device("cuda:0")
    p = Params(box=ps.box, n_h=ps.n_h, h_mode=ps.h_mode, precision=precision, timing=1,
               kernel=kernel)
    ctx = Context(p)
    R = p.real
    t = lambda a, dt=R: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    x, v, m, u, h = t(ps.x, torch.float64), t(ps.v), t(ps.m), t(ps.u), t(ps.h)
    wa = t(ps.w_a, torch.float64) if backward else None
    wu = t(ps.w_u, torch.float64) if backward else None
    ctx.reserve(ps.n)
    out = ctx.forward(x, v, m, u, h, stats=True)   # sizes workspace and lists
    stats = out["stats"]

    def step():
        ctx.forward(x, v, m, u, h, out=out)
        return ctx.backward(wa, wu) if backward else None

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.pass_times(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        g = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    passes = ctx.pass_times(reset=True)
    res = {k: val.cpu().numpy().astype(np.float64) for k, val in out.items()
           if isinstance(val, torch.Tensor)}
    if backward:
        res.update({k: val.cpu().numpy() for k, val in g.items()})
    ctx.close()
    ms = (t1 - t0) * 1e3 / steps
    return ms, stats, passes, res


# algorithmic HBM bytes per particle of the step's two elementwise kernels
# (FP32 state, FP64 positions and forces): first kick + drift + h update reads
# x 24, v 12, u 4, h 4, V 4, div v 12, a 24, du/dt 8 and writes x 24, v 12,
# u 4, h 4, predicted v 12 and u 4; the second kick reads v 12, u 4, a 24,
# du/dt 8 and writes v 12, u 4
STEP_BYTES_PER_PARTICLE = 92 + 60 + 48 + 16


def run_kdk(ps, steps, warmup, dt):
    """KDK steps (crk_kdk_step, FP32) from ps with h fixed at its solved value."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2511_21921_amd import FP32, Context, Params
    dev = torch.device("cuda:0")
    t = lambda a, dtype=torch.float32: torch.tensor(np.ascontiguousarray(a), dtype=dtype,
                                                    device=dev)
    # h: the solved smoothing lengths of the initial state
    p1 = Params(box=ps.box, n_h=ps.n_h, h_mode=1, precision=FP32)
    c1 = Context(p1)
    o1 = c1.forward(t(ps.x, torch.float64), t(ps.v), t(ps.m), t(ps.u), t(ps.h))
    h0 = o1["h"].clone()
    c1.close()
    p = dataclasses.replace(p1, h_mode=0, timing=1)
    ctx = Context(p)
    x, v, m, u = t(ps.x, torch.float64), t(ps.v), t(ps.m), t(ps.u)
    ctx.reserve(ps.n)
    out = ctx.forward(x, v, m, u, h0, stats=True)
    for _ in range(warmup):
        ctx.kdk_step(x, v, m, u, out, dt)
    torch.cuda.synchronize()
    ctx.pass_times(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.kdk_step(x, v, m, u, out, dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    passes = ctx.pass_times(reset=True)
    st = ctx.kdk_step(x, v, m, u, out, dt, stats=True)["stats"]
    torch.cuda.synchronize()
    ctx.close()
    return (t1 - t0) * 1e3 / steps, st, passes


def run_hkdk(ps, steps, warmup, dt):
    """One big step of the timestep hierarchy (crk_hkdk_step, FP32) from ps with
    h fixed at its solved value; levels from the signal speed s = c + |v|,
    level = clip(ceil(log2(s / median s)), 0, 3) (half the particles on level
    1, the hot core on level 3: eight substeps). Also times the same span as
    eight single-level steps of dt/8. Returns ms per big step, ms per eight
    single-level steps, the level counts."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2511_21921_amd import FP32, Context, Params
    dev = torch.device("cuda:0")
    t = lambda a, dtype=torch.float32: torch.tensor(np.ascontiguousarray(a), dtype=dtype,
                                                    device=dev)
    p1 = Params(box=ps.box, n_h=ps.n_h, h_mode=1, precision=FP32)
    c1 = Context(p1)
    o1 = c1.forward(t(ps.x, torch.float64), t(ps.v), t(ps.m), t(ps.u), t(ps.h))
    h0 = o1["h"].clone()
    c1.close()
    gam = p1.gamma
    sig = np.sqrt(gam * (gam - 1.0) * ps.u) + np.sqrt((ps.v ** 2).sum(0))
    lev = np.clip(np.ceil(np.log2(sig / np.median(sig))), 0, 3).astype(np.int32)
    levels = t(lev, torch.int32)
    p = dataclasses.replace(p1, h_mode=0)
    res = []
    for hier in (True, False):
        ctx = Context(p)
        x, v, m, u = t(ps.x, torch.float64), t(ps.v), t(ps.m), t(ps.u)
        ctx.reserve(ps.n)
        out = ctx.forward(x, v, m, u, h0.clone())

        def one():
            if hier:
                ctx.hkdk_step(x, v, m, u, out, levels, dt)
            else:
                for _ in range(8):
                    ctx.kdk_step(x, v, m, u, out, dt / 8)
        for _ in range(warmup):
            one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            one()
        torch.cuda.synchronize()
        res.append((time.perf_counter() - t0) * 1e3 / steps)
        ctx.close()
    return res[0], res[1], np.bincount(lev, minlength=4).tolist()


COOL_BYTES_PER_PARTICLE = 12  # FP32: read u and rho, write u


def run_cool(n, steps, warmup, seed=11):
    """Exact-integration cooling of n FP32 particles over a synthetic table:
    0.004 dex nodes over eight decades, a broken power law with a stable zero
    (heating below it, cooling above)."""
    import numpy as np
    import torch

    from paper_2511_21921_amd import FP32, Context, Params
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    dex, lu0 = 0.004, -3.0
    K = int(round(8 / dex)) + 1
    uk = 10 ** (lu0 + dex * np.arange(K))
    lam = (uk ** 1.5 - 0.1 ** 1.5) * np.exp(np.cumsum(rng.normal(0.0, 0.01, K)))
    ctx = Context(Params(precision=FP32, timing=1))
    ctx.cooling_table(lu0, dex, lam)
    u = torch.tensor(10 ** rng.uniform(-2.5, 4.5, n), dtype=torch.float32, device=dev)
    rho = torch.tensor(10 ** rng.uniform(-1, 1, n), dtype=torch.float32, device=dev)
    for _ in range(warmup):
        ctx.cool(rho, u, 1e-3)
    torch.cuda.synchronize()
    ctx.pass_times(reset=True)
    for _ in range(steps):
        ctx.cool(rho, u, 1e-3)
    torch.cuda.synchronize()
    us = pass_ms(ctx.pass_times(reset=True), "cool") * 1e3
    ctx.close()
    return us, K


def run_deposit(ng, ns, steps, warmup, seed=12):
    """Subgrid deposition of ns FP32 sources into ng FP32 gas particles, both
    uniform in the box; gas h for ~32 neighbours with a 20% spread, volumes
    1/ng; the sources hand over mass, metals, energy and momentum."""
    import numpy as np
    import torch

    from paper_2511_21921_amd import FP32, Context, Params, WENDLAND_C4
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    f = dict(dtype=torch.float32, device=dev)
    h0 = (32 / (4 * np.pi / 3) / ng) ** (1 / 3)
    gas = {"x": torch.tensor(rng.uniform(0, 1, (3, ng)), dtype=torch.float64, device=dev),
           "h": torch.tensor(h0 * (1 + 0.2 * rng.uniform(-1, 1, ng)), **f),
           "V": torch.full((ng,), 1.0 / ng, **f), "m": torch.full((ng,), 1.0 / ng, **f),
           "mZ": torch.full((ng,), 0.01 / ng, **f), "u": torch.ones(ng, **f),
           "v": torch.tensor(rng.normal(0, 0.1, (3, ng)), **f)}
    src = {"x": torch.tensor(rng.uniform(0, 1, (3, ns)), dtype=torch.float64, device=dev),
           "dM": torch.full((ns,), 1e-3 / ng, **f), "dMZ": torch.full((ns,), 1e-5 / ng, **f),
           "dE": torch.full((ns,), 1e-3 / ng, **f),
           "v": torch.tensor(rng.normal(0, 0.1, (3, ns)), **f)}
    ctx = Context(Params(precision=FP32, kernel=WENDLAND_C4, timing=1))
    for _ in range(warmup):
        ctx.deposit(gas, src, 2.25)
    torch.cuda.synchronize()
    ctx.pass_times(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.deposit(gas, src, 2.25)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e6
    dev_us = pass_ms(ctx.pass_times(reset=True), "deposit") * 1e3
    ctx.close()
    return wall, dev_us


def pass_ms(passes, name):
    tot, calls = passes[name]
    return tot / calls if calls else float("nan")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU form")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the time-step, hierarchy, cooling and deposition fields "
                         "(profiling runs of the forward + adjoint)")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the Wendland C4 n_h = 4 field (profiling runs of one workload)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="end with two plain 256 MiB device copies (untimed), the reference "
                         "for scaling the HBM byte counters of a profiling run")
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

    ps = synth.sedov64_v()
    ps0 = synth.sedov64()
    log("workload %s n=%d" % (ps.name, ps.n))
    ms32, st32, passes32, out32 = run_gpu(ps, FP32, args.steps, args.warmup, True)
    pairs = st32["n_pairs_force"]
    log("fp32 fwd+bwd: %.3f ms/step, pairs %d, passes %s" % (ms32, pairs, passes32))
    value = pairs / (ms32 * 1e-3)
    msf, stf, passesf, outf = run_gpu(ps0, FP32, args.steps, args.warmup, False)
    log("fp32 fwd (v = 0): %.3f ms/step" % msf)
    names = ("cells", "candidates", "hsolve", "nlist", "moments", "density", "force",
             "bwd_force", "bwd_density", "bwd_corr", "bwd_moments", "bwd_volume", "bwd_other")
    breakdown = {k: round(pass_ms(passes32, k), 4) for k in names}
    flops = {k: f * st32["n_" + unit] for k, (f, unit) in FLOPS_PER_PAIR.items()}
    pass_tflops = {k: round(f / (pass_ms(passes32, k) * 1e-3) / 1e12, 3) for k, f in flops.items()}
    # dominant kernel: the longest single-kernel pass of the step
    largest = max(SINGLE_KERNEL, key=lambda k: breakdown[k] if breakdown[k] == breakdown[k] else -1)
    rk = largest if largest in flops else max(flops, key=lambda k: breakdown[k])
    r_ms = pass_ms(passes32, rk)
    achieved = flops[rk] / (r_ms * 1e-3) / 1e12
    kname = "k_" + rk
    traffic = traffic_bytes(kname)

    # the paper's production resolution: Wendland C4, n_h = 4 (~268 neighbours)
    c4 = None
    if not args.no_c4:
        psc = synth.at_resolution(ps, 4.0)
        msc, stc, passesc, outc = run_gpu(psc, FP32, max(3, args.steps // 2), args.warmup, True,
                                          kernel=1)
        log("fp32 C4 n_h=4 fwd+bwd: %.3f ms/step" % msc)
        c4 = {"value": stc["n_pairs_force"] / (msc * 1e-3), "ms_per_step": round(msc, 4),
              "workload": "sedov64_v particles with the Wendland C4 kernel at n_h = 4 (~268 "
                          "neighbours, the paper's gas resolution), forward + adjoint",
              "pairs_force": stc["n_pairs_force"],
              "pass_ms": {k: round(pass_ms(passesc, k), 4) for k in names}}

    kdk = hkdk = cool = dep = None
    if not args.no_extras:
        # time integration around the passes: kick-drift-kick steps at fixed h
        # (the Thacker/continuity rate); dt is small enough that the ambient gas next
        # to the Sedov spike (u = 1e-2, du/dt up to ~1e4 from its half of the
        # pair work) stays positive over the timed steps
        msk, stk, passesk = run_kdk(ps, args.steps, args.warmup, 1e-9)
        step_us = pass_ms(passesk, "step") * 1e3  # two update launches per step
        kdk = {"ms_per_step": round(msk, 4), "value": stk["n_pairs_force"] / (msk * 1e-3),
               "unit": "interactions/s",
               "workload": "sedov64_v, kick-drift-kick steps (dt = 1e-9, lambda = 0.5) with h "
                           "integrated by the Thacker/continuity rate from the solved h",
               "speculative_forwards": stk["speculative"],
               "update_kernels": {"us_per_step": round(2 * step_us, 2),
                                  "bytes_per_particle": STEP_BYTES_PER_PARTICLE,
                                  "GBps": round(STEP_BYTES_PER_PARTICLE * ps.n /
                                                (2 * step_us * 1e-6) / 1e9, 1)}}
        log("kdk step: %.3f ms, update kernels %.1f us" % (msk, 2 * step_us))

        # timestep hierarchy (App. A.4): one big step on levels 0-3
        hk = max(2, args.steps // 4)
        msh, ms8, hcount = run_hkdk(ps, hk, 1, 8e-9)
        hkdk = {"ms_per_big_step": round(msh, 4), "ms_per_8_single_level_steps": round(ms8, 4),
                "levels_0_1_2_3": hcount,
                "workload": "sedov64_v, one big step dt = 8e-9 on levels clip(ceil(log2(s / "
                            "median s)), 0, 3), s = c + |v| (eight substeps; passive "
                            "particles skip the pair sums), against eight single-level "
                            "steps of dt / 8"}
        log("hkdk step: %.3f ms per big step vs %.3f ms for 8 single-level steps, levels %s"
            % (msh, ms8, hcount))

        # exact-integration cooling (Sec. 2.2), 2^24 particles
        ncool = 1 << 24
        cus, ck = run_cool(ncool, args.steps, args.warmup)
        cool_bps = COOL_BYTES_PER_PARTICLE * ncool / (cus * 1e-6)
        cool = {"us_per_launch": round(cus, 2), "value": ncool / (cus * 1e-6),
                "unit": "particles/s",
                "workload": "2^24 FP32 particles, u log-uniform over 7 decades, rho over 2; "
                            "table of %d nodes at 0.004 dex, a broken power law with a stable "
                            "zero" % ck,
                "hbm": {"bytes_per_particle": COOL_BYTES_PER_PARTICLE,
                        "GBps": round(cool_bps / 1e9, 1),
                        "frac_of_8TBps": round(cool_bps / 8e12, 3)}}
        log("cooling: %.1f us for %d particles" % (cus, ncool))

        # subgrid deposition (App. A.2 eq. (Vsg), eq. (Anorm)): 2^21 gas, 2^16 sources
        ngas, nsrc = 1 << 21, 1 << 16
        dwall, ddev = run_deposit(ngas, nsrc, args.steps, args.warmup)
        dep = {"us_per_call": round(dwall, 2), "device_us_per_call": round(ddev, 2),
               "value": nsrc / (dwall * 1e-6), "unit": "sources/s",
               "workload": "2^21 FP32 gas (uniform, ~32 neighbours, h spread 20%), 2^16 "
                           "uniform sources, Wendland C4, n_h,s = 2.25; one gas grid, one pair "
                           "sort, two host reads"}
        log("deposit: %.1f us per call (device %.1f us)" % (dwall, ddev))

    fp64 = None
    if not args.no_fp64:
        k64 = max(3, args.steps // 2)
        ms64, st64, passes64, _ = run_gpu(ps, FP64, k64, 1, True)
        ms64f, _, _, _ = run_gpu(ps0, FP64, k64, 1, False)
        log("fp64: fwd+bwd %.3f ms/step, fwd %.3f ms/step" % (ms64, ms64f))
        fp64 = {"value": st64["n_pairs_force"] / (ms64 * 1e-3), "ms_per_step": round(ms64, 4),
                "fp32_speedup": round(ms64 / ms32, 3),
                "fwd_value": stf["n_pairs_force"] / (ms64f * 1e-3),
                "fwd_ms_per_step": round(ms64f, 4), "fwd_fp32_speedup": round(ms64f / msf, 3),
                "pass_ms": {k: round(pass_ms(passes64, k), 4) for k in names}}

    cpu = None
    errs = None
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        # repeat the whole-workload forward until about 10 s of CPU work (at most 10 times)
        reps, tc = 0, 0.0
        while reps < 10 and (reps == 0 or tc < 10.0):
            t0 = time.perf_counter()
            ref = oracle.forward(ps.x, ps.v, ps.m, ps.u, ps.h, oracle.params_for(ps), nbr_mode=1)
            tc += time.perf_counter() - t0
            reps += 1
        cpu = {"value": reps * ref["pairs_force"] / tc, "unit": "interactions/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "the whole workload, %d times: FP64 forward of all 262144 particles "
                         "(%d force pairs, grid neighbour search), %.1f s in all; the oracle has "
                         "no reverse mode, so this is a forward-only rate"
                         % (reps, ref["pairs_force"], tc)}
        ref0 = oracle.forward(ps0.x, ps0.v, ps0.m, ps0.u, ps0.h, oracle.params_for(ps0),
                              nbr_mode=1)
        rng = np.random.default_rng(11)
        dx, dv = rng.normal(size=ps.x.shape), rng.normal(size=ps.x.shape)
        du = rng.normal(size=ps.n) * ps.u
        j = oracle.jvp(ps.x, ps.v, ps.m, ps.u, ps.h, oracle.params_for(ps), dx, dv, du, 0.0,
                       0.0, nbr_mode=1)
        jl = float((ps.w_a * j["d_accel"]).sum() + (ps.w_u * j["d_dudt"]).sum())
        gl = float((out32["g_x"] * dx).sum() + (out32["g_v"] * dv).sum() +
                   (out32["g_u"] * du).sum())
        rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
        errs = {"accel_relL2": rel(out32["accel"], ref["accel"]),
                "dudt_relL2": rel(out32["dudt"], ref["dudt"]),
                "grad_jvp_rel": abs(gl - jl) / abs(jl),
                "fwd_accel_relL2": rel(outf["accel"], ref0["accel"]),
                "h_relmax": float(np.max(np.abs(out32["h"] / ref["h"] - 1))),
                "rho_relmax": float(np.max(np.abs(out32["rho"] / ref["rho"] - 1))),
                "pairs_oracle": ref["pairs_force"]}
        log("errors", errs)
        if c4 is not None:
            refc = oracle.forward(psc.x, psc.v, psc.m, psc.u, psc.h,
                                  oracle.params_for(psc, kernel=1), nbr_mode=1)
            c4["errors"] = {"accel_relL2": rel(outc["accel"], refc["accel"]),
                            "dudt_relL2": rel(outc["dudt"], refc["dudt"]),
                            "pairs_oracle": refc["pairs_force"]}
            log("C4 errors", c4["errors"])

    line = {
        "metric": METRIC, "value": value, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms32, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sedov64_v: 64^3=262144-particle jittered lattice, Sedov spike, "
                               "N(0,0.1) velocities, adaptive h (64 neighbours), cubic spline; "
                               "forward + adjoint of sum w_a.a + sum w_u.du/dt",
                   "n": ps.n, "pairs_force": pairs, "pairs_gather": st32["n_pairs_gather"],
                   "step": "forward+backward"},
        "roofline": {"bound": "alu", "kernel": kname, "achieved": round(achieved, 3),
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "flops_per_unit": FLOPS_PER_PAIR[rk][0], "unit_count": FLOPS_PER_PAIR[rk][1],
                     "kernel_ms": round(r_ms, 4), "largest_pass": largest},
        "fwd": {"value": stf["n_pairs_force"] / (msf * 1e-3), "ms_per_step": round(msf, 4),
                "workload": "sedov64 (same particles, zero velocity), forward only",
                "pass_ms": {k: round(pass_ms(passesf, k), 4) for k in names[:7]}},
        "pass_ms": breakdown, "pass_tflops": pass_tflops,
        "c4_268": c4, "kdk_step": kdk, "hkdk_step": hkdk, "cooling": cool, "deposit": dep,
        "fp64": fp64, "errors": errs, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    if args.calibration_copy:
        import torch
        a = torch.ones(64 * 2 ** 20, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
