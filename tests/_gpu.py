"""Helpers for the GPU parity tests: run the HIP path on a synth.ParticleSet."""
import numpy as np
import torch

from paper_2511_21921_amd import FP32, FP64, Context, Params

DEV = torch.device("cuda:0")


def params_for(ps, precision=FP32, **kw):
    p = Params(box=ps.box, n_h=ps.n_h, h_mode=ps.h_mode, precision=precision)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def to_dev(ps, precision):
    R = torch.float64 if precision == FP64 else torch.float32
    t = lambda a, dt=R: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)
    return t(ps.x, torch.float64), t(ps.v), t(ps.m), t(ps.u), t(ps.h)


def run(ps, precision=FP32, ctx=None, stats=True, **kw):
    p = params_for(ps, precision, **kw)
    if ctx is None:
        ctx = Context(p)
    x, v, m, u, h = to_dev(ps, precision)
    out = ctx.forward(x, v, m, u, h, stats=stats)
    torch.cuda.synchronize()
    res = {k: (val.cpu().numpy().astype(np.float64) if isinstance(val, torch.Tensor) else val)
           for k, val in out.items()}
    return res, ctx


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def rel_max(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


def errors(g, o, h):
    """Error metrics of every output (GPU g vs oracle o); scaled where the value can vanish."""
    e = {}
    e["h"] = rel_max(g["h"], o["h"])
    e["V"] = rel_max(g["V"], o["V"])
    e["rho"] = rel_max(g["rho"], o["rho"])
    e["A"] = rel_max(g["A"], o["A"])
    hmin = float(np.min(h))
    for k, floor in (("B", 1 / hmin), ("gradA", 1 / hmin), ("gradB", 1 / hmin ** 2),
                     ("gradv", 0.0)):
        sc = max(np.abs(o[k]).max(), floor, 1e-300)
        e[k + "/max"] = np.max(np.abs(g[k] - o[k])) / sc
    e["accel_relL2"] = rel_l2(g["accel"], o["accel"])
    e["dudt_relL2"] = rel_l2(g["dudt"], o["dudt"])
    e["accel_scaled_max"] = np.max(np.abs(g["accel"] - o["accel"]).max(0) /
                                   np.maximum(o["scale_a"], 1e-300))
    e["dudt_scaled_max"] = np.max(np.abs(g["dudt"] - o["dudt"]) /
                                  np.maximum(o["scale_u"], 1e-300))
    return e
