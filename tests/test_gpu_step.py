"""The kick-drift-kick step on the GPU (crk_kdk_step) against the oracle's step.

Three steps from the same state on both sides (initial h: the oracle's exact
Thacker root; h then evolves by the step's own rate), compared after every
step: the state (x, v, u, h) and the end-of-step forward outputs. The GPU
keeps v, u and h in the working precision and x in FP64, like the oracle.
Bounds: FP64 1e-11 (relative, positions absolute in box units); FP32 the
single-evaluation bounds of the forward parity tests, plus 2e-6 on the state
(one FP32 rounding of v^1/2, u^1/2 and h per step, and the FP32 V and grad v
that feed the smoothing-length rate). The same in FP64 with the Wendland C4
kernel.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2511_21921_amd import FP32, FP64, WENDLAND_C4, Context, CrkError

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

from tests import _gpu  # noqa: E402
from tests.test_gpu_forward import FP32_BOUNDS, FP64_BOUNDS  # noqa: E402

STATE_BOUND = {FP64: 1e-11, FP32: 2e-6}


def _start(n, seed, mass_spread=0.0):
    ps = synth.random_small(n, seed, mass_spread=mass_spread)
    h = oracle.forward(ps.x, ps.v, ps.m, ps.u, ps.h, oracle.params_for(ps))["h"]
    ps.h = h
    ps.h_mode = 0
    return ps


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_three_steps_match_the_oracle(precision):
    ps = _start(3000, 301, mass_spread=0.1)
    print("case random3000 precision=%d" % precision, flush=True)
    dt, lam = 2e-4, 0.5  # no particle's u changes by more than ~2 % in a step
    p = oracle.params_for(ps)
    ctx = Context(_gpu.params_for(ps, precision))
    x, v, m, u, h = _gpu.to_dev(ps, precision)
    out = ctx.forward(x, v, m, u, h, stats=True)
    ox, ov, ou, oh = ps.x.copy(), ps.v.copy(), ps.u.copy(), ps.h.copy()
    prev = oracle.forward(ox, ov, ps.m, ou, oh, p)
    bounds = FP64_BOUNDS if precision == FP64 else FP32_BOUNDS
    sb = STATE_BOUND[precision]
    spec = []
    for it in range(3):
        out = ctx.kdk_step(x, v, m, u, out, dt, lam, stats=True)
        torch.cuda.synchronize()
        spec.append(out["stats"]["speculative"])
        o = oracle.kdk_step(ox, ov, ps.m, ou, oh, prev, p, dt, lam)
        ox, ov, ou, oh, prev = o["x"], o["v"], o["u"], o["h"], o
        dx = np.abs(_np(x) - ox)
        dx = np.minimum(dx, 1.0 - dx)  # periodic
        st = {"x": dx.max(), "v": np.abs(_np(v) - ov).max() / np.abs(ov).max(),
              "u": np.max(np.abs(_np(u) / ou - 1)), "h": np.max(np.abs(_np(out["h"]) / oh - 1))}
        g = {k: _np(t) for k, t in out.items() if isinstance(t, torch.Tensor)}
        e = _gpu.errors(g, o, o["h"])
        print("step", it, {k: "%.2e" % val for k, val in st.items()},
              {k: "%.2e" % val for k, val in e.items()}, out["stats"], flush=True)
        for k, val in st.items():
            assert val <= sb, (it, k, val)
        for k, b in bounds.items():
            assert e[k] <= b, (it, k, e[k], b)
    # after the first step the geometry of the previous evaluation usually holds
    assert sum(spec) >= 1


def test_steps_with_the_wendland_c4_kernel():
    # the same three steps with the C4 kernel at ~84 neighbours (h solved
    # with that kernel first), FP64
    ps = synth.random_small(2000, 331, n_ngb=100.0, mass_spread=0.1)
    p = oracle.params_for(ps, kernel=WENDLAND_C4)
    ps.h = oracle.forward(ps.x, ps.v, ps.m, ps.u, ps.h, p)["h"]
    ps.h_mode = 0
    print("case random2000 C4 FP64", flush=True)
    dt, lam = 2e-4, 0.5
    p = oracle.params_for(ps, kernel=WENDLAND_C4)
    ctx = Context(_gpu.params_for(ps, FP64, kernel=WENDLAND_C4))
    x, v, m, u, h = _gpu.to_dev(ps, FP64)
    out = ctx.forward(x, v, m, u, h)
    ox, ov, ou, oh = ps.x.copy(), ps.v.copy(), ps.u.copy(), ps.h.copy()
    prev = oracle.forward(ox, ov, ps.m, ou, oh, p)
    for it in range(3):
        out = ctx.kdk_step(x, v, m, u, out, dt, lam)
        torch.cuda.synchronize()
        o = oracle.kdk_step(ox, ov, ps.m, ou, oh, prev, p, dt, lam)
        ox, ov, ou, oh, prev = o["x"], o["v"], o["u"], o["h"], o
        dx = np.abs(_np(x) - ox)
        dx = np.minimum(dx, 1.0 - dx)
        st = {"x": dx.max(), "v": np.abs(_np(v) - ov).max() / np.abs(ov).max(),
              "u": np.max(np.abs(_np(u) / ou - 1)), "h": np.max(np.abs(_np(out["h"]) / oh - 1))}
        g = {k: _np(t) for k, t in out.items() if isinstance(t, torch.Tensor)}
        e = _gpu.errors(g, o, o["h"])
        print("step", it, {k: "%.2e" % val for k, val in st.items()},
              {k: "%.2e" % val for k, val in e.items()}, flush=True)
        for k, val in st.items():
            assert val <= STATE_BOUND[FP64], (it, k, val)
        for k, b in FP64_BOUNDS.items():
            assert e[k] <= b, (it, k, e[k], b)


def test_steps_conserve_momentum_and_track_energy():
    ps = _start(4000, 302)
    dt = 2e-4
    ctx = Context(_gpu.params_for(ps, FP64))
    x, v, m, u, h = _gpu.to_dev(ps, FP64)
    out = ctx.forward(x, v, m, u, h)
    mm = ps.m
    p0 = (mm * ps.v).sum(1)
    e0 = (mm * (0.5 * (ps.v ** 2).sum(0) + ps.u)).sum()
    scale = (mm * np.abs(ps.v)).sum()
    for it in range(5):
        out = ctx.kdk_step(x, v, m, u, out, dt, 0.5)
    torch.cuda.synchronize()
    vv, uu = _np(v), _np(u)
    assert np.abs((mm * vv).sum(1) - p0).max() < 1e-13 * scale
    e1 = (mm * (0.5 * (vv ** 2).sum(0) + uu)).sum()
    print("energy drift over 5 steps %.2e" % ((e1 - e0) / e0), flush=True)
    assert abs(e1 - e0) < 2e-5 * e0  # the oracle's own drift here is 3.5e-6


def test_step_argument_errors():
    ps = _start(500, 303)
    ctx = Context(_gpu.params_for(ps, FP32, h_mode=1))
    x, v, m, u, h = _gpu.to_dev(ps, FP32)
    out = ctx.forward(x, v, m, u, h)
    with pytest.raises(CrkError) as ei:
        ctx.kdk_step(x, v, m, u, out, 1e-3)
    assert ei.value.status == -1  # h_mode 1
    ctx.set_params(_gpu.params_for(ps, FP32, h_mode=0))
    for dt, lam in ((0.0, 0.5), (float("nan"), 0.5), (1e-3, 1.5)):
        with pytest.raises(CrkError) as ei:
            ctx.kdk_step(x, v, m, u, out, dt, lam)
        assert ei.value.status == -1
