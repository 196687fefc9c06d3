"""The hierarchical KDK step on the GPU (crk_hkdk_step) against the oracle's
(App. A.4 power-of-two levels; App. A.3 passive h, V and rho).

Two big steps from the same state on both sides, levels 0, 1 and 2 mixed
(four substeps per big step, passive particles in every evaluation but the
last), compared after each big step: the synchronised state (x, v, u, h) and
the last evaluation (every particle active there), on the set and step size of
the single-level step's test. Bounds: FP64 1e-11, the single evaluation's
(measured ~1e-14); FP32 the forward's single-evaluation bounds and 1e-5 on
the state (four substeps of FP32 roundings of v^1/2, u^1/2, h and of the
passive V and rho; measured <= 2.5e-6). A wrong passive state shows at
1e-3 and above. Also:
all levels 0 is crk_kdk_step and one level L everywhere is 2^L single-level
steps of dt / 2^L (up to the rounding of the two h-update forms), in FP64
and FP32; one big step with the Wendland C4 kernel (FP64); the argument errors.
Timestep refinement (App. A.5): two big steps on levels 0-2 with random
refinements to finer levels (up to 3: eight substeps), at substeps on their
new level's grid, midway through intervals and at their starts, against the
oracle's refined step to the same bounds; no refinement (refine_at -1 for
every particle) is the plain step bit for bit; refinements that break the
rules are CRK_EINVAL.
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

STATE_BOUND = {FP64: 1e-11, FP32: 1e-5}


def _start(n, seed):
    ps = synth.random_small(n, seed, mass_spread=0.1)
    ps.h = oracle.forward(ps.x, ps.v, ps.m, ps.u, ps.h, oracle.params_for(ps))["h"]
    ps.h_mode = 0
    return ps


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


class _Progress(list):
    """A trace that prints a line per substep of the oracle's big step."""

    def append(self, item):
        print("  oracle substep %d" % (len(self) + 1), flush=True)
        super().append(None)


def _state_errors(x, v, u, out, o):
    dx = np.abs(_np(x) - o["x"])
    dx = np.minimum(dx, 1.0 - dx)  # periodic
    return {"x": dx.max(), "v": np.abs(_np(v) - o["v"]).max() / np.abs(o["v"]).max(),
            "u": np.max(np.abs(_np(u) / o["u"] - 1)),
            "h": np.max(np.abs(_np(out["h"]) / o["h"] - 1))}


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_two_big_steps_match_the_oracle(precision):
    ps = _start(3000, 301)
    print("case random3000 levels 0-2 precision=%d" % precision, flush=True)
    # the single-level step's regime (its test's set and step): no particle's
    # u changes by more than ~2 % per step, so FP32 force errors (~1e-5 of
    # sum |F_ij| / m) are not amplified by near-vanishing energies
    dt, lam = 2e-4, 0.5
    lev = np.random.default_rng(312).integers(0, 3, ps.n)
    lev[0] = 2
    p = oracle.params_for(ps)
    ctx = Context(_gpu.params_for(ps, precision))
    x, v, m, u, h = _gpu.to_dev(ps, precision)
    levels = torch.tensor(lev, dtype=torch.int32, device=x.device)
    out = ctx.forward(x, v, m, u, h)
    ox, ov, ou, oh = ps.x.copy(), ps.v.copy(), ps.u.copy(), ps.h.copy()
    prev = oracle.forward(ox, ov, ps.m, ou, oh, p)
    bounds = FP64_BOUNDS if precision == FP64 else FP32_BOUNDS
    for it in range(2):
        out = ctx.hkdk_step(x, v, m, u, out, levels, dt, lam, stats=True)
        torch.cuda.synchronize()
        o = oracle.hkdk_step(ox, ov, ps.m, ou, oh, prev, lev, p, dt, lam)
        ox, ov, ou, oh, prev = o["x"], o["v"], o["u"], o["h"], o
        st = _state_errors(x, v, u, out, o)
        g = {k: _np(t) for k, t in out.items() if isinstance(t, torch.Tensor)}
        e = _gpu.errors(g, o, o["h"])
        print("big step", it, {k: "%.2e" % val for k, val in st.items()},
              {k: "%.2e" % val for k, val in e.items()}, flush=True)
        for k, val in st.items():
            assert val <= STATE_BOUND[precision], (it, k, val)
        for k, b in bounds.items():
            assert e[k] <= b, (it, k, e[k], b)


def test_big_step_with_the_wendland_c4_kernel():
    # the hierarchy's instances of the passes for the C4 kernel, ~100
    # neighbours, h solved with that kernel before the step; FP64
    ps = synth.random_small(2000, 321, n_ngb=100.0, mass_spread=0.1)
    ps.h = oracle.forward(ps.x, ps.v, ps.m, ps.u, ps.h,
                          oracle.params_for(ps, kernel=WENDLAND_C4))["h"]
    ps.h_mode = 0
    print("case random2000 C4 levels 0-2 FP64", flush=True)
    dt, lam = 2e-4, 0.5
    lev = np.random.default_rng(322).integers(0, 3, ps.n)
    lev[0] = 2
    p = oracle.params_for(ps, kernel=WENDLAND_C4)
    ctx = Context(_gpu.params_for(ps, FP64, kernel=WENDLAND_C4))
    x, v, m, u, h = _gpu.to_dev(ps, FP64)
    levels = torch.tensor(lev, dtype=torch.int32, device=x.device)
    out = ctx.forward(x, v, m, u, h)
    prev = oracle.forward(ps.x, ps.v, ps.m, ps.u, ps.h, p)
    out = ctx.hkdk_step(x, v, m, u, out, levels, dt, lam, stats=True)
    torch.cuda.synchronize()
    o = oracle.hkdk_step(ps.x, ps.v, ps.m, ps.u, ps.h, prev, lev, p, dt, lam,
                         trace=_Progress())
    st = _state_errors(x, v, u, out, o)
    g = {k: _np(t) for k, t in out.items() if isinstance(t, torch.Tensor)}
    e = _gpu.errors(g, o, o["h"])
    print({k: "%.2e" % val for k, val in st.items()},
          {k: "%.2e" % val for k, val in e.items()}, flush=True)
    for k, val in st.items():
        assert val <= STATE_BOUND[FP64], (k, val)
    for k, b in FP64_BOUNDS.items():
        assert e[k] <= b, (k, e[k], b)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_one_level_everywhere_is_repeated_single_level_steps(precision):
    ps = _start(2000, 313)
    print("case random2000 uniform levels precision=%d" % precision, flush=True)
    dt, lam = 4e-4, 0.5
    tol = 1e-11 if precision == FP64 else 1e-6
    for L in (0, 2):
        runs = []
        for hier in (True, False):
            ctx = Context(_gpu.params_for(ps, precision))
            x, v, m, u, h = _gpu.to_dev(ps, precision)
            out = ctx.forward(x, v, m, u, h)
            if hier:
                levels = torch.full((ps.n,), L, dtype=torch.int32, device=x.device)
                out = ctx.hkdk_step(x, v, m, u, out, levels, dt, lam)
            else:
                for _ in range(1 << L):
                    out = ctx.kdk_step(x, v, m, u, out, dt / (1 << L), lam)
            torch.cuda.synchronize()
            runs.append({"x": _np(x), "v": _np(v), "u": _np(u), "h": _np(out["h"]),
                         "accel": _np(out["accel"]), "rho": _np(out["rho"])})
        a, b = runs
        dx = np.abs(a["x"] - b["x"])
        assert np.minimum(dx, 1 - dx).max() < tol * 1e-2, L
        for k in ("v", "u", "h", "accel", "rho"):
            err = np.abs(a[k] - b[k]).max() / np.abs(b[k]).max()
            print("  L=%d %s %.2e" % (L, k, err), flush=True)
            assert err < tol, (L, k, err)


def test_hierarchy_errors():
    ps = _start(500, 314)
    ctx = Context(_gpu.params_for(ps, FP64))
    x, v, m, u, h = _gpu.to_dev(ps, FP64)
    out = ctx.forward(x, v, m, u, h)
    bad = torch.full((ps.n,), 31, dtype=torch.int32, device=x.device)
    with pytest.raises(CrkError):
        ctx.hkdk_step(x, v, m, u, out, bad, 1e-4)
    bad[:] = 0
    bad[7] = -1
    with pytest.raises(CrkError):
        ctx.hkdk_step(x, v, m, u, out, bad, 1e-4)
    lev = torch.zeros(ps.n, dtype=torch.int32, device=x.device)
    with pytest.raises(CrkError):
        ctx.hkdk_step(x, v, m, u, out, lev, -1.0)
    lev[3] = 1
    ctx.hkdk_step(x, v, m, u, out, lev, 1e-4)
    torch.cuda.synchronize()
    # the last evaluation had passive particles: no adjoint of it
    with pytest.raises(CrkError):
        ctx.backward(torch.zeros(3, ps.n, dtype=torch.float64, device=x.device),
                     torch.zeros(ps.n, dtype=torch.float64, device=x.device))


def test_sedov64_v_big_step_at_full_size():
    # the bench's configuration: 262,144 particles on levels from the signal
    # speed c + |v| (half on level 1, the hot core on level 3: eight
    # substeps), FP32 on the GPU against the FP64 oracle
    ps = synth.sedov64_v()
    print("case sedov64_v levels from c + |v|, one big step FP32", flush=True)
    p1 = oracle.params_for(ps)
    # the oracle's grid neighbour search (its brute force is quadratic in n)
    h = oracle.forward(ps.x, ps.v, ps.m, ps.u, ps.h, p1, nbr_mode=1)["h"]
    print("  oracle h solved", flush=True)
    ps.h, ps.h_mode = h, 0
    p = oracle.params_for(ps)
    sig = np.sqrt(p.gamma * (p.gamma - 1.0) * ps.u) + np.sqrt((ps.v ** 2).sum(0))
    lev = np.clip(np.ceil(np.log2(sig / np.median(sig))), 0, 3).astype(np.int64)
    assert lev.max() == 3 and (lev == 3).sum() == 27 and (lev == 1).sum() > 100000
    dt, lam = 8e-9, 0.5
    ctx = Context(_gpu.params_for(ps, FP32))
    x, v, m, u, hh = _gpu.to_dev(ps, FP32)
    out = ctx.forward(x, v, m, u, hh)
    levels = torch.tensor(lev, dtype=torch.int32, device=x.device)
    out = ctx.hkdk_step(x, v, m, u, out, levels, dt, lam)
    torch.cuda.synchronize()
    print("  GPU step done", flush=True)
    prev = oracle.forward(ps.x, ps.v, ps.m, ps.u, h, p, nbr_mode=1)
    trace = _Progress()
    o = oracle.hkdk_step(ps.x, ps.v, ps.m, ps.u, h, prev, lev, p, dt, lam, nbr_mode=1,
                         trace=trace)
    st = _state_errors(x, v, u, out, o)
    g = {k: _np(t) for k, t in out.items() if isinstance(t, torch.Tensor)}
    e = _gpu.errors(g, o, o["h"])
    print({k: "%.2e" % val for k, val in st.items()}, {k: "%.2e" % val for k, val in e.items()},
          flush=True)
    for k, val in st.items():
        assert val <= STATE_BOUND[FP32], (k, val)
    for k, b in FP32_BOUNDS.items():
        assert e[k] <= b, (k, e[k], b)


def test_big_step_on_the_tree_search_path():
    # the tree (the search for strongly clustered sets) with passive particles
    ps = _start(3000, 301)
    print("case random3000 levels 0-2 tree search FP64", flush=True)
    dt, lam = 2e-4, 0.5
    lev = np.random.default_rng(315).integers(0, 3, ps.n)
    lev[0] = 2
    p = oracle.params_for(ps)
    ctx = Context(_gpu.params_for(ps, FP64, search=2))
    x, v, m, u, h = _gpu.to_dev(ps, FP64)
    levels = torch.tensor(lev, dtype=torch.int32, device=x.device)
    out = ctx.forward(x, v, m, u, h)
    out = ctx.hkdk_step(x, v, m, u, out, levels, dt, lam)
    torch.cuda.synchronize()
    prev = oracle.forward(ps.x, ps.v, ps.m, ps.u, ps.h, p)
    o = oracle.hkdk_step(ps.x, ps.v, ps.m, ps.u, ps.h, prev, lev, p, dt, lam)
    st = _state_errors(x, v, u, out, o)
    g = {k: _np(t) for k, t in out.items() if isinstance(t, torch.Tensor)}
    e = _gpu.errors(g, o, o["h"])
    print({k: "%.2e" % val for k, val in st.items()}, {k: "%.2e" % val for k, val in e.items()},
          flush=True)
    for k, val in st.items():
        assert val <= STATE_BOUND[FP64], (k, val)
    for k, b in FP64_BOUNDS.items():
        assert e[k] <= b, (k, e[k], b)


def test_deep_hierarchy_sixteen_substeps():
    ps = _start(1000, 316)
    print("case random1000 levels 0-4 FP64", flush=True)
    dt, lam = 4e-4, 0.5
    lev = np.random.default_rng(317).integers(0, 5, ps.n)
    lev[0] = 4
    p = oracle.params_for(ps)
    ctx = Context(_gpu.params_for(ps, FP64))
    x, v, m, u, h = _gpu.to_dev(ps, FP64)
    levels = torch.tensor(lev, dtype=torch.int32, device=x.device)
    out = ctx.forward(x, v, m, u, h)
    out = ctx.hkdk_step(x, v, m, u, out, levels, dt, lam)
    torch.cuda.synchronize()
    prev = oracle.forward(ps.x, ps.v, ps.m, ps.u, ps.h, p)
    o = oracle.hkdk_step(ps.x, ps.v, ps.m, ps.u, ps.h, prev, lev, p, dt, lam)
    st = _state_errors(x, v, u, out, o)
    g = {k: _np(t) for k, t in out.items() if isinstance(t, torch.Tensor)}
    e = _gpu.errors(g, o, o["h"])
    print({k: "%.2e" % val for k, val in st.items()}, flush=True)
    for k, val in st.items():
        assert val <= STATE_BOUND[FP64], (k, val)
    for k, b in FP64_BOUNDS.items():
        assert e[k] <= b, (k, e[k], b)


def test_big_step_with_relaxation():
    # relaxation on (exp(|div v| dt_relax) > 8): passive particles take their
    # flag from the stored grad v, active ones from the new evaluation
    ps = _start(1500, 318)
    print("case random1500 levels 0-2 relaxation FP64", flush=True)
    dt, lam = 2e-4, 0.5
    lev = np.random.default_rng(319).integers(0, 3, ps.n)
    lev[0] = 2
    p = oracle.params_for(ps, dt_relax=3.0)
    ctx = Context(_gpu.params_for(ps, FP64, dt_relax=3.0))
    x, v, m, u, h = _gpu.to_dev(ps, FP64)
    levels = torch.tensor(lev, dtype=torch.int32, device=x.device)
    out = ctx.forward(x, v, m, u, h)
    out = ctx.hkdk_step(x, v, m, u, out, levels, dt, lam, stats=True)
    torch.cuda.synchronize()
    prev = oracle.forward(ps.x, ps.v, ps.m, ps.u, ps.h, p)
    assert 0 < prev["relaxed"] < ps.n
    o = oracle.hkdk_step(ps.x, ps.v, ps.m, ps.u, ps.h, prev, lev, p, dt, lam)
    st = _state_errors(x, v, u, out, o)
    g = {k: _np(t) for k, t in out.items() if isinstance(t, torch.Tensor)}
    e = _gpu.errors(g, o, o["h"])
    print({k: "%.2e" % val for k, val in st.items()}, out["stats"]["relaxed"], flush=True)
    for k, val in st.items():
        assert val <= STATE_BOUND[FP64], (k, val)
    for k, b in FP64_BOUNDS.items():
        assert e[k] <= b, (k, e[k], b)


def _refine(n, rng, lev, lmax):
    at = np.full(n, -1, dtype=np.int64)
    to = lev.copy()
    for i in np.nonzero(rng.uniform(size=n) < 0.3)[0]:
        if lev[i] >= lmax:
            continue
        L = int(rng.integers(lev[i] + 1, lmax + 1))
        at[i] = int(rng.integers(0, 1 << L)) << (lmax - L)
        to[i] = L
    return at, to


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_refined_big_steps_match_the_oracle(precision):
    ps = _start(3000, 331)
    print("case random3000 levels 0-2 refined to 3, precision=%d" % precision, flush=True)
    dt, lam = 2e-4, 0.5
    rng = np.random.default_rng(332)
    lev = rng.integers(0, 3, ps.n)
    lev[0] = 2
    p = oracle.params_for(ps)
    ctx = Context(_gpu.params_for(ps, precision))
    x, v, m, u, h = _gpu.to_dev(ps, precision)
    levels = torch.tensor(lev, dtype=torch.int32, device=x.device)
    out = ctx.forward(x, v, m, u, h)
    ox, ov, ou, oh = ps.x.copy(), ps.v.copy(), ps.u.copy(), ps.h.copy()
    prev = oracle.forward(ox, ov, ps.m, ou, oh, p)
    bounds = FP64_BOUNDS if precision == FP64 else FP32_BOUNDS
    for it in range(2):
        at, to = _refine(ps.n, rng, lev, 3)
        print("big step", it, "refinements", int((at >= 0).sum()), "midway",
              int(((at >= 0) & (at % (1 << (3 - lev)) != 0)).sum()), flush=True)
        ref = (torch.tensor(at, dtype=torch.int32, device=x.device),
               torch.tensor(to, dtype=torch.int32, device=x.device))
        out = ctx.hkdk_step(x, v, m, u, out, levels, dt, lam, stats=True, refine=ref)
        torch.cuda.synchronize()
        o = oracle.hkdk_step(ox, ov, ps.m, ou, oh, prev, lev, p, dt, lam, refine=(at, to))
        ox, ov, ou, oh, prev = o["x"], o["v"], o["u"], o["h"], o
        st = _state_errors(x, v, u, out, o)
        g = {k: _np(t) for k, t in out.items() if isinstance(t, torch.Tensor)}
        e = _gpu.errors(g, o, o["h"])
        print("big step", it, {k: "%.2e" % val for k, val in st.items()},
              {k: "%.2e" % val for k, val in e.items()}, flush=True)
        for k, val in st.items():
            assert val <= STATE_BOUND[precision], (it, k, val)
        for k, b in bounds.items():
            assert e[k] <= b, (it, k, e[k], b)


def test_empty_refinement_is_the_plain_step():
    ps = _start(1500, 341)
    print("case random1500 refine_at all -1", flush=True)
    lev = np.random.default_rng(342).integers(0, 3, ps.n)
    runs = []
    for refine in (False, True):
        ctx = Context(_gpu.params_for(ps, FP32))
        x, v, m, u, h = _gpu.to_dev(ps, FP32)
        levels = torch.tensor(lev, dtype=torch.int32, device=x.device)
        out = ctx.forward(x, v, m, u, h)
        ref = None
        if refine:
            ref = (torch.full((ps.n,), -1, dtype=torch.int32, device=x.device), levels.clone())
        out = ctx.hkdk_step(x, v, m, u, out, levels, 2e-4, 0.5, refine=ref)
        torch.cuda.synchronize()
        runs.append({"x": _np(x), "v": _np(v), "u": _np(u),
                     **{k: _np(t) for k, t in out.items() if isinstance(t, torch.Tensor)}})
    for k in runs[0]:
        assert np.array_equal(runs[0][k], runs[1][k]), k


def test_refinement_errors():
    ps = _start(300, 351)
    print("case random300 bad refinements", flush=True)
    ctx = Context(_gpu.params_for(ps, FP32))
    x, v, m, u, h = _gpu.to_dev(ps, FP32)
    out = ctx.forward(x, v, m, u, h)
    lev = torch.ones(ps.n, dtype=torch.int32, device=x.device)
    at = torch.full((ps.n,), -1, dtype=torch.int32, device=x.device)
    at[5] = 0
    with pytest.raises(CrkError):  # not a finer level
        ctx.hkdk_step(x, v, m, u, out, lev, 1e-4, refine=(at, lev.clone()))
    to = lev.clone()
    to[5] = 2
    to[6] = 3
    at[6] = 0
    at[5] = 1  # level 2 of lmax 3 starts on even substeps only
    with pytest.raises(CrkError):
        ctx.hkdk_step(x, v, m, u, out, lev, 1e-4, refine=(at, to))
    at[5] = 2
    ctx.hkdk_step(x, v, m, u, out, lev, 1e-4, refine=(at, to))
