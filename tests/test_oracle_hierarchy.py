"""Pins of the oracle's timestep hierarchy (App. A.4 hierarchical KDK, App. A.3
passive updates) and of its forward with passive particles.

What fixes them independently of their own formulas:
* substituting, for a passive subset, exactly the values a full forward
  computes for it leaves every output of the forward unchanged, and an empty
  passive set is the plain forward;
* a passive particle's stored state reaches only particles within the
  interaction range (two smoothing lengths);
* with one level L everywhere the hierarchy is 2^L single-level KDK steps of
  dt / 2^L (themselves pinned in tests/test_oracle_step.py), bit for bit;
* a lattice in uniform motion on mixed levels feels no force and advances by
  v dt exactly;
* a particle that stays passive through the substeps moves on the parabola
  of constant acceleration, x(t) = x^0 + v^0 t + a^0 t^2 / 2 at every
  substep, and its velocity obeys the KDK identity
  v^1 = v^0 + (a^0 + a^1) dt_a / 2;
* with lambda = 0, after a passive particle's first substep its carried
  density times its volume equals rho^0 (h^0 / n_h)^3: the continuity
  update of rho and the continuity part of h (cubed into V) cancel; over
  later substeps (hdot held while h changes) the product drifts only at
  second order in div(v) dt.

Timestep refinement (App. A.5), pinned by:
* an empty refinement is the plain big step, bit for bit;
* a refinement at the start of the big step is the big step with the finer
  level from the start, bit for bit;
* under accelerations that are constant in time the velocity, energy and
  position at the end are the closed forms v^0 + a dt, u^0 + b dt,
  x^0 + v^0 dt + a dt^2 / 2, whatever the levels and refinements;
* a particle refined midway through its interval ends its cycle with the
  piecewise-constant final kick v^1 = v^0 + a^0 (dt_b - dt_c)
  + (a^0 + a^1) dt_c / 2 and keeps the parabola of a^0 until then, with
  accelerations that change from one evaluation to the next.
"""
import numpy as np

import oracle
import synth


def _state(ns=12, seed=3, amp=0.05):
    rng = np.random.default_rng(seed)
    g = (np.arange(ns) + 0.5) / ns
    x = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    n = x.shape[1]
    x = np.mod(x + rng.uniform(-0.1, 0.1, x.shape) / ns, 1.0)
    n_h = synth.n_h_for_neighbours(32)
    m = np.full(n, 1.0 / n)
    u = 10 ** rng.normal(0, 0.3, n)
    v = amp * rng.normal(0, 1, (3, n))
    h = oracle.forward(x, v, m, u, np.full(n, n_h / ns), oracle.Params(n_h=n_h, h_mode=1))["h"]
    return x, v, m, u, h, oracle.Params(n_h=n_h, h_mode=0), rng


def _levels(n, rng, lmax=2):
    lev = rng.integers(0, lmax + 1, n)
    lev[0] = lmax
    return lev


def test_passive_substitution_of_the_computed_values_changes_nothing():
    x, v, m, u, h, p, rng = _state()
    full = oracle.forward(x, v, m, u, h, p)
    mask = rng.uniform(size=m.size) < 0.4
    pas = dict({k: full[k] for k in oracle.PASSIVE_KEYS}, mask=mask)
    sub = oracle.forward(x, v, m, u, h, p, passive=pas)
    for k in ("V", "rho", "A", "B", "gradA", "gradB", "gradv", "P", "c", "accel", "dudt"):
        assert np.array_equal(sub[k], full[k]), k
    none = oracle.forward(x, v, m, u, h, p, passive=dict(pas, mask=np.zeros(m.size, bool)))
    for k in ("accel", "dudt", "V", "rho"):
        assert np.array_equal(none[k], full[k]), k


def test_passive_state_reaches_only_the_interaction_range():
    x, v, m, u, h, p, rng = _state()
    full = oracle.forward(x, v, m, u, h, p)
    mask = np.zeros(m.size, bool)
    k0 = 100
    mask[k0] = True
    pas = {k: full[k].copy() for k in oracle.PASSIVE_KEYS}
    pas["V"][k0] *= 1.3
    pas["rho"][k0] *= 0.7
    pas["B"][:, k0] += 0.1 / h[k0]
    sub = oracle.forward(x, v, m, u, h, p, passive=dict(pas, mask=mask))
    d = x - x[:, k0:k0 + 1]
    d -= np.round(d)
    r = np.sqrt((d * d).sum(0))
    changed = np.abs(sub["accel"] - full["accel"]).max(0) > 0
    changed[k0] = False
    assert changed.sum() > 10
    assert r[changed].max() < 2 * h.max()


def test_one_level_everywhere_is_repeated_single_level_steps():
    x, v, m, u, h, p, _ = _state(10)
    prev = oracle.forward(x, v, m, u, h, p)
    dt, lam = 4e-3, 0.5
    for L in (0, 2):
        hs = oracle.hkdk_step(x, v, m, u, h, prev, np.full(m.size, L), p, dt, lam)
        s = dict(prev, x=x, v=v, u=u, h=h)
        for _ in range(1 << L):
            s = oracle.kdk_step(s["x"], s["v"], m, s["u"], s["h"], s, p, dt / (1 << L), lam)
        for k in ("x", "v", "u", "h", "accel", "dudt", "V", "rho", "A", "B", "gradv"):
            assert np.array_equal(hs[k], s[k]), (L, k)


def test_mixed_levels_uniform_motion_is_force_free():
    ns = 10
    g = (np.arange(ns) + 0.5) / ns
    x = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    n = x.shape[1]
    n_h = synth.n_h_for_neighbours(32)
    m = np.full(n, 1.0 / n)
    u = np.ones(n)
    h = oracle.forward(x, np.zeros((3, n)), m, u, np.full(n, n_h / ns),
                       oracle.Params(n_h=n_h, h_mode=1))["h"]
    p = oracle.Params(n_h=n_h, h_mode=0)
    v0 = np.array([0.3, -0.2, 0.1])[:, None] * np.ones_like(x)
    prev = oracle.forward(x, v0, m, u, h, p)
    lev = _levels(n, np.random.default_rng(5), 3)
    dt = 1e-2
    s = oracle.hkdk_step(x, v0, m, u, h, prev, lev, p, dt, 0.5)
    assert np.abs(s["x"] - np.mod(x + dt * v0, 1.0)).max() < 1e-15
    assert np.abs(s["v"] - v0).max() < 1e-13
    assert np.abs(s["h"] / h - 1).max() < 1e-13


def test_passive_particles_follow_the_parabola_and_the_kdk_identity():
    x, v, m, u, h, p, rng = _state(10, seed=4, amp=0.3)
    prev = oracle.forward(x, v, m, u, h, p)
    lev = _levels(m.size, rng, 2)
    dt = 2e-3
    trace = []
    s = oracle.hkdk_step(x, v, m, u, h, prev, lev, p, dt, 0.5, trace=trace)
    top = lev == 0  # one interval over the whole big step, passive in between
    a0 = prev["accel"][:, top]
    for j, t in enumerate(trace):
        tt = (j + 1) * dt / 4
        d = t["x"][:, top] - (x[:, top] + v[:, top] * tt + 0.5 * a0 * tt * tt)
        d -= np.round(d)
        assert np.abs(d).max() < 1e-15, j
    d = s["x"][:, top] - (x[:, top] + v[:, top] * dt + 0.5 * a0 * dt * dt)
    d -= np.round(d)
    assert np.abs(d).max() < 1e-15
    assert np.abs(s["v"][:, top] - (v[:, top] + 0.5 * (a0 + s["accel"][:, top]) * dt)).max() \
        < 1e-12 * np.abs(v).max()
    # the others moved differently from a single constant-acceleration arc
    fine = lev == 2
    arc = x[:, fine] + v[:, fine] * dt + 0.5 * prev["accel"][:, fine] * dt * dt
    d = s["x"][:, fine] - arc
    d -= np.round(d)
    assert np.abs(d).max() > 1e-12


def test_carried_density_times_volume_while_passive():
    x, v, m, u, h, p, rng = _state(10, seed=6, amp=0.3)
    prev = oracle.forward(x, v, m, u, h, p)
    lev = _levels(m.size, rng, 2)
    dt = 4e-3
    trace = []
    oracle.hkdk_step(x, v, m, u, h, prev, lev, p, dt, 0.0, trace=trace)
    top = lev == 0
    assert all(t["passive"][top].all() for t in trace[:-1]) and not trace[-1]["passive"].any()
    start = prev["rho"][top] * (h[top] / p.n_h) ** 3
    first = trace[0]["rho"][top] * trace[0]["V"][top]
    assert np.abs(first / start - 1).max() < 1e-13
    g = prev["gradv"]
    divdt = np.abs(g[0] + g[4] + g[8])[top] * dt
    for t in trace[1:-1]:
        dev = np.abs(t["rho"][top] * t["V"][top] / start - 1)
        assert np.all(dev <= divdt ** 2 + 1e-13)
    # with lambda > 0 the Thacker term moves h alone, and the product moves
    trace = []
    oracle.hkdk_step(x, v, m, u, h * 1.05, prev, lev, p, dt, 0.5, trace=trace)
    start = prev["rho"][top] * (1.05 * h[top] / p.n_h) ** 3
    moved = trace[0]["rho"][top] * trace[0]["V"][top] / start
    assert np.abs(moved - 1).max() > 1e-6


# ------------------------------------------------ refinement (App. A.5) --

def _refinement(n, rng, lev, lmax):
    """Random refinements: about a third of the particles move, at a random
    substep on the grid of their new level, to a finer level up to lmax."""
    at = np.full(n, -1)
    to = lev.copy()
    for i in np.nonzero(rng.uniform(size=n) < 0.35)[0]:
        if lev[i] >= lmax:
            continue
        L = int(rng.integers(lev[i] + 1, lmax + 1))
        at[i] = int(rng.integers(0, 1 << L)) << (lmax - L)
        to[i] = L
    return at, to


def test_empty_refinement_is_the_plain_big_step():
    x, v, m, u, h, p, rng = _state(ns=8, seed=21)
    prev = oracle.forward(x, v, m, u, h, p)
    lev = _levels(m.size, rng)
    a = oracle.hkdk_step(x, v, m, u, h, prev, lev, p, 1e-3, 0.5)
    b = oracle.hkdk_step(x, v, m, u, h, prev, lev, p, 1e-3, 0.5,
                         refine=(np.full(m.size, -1), lev))
    for k in ("x", "v", "u", "h", "accel", "dudt", "V", "rho"):
        assert np.array_equal(a[k], b[k]), k


def test_refinement_at_the_start_is_the_finer_level():
    x, v, m, u, h, p, rng = _state(ns=8, seed=22)
    prev = oracle.forward(x, v, m, u, h, p)
    lev = np.zeros(m.size, dtype=np.int64)
    lev[0] = 2
    at = np.full(m.size, -1)
    to = lev.copy()
    moved = np.nonzero(rng.uniform(size=m.size) < 0.3)[0]
    moved = moved[moved != 0]
    at[moved] = 0
    to[moved] = rng.integers(1, 3, moved.size)
    a = oracle.hkdk_step(x, v, m, u, h, prev, lev, p, 1e-3, 0.5, refine=(at, to))
    b = oracle.hkdk_step(x, v, m, u, h, prev, np.where(at >= 0, to, lev), p, 1e-3, 0.5)
    for k in ("x", "v", "u", "h", "accel", "dudt", "V", "rho"):
        assert np.array_equal(a[k], b[k]), k


def test_constant_acceleration_gives_the_closed_form():
    rng = np.random.default_rng(23)
    n, lmax, dt, box = 200, 3, 0.5, 1.0
    x0 = rng.uniform(0, box, (3, n))
    v0 = rng.normal(0, 0.3, (3, n))
    u0 = rng.uniform(1, 2, n)
    acc = rng.normal(0, 2.0, (3, n))
    du = rng.normal(0, 1.0, n)
    lev = rng.integers(0, lmax + 1, n)
    lev[0] = lmax
    refine = _refinement(n, rng, lev, lmax)
    assert (refine[0] >= 0).sum() > 20

    def evaluate(x_, v_, u_, h_, passive):
        return {"accel": acc.copy(), "dudt": du.copy()}
    p = oracle.Params(box=box, h_mode=0)
    o = oracle.hkdk_step(x0, v0, np.ones(n), u0, np.full(n, 0.1), {"accel": acc, "dudt": du},
                         lev, p, dt, 0.5, refine=refine, evaluate=evaluate)
    np.testing.assert_allclose(o["v"], v0 + acc * dt, rtol=0, atol=1e-13)
    np.testing.assert_allclose(o["u"], u0 + du * dt, rtol=0, atol=1e-13)
    d = o["x"] - (x0 + v0 * dt + 0.5 * acc * dt * dt)
    d -= box * np.round(d / box)
    assert np.abs(d).max() < 1e-13


def test_midway_refinement_takes_the_piecewise_constant_final_kick():
    # level 1 (two intervals of dt / 2); in the second one, a quarter step in
    # (e = dt / 4), the particle moves to level 2 (dt_c = dt / 4): its cycle
    # is dt_b = e + dt_c = dt / 2 long and closes at dt
    rng = np.random.default_rng(24)
    n, dt = 3, 0.8
    x0 = rng.uniform(0, 1, (3, n))
    v0 = rng.normal(0, 0.3, (3, n))
    u0 = np.array([1.0, 2.0, 3.0])
    A = [rng.normal(0, 1, (3, n)) for _ in range(5)]   # a at t = k dt / 4
    B = [rng.normal(0, 1, n) for _ in range(5)]
    calls = []

    def evaluate(x_, v_, u_, h_, passive):
        calls.append(1)
        k = len(calls)
        return {"accel": A[k].copy(), "dudt": B[k].copy()}
    lev = np.array([1, 1, 2])
    at = np.array([3, -1, -1])
    to = np.array([2, 1, 2])
    p = oracle.Params(h_mode=0)
    o = oracle.hkdk_step(x0, v0, np.ones(n), u0, np.full(n, 0.1), {"accel": A[0], "dudt": B[0]},
                         lev, p, dt, 0.0, refine=(at, to), evaluate=evaluate)
    half = dt / 2
    v_half = v0 + 0.5 * (A[0] + A[2]) * half           # first interval, t = dt / 2
    u_half = u0 + 0.5 * (B[0] + B[2]) * half
    x_half = x0 + v0 * half + 0.5 * A[0] * half ** 2
    dt_b, dt_c = half, dt / 4
    v1 = v_half + A[2] * (dt_b - dt_c) + 0.5 * (A[2] + A[4]) * dt_c
    u1 = u_half + B[2] * (dt_b - dt_c) + 0.5 * (B[2] + B[4]) * dt_c
    x1 = x_half + v_half * half + 0.5 * A[2] * half ** 2
    np.testing.assert_allclose(o["v"][:, 0], v1[:, 0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(o["u"][0], u1[0], rtol=0, atol=1e-14)
    d = o["x"][:, 0] - x1[:, 0]
    assert np.abs(d - np.round(d)).max() < 1e-14
    # the unrefined level-1 particle takes the plain KDK of its second interval
    v1b = v_half + 0.5 * (A[2] + A[4]) * half
    np.testing.assert_allclose(o["v"][:, 1], v1b[:, 1], rtol=0, atol=1e-14)


def test_refinement_errors():
    x, v, m, u, h, p, rng = _state(ns=6, seed=25)
    prev = oracle.forward(x, v, m, u, h, p)
    lev = np.ones(m.size, dtype=np.int64)
    at = np.full(m.size, -1)
    at[3] = 0
    import pytest
    with pytest.raises(ValueError):  # not finer
        oracle.hkdk_step(x, v, m, u, h, prev, lev, p, 1e-3, 0.5, refine=(at, lev))
    to = lev.copy()
    to[3] = 3
    at[3] = 1  # level 3 with lmax 3: any substep; level 2 needs even substeps
    oracle.hkdk_step(x, v, m, u, h, prev, lev, p, 1e-3, 0.5, refine=(at, to))
    to[3] = 2
    to[4] = 3
    at[4] = 0
    with pytest.raises(ValueError):  # off the grid of level 2 (lmax 3)
        oracle.hkdk_step(x, v, m, u, h, prev, lev, p, 1e-3, 0.5, refine=(at, to))
