"""Pins of the oracle's KDK step (App. A.4) with the smoothing-length update of App. A.3.

What fixes the step independently of its own formulas:
* a perfect lattice at rest, with h at the exact Thacker root (the oracle's h
  solve), is an equilibrium: nothing moves and Delta_N = 1 keeps h;
* from a wrong h, repeated steps at rest drive h to that same root (the time-
  integrated Thacker estimate has the h solve's root as its fixed point);
* a lattice in uniform motion feels no force (Galilean invariance): positions
  advance by v dt exactly, velocities stay;
* with lambda = 0 the smoothing length follows the continuity equation: for a
  sinusoidal velocity field, log(h_new / h) = div(v) dt / 3 with the analytic
  divergence, to the accuracy of the corrected gradient at that resolution;
* momentum is conserved to rounding (antisymmetric pair forces), and the
  energy error of one step falls by ~8x when dt halves (a second-order
  integrator has a local error of order dt^3).
"""
import numpy as np
import pytest

import oracle
import synth


def _lattice(ns=12):
    g = (np.arange(ns) + 0.5) / ns
    x = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    n = x.shape[1]
    n_h = synth.n_h_for_neighbours(32)
    m = np.full(n, 1.0 / n)
    u = np.ones(n)
    root = oracle.forward(x, np.zeros((3, n)), m, u, np.full(n, n_h / ns),
                          oracle.Params(n_h=n_h, h_mode=1))["h"]
    return x, m, u, root, oracle.Params(n_h=n_h, h_mode=0)


def test_lattice_at_rest_is_an_equilibrium():
    x, m, u, h, p = _lattice()
    v = np.zeros_like(x)
    prev = oracle.forward(x, v, m, u, h, p)
    s = oracle.kdk_step(x, v, m, u, h, prev, p, 1e-3, 0.5)
    assert np.array_equal(s["x"], x)
    assert np.abs(s["v"]).max() < 1e-15
    assert np.abs(s["u"] - u).max() < 1e-15
    assert np.abs(s["h"] / h - 1).max() < 1e-14


def test_thacker_steps_relax_h_to_the_exact_root():
    x, m, u, root, p = _lattice()
    h = 1.15 * root
    v = np.zeros_like(x)
    prev = oracle.forward(x, v, m, u, h, p)
    err = []
    for it in range(40):
        s = oracle.kdk_step(x, v, m, u, h, prev, p, 1e-3, 0.5)
        x, v, u, h, prev = s["x"], s["v"], s["u"], s["h"], s
        err.append(np.abs(h / root - 1).max())
    assert err[9] < 1e-3 and err[19] < 1e-6 and err[39] < 1e-12
    assert all(b <= a * 1.01 for a, b in zip(err, err[1:]))  # monotone approach


def test_uniform_translation_is_force_free():
    x, m, u, h, p = _lattice()
    v0 = np.array([0.3, -0.2, 0.1])[:, None] * np.ones_like(x)
    prev = oracle.forward(x, v0, m, u, h, p)
    dt = 1e-2
    s = oracle.kdk_step(x, v0, m, u, h, prev, p, dt, 0.5)
    assert np.abs(s["x"] - np.mod(x + dt * v0, 1.0)).max() < 1e-15
    assert np.abs(s["v"] - v0).max() < 1e-14
    assert np.abs(s["h"] / h - 1).max() < 1e-14


def test_continuity_part_follows_the_analytic_divergence():
    ns = 16
    x, m, u, h, p = _lattice(ns)
    amp, dt = 0.05, 1e-2
    v = np.zeros_like(x)
    v[0] = amp * np.sin(2 * np.pi * x[0])
    prev = oracle.forward(x, v, m, u, h, p)
    s = oracle.kdk_step(x, v, m, u, h, prev, p, dt, 0.0)
    want = 2 * np.pi * amp * np.cos(2 * np.pi * x[0]) * dt / 3
    got = np.log(s["h"] / h)
    slope = np.polyfit(want, got, 1)[0]
    assert 0.95 < slope < 1.02
    assert np.abs(got - want).max() < 0.05 * np.abs(want).max()


def test_momentum_exact_and_energy_error_third_order():
    ps = synth.random_small(1500, 7)
    h = oracle.forward(ps.x, ps.v, ps.m, ps.u, ps.h, oracle.params_for(ps))["h"]
    p = oracle.params_for(ps, h_mode=0)
    prev = oracle.forward(ps.x, ps.v, ps.m, ps.u, h, p)
    e0 = (ps.m * (0.5 * (ps.v ** 2).sum(0) + ps.u)).sum()
    p0 = (ps.m * ps.v).sum(1)
    scale = (ps.m * np.abs(ps.v)).sum()
    de = []
    for dt in (4e-3, 2e-3, 1e-3):
        s = oracle.kdk_step(ps.x, ps.v, ps.m, ps.u, h, prev, p, dt, 0.5)
        assert np.abs((ps.m * s["v"]).sum(1) - p0).max() < 1e-15 * scale * 1e3
        de.append(abs((ps.m * (0.5 * (s["v"] ** 2).sum(0) + s["u"])).sum() - e0) / e0)
    r1, r2 = de[0] / de[1], de[1] / de[2]
    print("energy errors", de, "ratios", r1, r2)
    assert 4.0 < r1 < 12.0 and 6.0 < r2 < 10.0


def test_step_needs_fixed_h_mode():
    x, m, u, h, p = _lattice(6)
    with pytest.raises(ValueError):
        oracle.kdk_step(x, np.zeros_like(x), m, u, h, {}, oracle.Params(h_mode=1), 1e-3, 0.5)
