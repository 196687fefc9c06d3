"""Pins of the oracle's exact-integration cooling (Sec. 2.2, exact integration).

The oracle walks I(u) bin by bin from the anchor u_a = u^0 and inverts the
final bin, eq. (Iu) and (Iinv). What fixes it independently:
* a table sampling a pure power law lam = A u^beta is interpolated exactly, so
  u^1 must equal the closed-form solution of du/dt = -rho A u^beta: beta = 1.5
  (the self-similar cooling slope of App. B) cooling and heating, and beta = 1
  (the alpha_k = 1 branch: exponential decay);
* a general piecewise power law: u^1 equals a high-order ODE integration of
  du/dt = -rho lam(u) with the same interpolant;
* the table ends clamp u; a stable zero of lam is approached from both sides,
  never crossed, and reached by every particle after a long step; an unstable
  zero is left.
"""
import numpy as np
import pytest

import oracle

DEX, LU0 = 0.004, -2.0
K = int(round(6 / DEX)) + 1
UK = 10 ** (LU0 + DEX * np.arange(K))
A = 0.7


def _particles(n=300, seed=1):
    rng = np.random.default_rng(seed)
    return 10 ** rng.uniform(-1, 3, n), 10 ** rng.uniform(-1, 1, n)


@pytest.mark.parametrize("beta", [1.5, 1.0])
def test_power_law_cooling_closed_form(beta):
    u0, rho = _particles()
    tab = oracle.CoolingTable(LU0, DEX, A * UK ** beta)
    dt = 0.3
    got = oracle.cool(tab, u0, rho, dt)
    if beta == 1.0:
        want = u0 * np.exp(-rho * A * dt)
    else:
        want = (u0 ** (1 - beta) + (beta - 1) * rho * A * dt) ** (1 / (1 - beta))
    want = np.maximum(want, UK[0])  # the table floor
    assert np.max(np.abs(got / want - 1)) < 1e-13


def test_power_law_heating_closed_form():
    u0, rho = _particles()
    tab = oracle.CoolingTable(LU0, DEX, -A * UK ** 1.5)
    dt = 0.01
    got = oracle.cool(tab, u0, rho, dt)
    want = np.minimum((u0 ** -0.5 - 0.5 * rho * A * dt) ** -2, UK[-1])
    assert np.all(got >= u0)
    assert np.max(np.abs(got / want - 1)) < 1e-13


def test_general_table_matches_ode_integration():
    from scipy.integrate import solve_ivp
    rng = np.random.default_rng(2)
    lam = np.exp(np.cumsum(rng.normal(0, 0.02, K))) * UK ** 1.2
    tab = oracle.CoolingTable(LU0, DEX, lam)
    u0, rho = _particles(12, 3)
    dt = 0.05
    got = oracle.cool(tab, u0, rho, dt)
    for i in range(u0.size):
        sol = solve_ivp(lambda t, y: [-rho[i] * tab.lam_at(y[0])], (0, dt), [u0[i]],
                        method="DOP853", rtol=1e-12, atol=1e-14)
        assert abs(sol.y[0, -1] / got[i] - 1) < 1e-6


def test_table_ends_clamp():
    tab = oracle.CoolingTable(LU0, DEX, A * UK ** 1.5)
    got = oracle.cool(tab, np.array([5.0, 1e-5, 1e9]), np.ones(3), 1e6)
    assert np.all(got == UK[0])
    tab = oracle.CoolingTable(LU0, DEX, -A * UK ** 1.5)
    got = oracle.cool(tab, np.array([5.0, 1e9]), np.ones(2), 10.0)
    assert np.all(got == UK[-1])


def test_stable_equilibrium_is_approached_not_crossed():
    ueq = 3.0
    tab = oracle.CoolingTable(LU0, DEX, A * (UK ** 1.5 - ueq ** 1.5))
    u0, rho = _particles()
    short = oracle.cool(tab, u0, rho, 0.05)
    k = np.searchsorted(UK, ueq) - 1
    lk, lk1 = tab.lam[k], tab.lam[k + 1]
    zero = UK[k] - lk * (UK[k + 1] - UK[k]) / (lk1 - lk)
    assert np.all((short - zero) * (u0 - zero) >= 0)        # never crossed
    assert np.all(np.abs(short - zero) <= np.abs(u0 - zero))  # approached
    long = oracle.cool(tab, u0, rho, 1e6)
    assert np.all(long == long[0]) and abs(long[0] - zero) < 1e-12 * zero


def test_unstable_equilibrium_is_left():
    ueq = 3.0
    tab = oracle.CoolingTable(LU0, DEX, -A * (UK ** 1.5 - ueq ** 1.5))
    k = np.searchsorted(UK, ueq) - 1
    u0 = np.array([UK[k] * 1.0001, UK[k + 1] * 0.9999, 1.0, 10.0])
    got = oracle.cool(tab, u0, np.ones(4), 1e-3)
    lk, lk1 = tab.lam[k], tab.lam[k + 1]
    zero = UK[k] - lk * (UK[k + 1] - UK[k]) / (lk1 - lk)
    assert np.all(np.sign(got - u0) == np.sign(u0 - zero))
