"""Pins of the oracle's subgrid deposition (App. A.2 eq. (Vsg); eqs. (windmetal),
(Anorm), (starmetal), (stellarmom), (AGNE)).

* The normalised weights of a source sum to one over its eligible gas, so the
  deposited mass, metal mass and energy and the carried momentum appear in
  the gas exactly (conservation to rounding), whatever the configuration.
* A source that coincides with a gas particle of a uniform lattice (equal h,
  equal masses) sees the gas particle's own SPH sum, so V_s = (1 - C w(0) /
  n_h,s^3) V_gas with V_gas from the oracle's forward (the C++ gas volume).
* Equidistant eligible gas of equal volume receives equal shares; a single
  eligible neighbour receives everything; ineligible gas (metallicity above
  z_max, mass above m_max) is untouched.
"""
import numpy as np

import oracle
import synth


def _lattice(ns=10):
    g = (np.arange(ns) + 0.5) / ns
    return np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)


def _gas(x, h, rng, zfrac=0.01):
    n = x.shape[1]
    m = np.full(n, 1.0 / n) * (1 + 0.1 * rng.uniform(-1, 1, n))
    return {"x": x, "h": np.full(n, h) if np.isscalar(h) else h, "V": m.copy() * 1.0,
            "m": m, "v": rng.normal(0, 0.1, (3, n)), "mZ": zfrac * m,
            "u": 10 ** rng.normal(0, 0.3, n)}


def _src(xs, rng):
    ns = xs.shape[1]
    return {"x": xs, "dM": rng.uniform(0.1, 1.0, ns) * 1e-4,
            "dMZ": rng.uniform(0.0, 0.1, ns) * 1e-4, "dE": rng.uniform(0.0, 1.0, ns) * 1e-3,
            "v": rng.normal(0, 0.2, (3, ns))}


def test_conservation_of_mass_metals_energy_momentum():
    rng = np.random.default_rng(1)
    xg = rng.uniform(0, 1, (3, 3000))
    gas = _gas(xg, 0.12 * (1 + 0.3 * rng.uniform(-1, 1, 3000)), rng)
    src = _src(rng.uniform(0, 1, (3, 60)), rng)
    out = oracle.deposit(gas, src, 2.25, kernel=1)
    assert np.all(out["A_s"] > 0)
    m0, m1 = gas["m"].sum(), out["m"].sum()
    assert abs(m1 - m0 - src["dM"].sum()) < 1e-15 * m0
    assert abs(out["mZ"].sum() - gas["mZ"].sum() - src["dMZ"].sum()) < 1e-15 * m0
    e0 = (gas["m"] * gas["u"]).sum()
    assert abs((out["m"] * out["u"]).sum() - e0 - src["dE"].sum()) < 1e-14 * e0
    p0 = (gas["m"] * gas["v"]).sum(1)
    p1 = (out["m"] * out["v"]).sum(1)
    assert np.abs(p1 - p0 - (src["dM"] * src["v"]).sum(1)).max() < 1e-15


def test_source_on_a_lattice_site_sees_the_gas_volume():
    ns = 12
    x = _lattice(ns)
    n = x.shape[1]
    n_h = synth.n_h_for_neighbours(48)
    h = n_h / ns
    m = np.full(n, 1.0 / n)
    o = oracle.forward(x, np.zeros((3, n)), m, np.ones(n), np.full(n, h),
                       oracle.Params(n_h=n_h, h_mode=0, kernel=1))
    rng = np.random.default_rng(2)
    gas = {"x": x, "h": np.full(n, h), "V": o["V"], "m": m, "v": np.zeros((3, n)),
           "mZ": 0.01 * m, "u": np.ones(n)}
    k = [5, 77, 1000]
    src = _src(x[:, k], rng)
    n_hs = 2.25
    out = oracle.deposit(gas, src, n_hs, kernel=1)
    _, _, norm = oracle.kernel_eval(1, np.zeros(1))
    w0 = oracle.kernel_eval(1, np.zeros(1))[0][0]
    want = (1 - norm * w0 / n_hs ** 3) * o["V"][k]
    assert np.max(np.abs(out["V_s"] / want - 1)) < 1e-13


def test_equal_shares_single_neighbour_and_exclusion():
    ns = 8
    x = _lattice(ns)
    rng = np.random.default_rng(3)
    gas = _gas(x, 1.6 / ns, rng)
    gas["V"] = np.full(x.shape[1], 1.0 / x.shape[1])
    gas["m"] = np.full(x.shape[1], 1.0 / x.shape[1])
    gas["mZ"] = 0.01 * gas["m"]
    # a source at a cell corner of the lattice: its 8 nearest gas are equidistant
    src = _src(np.array([[3.0 / ns], [3.0 / ns], [3.0 / ns]]), rng)
    out = oracle.deposit(gas, src, 2.25, kernel=1)
    d = x - src["x"]
    r = np.sqrt((d * d).sum(0))
    got = out["m"] - gas["m"]
    near8 = np.argsort(r)[:8]
    assert np.ptp(got[near8]) < 1e-15 * got[near8].max() and got[near8].min() > 0
    # only one eligible neighbour within reach: it receives everything
    gas2 = dict(gas)
    gas2["mZ"] = gas["mZ"].copy()
    gas2["mZ"][np.argsort(r)[1:]] = gas["m"][np.argsort(r)[1:]]  # metallicity 1 > z_max
    out2 = oracle.deposit(gas2, src, 2.25, kernel=1, z_max=0.1)
    got2 = out2["m"] - gas2["m"]
    assert abs(got2[np.argsort(r)[0]] - src["dM"][0]) < 1e-18
    assert np.all(got2[np.argsort(r)[1:]] == 0.0)
    assert np.array_equal(out2["mZ"][np.argsort(r)[1:]] - gas2["mZ"][np.argsort(r)[1:]],
                          np.zeros(x.shape[1] - 1))
    # mass cap: every gas particle above m_max is left alone
    out3 = oracle.deposit(gas, src, 2.25, kernel=1, m_max=0.5 / x.shape[1])
    assert np.all(out3["A_s"] == 0) and np.array_equal(out3["m"], gas["m"])


def test_resolution_below_the_self_term_is_rejected():
    import pytest
    rng = np.random.default_rng(4)
    gas = _gas(_lattice(4), 0.3, rng)
    with pytest.raises(ValueError):
        oracle.deposit(gas, _src(np.full((3, 1), 0.5), rng), 1.0, kernel=1)
