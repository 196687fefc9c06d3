"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the property it pins. None re-types the oracle's own
arithmetic: they check integrals, symmetries, conservation laws, reproducing
conditions, closed forms on a perfect lattice, the textbook-SPH limit, and
finite differences of the oracle itself.
"""
import math

import numpy as np
import pytest

import synth
from tests import _pins

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ------------------------------------------------------------------ kernels --

@pytest.mark.parametrize("kernel", [0, 1])
def test_kernel_normalisation(oracle_lib, kernel):
    """4 pi C int_0^1 q^2 w(q) dq = 1: radius-h support (App. A.2 footnote)."""
    xg, wg = np.polynomial.legendre.leggauss(40)
    total = 0.0
    for a, b in [(0.0, 0.5), (0.5, 1.0)]:   # the cubic spline is piecewise at q = 1/2
        q = 0.5 * (b - a) * xg + 0.5 * (b + a)
        w, _, norm = oracle_lib.kernel_eval(kernel, q)
        total += 0.5 * (b - a) * np.sum(wg * q * q * w)
    assert abs(4 * math.pi * norm * total - 1.0) < 1e-13


@pytest.mark.parametrize("kernel", [0, 1])
def test_kernel_derivative_and_support(oracle_lib, kernel):
    q = np.linspace(0.01, 0.99, 97)
    eps = 1e-6
    w, dw, _ = oracle_lib.kernel_eval(kernel, q)
    wp, _, _ = oracle_lib.kernel_eval(kernel, q + eps)
    wm, _, _ = oracle_lib.kernel_eval(kernel, q - eps)
    assert np.max(np.abs((wp - wm) / (2 * eps) - dw)) < 1e-8
    w1, dw1, _ = oracle_lib.kernel_eval(kernel, np.array([1.0, 1.5, 3.0]))
    assert np.all(w1 == 0) and np.all(dw1 == 0)
    w0, dw0, _ = oracle_lib.kernel_eval(kernel, np.array([0.0]))
    assert w0[0] == 1.0 and dw0[0] == 0.0


def test_cubic_matches_textbook_m4(oracle_lib):
    q = np.linspace(0, 1.2, 121)
    w, dw, norm = oracle_lib.kernel_eval(0, q)
    assert np.allclose(w, _pins.cubic_w(q), rtol=0, atol=1e-15)
    assert np.allclose(dw, _pins.cubic_dw(q), rtol=0, atol=1e-14)
    assert norm == pytest.approx(8 / math.pi, rel=1e-15)


# ---------------------------------------------------------- neighbour sets --

@pytest.mark.parametrize("make", [
    lambda: synth.lattice16(),
    lambda: synth.random_small(600, 3),
    lambda: synth.plummer_clumps(3000, 6, 11),
])
def test_brute_and_grid_neighbour_sets_equal(oracle_lib, make):
    ps = make()
    h = ps.h * (1 + 0.3 * np.sin(np.arange(ps.n)))  # varied h, exercises max(h_i, h_j)
    for kind in (0, 1):
        a = oracle_lib.neighbours(ps.x, h, kind=kind, mode=0, lists=True)
        b = oracle_lib.neighbours(ps.x, h, kind=kind, mode=1, lists=True)
        assert all(np.array_equal(p, q) for p, q in zip(a, b))


# -------------------------------------------------------- h and the volume --

def test_volume_equals_thacker_fixed_point(oracle_lib):
    """At the root of Delta_N = 1 (App. A.3), V = h^3 / n_h^3 and N = 4pi/3 h^3/V."""
    ps = synth.random_small(500, 7, mass_spread=0.5)
    o = oracle_lib.forward(ps.x, ps.v, ps.m, ps.u, ps.h, oracle_lib.params_for(ps))
    assert o["h_unconverged"] == 0
    rel = np.abs(o["V"] * ps.n_h ** 3 / o["h"] ** 3 - 1)
    assert rel.max() < 1e-12


def test_perfect_lattice_uniform_h_and_volume(oracle_lib):
    ps = synth.perfect_lattice(10, n_ngb=40)
    ps.h_mode = 1
    ps.h = ps.h * (1 + 0.05 * np.cos(np.arange(ps.n)))  # varied guesses, same root
    o = oracle_lib.forward(ps.x, ps.v, ps.m, ps.u, ps.h, oracle_lib.params_for(ps))
    assert np.ptp(o["h"]) / o["h"].mean() < 1e-12
    assert np.ptp(o["V"]) / o["V"].mean() < 1e-12
    # equal masses + identical volumes => rho = m / V (Sec. 2.5.1 eq. rhow)
    assert np.allclose(o["rho"], ps.m / o["V"], rtol=1e-12)


def test_perfect_lattice_closed_form_corrections_and_zero_force(oracle_lib):
    """Perfect lattice: B = grad A = 0, grad B = -(c1/c2) I, and a = du/dt = 0."""
    ps = synth.perfect_lattice(8, n_ngb=32)
    o = oracle_lib.forward(ps.x, ps.v, ps.m, ps.u, ps.h, oracle_lib.params_for(ps))
    h = ps.h[0]
    gB, V = _pins.lattice_corr_closed_form(8, h)
    assert np.allclose(o["V"], V, rtol=1e-12)
    assert np.abs(o["B"]).max() * h < 1e-12
    assert np.abs(o["gradA"]).max() * h < 1e-11
    expect = np.zeros((9, ps.n))
    expect[[0, 4, 8]] = gB
    assert np.abs(o["gradB"] - expect).max() * h * h < 1e-11
    assert np.all(np.abs(o["accel"]) <= 1e-13 * o["scale_a"])
    assert np.all(np.abs(o["dudt"]) <= 1e-13 * np.maximum(o["scale_u"], 1e-300))


# --------------------------------------------------- reproducing conditions --

@pytest.mark.parametrize("h_mode", [0, 1])
def test_reproducing_conditions(oracle_lib, h_mode):
    """W^R = A(1 + B.x)W (App. A.1 eq. RK) reproduces constants and linear fields."""
    ps = synth.random_small(400, 5, mass_spread=0.15, h_mode=h_mode)
    o = oracle_lib.forward(ps.x, ps.v, ps.m, ps.u, ps.h, oracle_lib.params_for(ps))
    assert o["m2_singular"] == 0
    lists = oracle_lib.neighbours(ps.x, o["h"], kind=0, lists=True)
    ii, jj, d = _pins.pair_table(ps.x, lists, 1.0)
    r = np.sqrt((d ** 2).sum(0))
    hi = o["h"][ii]
    Wv = _pins.W(r, hi)
    nz = r > 0
    gW = np.zeros_like(d)
    gW[:, nz] = _pins.dWdr(r[nz], hi[nz]) * d[:, nz] / r[nz]
    A, B, gA, gB = o["A"][ii], o["B"][:, ii], o["gradA"][:, ii], o["gradB"][:, ii]
    lin = 1 + (B * d).sum(0)
    WR = A * lin * Wv
    dbx = np.stack([(gB[3 * g:3 * g + 3] * d).sum(0) for g in range(3)])
    gWR = gA * lin * Wv + A * (dbx + B) * Wv + A * lin * gW
    Vj = o["V"][jj]
    n = ps.n
    s0 = np.bincount(ii, Vj * WR, n)
    assert np.abs(s0 - 1).max() < 1e-12
    for a in range(3):
        s1 = np.bincount(ii, Vj * d[a] * WR, n)
        assert np.abs(s1).max() < 1e-12 * o["h"].max()
        sg = np.bincount(ii, Vj * gWR[a], n)
        assert np.abs(sg).max() * o["h"].min() < 1e-10
        for g in range(3):
            sxg = np.bincount(ii, Vj * d[a] * gWR[g], n)
            assert np.abs(sxg + (1.0 if a == g else 0.0)).max() < 1e-11


@pytest.mark.parametrize("h_mode", [0, 1])
def test_density_off_lattice(oracle_lib, h_mode):
    """Sec. 2.5.1 eq. (rhow): rho_i = sum_j m_j V_j W^R_ij / sum_j V_j^2 W^R_ij, self included,
    evaluated here with the textbook kernel of _pins and the oracle's V, A, B (pinned by the
    volume and reproducing-condition tests) on random, unequal-mass particles, where W in
    place of W^R, or a dropped V_j, give visibly different densities."""
    ps = synth.random_small(400, 7, mass_spread=0.3, h_mode=h_mode)
    o = oracle_lib.forward(ps.x, ps.v, ps.m, ps.u, ps.h, oracle_lib.params_for(ps))
    lists = oracle_lib.neighbours(ps.x, o["h"], kind=0, lists=True)
    ii, jj, d = _pins.pair_table(ps.x, lists, 1.0)
    r = np.sqrt((d ** 2).sum(0))
    assert np.all(r[ii == jj] == 0) and np.sum(ii == jj) == ps.n  # self terms listed once
    Wv = _pins.W(r, o["h"][ii])
    WR = o["A"][ii] * (1 + (o["B"][:, ii] * d).sum(0)) * Wv
    Vj, mj = o["V"][jj], ps.m[jj]
    n = ps.n
    rho = np.bincount(ii, mj * Vj * WR, n) / np.bincount(ii, Vj * Vj * WR, n)
    assert np.abs(rho / o["rho"] - 1).max() < 1e-12
    # the pin separates the readings a slip would give
    rho_w = np.bincount(ii, mj * Vj * Wv, n) / np.bincount(ii, Vj * Vj * Wv, n)
    rho_nov = np.bincount(ii, mj * WR, n) / np.bincount(ii, Vj * WR, n)
    assert np.abs(rho_w / o["rho"] - 1).max() > 1e-2
    assert np.abs(rho_nov / o["rho"] - 1).max() > 1e-2


def test_velocity_gradient_exact_for_linear_field(oracle_lib):
    """grad v (App. A.1 eq. gradv) is exact for v = v0 + M x (linear reproduction, Sec. 2.1)."""
    ps = synth.sedov(12, k=9)
    ps.h_mode = 0
    rng = np.random.default_rng(1)
    M = rng.normal(size=(3, 3))
    v0 = rng.normal(size=3)
    v = v0[:, None] + M @ ps.x
    o = oracle_lib.forward(ps.x, v, ps.m, ps.u, ps.h, oracle_lib.params_for(ps))
    inner = np.all((ps.x > ps.h) & (ps.x < 1 - ps.h), axis=0)
    assert inner.sum() > 50
    gv = o["gradv"][:, inner].reshape(3, 3, -1)
    assert np.abs(gv - M[:, :, None]).max() < 1e-11


# -------------------------------------------------------- conservation laws --

@pytest.mark.parametrize("make,kw", [
    (lambda: synth.lattice16(), {}),
    (lambda: synth.random_small(500, 2, mass_spread=0.5), {}),
    (lambda: synth.random_small(500, 4), {"kernel": 1}),
    (lambda: synth.random_small(500, 6), {"dt_relax": 3.0}),
])
def test_momentum_and_energy_conservation(oracle_lib, make, kw):
    """Pairwise antisymmetry => sum m a = 0 and d/dt sum m (v^2/2 + u) = 0 (Sec. 2.1)."""
    ps = make()
    p = oracle_lib.params_for(ps, **kw)
    if "kernel" in kw:
        p.n_h = synth.n_h_for_neighbours(100)
    o = oracle_lib.forward(ps.x, ps.v, ps.m, ps.u, ps.h, p)
    if "dt_relax" in kw:
        assert 0 < o["relaxed"] < ps.n
    mom = (ps.m * o["accel"]).sum(1)
    assert np.abs(mom).max() <= 1e-13 * (ps.m * o["scale_a"]).sum()
    e = (ps.m * ((ps.v * o["accel"]).sum(0) + o["dudt"])).sum()
    escale = (ps.m * (np.linalg.norm(ps.v, axis=0) * o["scale_a"] + o["scale_u"])).sum()
    assert abs(e) <= 1e-13 * escale


# --------------------------------------------------------------- invariance --

def _fwd(oracle_lib, ps, x=None, v=None, **kw):
    return oracle_lib.forward(ps.x if x is None else x, ps.v if v is None else v, ps.m, ps.u,
                              ps.h, oracle_lib.params_for(ps, **kw))


def test_galilean_translation_permutation_reflection(oracle_lib):
    ps = synth.random_small(400, 8)
    o = _fwd(oracle_lib, ps)
    tol_a = 1e-10 * o["scale_a"].max()
    tol_u = 1e-10 * o["scale_u"].max()
    # Galilean boost
    g = _fwd(oracle_lib, ps, v=ps.v + np.array([[0.3], [-0.2], [0.5]]))
    assert np.abs(g["accel"] - o["accel"]).max() < tol_a
    assert np.abs(g["dudt"] - o["dudt"]).max() < tol_u
    # periodic translation
    t = _fwd(oracle_lib, ps, x=np.mod(ps.x + np.array([[0.37], [0.81], [0.05]]), 1.0))
    assert np.abs(t["accel"] - o["accel"]).max() < tol_a
    assert np.abs(t["dudt"] - o["dudt"]).max() < tol_u
    # axis permutation (x, y, z) -> (y, z, x)
    perm = [1, 2, 0]
    p = _fwd(oracle_lib, ps, x=ps.x[perm], v=ps.v[perm])
    assert np.abs(p["accel"] - o["accel"][perm]).max() < tol_a
    assert np.abs(p["gradv"].reshape(3, 3, -1) -
                  o["gradv"].reshape(3, 3, -1)[perm][:, perm]).max() < 1e-9 * np.abs(o["gradv"]).max()
    # reflection x -> -x
    xr = ps.x.copy()
    xr[0] = np.mod(-xr[0], 1.0)
    vr = ps.v.copy()
    vr[0] = -vr[0]
    r = _fwd(oracle_lib, ps, x=xr, v=vr)
    ar = r["accel"].copy()
    ar[0] = -ar[0]
    assert np.abs(ar - o["accel"]).max() < tol_a
    assert np.abs(r["dudt"] - o["dudt"]).max() < tol_u


# -------------------------------------------------------- viscosity pins ----

def test_viscosity_vanishes_for_exact_linear_flow(oracle_lib):
    """Linear v with exact grad v: limiter = 1, midpoint jump = 0 => Q = 0."""
    ps = synth.sedov(20, k=9)
    ps.h_mode = 0
    rng = np.random.default_rng(3)
    M = rng.normal(size=(3, 3))
    v = M @ ps.x
    o1 = oracle_lib.forward(ps.x, v, ps.m, ps.u, ps.h,
                            oracle_lib.params_for(ps, alpha=1.0, beta=2.0), nbr_mode=1)
    o0 = oracle_lib.forward(ps.x, v, ps.m, ps.u, ps.h,
                            oracle_lib.params_for(ps, alpha=0.0, beta=0.0), nbr_mode=1)
    # only particles whose whole two-hop neighbourhood avoids the periodic seam
    inner = np.all((ps.x > 2 * ps.h) & (ps.x < 1 - 2 * ps.h), axis=0)
    assert inner.sum() > 5
    assert np.abs(o1["accel"][:, inner] - o0["accel"][:, inner]).max() < \
        1e-10 * o0["scale_a"][inner].max()


def test_outputs_affine_in_alpha_beta(oracle_lib):
    """a and du/dt are affine in (alpha, beta); pins the oracle's alpha/beta tangents."""
    ps = synth.random_small(3000, 12)
    p = oracle_lib.params_for(ps)
    base = oracle_lib.forward(ps.x, ps.v, ps.m, ps.u, ps.h, p)
    pa = oracle_lib.params_for(ps, alpha=p.alpha + 1.0)
    pb = oracle_lib.params_for(ps, beta=p.beta + 1.0)
    fa = oracle_lib.forward(ps.x, ps.v, ps.m, ps.u, ps.h, pa)
    fb = oracle_lib.forward(ps.x, ps.v, ps.m, ps.u, ps.h, pb)
    z3, z1 = np.zeros((3, ps.n)), np.zeros(ps.n)
    ja = oracle_lib.jvp(ps.x, ps.v, ps.m, ps.u, ps.h, p, z3, z3, z1, dalpha=1.0)
    jb = oracle_lib.jvp(ps.x, ps.v, ps.m, ps.u, ps.h, p, z3, z3, z1, dbeta=1.0)
    sa = base["scale_a"].max()
    assert np.abs(ja["d_accel"] - (fa["accel"] - base["accel"])).max() < 1e-11 * sa
    assert np.abs(jb["d_accel"] - (fb["accel"] - base["accel"])).max() < 1e-11 * sa
    assert np.abs(ja["d_dudt"] - (fa["dudt"] - base["dudt"])).max() < 1e-11 * base["scale_u"].max()
    # pure expansion: every mu = 0 => no viscosity at all
    pe = oracle_lib.forward(ps.x, 0.5 * (ps.x - 0.5), ps.m, ps.u, ps.h,
                            oracle_lib.params_for(ps, alpha=0.0, beta=0.0))
    pe1 = oracle_lib.forward(ps.x, 0.5 * (ps.x - 0.5), ps.m, ps.u, ps.h, p)
    hm = pe["h"].max()
    inner = np.all((ps.x > 2 * hm) & (ps.x < 1 - 2 * hm), axis=0)
    assert inner.sum() >= 5
    assert np.abs(pe["accel"][:, inner] - pe1["accel"][:, inner]).max() <= \
        1e-12 * pe["scale_a"].max()


def test_relaxed_pairs_reduce_to_textbook_sph(oracle_lib):
    """Relaxation (App. A.1): A = 1, B = 0 on every pair => kernel-averaged SPH force."""
    ps = synth.random_small(300, 13)
    ps.h_mode = 0
    v = np.random.default_rng(2).normal(size=ps.x.shape)   # |div v| >> 0 everywhere
    p = oracle_lib.params_for(ps, alpha=0.0, beta=0.0, dt_relax=1e3)
    o = oracle_lib.forward(ps.x, v, ps.m, ps.u, ps.h, p)
    assert o["relaxed"] == ps.n
    sym = oracle_lib.neighbours(ps.x, ps.h, kind=1, lists=True)
    a = _pins.textbook_sph_accel(ps.x, ps.m, o["V"], o["P"], ps.h, 1.0, sym)
    assert np.abs(a - o["accel"]).max() < 1e-12 * o["scale_a"].max()


@pytest.mark.parametrize("h_mode", [0, 1])
def test_compatible_energy_splits_work_equally(oracle_lib, h_mode):
    """Compatible energy (Sec. 2.1): each pair's work (v_i - v_j).F_ij goes half to i, half to j.

    With the viscosity off F_ij does not depend on v. Move one particle k with
    w and hold the rest: the heat w.(m_k a_k) taken from k's kinetic energy
    lands half on k and half on its neighbours together, -1/2 w.(m_k a_k) each.
    Any other split (by P/rho^2, by mass) moves the mover's share off one half.
    """
    ps = synth.random_small(500, 21, mass_spread=0.5)
    ps.h_mode = h_mode
    p = oracle_lib.params_for(ps, alpha=0.0, beta=0.0)
    zero = np.zeros_like(ps.x)
    base = oracle_lib.forward(ps.x, zero, ps.m, ps.u, ps.h, p)
    assert np.abs(base["dudt"]).max() == 0.0
    rng = np.random.default_rng(5)
    for k in rng.choice(ps.n, 4, replace=False):
        v = zero.copy()
        v[:, k] = rng.normal(size=3)
        o = oracle_lib.forward(ps.x, v, ps.m, ps.u, ps.h, p)
        assert np.abs(o["accel"] - base["accel"]).max() == 0.0
        work = float(v[:, k] @ (ps.m[k] * o["accel"][:, k]))
        assert abs(work) > 0
        mdu = ps.m * o["dudt"]
        assert abs(mdu[k] + 0.5 * work) <= 1e-12 * abs(work)
        others = np.delete(mdu, k)
        assert abs(others.sum() + 0.5 * work) <= 1e-12 * abs(work)
        assert np.count_nonzero(others) >= 10


def test_relaxed_pairs_compatible_energy_is_textbook(oracle_lib):
    """Relaxed pairs (App. A.1): du_i/dt = -1/(2 m_i) sum_j (v_i - v_j).F_ij with textbook F_ij."""
    ps = synth.random_small(300, 13)
    ps.h_mode = 0
    v = np.random.default_rng(2).normal(size=ps.x.shape)
    p = oracle_lib.params_for(ps, alpha=0.0, beta=0.0, dt_relax=1e3)
    o = oracle_lib.forward(ps.x, v, ps.m, ps.u, ps.h, p)
    assert o["relaxed"] == ps.n
    sym = oracle_lib.neighbours(ps.x, ps.h, kind=1, lists=True)
    du = np.zeros(ps.n)
    for i in range(ps.n):
        js = sym[i]
        if len(js) == 0:
            continue
        d = _pins.min_image(ps.x[:, [i]], ps.x[:, js], 1.0)
        r = np.sqrt((d ** 2).sum(0))
        g = 0.5 * (_pins.dWdr(r, ps.h[i]) + _pins.dWdr(r, ps.h[js])) * d / r
        F = -o["V"][i] * o["V"][js] * (o["P"][i] + o["P"][js]) * g
        du[i] = -0.5 * ((v[:, [i]] - v[:, js]) * F).sum() / ps.m[i]
    assert np.abs(du - o["dudt"]).max() < 1e-12 * o["scale_u"].max()


def test_equation_of_state(oracle_lib):
    ps = synth.random_small(200, 14)
    o = _fwd(oracle_lib, ps)
    assert np.allclose(o["P"], (5 / 3 - 1) * o["rho"] * ps.u, rtol=1e-14)
    assert np.allclose(o["c"], np.sqrt(5 / 3 * 2 / 3 * ps.u), rtol=1e-14)


# ------------------------------------------------------- derivatives (JVP) --

def _loss(o, ps):
    return float((ps.w_a * o["accel"]).sum() + (ps.w_u * o["dudt"]).sum())


@pytest.mark.parametrize("h_mode", [0, 1])
def test_jvp_matches_central_differences(oracle_lib, h_mode):
    """Dual-number JVP of the loss vs central FD of the oracle (random direction)."""
    ps = synth.random_small(216, 21, mass_spread=0.2, h_mode=h_mode)
    p = oracle_lib.params_for(ps)
    rng = np.random.default_rng(5)
    dx = rng.normal(size=(3, ps.n))
    dv = rng.normal(size=(3, ps.n))
    du = rng.normal(size=ps.n) * ps.u
    da, db = 0.7, -0.4
    j = oracle_lib.jvp(ps.x, ps.v, ps.m, ps.u, ps.h, p, dx, dv, du, da, db)
    jl = float((ps.w_a * j["d_accel"]).sum() + (ps.w_u * j["d_dudt"]).sum())
    eps = 1e-7

    def L(s):
        q = oracle_lib.params_for(ps, alpha=p.alpha + s * da, beta=p.beta + s * db)
        o = oracle_lib.forward(ps.x + s * dx, ps.v + s * dv, ps.m, ps.u + s * du, ps.h, q)
        return _loss(o, ps)

    fd = (L(eps) - L(-eps)) / (2 * eps)
    assert abs(fd - jl) <= 1e-5 * abs(jl)


def test_h_tangent_matches_resolve(oracle_lib):
    """Implicit-function h tangent vs finite differences of the re-solved h."""
    ps = synth.random_small(300, 22)
    p = oracle_lib.params_for(ps)
    rng = np.random.default_rng(6)
    dx = rng.normal(size=(3, ps.n))
    z3, z1 = np.zeros((3, ps.n)), np.zeros(ps.n)
    j = oracle_lib.jvp(ps.x, ps.v, ps.m, ps.u, ps.h, p, dx, z3, z1)
    eps = 1e-7
    hp = oracle_lib.forward(ps.x + eps * dx, ps.v, ps.m, ps.u, ps.h, p)["h"]
    hm = oracle_lib.forward(ps.x - eps * dx, ps.v, ps.m, ps.u, ps.h, p)["h"]
    fd = (hp - hm) / (2 * eps)
    assert np.abs(fd - j["d_h"]).max() <= 1e-5 * np.abs(j["d_h"]).max()
    # V = h^3 / n_h^3 at the root => dV = 3 V dh / h
    o = oracle_lib.forward(ps.x, ps.v, ps.m, ps.u, ps.h, p)
    assert np.allclose(j["d_V"], 3 * o["V"] * j["d_h"] / o["h"], rtol=1e-8,
                       atol=1e-10 * np.abs(j["d_V"]).max())
