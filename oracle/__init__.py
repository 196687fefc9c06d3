"""Python wrapper of the FP64 CPU oracle (``crk_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg. The GPU library never imports or links it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "crk_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

# Plain optimisation, no fast-math, no FMA contraction, portable ISA.
CXXFLAGS = ["-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
            "-ffp-contract=off"]


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", *CXXFLAGS, _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        D = C.POINTER(C.c_double)
        I64 = C.POINTER(C.c_int64)
        _lib.oracle_num_threads.argtypes = []
        _lib.oracle_num_threads.restype = C.c_int
        _lib.oracle_set_threads.argtypes = [C.c_int]
        _lib.oracle_set_threads.restype = None
        _lib.oracle_kernel_eval.argtypes = [C.c_int, C.c_int64, D, D, D, D]
        _lib.oracle_neighbours.argtypes = [C.c_int64, D, D, C.c_double, C.c_int, C.c_int, I64, I64]
        _lib.oracle_neighbours.restype = C.c_int
        common = [C.c_int64, D, D, D, D, D, C.c_double, C.c_double, C.c_double, C.c_double,
                  C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int]
        _lib.oracle_forward.argtypes = common + [D] * 14 + [I64]
        _lib.oracle_forward.restype = C.c_int
        _lib.oracle_forward_passive.argtypes = (common + [C.POINTER(C.c_uint8)] + [D] * 7
                                                + [D] * 14 + [I64])
        _lib.oracle_forward_passive.restype = C.c_int
        _lib.oracle_jvp.argtypes = common + [D, D, D, C.c_double, C.c_double] + [D] * 7
        _lib.oracle_jvp.restype = C.c_int
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pi(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _c(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


@dataclass
class Params:
    box: float = 1.0
    gamma: float = 5.0 / 3.0
    alpha: float = 1.0
    beta: float = 2.0
    eps2: float = 0.01
    n_h: float = 2.4814
    dt_relax: float = 0.0
    kernel: int = 0          # 0 cubic spline, 1 Wendland C4
    h_mode: int = 1          # 0 fixed, 1 solve

    def args(self):
        return [self.box, self.gamma, self.alpha, self.beta, self.eps2, self.n_h, self.dt_relax,
                self.kernel, self.h_mode]


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (the benchmark's one-core timing)."""
    lib().oracle_set_threads(int(n))


def kernel_eval(kernel: int, q):
    q = _c(q).ravel()
    w = np.empty_like(q)
    dw = np.empty_like(q)
    norm = np.zeros(1)
    lib().oracle_kernel_eval(kernel, q.size, _p(q), _p(w), _p(dw), _p(norm))
    return w, dw, float(norm[0])


def neighbours(x, h, box=1.0, mode=0, kind=0, lists=False):
    x = _c(x)
    h = _c(h)
    n = h.size
    counts = np.zeros(n, dtype=np.int64)
    rc = lib().oracle_neighbours(n, _p(x), _p(h), box, mode, kind, _pi(counts), None)
    if rc:
        raise RuntimeError("oracle_neighbours failed: %d" % rc)
    if not lists:
        return counts
    out = np.zeros(int(counts.sum()), dtype=np.int64)
    rc = lib().oracle_neighbours(n, _p(x), _p(h), box, mode, kind, _pi(counts), _pi(out))
    if rc:
        raise RuntimeError("oracle_neighbours failed: %d" % rc)
    off = np.concatenate([[0], np.cumsum(counts)])
    return [out[off[i]:off[i + 1]] for i in range(n)]


PASSIVE_KEYS = ("V", "A", "B", "gradA", "gradB", "rho", "gradv")


def forward(x, v, m, u, h, params: Params, nbr_mode: int = 0, passive: dict = None) -> dict:
    """FP64 forward. Returns a dict of numpy arrays (SoA) and the pair stats.

    passive: optional stored state of the particles that are passive in a
    timestep hierarchy: "mask" (True = passive) and their V, A, B, gradA,
    gradB, rho, gradv (caller layouts, all particles; only the masked ones
    are read). Those particles keep these values; their P and c follow
    from rho and u; their other outputs carry no meaning."""
    x, v, m, u, h = _c(x), _c(v), _c(m), _c(u), _c(h)
    n = m.size
    o = {k: np.zeros(s) for k, s in [("h", n), ("V", n), ("rho", n), ("A", n), ("B", (3, n)),
                                      ("gradA", (3, n)), ("gradB", (9, n)), ("gradv", (9, n)),
                                      ("P", n), ("c", n), ("accel", (3, n)), ("dudt", n),
                                      ("scale_a", n), ("scale_u", n)]}
    stats = np.zeros(6, dtype=np.int64)
    outs = [_p(o[k]) for k in ["h", "V", "rho", "A", "B", "gradA", "gradB", "gradv", "P", "c",
                               "accel", "dudt", "scale_a", "scale_u"]]
    if passive is None:
        rc = lib().oracle_forward(n, _p(x), _p(v), _p(m), _p(u), _p(h), *params.args(),
                                  nbr_mode, *outs, _pi(stats))
    else:
        mask = np.ascontiguousarray(passive["mask"], dtype=np.uint8)
        if mask.shape != (n,):
            raise ValueError("passive mask must have shape (n,)")
        shapes = {"V": n, "A": n, "B": (3, n), "gradA": (3, n), "gradB": (9, n), "rho": n,
                  "gradv": (9, n)}
        st = [_c(passive[k], shapes[k]) for k in PASSIVE_KEYS]
        rc = lib().oracle_forward_passive(
            n, _p(x), _p(v), _p(m), _p(u), _p(h), *params.args(), nbr_mode,
            mask.ctypes.data_as(C.POINTER(C.c_uint8)), *[_p(a) for a in st], *outs, _pi(stats))
    if rc:
        raise RuntimeError("oracle_forward failed: %d" % rc)
    o["pairs_gather"], o["pairs_force"], o["h_iters_max"], o["h_unconverged"], \
        o["m2_singular"], o["relaxed"] = [int(s) for s in stats]
    return o


def jvp(x, v, m, u, h, params: Params, dx, dv, du, dalpha=0.0, dbeta=0.0,
        nbr_mode: int = 0) -> dict:
    """Exact directional derivative of the forward along (dx, dv, du, dalpha, dbeta)."""
    x, v, m, u, h = _c(x), _c(v), _c(m), _c(u), _c(h)
    dx, dv, du = _c(dx, x.shape), _c(dv, v.shape), _c(du, u.shape)
    n = m.size
    o = {k: np.zeros(s) for k, s in [("accel", (3, n)), ("dudt", n), ("d_accel", (3, n)),
                                      ("d_dudt", n), ("d_h", n), ("d_V", n), ("d_rho", n)]}
    rc = lib().oracle_jvp(n, _p(x), _p(v), _p(m), _p(u), _p(h), *params.args(), nbr_mode,
                          _p(dx), _p(dv), _p(du), float(dalpha), float(dbeta),
                          *[_p(o[k]) for k in ["accel", "dudt", "d_accel", "d_dudt", "d_h",
                                               "d_V", "d_rho"]])
    if rc:
        raise RuntimeError("oracle_jvp failed: %d" % rc)
    return o


def params_for(ps, **kw) -> Params:
    """Oracle parameters for a synth.ParticleSet (kernel radius h, n_h, h mode, box)."""
    p = Params(box=ps.box, n_h=ps.n_h, h_mode=ps.h_mode)
    for k, val in kw.items():
        setattr(p, k, val)
    return p


# ------------------------------------------------------------ time step --
# One kick-drift-kick cycle on a single timestep level, App. A.4 (the KDK
# update) with the smoothing-length evolution of App. A.3: the Thacker
# estimate h^T = h (1 - lambda + lambda Delta_N), Delta_N^3 = V n_h^3 / h^3,
# gives hdot^T = (h^T - h) / dt; continuity gives hdot^cont = h div(v) / 3;
# each drift of dt updates h <- h exp(hdot dt / h). Positions accumulate in
# FP64 (App. A.4, last paragraph). The evaluation at the end of the step
# takes the predicted velocity and energy v^1/2 + a^0 dt / 2, u^1/2 +
# du^0 dt / 2 (the paper leaves the velocity of that evaluation open).

def kdk_step(x, v, m, u, h, prev: dict, params: Params, dt: float, lam: float,
             nbr_mode: int = 0) -> dict:
    """One KDK step from the state (x, v, u, h) and the evaluation prev at it.

    prev holds accel, dudt, V and gradv of the forward at (x, v, u, h) with h
    fixed. Returns the new x, v, u, h and the forward at the new state (its
    accel, dudt, V, gradv serve as prev of the next step).
    """
    if params.h_mode != 0:
        raise ValueError("the time-integrated smoothing length needs h_mode = 0")
    x, v, m, u, h = _c(x), _c(v), _c(m), _c(u), _c(h)
    a0, du0 = _c(prev["accel"]), _c(prev["dudt"])
    # first kick
    v_half = v + 0.5 * dt * a0
    u_half = u + 0.5 * dt * du0
    # hdot from the evaluation at the start of the step
    div_v = prev["gradv"][0] + prev["gradv"][4] + prev["gradv"][8]
    delta_n = params.n_h * np.cbrt(prev["V"]) / h
    h_thacker = h * (1.0 - lam + lam * delta_n)
    hdot = (h_thacker - h) / dt + h * div_v / 3.0
    # drift
    x_new = np.mod(x + dt * v_half, params.box)
    h_new = h * np.exp(hdot * dt / h)
    # evaluation at the end of the step, then the second kick
    o = forward(x_new, v_half + 0.5 * dt * a0, m, u_half + 0.5 * dt * du0, h_new, params,
                nbr_mode=nbr_mode)
    o["x"] = x_new
    o["v"] = v_half + 0.5 * dt * o["accel"]
    o["u"] = u_half + 0.5 * dt * o["dudt"]
    o["h"] = h_new
    return o


# ------------------------------------------------- timestep hierarchy --
# One big step dt of the hierarchical KDK integrator, App. A.4, on
# power-of-two levels: a particle of level L is active on intervals
# dt_a = dt / 2^L and all particles drift on the smallest interval
# dt_min = dt / 2^Lmax. At the start of its interval a particle takes its
# first kick and its hdot (App. A.3: Thacker plus continuity, with dt_a);
# every substep drifts every particle, x on the piecewise-parabolic path
# v_j = v^1/2 + a^0 (t_elapsed + (dt_min - dt_a) / 2) (FP64), h by
# h exp(hdot dt_min / h), and updates the passive state V = (h / n_h)^3,
# rho <- rho exp(-div v dt_min); at the end of each substep the particles
# whose interval ends are evaluated (the others passive, with their stored
# V, rho, corrections and grad v), kicked a second time and, unless the big
# step is over, open their next interval. The evaluation takes each
# particle's velocity and energy at that time under its constant a^0 and
# du^0 (the predicted values of the single-level step, R14, for the active
# ones).
#
# Timestep refinement, App. A.5: a particle may be moved to a finer level L'
# at the start of substep j_r (a limiter's decision, given by the caller).
# Its interval opened at t_0 with its level L; at t_r = j_r dt_min, e = t_r
# - t_0 into it, the half-kicked state is re-synchronised: the velocity and
# energy advance under the constant a^0, du^0 to t_r (v <- v^0 + a^0 e), and
# a new interval of dt_c = dt / 2^L' opens there as any interval opens. The
# cycle then ends with v^1 = v^0 + a^0 e + (a^0 + a^1) dt_c / 2, which is
# App. A.5's piecewise-constant final kick with dt_b = e + dt_c (for e = 0
# its corrected half kick, v^1/2 = v^0 + a^0 dt_b / 2); the drift keeps the
# parabola of a^0, and the particle stays on level L' to the end of the big
# step. j_r must lie on the grid of L' (a multiple of 2^(Lmax - L')) so that
# the refined intervals end on it; at an interval start of L (e = 0) the
# refinement is the same as having level L' from there on.

def hkdk_step(x, v, m, u, h, prev: dict, levels, params: Params, dt: float, lam: float,
              nbr_mode: int = 0, trace: list = None, refine=None, evaluate=None) -> dict:
    """One big step of the hierarchy from the synchronised state (x, v, u, h).

    prev holds the evaluation at that state with h fixed (accel, dudt, V,
    rho, A, B, gradA, gradB, gradv). levels: int per particle, >= 0.
    refine: None, or (refine_at, refine_level) per particle: refine_at = -1
    for none, else the substep j_r at whose start the particle moves to the
    finer level refine_level (Lmax counts these levels too).
    evaluate: None (the CRKSPH forward), or a function (x, v, u, h, passive)
    returning at least accel and dudt (the integrator's own tests).
    Returns the synchronised x, v, u, h and each particle's latest
    evaluation (the prev of the next big step). trace, when given, collects
    per substep the passive mask and the x, h, V, rho the evaluation used.
    """
    if params.h_mode != 0:
        raise ValueError("the time-integrated smoothing length needs h_mode = 0")
    levels = np.asarray(levels, dtype=np.int64).copy()
    if levels.min() < 0:
        raise ValueError("levels must be >= 0")
    x, v, m, u, h = _c(x).copy(), _c(v).copy(), _c(m), _c(u).copy(), _c(h).copy()
    r_at = np.full(m.size, -1, dtype=np.int64)
    r_lev = levels.copy()
    if refine is not None:
        r_at = np.asarray(refine[0], dtype=np.int64)
        r_lev = np.asarray(refine[1], dtype=np.int64)
    ref = r_at >= 0
    lmax = int(max(levels.max(), r_lev[ref].max() if ref.any() else 0))
    nsub = 1 << lmax
    if ref.any():
        if np.any(r_lev[ref] <= levels[ref]):
            raise ValueError("a refinement moves a particle to a finer level")
        if np.any(r_at[ref] >= nsub) or np.any(r_at[ref] % (1 << (lmax - r_lev[ref])) != 0):
            raise ValueError("a refinement starts on the grid of its new level")
    dt_min = dt / nsub
    if evaluate is None:
        def evaluate(x_, v_, u_, h_, passive):
            return forward(x_, v_, m, u_, h_, params, nbr_mode=nbr_mode, passive=passive)
    keys = ("accel", "dudt") + tuple(k for k in PASSIVE_KEYS if k in prev)
    st = {k: _c(prev[k]).copy() for k in keys}
    vh = np.empty_like(v)
    uh = np.empty_like(u)
    hdot = np.empty_like(h)
    per = np.left_shift(1, lmax - levels)  # substeps per active interval
    dta = per * dt_min
    start = np.zeros(m.size, dtype=np.int64)  # substep that opened each interval

    def open_interval(sel):
        vh[:, sel] = v[:, sel] + 0.5 * dta[sel] * st["accel"][:, sel]
        uh[sel] = u[sel] + 0.5 * dta[sel] * st["dudt"][sel]
        if "gradv" in st:
            g = st["gradv"]
            div_v = g[0, sel] + g[4, sel] + g[8, sel]
            delta_n = params.n_h * np.cbrt(st["V"][sel]) / h[sel]
            h_thacker = h[sel] * (1.0 - lam + lam * delta_n)
            hdot[sel] = (h_thacker - h[sel]) / dta[sel] + h[sel] * div_v / 3.0
        else:
            hdot[sel] = 0.0

    open_interval(np.ones(m.size, dtype=bool))
    for j in range(nsub):
        sel = r_at == j
        if sel.any():
            # re-synchronise at t_r under the constant a^0, du^0 and open the
            # refined interval there
            e = (j - start[sel]) * dt_min
            v[:, sel] = v[:, sel] + st["accel"][:, sel] * e
            u[sel] = u[sel] + st["dudt"][sel] * e
            levels[sel] = r_lev[sel]
            per[sel] = 1 << (lmax - levels[sel])
            dta[sel] = per[sel] * dt_min
            start[sel] = j
            open_interval(sel)
        elapsed = (j - start) * dt_min
        # drift
        v_j = vh + st["accel"] * (elapsed + 0.5 * (dt_min - dta))
        x = np.mod(x + v_j * dt_min, params.box)
        h = h * np.exp(hdot * dt_min / h)
        if "gradv" in st:
            g = st["gradv"]
            st["V"] = (h / params.n_h) ** 3
            st["rho"] = st["rho"] * np.exp(-(g[0] + g[4] + g[8]) * dt_min)
        # evaluation for the particles whose interval ends now
        j_end = j + 1
        active = (j_end - start) == per
        t_rel = (j_end - start) * dt_min - 0.5 * dta  # time since the half kick's centre
        v_p = vh + st["accel"] * t_rel
        u_p = uh + st["dudt"] * t_rel
        pas = dict({k: st[k] for k in PASSIVE_KEYS if k in st}, mask=~active)
        if trace is not None:
            trace.append({"passive": ~active, "x": x.copy(), "h": h.copy(),
                          "V": st["V"].copy() if "V" in st else None,
                          "rho": st["rho"].copy() if "rho" in st else None})
        o = evaluate(x, v_p, u_p, h, pas)
        # second kick of the active particles; their evaluation is stored
        v[:, active] = vh[:, active] + 0.5 * dta[active] * o["accel"][:, active]
        u[active] = uh[active] + 0.5 * dta[active] * o["dudt"][active]
        for k in keys:
            st[k][..., active] = o[k][..., active]
        if j_end < nsub:
            start[active] = j_end
            open_interval(active)
    # every interval ends at dt: the last evaluation had every particle active
    out = dict(o)
    out.update(st)
    out.update(x=x, v=v, u=u, h=h)
    return out


# ------------------------------------------------------------- cooling --
# Exact integration of du/dt = -s Lambda / rho over dt (Sec. 2.2, exact
# integration) for a source function tabulated at log-spaced energies and
# interpolated by piecewise power laws. The composition is folded into the
# table: Lambda(u; rho) = rho^2 lam(u), so du/dt = -rho lam(u) (cooling where
# lam > 0, heating where lam < 0). Each particle is anchored at u_a = u^0, so
# I(u^0) = 0 and I(u^1) = Lambda_a dt / (u_a rho); I is accumulated bin by bin
# from the anchor in the direction of evolution (down for cooling, up for
# heating) with the per-bin closed form, and the final bin is inverted.
# A bin where lam changes sign holds the equilibrium: there the source is
# held at the larger of the two edge magnitudes, in the direction of the
# anchor's side, and u stops at the zero of the linear interpolant. Below
# the first node or above the last, u is clamped to the table.

class CoolingTable:
    """lam_k at u_k = 10^(log10_u0 + k dex), k = 0 .. K-1."""

    def __init__(self, log10_u0: float, dex: float, lam):
        self.lu0, self.dex = float(log10_u0), float(dex)
        self.lam = np.asarray(lam, dtype=np.float64)
        self.K = self.lam.size

    def u(self, k):
        return 10.0 ** (self.lu0 + k * self.dex)

    def slope(self, k):
        """alpha_k of bin [u_k, u_k+1] (same-sign edges)."""
        return np.log(self.lam[k + 1] / self.lam[k]) / np.log(self.u(k + 1) / self.u(k))

    def lam_at(self, u):
        k = min(max(int(np.floor((np.log10(u) - self.lu0) / self.dex)), 0), self.K - 2)
        lk, lk1 = self.lam[k], self.lam[k + 1]
        if lk * lk1 <= 0.0:  # the equilibrium bin: linear
            return lk + (lk1 - lk) * (u - self.u(k)) / (self.u(k + 1) - self.u(k))
        return lk * (u / self.u(k)) ** self.slope(k)


def _I_in_bin(tab, k, u, Ik, s, la, ua):
    """I(u) in power-law bin k from I_k = I(u_k), eq. (Iu); la = |lam(u_a)|."""
    uk, lk = tab.u(k), abs(tab.lam[k])
    a = tab.slope(k)
    c = s * la * uk / (lk * ua)
    if a == 1.0:
        return Ik + c * (-np.log(u / uk))
    # [1 - (u/u_k)^(1 - a)] / (1 - a), written with expm1 so that slopes
    # near 1 keep their accuracy (the same function, tending to -ln(u/u_k))
    return Ik + c * (-np.expm1((1.0 - a) * np.log(u / uk)) / (1.0 - a))


def _I_inverse(tab, k, I, Ik, s, la, ua):
    """u in power-law bin k with I(u) = I, eq. (Iinv)."""
    uk, lk = tab.u(k), abs(tab.lam[k])
    a = tab.slope(k)
    c = s * lk * ua / (la * uk)
    if a == 1.0:
        return uk * np.exp(-c * (I - Ik))
    # [1 - (I - I_k)(1 - a) c]^(1 / (1 - a)) with log1p (same reason)
    return uk * np.exp(np.log1p(-(I - Ik) * (1.0 - a) * c) / (1.0 - a))


def cool(tab: CoolingTable, u0, rho, dt: float):
    """u^1 of every particle after dt (FP64, one particle at a time)."""
    u0 = np.asarray(u0, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    out = np.empty_like(u0)
    lo, hi = tab.u(0), tab.u(tab.K - 1)
    for i in range(u0.size):
        u = min(max(u0[i], lo), hi)
        left = rho[i] * dt   # rho times the time still to integrate
        # a particle that starts on the outer side of an unstable zero leaves
        # its bin and is anchored again at the bin edge (at most once per side)
        for _ in range(3):
            u, left = _cool_from(tab, u, left)
            if left <= 0.0:
                break
        out[i] = u
    return out


def _bin_of(tab, u):
    return min(max(int(np.floor((np.log10(u) - tab.lu0) / tab.dex)), 0), tab.K - 2)


def _equilibrium_bin(tab, k, u, left):
    """Bin k holds the sign change: constant source of the larger edge
    magnitude (left = rho t). Toward the zero of the linear interpolant u
    stops there; away from it (an unstable zero) u runs to the bin edge and
    the time still left is returned."""
    uk, uk1 = tab.u(k), tab.u(k + 1)
    lk, lk1 = tab.lam[k], tab.lam[k + 1]
    ueq = uk - lk * (uk1 - uk) / (lk1 - lk) if lk1 != lk else uk
    lin = lk + (lk1 - lk) * (u - uk) / (uk1 - uk)
    mag = max(abs(lk), abs(lk1))
    if lin == 0.0 or mag == 0.0:
        return u, 0.0
    down = lin > 0.0                  # cooling moves u down
    target = ueq if (ueq < u) == down else (uk if down else uk1)
    dist = abs(u - target)
    if mag * left <= dist:
        return (u - mag * left if down else u + mag * left), 0.0
    if target == ueq:
        return ueq, 0.0
    return target, left - dist / mag


def _cool_from(tab, ua, left):
    """Integrate from the anchor u_a for rho t = left; returns (u, left')."""
    k = _bin_of(tab, ua)
    if tab.lam[k] * tab.lam[k + 1] <= 0.0:
        return _equilibrium_bin(tab, k, ua, left)
    la = abs(tab.lam_at(ua))          # Lambda_a / rho^2
    s = 1.0 if tab.lam[k] > 0.0 else -1.0   # +1 cooling, -1 heating
    I1 = la * left / ua               # I(u^1) = Lambda_a dt / (u_a rho), with I(u^0) = 0
    Ik = -_I_in_bin(tab, k, ua, 0.0, s, la, ua)   # I_k of the anchor's bin
    while True:
        # the far edge of bin k in the direction of evolution, and I there
        if s > 0:
            edge, Iedge = tab.u(k), Ik
        else:
            edge, Iedge = tab.u(k + 1), _I_in_bin(tab, k, tab.u(k + 1), Ik, s, la, ua)
        if Iedge >= I1:
            return _I_inverse(tab, k, I1, Ik, s, la, ua), 0.0
        kn = k - 1 if s > 0 else k + 1
        if kn < 0 or kn > tab.K - 2:
            return edge, 0.0          # clamped at the end of the table
        if tab.lam[kn] * tab.lam[kn + 1] <= 0.0:
            # the equilibrium bin, entered toward its zero: rho t left is
            # (I1 - I(edge)) u_a / |lam_a|
            return _equilibrium_bin(tab, kn, edge, (I1 - Iedge) * ua / la)
        # I_k of the next bin: for cooling its upper edge is the edge just
        # reached, for heating its lower edge
        Ik = Iedge - _I_in_bin(tab, kn, edge, 0.0, s, la, ua) if s > 0 else Iedge
        k = kn


# ---------------------------------------------------------- deposition --
# Subgrid sources (stars, winds, black holes) coupling to the gas, App. A.2
# eq. (Vsg) and the SPH-weighted deposition of Sec. 2.5 / 2.6 / 2.7 (eqs.
# windmetal and Anorm, starmetal and stellarmom, AGNE):
#   V_s^-1 = sum over gas j and the source itself of W(|x_sj|, h_j) (the
#     scatter definition: each gas neighbour's own h; the self term takes h_s);
#   h_s = n_h,s V_s^(1/3), so the self term is C w(0) / (n_h,s^3 V_s) and
#     V_s = (1 - C w(0) / n_h,s^3) / (sum over gas of W(|x_sj|, h_j));
#   A_s^-1 = sum over eligible gas j of V_j W(|x_sj|, h_s) (gather: h_s);
#   gas j receives A_s V_j W(|x_sj|, h_s) of each deposited amount of every
#     source s (mass, metal mass, energy), and the mass carries the source's
#     velocity: v_j <- (m_j v_j + sum_s dm_js v_s) / (m_j + sum_s dm_js);
#     u_j <- (m_j u_j + dE_j) / (m_j + dm_j) (the deposited energy is added to
#     the internal energy of the grown particle).
# Gas with metallicity above z_max or mass above m_max is not eligible (it
# neither receives nor enters A). All minimum-image separations, box L.

def _kernel_w(kernel, r, h):
    q = np.asarray(r / h, dtype=np.float64)
    w, _, norm = kernel_eval(kernel, q)
    return norm * w.reshape(q.shape) / h ** 3


def deposit(gas: dict, src: dict, n_h_s: float, kernel: int = 1, box: float = 1.0,
            z_max: float = np.inf, m_max: float = np.inf) -> dict:
    """gas: x [3][n], h, V, m, v [3][n], mZ, u; src: x [3][s], dM, dMZ, dE, v [3][s].
    Returns the updated gas fields and the sources' V, h and A (A = 0 when a
    source has no eligible gas in reach: it deposits nothing)."""
    xg, hg, Vg = _c(gas["x"]), _c(gas["h"]), _c(gas["V"])
    m, v, mZ, u = _c(gas["m"]), _c(gas["v"]), _c(gas["mZ"]), _c(gas["u"])
    xs = _c(src["x"])
    ns = xs.shape[1]
    elig = (mZ <= z_max * m) & (m <= m_max)
    _, _, norm = kernel_eval(kernel, np.zeros(1))
    w0 = kernel_eval(kernel, np.zeros(1))[0][0]
    self_frac = norm * w0 / n_h_s ** 3
    if not self_frac < 1.0:
        raise ValueError("n_h,s^3 must exceed C w(0): the self term alone would exceed 1/V_s")
    Vs, hs, As = np.zeros(ns), np.zeros(ns), np.zeros(ns)
    dm = np.zeros_like(m)
    dmz = np.zeros_like(m)
    de = np.zeros_like(m)
    dp = np.zeros_like(v)
    for s in range(ns):
        d = xg - xs[:, s:s + 1]
        d -= box * np.round(d / box)
        r = np.sqrt((d * d).sum(0))
        inside = r < hg
        sg = _kernel_w(kernel, r[inside], hg[inside]).sum()
        if not sg > 0.0:
            continue
        Vs[s] = (1.0 - self_frac) / sg
        hs[s] = n_h_s * np.cbrt(Vs[s])
        near = (r < hs[s]) & elig
        wt = Vg[near] * _kernel_w(kernel, r[near], hs[s])
        tot = wt.sum()
        if not tot > 0.0:
            continue
        As[s] = 1.0 / tot
        f = As[s] * wt
        dm[near] += f * src["dM"][s]
        dmz[near] += f * src["dMZ"][s]
        de[near] += f * src["dE"][s]
        dp[:, near] += np.outer(src["v"][:, s], f * src["dM"][s])
    out = {"m": m + dm, "mZ": mZ + dmz, "V_s": Vs, "h_s": hs, "A_s": As}
    out["v"] = (m * v + dp) / out["m"]
    out["u"] = (m * u + de) / out["m"]
    return out
