"""Seeded synthetic particle sets shaped like cosmological gas.

This module is shared by the tests, the benchmark and the oracle checks. It
draws inputs only (positions, velocities, masses, internal energies, a first
smoothing-length guess and loss weights); it contains none of the hydro
method's arithmetic.

Workloads (all in a periodic unit box, equal particle masses m = 1/N so the
mean density is 1):

* ``lattice16``  16^3 cubic lattice, each site jittered by U(-0.1, 0.1) of the
  spacing per axis, u = 1, velocities N(0, 0.1) per axis, fixed smoothing
  length n_h * spacing with n_h chosen for 32 neighbours (the paper's
  neighbour number N = 4 pi/3 n_h^3, App. A.2).
* ``sedov64``    64^3 jittered lattice, u = 1e4 on the 27 sites nearest the
  box centre and 1e-2 elsewhere, zero velocity, adaptive smoothing length
  for 64 neighbours.
* ``sedov64_v``  the same particles with velocities N(0, 0.1) per axis and
  N(0, 1) loss weights on the accelerations and du/dt (the gradient
  workload).
* ``clumps128`` / ``clumps256``  50% uniform background plus Plummer clumps
  (512 / 4096), clump masses log-normal with sigma 1 dex, scale radii
  U(0.002, 0.02), velocities N(0, 0.05), log10 u ~ N(0, 0.5).

Seeds: ``numpy.random.SeedSequence(20251121 + k).spawn(4)`` gives the
generators for positions, velocities, internal energy and loss weights of
workload k.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 20251121


def n_h_for_neighbours(n_ngb: float) -> float:
    """Particles per kernel radius that give ``n_ngb`` neighbours, N = 4 pi/3 n_h^3."""
    return (3.0 * n_ngb / (4.0 * math.pi)) ** (1.0 / 3.0)


@dataclass
class ParticleSet:
    """One synthetic workload. Arrays are float64, SoA, [3][n] for vectors."""

    name: str
    x: np.ndarray          # [3][n] positions in [0, box)
    v: np.ndarray          # [3][n]
    m: np.ndarray          # [n]
    u: np.ndarray          # [n]
    h: np.ndarray          # [n] fixed smoothing length, or the first guess
    n_h: float             # particles per kernel radius
    h_mode: int            # 0 fixed, 1 solve
    box: float = 1.0
    w_a: np.ndarray | None = None   # [3][n] loss weights on accelerations
    w_u: np.ndarray | None = None   # [n] loss weights on du/dt
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.m.shape[0])


def _rngs(k: int):
    ss = np.random.SeedSequence(BASE_SEED + k).spawn(4)
    return [np.random.default_rng(s) for s in ss]


def jittered_lattice(n_side: int, rng: np.random.Generator, jitter: float = 0.1,
                     box: float = 1.0) -> np.ndarray:
    """Sites at i*dx (i = 0..n-1) per axis, per-axis jitter U(-jitter, jitter)*dx, wrapped."""
    dx = box / n_side
    g = np.arange(n_side, dtype=np.float64) * dx
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    if jitter:
        x = x + rng.uniform(-jitter, jitter, size=x.shape) * dx
    return np.mod(x, box)


def _nearest_sites(x: np.ndarray, centre, k: int, box: float) -> np.ndarray:
    d = x - np.asarray(centre, dtype=np.float64)[:, None]
    d -= box * np.round(d / box)
    r2 = (d * d).sum(0)
    # lower index wins ties (stable sort)
    return np.argsort(r2, kind="stable")[:k]


def lattice16(k: int = 1) -> ParticleSet:
    rx, rv, ru, rw = _rngs(k)
    n_side = 16
    x = jittered_lattice(n_side, rx)
    n = x.shape[1]
    v = rv.normal(0.0, 0.1, size=(3, n))
    n_h = n_h_for_neighbours(32)
    h = np.full(n, n_h / n_side)
    return ParticleSet("lattice16", x, v, np.full(n, 1.0 / n), np.ones(n), h, n_h, 0)


def _sedov(n_side: int, k: int, with_velocity: bool) -> ParticleSet:
    rx, rv, ru, rw = _rngs(k)
    x = jittered_lattice(n_side, rx)
    n = x.shape[1]
    u = np.full(n, 1e-2)
    u[_nearest_sites(x, (0.5, 0.5, 0.5), 27, 1.0)] = 1e4
    n_h = n_h_for_neighbours(64)
    h = np.full(n, n_h / n_side)
    v = rv.normal(0.0, 0.1, size=(3, n)) if with_velocity else np.zeros((3, n))
    ps = ParticleSet("sedov%d%s" % (n_side, "_v" if with_velocity else ""), x, v,
                     np.full(n, 1.0 / n), u, h, n_h, 1)
    if with_velocity:
        ps.w_a = rw.normal(0.0, 1.0, size=(3, n))
        ps.w_u = rw.normal(0.0, 1.0, size=n)
    return ps


def sedov64(k: int = 2) -> ParticleSet:
    return _sedov(64, k, False)


def sedov64_v(k: int = 4) -> ParticleSet:
    return _sedov(64, k, True)


def at_resolution(ps: ParticleSet, n_h: float) -> ParticleSet:
    """The same particles with n_h particles per kernel radius (first h guess scaled to match).

    n_h = 4 is the paper's production resolution for gas (about 268 neighbours)."""
    q = dataclasses.replace(ps, h=ps.h * (n_h / ps.n_h), n_h=n_h, meta=dict(ps.meta))
    q.name = "%s_nh%g" % (ps.name, n_h)
    return q


def sedov(n_side: int, k: int = 2, with_velocity: bool = False) -> ParticleSet:
    """Sedov-like jittered lattice at any size (test variants)."""
    return _sedov(n_side, k, with_velocity)


# Plummer enclosed-mass fraction at 10 scale radii: (r^2/(r^2+a^2))^(3/2).
_PLUMMER_TRUNC = (100.0 / 101.0) ** 1.5


def plummer_clumps(n: int, n_clumps: int, k: int, box: float = 1.0) -> ParticleSet:
    """Half the particles uniform, half in Plummer spheres truncated at 10 a."""
    rx, rv, ru, rw = _rngs(k)
    n_bg = n // 2
    n_cl = n - n_bg
    centres = rx.uniform(0.0, box, size=(n_clumps, 3))
    logm = rx.normal(0.0, 1.0, size=n_clumps)
    mass = 10.0 ** logm
    share = n_cl * mass / mass.sum()
    counts = np.floor(share).astype(np.int64)
    rem = n_cl - counts.sum()
    order = np.argsort(-(share - counts), kind="stable")
    counts[order[:rem]] += 1
    a = rx.uniform(0.002, 0.02, size=n_clumps)
    xs = [rx.uniform(0.0, box, size=(3, n_bg))]
    for c in range(n_clumps):
        nc = int(counts[c])
        if nc == 0:
            continue
        uu = rx.uniform(0.0, _PLUMMER_TRUNC, size=nc)
        uu = np.maximum(uu, 1e-300)
        r = a[c] / np.sqrt(uu ** (-2.0 / 3.0) - 1.0)
        d = rx.normal(size=(3, nc))
        d /= np.linalg.norm(d, axis=0, keepdims=True)
        xs.append(centres[c][:, None] + r[None, :] * d)
    x = np.mod(np.concatenate(xs, axis=1), box)
    v = rv.normal(0.0, 0.05, size=(3, n))
    u = 10.0 ** ru.normal(0.0, 0.5, size=n)
    n_h = n_h_for_neighbours(64)
    h = np.full(n, n_h * (box ** 3 / n) ** (1.0 / 3.0))
    ps = ParticleSet("clumps%d" % round(n ** (1 / 3)), x, v, np.full(n, 1.0 / n), u, h, n_h, 1)
    ps.meta.update(n_clumps=n_clumps, clump_counts=counts, clump_a=a, clump_centres=centres)
    # loss weights N(0, 1) from the fourth generator (the other draws are unaffected)
    ps.w_a = rw.normal(size=(3, n))
    ps.w_u = rw.normal(size=n)
    return ps


def clumps128(k: int = 3) -> ParticleSet:
    return plummer_clumps(128 ** 3, 512, k)


def clumps256(k: int = 5) -> ParticleSet:
    return plummer_clumps(256 ** 3, 4096, k)


def perfect_lattice(n_side: int, n_ngb: float = 32.0, box: float = 1.0) -> ParticleSet:
    """Unperturbed lattice, u = 1, v = 0, equal masses, fixed h (invariant tests)."""
    x = jittered_lattice(n_side, None, jitter=0.0, box=box)
    n = x.shape[1]
    n_h = n_h_for_neighbours(n_ngb)
    h = np.full(n, n_h * box / n_side)
    return ParticleSet("lattice%d_perfect" % n_side, x, np.zeros((3, n)), np.full(n, 1.0 / n),
                       np.ones(n), h, n_h, 0, box=box)


def random_small(n: int, seed: int, n_ngb: float = 32.0, box: float = 1.0,
                 mass_spread: float = 0.0, h_mode: int = 1) -> ParticleSet:
    """Uniform random positions; optional log-uniform mass spread (general eq. Vg path)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, box, size=(3, n))
    v = rng.normal(0.0, 0.1, size=(3, n))
    u = 10.0 ** rng.normal(0.0, 0.3, size=n)
    m = np.full(n, 1.0 / n)
    if mass_spread:
        m = m * 10.0 ** rng.uniform(-mass_spread, mass_spread, size=n)
    n_h = n_h_for_neighbours(n_ngb)
    h = np.full(n, n_h * (box ** 3 / n) ** (1.0 / 3.0))
    ps = ParticleSet("random%d" % n, x, v, m, u, h, n_h, h_mode, box=box)
    ps.w_a = rng.normal(size=(3, n))
    ps.w_u = rng.normal(size=n)
    return ps


WORKLOADS = {
    "lattice16": lattice16,
    "sedov64": sedov64,
    "sedov64_v": sedov64_v,
    "clumps128": clumps128,
    "clumps256": clumps256,
}


def make(name: str) -> ParticleSet:
    return WORKLOADS[name]()
