"""GPU parity of the tree neighbour search (clustered particle sets).

The tree path (Morton-ordered 16-particle leaves over a 1024^3 lattice) must
give the same results as the cell-list path and the oracle: the same bounds
as test_gpu_forward.py, forced on uniform inputs and chosen automatically on
Plummer-clump inputs whose smoothing lengths span more than an order of
magnitude; with the cubic spline and with the Wendland C4 kernel.
"""
import numpy as np
import pytest

import synth
from paper_2511_21921_amd import FP32, FP64, WENDLAND_C4

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

from tests import _gpu  # noqa: E402
from tests.test_gpu_forward import FP32_BOUNDS, FP64_BOUNDS, _compare  # noqa: E402

TREE = 2


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_tree_forced_on_lattice_fixed_h(precision):
    ps = synth.lattice16()
    g, o, _ = _compare(ps, precision, FP64_BOUNDS if precision == FP64 else FP32_BOUNDS,
                       search=TREE)
    assert g["stats"]["n_pairs_force"] == o["pairs_force"]
    assert g["stats"]["grid"] == 1024


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_tree_forced_adaptive_random_masses(precision):
    ps = synth.random_small(3001, 61, mass_spread=0.1)
    _compare(ps, precision, FP64_BOUNDS if precision == FP64 else FP32_BOUNDS, search=TREE)


def _clumps(n, nc, seed):
    ps = synth.plummer_clumps(n, nc, seed)
    rng = np.random.default_rng(seed)
    ps.w_a, ps.w_u = rng.normal(size=(3, ps.n)), rng.normal(size=ps.n)
    return ps


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_clustered_switches_to_tree_and_matches_oracle(precision):
    ps = _clumps(20000, 8, 62)
    g, o, e = _compare(ps, precision, FP64_BOUNDS if precision == FP64 else FP32_BOUNDS, nbr=1)
    hr = o["h"].max() / o["h"].min()
    print("h range %.1f, grid %d" % (hr, g["stats"]["grid"]))
    assert hr > 30
    assert g["stats"]["grid"] == 1024          # automatic choice of the tree path
    assert g["stats"]["h_unconverged"] == 0
    if precision == FP64:
        assert g["stats"]["n_pairs_force"] == o["pairs_force"]


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_tree_with_the_wendland_c4_kernel(precision):
    # the tree search's instances for the C4 kernel: forced on a random set
    # at ~84 neighbours, and chosen automatically on Plummer clumps
    from tests.test_gpu_c4 import C4_FP32_BOUNDS
    bounds = FP64_BOUNDS if precision == FP64 else C4_FP32_BOUNDS
    ps = synth.random_small(3001, 64, n_ngb=100.0, mass_spread=0.1)
    g, _, _ = _compare(ps, precision, bounds, search=TREE, kernel=WENDLAND_C4)
    assert g["stats"]["grid"] == 1024
    ps = _clumps(20000, 8, 62)
    g, o, _ = _compare(ps, precision, bounds, nbr=1, kernel=WENDLAND_C4)
    assert g["stats"]["grid"] == 1024
    assert g["stats"]["h_unconverged"] == 0
    if precision == FP64:
        assert g["stats"]["n_pairs_force"] == o["pairs_force"]


def test_clustered_adjoint_fp64_matches_oracle_jvp():
    from tests.test_gpu_backward import _check_jvps, _grad
    ps = _clumps(6000, 4, 63)
    print("case clumps n=%d" % ps.n, flush=True)
    g, _ = _grad(ps, FP64, search=TREE)
    _check_jvps(ps, g, 1e-9)


def test_tree_and_cell_list_agree_fp64():
    ps = synth.sedov(16, k=4, with_velocity=True)
    a, _ = _gpu.run(ps, FP64, search=1)
    b, _ = _gpu.run(ps, FP64, search=TREE)
    for k in ("h", "V", "rho", "accel", "dudt"):
        assert np.abs(a[k] - b[k]).max() <= 1e-11 * np.abs(a[k]).max(), k
    assert a["stats"]["n_pairs_force"] == b["stats"]["n_pairs_force"]


def test_tree_and_cell_list_agree_many_neighbours():
    """~1000 neighbours on 100,000 uniform particles, FP64. The common sphere of a wave's
    four rows reaches many level-2 nodes (a frontier that outgrows its buffer sends the rows
    on alone), and every row takes hundreds of candidates: tree and cell list must give the
    same pairs and outputs."""
    ps = synth.random_small(100000, 93, n_ngb=1000)
    a, _ = _gpu.run(ps, FP64, search=1)
    b, _ = _gpu.run(ps, FP64, search=TREE)
    for k in ("h", "V", "rho", "accel", "dudt"):
        assert np.abs(a[k] - b[k]).max() <= 1e-11 * np.abs(a[k]).max(), k
    assert a["stats"]["n_pairs_force"] == b["stats"]["n_pairs_force"]
    assert b["stats"]["grid"] == 1024


@pytest.mark.parametrize("n", [37, 64, 129])
def test_tree_tiny_and_ragged(n):
    """One partial leaf, exactly one leaf, and a ragged third leaf.

    With 14 neighbours and so few particles a quarter of the moment matrices
    are singular and several more are nearly so; rounding in the inverse is
    amplified by their condition numbers (grad B differs by up to 3.6e-11 of
    its largest value), so the bounds are a hundred times the
    well-conditioned FP64 ones.
    """
    ps = synth.random_small(n, 80 + n, n_ngb=14, mass_spread=0.1)
    _compare(ps, FP64, {k: 100 * b for k, b in FP64_BOUNDS.items()}, search=TREE)


def test_tree_fixed_h_unequal_masses():
    ps = synth.random_small(2000, 90, mass_spread=0.1)
    ps.h_mode = 0
    g, o, _ = _compare(ps, FP64, FP64_BOUNDS, search=TREE)
    assert g["stats"]["n_pairs_force"] == o["pairs_force"]


def test_tree_particle_without_candidates():
    """Fixed h, one particle farther than h from every other: its row keeps no
    candidate at all, and the h solve and the list filter read no entry of the
    pool for it (the word at its position belongs to another row or was never
    written). Regression test: reading it as a particle index went out of bounds."""
    ps = synth.random_small(2000, 92, mass_spread=0.1)
    ps.h_mode = 0
    ps.x[0] *= 0.5
    ps.x[:, 0] = (0.75, 0.5, 0.5)
    g, o, _ = _compare(ps, FP64, FP64_BOUNDS, search=TREE)
    assert g["stats"]["n_pairs_force"] == o["pairs_force"]
    assert g["stats"]["m2_singular"] == 1


def test_tree_empty_input():
    ps = synth.random_small(300, 91)
    g, ctx = _gpu.run(ps, FP32, search=TREE)
    x, v, m, u, h = _gpu.to_dev(ps, FP32)
    out = ctx.forward(x[:, :0].contiguous(), v[:, :0].contiguous(), m[:0], u[:0], h[:0],
                      stats=True)
    assert out["stats"]["n_pairs_force"] == 0


def test_tree_candidate_pool_that_must_grow():
    """A context whose candidate pool was sized by a forward on a uniform set
    with 16 neighbours per particle: the next forward, on clumps with more,
    fills the pool in its first round, the blocks that find it full leave
    their particles to the retry rounds (which grow it), and the results
    equal a fresh context's."""
    first = synth.random_small(20000, 64, n_ngb=16)
    ps = _clumps(20000, 8, 63)
    print("case uniform 20000 (16 neighbours) then clumps 20000 seed 63", flush=True)
    _, ctx = _gpu.run(first, FP64, search=TREE)  # sizes the pool
    ctx.set_params(_gpu.params_for(ps, FP64, search=TREE))
    b, _ = _gpu.run(ps, FP64, ctx=ctx)
    c, _ = _gpu.run(ps, FP64, search=TREE)
    for k in ("h", "V", "rho", "accel", "dudt"):
        assert np.abs(b[k] - c[k]).max() <= 1e-11 * np.abs(c[k]).max(), k
    assert b["stats"]["n_pairs_force"] == c["stats"]["n_pairs_force"]
    print("searched", b["stats"]["n_searched"], c["stats"]["n_searched"], flush=True)
    assert b["stats"]["n_searched"] > c["stats"]["n_searched"]  # the full pool's retries


@pytest.mark.parametrize("precision", [FP32, FP64])
def test_tree_bitwise_deterministic(precision):
    """Two fresh contexts on the same clumps give bitwise equal outputs: the
    candidate pool's block placement and the scatter-only lists' fill order
    follow the order of atomics, but every list is sorted (in registers, or
    in LDS when long) before the pair passes sum over it."""
    ps = _clumps(20000, 8, 65)
    print("case clumps 20000 seed 65 precision=%d" % precision, flush=True)
    a, _ = _gpu.run(ps, precision)
    b, _ = _gpu.run(ps, precision)
    assert a["stats"]["grid"] == 1024
    for k in ("h", "V", "rho", "A", "B", "gradA", "gradB", "gradv", "accel", "dudt"):
        assert np.array_equal(a[k], b[k]), k
    assert a["stats"]["n_pairs_force"] > a["stats"]["n_pairs_gather"]  # scatter-only entries
