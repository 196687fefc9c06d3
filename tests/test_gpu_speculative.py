"""Forwards that reuse the previous forward's cell-list geometry.

After a forward that settled on the cell list at its first grid, the next
forward with the same n and precision launches every pass with that
geometry and checks once at the end whether the careful order would have
chosen the same (crk_forward in include/crk.h). Accepted or rejected, its
outputs and the adjoint after it must equal those of a fresh context bit
for bit: the check only accepts when every choice (grid, mass form,
capacities that fit, no capped h root, no clustering switch) is the same.
"""
import dataclasses

import numpy as np
import pytest

import synth
from paper_2511_21921_amd import FP32, FP64, Context

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

from tests import _gpu  # noqa: E402

KEYS = ("h", "V", "rho", "A", "B", "gradA", "gradB", "gradv", "accel", "dudt")


def _same(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k
    for k in ("n_pairs_gather", "n_pairs_force", "grid"):
        assert a["stats"][k] == b["stats"][k], k


def _grads(ctx, ps, seed):
    rng = np.random.default_rng(seed)
    wa = torch.tensor(rng.normal(size=(3, ps.n)), dtype=torch.float64, device=_gpu.DEV)
    wu = torch.tensor(rng.normal(size=ps.n), dtype=torch.float64, device=_gpu.DEV)
    g = ctx.backward(wa, wu)
    torch.cuda.synchronize()
    return {k: t.cpu().numpy() for k, t in g.items()}


@pytest.mark.parametrize("precision", [FP32, FP64])
def test_repeat_is_speculative_and_bitwise(precision):
    ps = synth.random_small(4000, 101)
    print("case random4000 precision=%d" % precision, flush=True)
    g1, ctx = _gpu.run(ps, precision)
    b1 = _grads(ctx, ps, 5)
    assert g1["stats"]["speculative"] == 0
    g2, _ = _gpu.run(ps, precision, ctx=ctx)
    assert g2["stats"]["speculative"] == 1
    _same(g1, g2)
    b2 = _grads(ctx, ps, 5)
    for k in b1:
        assert np.array_equal(b1[k], b2[k]), k


def _rejected_then_fresh(ps1, ps2, precision=FP32, expect_reject=True):
    # the second forward reuses the context, and with it ps1's parameters
    assert (ps1.box, ps1.n_h, ps1.h_mode) == (ps2.box, ps2.n_h, ps2.h_mode)
    _, ctx = _gpu.run(ps1, precision)
    g, _ = _gpu.run(ps2, precision, ctx=ctx)
    if expect_reject:
        assert g["stats"]["speculative"] == 0
    fresh, _ = _gpu.run(ps2, precision)
    assert fresh["stats"]["speculative"] == 0
    _same(g, fresh)
    return g


def test_fixed_h_grown_beyond_the_candidate_radius():
    ps1 = synth.random_small(3000, 102)
    ps1 = dataclasses.replace(ps1, h_mode=0, h=ps1.h * 0.8)
    ps2 = dataclasses.replace(ps1, h=ps1.h * 1.5)
    print("case fixed h x1.5", flush=True)
    _rejected_then_fresh(ps1, ps2)


def test_masses_no_longer_equal():
    ps1 = synth.random_small(3000, 103)
    ps2 = synth.random_small(3000, 103, mass_spread=0.1)
    print("case equal -> unequal masses", flush=True)
    _rejected_then_fresh(ps1, ps2)


def test_clustered_input_of_the_same_size():
    ps1 = synth.random_small(6000, 104)
    # the context keeps ps1's parameters: same resolution n_h for both sets
    ps2 = dataclasses.replace(synth.plummer_clumps(6000, 4, 104), n_h=ps1.n_h)
    print("case uniform -> clumps, n=6000", flush=True)
    _rejected_then_fresh(ps1, ps2)


def test_new_h_guess_either_way_equal():
    ps1 = synth.random_small(3000, 105)
    ps2 = dataclasses.replace(ps1, h=ps1.h * 1.3)
    print("case h guess x1.3", flush=True)
    _rejected_then_fresh(ps1, ps2, expect_reject=False)


def test_set_params_keeps_or_drops_the_geometry():
    """A parameter the cell-list geometry does not depend on (alpha) keeps the
    speculative forward, which then equals a fresh context's bit for bit; one it
    depends on (n_h) drops it."""
    ps = synth.random_small(3000, 106)
    _, ctx = _gpu.run(ps, FP32)
    ctx.set_params(_gpu.params_for(ps, FP32, alpha=1.5))
    g, _ = _gpu.run(ps, FP32, ctx=ctx, alpha=1.5)
    assert g["stats"]["speculative"] == 1
    f, _ = _gpu.run(ps, FP32, alpha=1.5)
    for k in ("h", "V", "rho", "A", "B", "gradv", "accel", "dudt"):
        assert np.array_equal(g[k], f[k]), k
    ctx.set_params(_gpu.params_for(ps, FP32, alpha=1.5, n_h=ps.n_h * 1.01))
    g, _ = _gpu.run(ps, FP32, ctx=ctx, alpha=1.5, n_h=ps.n_h * 1.01)
    assert g["stats"]["speculative"] == 0


@pytest.mark.parametrize("precision", [FP32, FP64])
def test_kept_cell_list_and_a_particle_that_changes_cell(precision):
    """A speculative forward keeps the last cell list when a check found it
    still sorted; once a particle has moved to another cell that forward is
    rejected, equals a fresh context's, and the next one builds the list again."""
    ps = synth.random_small(4000, 103)
    print("case random4000 seed 103 precision=%d" % precision, flush=True)
    g1, ctx = _gpu.run(ps, precision)          # careful: builds the list
    g2, _ = _gpu.run(ps, precision, ctx=ctx)   # checks the list and builds it again
    g3, _ = _gpu.run(ps, precision, ctx=ctx)   # keeps it
    assert g2["stats"]["speculative"] == 1 and g3["stats"]["speculative"] == 1
    _same(g1, g2)
    _same(g1, g3)
    grid = g1["stats"]["grid"]
    assert grid >= 2
    x2 = ps.x.copy()
    x2[0, 7] = (x2[0, 7] + ps.box / grid) % ps.box  # one cell side along x
    ps2 = dataclasses.replace(ps, x=x2)
    fresh, _ = _gpu.run(ps2, precision)
    g4, _ = _gpu.run(ps2, precision, ctx=ctx)
    assert g4["stats"]["speculative"] == 0
    _same(g4, fresh)
    g5, _ = _gpu.run(ps2, precision, ctx=ctx)
    assert g5["stats"]["speculative"] == 1
    _same(g5, fresh)
