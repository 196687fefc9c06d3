"""Error paths of the library on the GPU, each forced from the host.

Every condition here is made by the inputs or the parameters a caller
passes; every kernel still runs to its normal end:
  - CRK_ENONFINITE: check_finite = 1 and one NaN velocity (no index, count or
    loop bound depends on a velocity), on the careful and the speculative
    forward;
  - CRK_ENOTCONV: an h solve capped at one iteration (h_max_iter = 1), with
    and without stats, on the cell list and on the tree; the outputs are
    still written and finite;
  - CRK_EINVAL for non-finite positions, on the careful forward and on the
    speculative one (whose cell keys are computed from the positions before
    the input check is read: the key kernels map such a coordinate to cell 0);
    a good forward afterwards equals a fresh context's bit for bit;
  - the state kept for crk_backward is dropped by a parameter change and by a
    reserve that grows the workspace (CRK_EINVAL), and kept by a change of
    timing alone.
"""
import dataclasses

import numpy as np
import pytest

import synth
from paper_2511_21921_amd import FP32, FP64, Context, CrkError

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

from tests import _gpu  # noqa: E402

EINVAL, ENOTCONV, ENONFINITE = -1, -5, -6


def _outputs(n, R):
    e = lambda *s, dt=R: torch.empty(*s, dtype=dt, device=_gpu.DEV)
    return {"h": e(n), "V": e(n), "rho": e(n), "A": e(n), "B": e(3, n), "gradA": e(3, n),
            "gradB": e(9, n), "gradv": e(9, n), "accel": e(3, n, dt=torch.float64),
            "dudt": e(n, dt=torch.float64)}


def _weights(ps):
    rng = np.random.default_rng(4)
    wa = torch.tensor(rng.normal(size=(3, ps.n)), dtype=torch.float64, device=_gpu.DEV)
    wu = torch.tensor(rng.normal(size=ps.n), dtype=torch.float64, device=_gpu.DEV)
    return wa, wu


@pytest.mark.parametrize("precision", [FP32, FP64])
def test_nonfinite_velocity_gives_enonfinite(precision):
    ps = synth.sedov(12, k=2, with_velocity=True)
    print("case nan velocity n=%d precision=%d" % (ps.n, precision), flush=True)
    ctx = Context(_gpu.params_for(ps, precision, check_finite=1))
    x, v, m, u, h = _gpu.to_dev(ps, precision)
    out = ctx.forward(x, v, m, u, h, stats=True)  # clean: accepted
    assert out["stats"]["nonfinite"] == 0
    vb = v.clone()
    vb[1, 100] = float("nan")
    for attempt in ("speculative", "careful"):
        if attempt == "careful":
            ctx.set_params(_gpu.params_for(ps, precision, check_finite=1, search=1))
        with pytest.raises(CrkError) as ei:
            ctx.forward(x, vb, m, u, h)
        print(attempt, ei.value, flush=True)
        assert ei.value.status == ENONFINITE
    # without the check the call succeeds (the NaN reaches du/dt of the neighbours)
    ctx.set_params(_gpu.params_for(ps, precision, check_finite=0))
    o = ctx.forward(x, vb, m, u, h, stats=True)
    assert o["stats"]["nonfinite"] == 0
    assert not np.all(np.isfinite(o["dudt"].cpu().numpy()))


@pytest.mark.parametrize("search", [1, 2])
def test_capped_h_solve_gives_enotconv(search):
    ps = synth.random_small(2000, 21)
    ps.h = ps.h * 1.7  # a guess far from the root
    print("case h_max_iter=1 search=%d n=%d" % (search, ps.n), flush=True)
    for stats in (False, True):
        ctx = Context(_gpu.params_for(ps, FP32, h_max_iter=1, search=search))
        x, v, m, u, h = _gpu.to_dev(ps, FP32)
        out = _outputs(ps.n, torch.float32)
        out["h"].copy_(h)
        with pytest.raises(CrkError) as ei:
            ctx.forward(x, v, m, u, h, out=out, stats=stats)
        print(" stats=%s" % stats, ei.value, flush=True)
        assert ei.value.status == ENOTCONV
        torch.cuda.synchronize()
        for k in ("h", "V", "rho", "accel", "dudt"):
            assert np.all(np.isfinite(out[k].cpu().numpy())), k
        assert np.all(out["h"].cpu().numpy() > 0)
    # the same inputs with the default cap converge
    g, _ = _gpu.run(ps, FP32, search=search)
    assert g["stats"]["h_unconverged"] == 0


def test_nonfinite_positions_rejected():
    ps = synth.sedov(16, k=2, with_velocity=True)
    print("case non-finite positions n=%d" % ps.n, flush=True)
    p = _gpu.params_for(ps, FP32)
    ctx = Context(p)
    x, v, m, u, h = _gpu.to_dev(ps, FP32)
    first = ctx.forward(x, v, m, u, h, stats=True)  # settles: the next one speculates
    ref = {k: t.cpu().numpy() for k, t in first.items() if isinstance(t, torch.Tensor)}
    for bad in (float("nan"), float("inf"), -float("inf")):
        xb = x.clone()
        xb[2, 77] = bad
        with pytest.raises(CrkError) as ei:  # speculative attempt, then the careful check
            ctx.forward(xb, v, m, u, h)
        print(" x = %r:" % bad, ei.value, flush=True)
        assert ei.value.status == EINVAL
    fresh = Context(p)
    xb = x.clone()
    xb[0, 5] = float("nan")
    with pytest.raises(CrkError) as ei:  # careful path: the check is read before any key
        fresh.forward(xb, v, m, u, h)
    assert ei.value.status == EINVAL
    again = ctx.forward(x, v, m, u, h, stats=True)
    for k, want in ref.items():
        assert np.array_equal(again[k].cpu().numpy(), want), k


def test_backward_state_follows_the_parameters():
    ps = synth.sedov(12, k=2, with_velocity=True)
    print("case backward state n=%d" % ps.n, flush=True)
    p = _gpu.params_for(ps, FP64)
    ctx = Context(p)
    x, v, m, u, h = _gpu.to_dev(ps, FP64)
    wa, wu = _weights(ps)
    ctx.forward(x, v, m, u, h)
    g0 = ctx.backward(wa, wu)
    # timing alone keeps the state
    ctx.set_params(dataclasses.replace(p, timing=1))
    g1 = ctx.backward(wa, wu)
    assert torch.equal(g0["g_x"], g1["g_x"])
    for change in ({"store_corrections": 1}, {"alpha": 1.5}, {"kernel": 1}, {"box": 1.0 + 1e-9}):
        ctx.set_params(dataclasses.replace(p, **change))
        with pytest.raises(CrkError) as ei:
            ctx.backward(wa, wu)
        print(" after %s:" % change, ei.value, flush=True)
        assert ei.value.status == EINVAL
        ctx.set_params(p)
        ctx.forward(x, v, m, u, h)
        ctx.backward(wa, wu)
    # a reserve that grows the workspace drops the state; one that does not keeps it
    ctx.reserve(ps.n)
    ctx.backward(wa, wu)
    ctx.reserve(4 * ps.n)
    with pytest.raises(CrkError) as ei:
        ctx.backward(wa, wu)
    assert ei.value.status == EINVAL
    ctx.forward(x, v, m, u, h)
    g2 = ctx.backward(wa, wu)
    torch.cuda.synchronize()
    assert torch.equal(g0["g_x"], g2["g_x"]) and torch.equal(g0["g_u"], g2["g_u"])
