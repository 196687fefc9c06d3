"""crk_backward_noalloc, the adjoint with its workspace in the library's static
device array (no allocation), against crk_backward on the same forward state.

Two forwards in a row, the second with fewer particles, each followed by both
adjoints (in either order): the gradients must be identical (the same kernels
run on the same state; only the workspace address differs), in FP64 and FP32.
Sizes beyond the array's limit (65,536 particles) are refused with CRK_EINVAL.
"""
import ctypes as C

import numpy as np
import pytest

import synth
from paper_2511_21921_amd import FP32, FP64, Context, crk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

from tests import _gpu  # noqa: E402


def _lib():
    return crk.lib()


def _grads(ctx, n, wa, wu, noalloc):
    o = {"g_x": torch.full((3, n), np.nan, dtype=torch.float64, device=_gpu.DEV),
         "g_v": torch.full((3, n), np.nan, dtype=torch.float64, device=_gpu.DEV),
         "g_u": torch.full((n,), np.nan, dtype=torch.float64, device=_gpu.DEV),
         "g_alpha_beta": torch.full((2,), np.nan, dtype=torch.float64, device=_gpu.DEV)}
    stream = C.c_void_p(torch.cuda.current_stream(_gpu.DEV).cuda_stream)
    fn = _lib().crk_backward_noalloc if noalloc else crk.lib().crk_backward
    p = lambda t: C.c_void_p(t.data_ptr())
    rc = fn(ctx._h, stream, n, p(wa), p(wu), p(o["g_x"]), p(o["g_v"]), p(o["g_u"]),
            p(o["g_alpha_beta"]))
    assert rc == 0, (rc, ctx.last_error())
    torch.cuda.synchronize()
    return {k: t.cpu().numpy() for k, t in o.items()}


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_noalloc_backward_equals_backward(precision):
    ctx = None
    for step, (side, seed) in enumerate(((36, 1), (20, 2))):  # 46,656 then 8,000 particles
        ps = synth.sedov(side, k=seed, with_velocity=True)
        print("noalloc precision=%d call %d n=%d" % (precision, step, ps.n), flush=True)
        if ctx is None:
            ctx = Context(_gpu.params_for(ps, precision))
        x, v, m, u, h = _gpu.to_dev(ps, precision)
        ctx.forward(x, v, m, u, h)
        rng = np.random.default_rng(seed)
        wa = torch.tensor(rng.normal(size=(3, ps.n)), dtype=torch.float64, device=_gpu.DEV)
        wu = torch.tensor(rng.normal(size=ps.n), dtype=torch.float64, device=_gpu.DEV)
        order = (True, False) if step else (False, True)
        first = _grads(ctx, ps.n, wa, wu, order[0])
        second = _grads(ctx, ps.n, wa, wu, order[1])
        for k in first:
            assert np.all(np.isfinite(first[k])), k
            assert np.array_equal(first[k], second[k]), (k, step)


def test_noalloc_backward_refuses_beyond_its_limit():
    ps = synth.random_small(70000, 3)
    print("noalloc limit n=%d" % ps.n, flush=True)
    ctx = Context(_gpu.params_for(ps, FP32))
    x, v, m, u, h = _gpu.to_dev(ps, FP32)
    ctx.forward(x, v, m, u, h)
    z = lambda *s: torch.zeros(*s, dtype=torch.float64, device=_gpu.DEV)
    wa, wu, gx, gv, gu, gab = z(3, ps.n), z(ps.n), z(3, ps.n), z(3, ps.n), z(ps.n), z(2)
    stream = C.c_void_p(torch.cuda.current_stream(_gpu.DEV).cuda_stream)
    p = lambda t: C.c_void_p(t.data_ptr())
    rc = _lib().crk_backward_noalloc(ctx._h, stream, ps.n, p(wa), p(wu), p(gx), p(gv), p(gu),
                                     p(gab))
    assert rc == -1
    assert "65536" in ctx.last_error()
    # the ordinary adjoint takes it
    ctx.backward(wa, wu)
