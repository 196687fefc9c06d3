"""Full-size clustered workloads on the GPU, checked where the oracle can reach.

The 2.1M-particle clump set (FP32 forward) and the 16.8M-particle clump set
(FP32 forward and adjoint with the corrections recomputed, one GPU's share of
a large volume) are far beyond what the oracle runs whole. They are checked
by (1) oracle values at sampled particles, computed on subsets that hold each
sample's whole dependency chain (oracle/sampled.py); (2) oracle JVPs of a
loss whose weights sit on sampled particles only, which is then exact on the
union of their subsets; (3) identities that hold at any size: momentum and
energy conservation, the affine dependence of a and du/dt on (alpha, beta),
and the invariance of L under a common shift of all positions or of all
velocities (so the position and velocity gradients sum to zero).

Sampled bounds (FP32 pairs, FP64 solve and accumulators): relative 1e-5 on h
and 2e-5 on V, rho, A; the per-field scaled bounds of the forward parity
tests for B, grad A, grad B, grad v; acceleration and du/dt errors scaled per
particle by s_i = sum_j |F_ij| / m_i (cancellation-aware), 5e-5.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2511_21921_amd import FP32, Context

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

from tests import _gpu  # noqa: E402
from oracle.sampled import localized_jvp, sampled_oracle  # noqa: E402

SAMPLE_BOUNDS = {"h": 1e-5, "V": 2e-5, "rho": 2e-5, "A": 2e-5, "B/max": 2e-5, "gradA/max": 2e-5,
                 "gradB/max": 2e-5, "gradv/max": 2e-5, "accel_scaled_max": 5e-5,
                 "dudt_scaled_max": 5e-5}


def _check_samples(name, g, o, samples):
    gs = {k: v[..., samples] for k, v in g.items() if isinstance(v, np.ndarray)}
    e = _gpu.errors(gs, o, o["h"])
    print(name, {k: "%.2e" % v for k, v in e.items()}, flush=True)
    for k, b in SAMPLE_BOUNDS.items():
        assert e[k] <= b, (k, e[k], b)


def _conservation(ps, g):
    ma = ps.m * g["accel"]
    mom = np.abs(ma.sum(1)).max() / np.abs(ma).sum()
    e = (ps.m * ((ps.v * g["accel"]).sum(0) + g["dudt"])).sum()
    escale = (ps.m * (np.abs(ps.v * g["accel"]).sum(0) + np.abs(g["dudt"]))).sum()
    return mom, abs(e) / escale


def _sampled_oracle(ps, k, seed, dense=2):
    """k samples (each with a complete subset of at most 40k particles) plus the `dense`
    densest core particles (any subset size), and their oracle values."""
    kept, subsets, o = sampled_oracle(ps, oracle.params_for(ps), k, seed, dense=dense)
    print("samples", kept.tolist(), "h", o["h"].tolist(), flush=True)
    return kept, subsets, o


def test_clumps128_fp32_forward_sampled_parity():
    ps = synth.clumps128()
    print("case clumps128 n=%d" % ps.n, flush=True)
    g, _ = _gpu.run(ps, FP32)
    st = g["stats"]
    print(st, flush=True)
    assert st["grid"] == 1024 and st["h_unconverged"] == 0 and st["nonfinite"] == 0
    hr = g["h"].max() / g["h"].min()
    print("h range %.1f" % hr, flush=True)
    assert hr > 30
    mom, en = _conservation(ps, g)
    print("momentum %.2e energy %.2e" % (mom, en), flush=True)
    assert mom < 1e-6 and en < 1e-6
    samples, _, o = _sampled_oracle(ps, 12, 71)
    _check_samples("clumps128", g, o, samples)


def test_clumps256_fp32_fwd_bwd_recompute_sampled():
    ps = synth.clumps256()
    print("case clumps256 n=%d" % ps.n, flush=True)
    # samples and their oracle values first: the loss weights sit on them
    samples, subsets, o = _sampled_oracle(ps, 8, 72)
    print("samples", samples.tolist(), "subsets", [s.size for s in subsets], flush=True)
    rng = np.random.default_rng(73)
    # loss weights on the sampled particles only: L depends on a few thousand particles
    w_a = np.zeros((3, ps.n))
    w_u = np.zeros(ps.n)
    w_a[:, samples] = rng.normal(size=(3, samples.size))
    w_u[samples] = rng.normal(size=samples.size)
    p = _gpu.params_for(ps, FP32, store_corrections=0)
    ctx = Context(p)
    x, v, m, u, h = _gpu.to_dev(ps, FP32)
    out = ctx.forward(x, v, m, u, h, stats=True)
    wa_d = torch.tensor(w_a, dtype=torch.float64, device=_gpu.DEV)
    wu_d = torch.tensor(w_u, dtype=torch.float64, device=_gpu.DEV)
    grad = ctx.backward(wa_d, wu_d)
    torch.cuda.synchronize()
    g = {k: t.cpu().numpy().astype(np.float64) for k, t in out.items()
         if isinstance(t, torch.Tensor)}
    gr = {k: t.cpu().numpy() for k, t in grad.items()}
    st = out["stats"]
    print(st, flush=True)
    assert st["grid"] == 1024 and st["h_unconverged"] == 0 and st["nonfinite"] == 0
    mom, en = _conservation(ps, g)
    print("momentum %.2e energy %.2e" % (mom, en), flush=True)
    assert mom < 1e-6 and en < 1e-6

    def loss(o_):
        return float((w_a * o_["accel"]).sum() + (w_u * o_["dudt"]).sum())

    L0 = loss(g)
    # a and du/dt are affine in (alpha, beta): the gradient is the exact difference
    for t, kw in enumerate(({"alpha": p.alpha + 1.0}, {"beta": p.beta + 1.0})):
        ctx.set_params(_gpu.params_for(ps, FP32, store_corrections=0, **kw))
        o1, _ = _gpu.run(ps, FP32, ctx=ctx, stats=False)
        diff = loss(o1) - L0
        ga = gr["g_alpha_beta"][t]
        print("alpha/beta[%d] gradient % .8e difference % .8e" % (t, ga, diff), flush=True)
        assert abs(ga - diff) <= 1e-4 * max(abs(diff), 1e-300)
    # common shifts of all positions or all velocities leave L unchanged
    for k in ("g_x", "g_v"):
        rel = np.abs(gr[k].sum(1)).max() / np.abs(gr[k]).sum(1).max()
        print("%s sum / sum|.| %.2e" % (k, rel), flush=True)
        assert rel < 1e-5
    # oracle: forward values at the samples and the JVP of the localised loss
    _check_samples("clumps256", g, o, samples)
    drng = np.random.default_rng(74)

    def dirs(U):
        dx = drng.normal(size=(3, U.size)) * 1e-3
        dv = drng.normal(size=(3, U.size))
        du = drng.normal(size=U.size) * ps.u[U]
        return dx, dv, du, 0.0, 0.0

    jl, U, (dx, dv, du, _, _) = localized_jvp(ps, samples, subsets, oracle.params_for(ps),
                                             w_a[:, samples], w_u[samples], dirs)
    gl = float((gr["g_x"][:, U] * dx).sum() + (gr["g_v"][:, U] * dv).sum() +
               (gr["g_u"][U] * du).sum())
    print("localised JVP over %d particles: oracle % .8e adjoint % .8e rel %.2e"
          % (U.size, jl, gl, abs(gl - jl) / abs(jl)), flush=True)
    assert abs(gl - jl) <= 2e-4 * abs(jl)
    # the gradient vanishes outside the union (L does not depend on those particles)
    outside = np.ones(ps.n, dtype=bool)
    outside[U] = False
    assert np.abs(gr["g_x"][:, outside]).max() == 0.0
