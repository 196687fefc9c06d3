"""Exact-integration cooling on the GPU (crk_cool) against the oracle's bin walk.

The GPU prepares the table once (prefix integrals within runs of same-sign
bins) and finds each particle's final bin by binary search; the oracle walks
I(u) bin by bin from the anchor. Same function, different summation order:
FP64 within 1e-11 relative; FP32 (u and rho stored in float, FP64 arithmetic)
within 2e-7, the oracle fed the same float-rounded inputs.
Tables: the pinned shapes of tests/test_oracle_cooling.py (pure power laws,
a random broken power law, stable and unstable zeros) plus one with three
zeros, on 0.004 dex nodes (the paper's bin width); particles span beyond
both table ends.
"""
import numpy as np
import pytest

import oracle
from paper_2511_21921_amd import FP32, FP64, Context, CrkError, Params

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

DEX, LU0 = 0.004, -2.0
K = int(round(6 / DEX)) + 1
UK = 10 ** (LU0 + DEX * np.arange(K))
A = 0.7
DEV = torch.device("cuda:0")


def _tables():
    rng = np.random.default_rng(4)
    return {
        "pow1.5": (A * UK ** 1.5, 0.3),
        "beta1": (A * UK, 0.3),
        "heating": (-A * UK ** 1.5, 0.01),
        "broken": (np.exp(np.cumsum(rng.normal(0, 0.02, K))) * UK ** 1.2, 0.05),
        "stable": (A * (UK ** 1.5 - 3.0 ** 1.5), 0.05),
        "unstable": (-A * (UK ** 1.5 - 3.0 ** 1.5), 1e-3),
        "three_zeros": (A * (UK - 0.5) * (UK - 5.0) * (UK - 50.0), 0.02),
    }


def _particles(n, seed):
    rng = np.random.default_rng(seed)
    return 10 ** rng.uniform(-2.5, 4.5, n), 10 ** rng.uniform(-1, 1, n)


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("name", list(_tables()))
def test_cooling_matches_the_oracle(name, precision):
    lam, dt = _tables()[name]
    u0, rho = _particles(1500, 5)
    print("case %s precision=%d" % (name, precision), flush=True)
    R = torch.float64 if precision == FP64 else torch.float32
    u0 = u0.astype(np.float32).astype(np.float64) if precision == FP32 else u0
    rho = rho.astype(np.float32).astype(np.float64) if precision == FP32 else rho
    ctx = Context(Params(precision=precision))
    ctx.cooling_table(LU0, DEX, lam)
    u = torch.tensor(u0, dtype=R, device=DEV)
    ctx.cool(torch.tensor(rho, dtype=R, device=DEV), u, dt)
    torch.cuda.synchronize()
    got = u.cpu().numpy().astype(np.float64)
    want = oracle.cool(oracle.CoolingTable(LU0, DEX, lam), u0, rho, dt)
    err = np.max(np.abs(got / want - 1))
    print("  max rel err %.2e" % err, flush=True)
    assert err <= (1e-11 if precision == FP64 else 2e-7)


def test_cooling_edges_and_errors():
    lam, _ = _tables()["stable"]
    ctx = Context(Params(precision=FP64))
    u = torch.tensor([3.0, 1e-9, 1e9], dtype=torch.float64, device=DEV)
    rho = torch.ones(3, dtype=torch.float64, device=DEV)
    with pytest.raises(CrkError):
        ctx.cool(rho, u, 0.1)  # no table yet
    with pytest.raises(CrkError):
        ctx.cooling_table(LU0, 0.0, lam)
    with pytest.raises(CrkError):
        ctx.cooling_table(LU0, DEX, np.array([1.0]))
    with pytest.raises(CrkError):
        ctx.cooling_table(LU0, DEX, np.array([1.0, np.nan, 2.0]))
    ctx.cooling_table(LU0, DEX, lam)
    with pytest.raises(CrkError):
        ctx.cool(rho, u, -1.0)
    ctx.cool(rho[:0], u[:0], 0.1)  # n = 0
    ctx.cool(rho, u, 0.0)          # dt = 0 clamps to the table only
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    assert got[0] == 3.0 and np.allclose(got[1:], [UK[0], UK[-1]], rtol=1e-15, atol=0)


def test_cooling_million_particles_sampled():
    lam, dt = _tables()["three_zeros"]
    n = 1 << 20
    u0, rho = _particles(n, 6)
    ctx = Context(Params(precision=FP64))
    ctx.cooling_table(LU0, DEX, lam)
    u = torch.tensor(u0, dtype=torch.float64, device=DEV)
    ctx.cool(torch.tensor(rho, dtype=torch.float64, device=DEV), u, dt)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    idx = np.random.default_rng(7).choice(n, 400, replace=False)
    want = oracle.cool(oracle.CoolingTable(LU0, DEX, lam), u0[idx], rho[idx], dt)
    assert np.max(np.abs(got[idx] / want - 1)) <= 1e-11
    assert np.all(np.isfinite(got)) and got.min() >= UK[0] and got.max() <= UK[-1]


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_cooling_table_beyond_the_lds_size(precision):
    # 3001 nodes (0.002 dex over six decades): more than the LDS copy holds,
    # so the table is read from global memory; same arithmetic
    dex = 0.002
    k = int(round(6 / dex)) + 1
    uk = 10 ** (LU0 + dex * np.arange(k))
    rng = np.random.default_rng(8)
    lam = A * (uk ** 1.5 - 3.0 ** 1.5) * np.exp(np.cumsum(rng.normal(0, 0.01, k)))
    u0, rho = _particles(1500, 9)
    print("case %d nodes precision=%d" % (k, precision), flush=True)
    R = torch.float64 if precision == FP64 else torch.float32
    u0 = u0.astype(np.float32).astype(np.float64) if precision == FP32 else u0
    rho = rho.astype(np.float32).astype(np.float64) if precision == FP32 else rho
    ctx = Context(Params(precision=precision))
    ctx.cooling_table(LU0, dex, lam)
    u = torch.tensor(u0, dtype=R, device=DEV)
    ctx.cool(torch.tensor(rho, dtype=R, device=DEV), u, 0.05)
    torch.cuda.synchronize()
    got = u.cpu().numpy().astype(np.float64)
    want = oracle.cool(oracle.CoolingTable(LU0, dex, lam), u0, rho, 0.05)
    err = np.max(np.abs(got / want - 1))
    print("  max rel err %.2e" % err, flush=True)
    assert err <= (1e-11 if precision == FP64 else 2e-7)
