// Exact integration of radiative cooling and heating (Sec. 2.2, exact
// integration): du/dt = -rho lam(u) per particle over dt, lam tabulated at
// log-spaced energies u_k = 10^(log10_u0 + k dex) and interpolated by piecewise
// power laws (the composition folded into the table: Lambda = rho^2 lam).
//
// The paper walks I(u) bin by bin from each particle's anchor u_a = u^0. The
// integral of du / lam over a bin does not depend on the particle, so here the
// table is prepared once: within every run of bins where lam keeps its sign,
// G(u_k) = int from the run's first node to u_k of du / lam (a prefix sum of
// per-bin closed forms). A particle then needs G at u^0 (its bin's node value
// plus the in-bin closed form), a binary search for G(u^0) - rho dt among the
// run's nodes and the in-bin inverse: O(log K) table reads instead of a walk
// over every bin crossed. A bin where lam changes sign holds the equilibrium:
// constant source of the larger edge magnitude, u stopped at the zero of the
// linear interpolant when moving toward it; moving away (an unstable zero) it
// runs to the bin edge and continues in the neighbouring run. The table ends
// clamp u. Arithmetic is FP64 in both precisions (u and rho are Real), in log
// space where it can be: ln(u / u_k) = ln 10 (log10 u - log10 u_k) from the
// one log10 of the bin lookup, and the inverse as exp(ln u_k + ...), so that a
// particle in a run costs four transcendentals (log10, expm1, log1p, exp).
#include <cmath>

#include "crk_internal.h"

namespace crk {
namespace {

constexpr double kLn10 = 2.302585092994045684;

// Per power-law bin k with slope a_k and c_k = u_k / lam_k (the in-bin integral
// is c_k ln(u / u_k) for a_k = 1, else c_k expm1((1 - a_k) ln(u / u_k)) / (1 - a_k))
// the table holds oma_k = 1 - a_k and co_k = c_k / oma_k (c_k where oma_k = 0),
// so that the integral and its inverse need no division but the last one.
struct CoolTab {
  int K;
  double lu0, dex, inv_dex;
  double u_lo, u_hi;    // the first and last node energies
  const double* lam;    // [K]
  const double* co;     // [K - 1] c_k / (1 - a_k), or c_k (0 for a sign-change bin)
  const double* oma;    // [K - 1] 1 - a_k (0 for a sign-change bin)
  const double* G;      // [K] prefix integral within the node's run (see above)
  const int2* run;      // [K - 1] first and last bin of the bin's run ({-1, -1}: sign change)
};

__device__ inline double node_lnu(const CoolTab& T, int k) {
  return kLn10 * (T.lu0 + (double)k * T.dex);
}

__device__ inline double node_u(const CoolTab& T, int k) {
  return exp10(T.lu0 + (double)k * T.dex);
}

__device__ inline int bin_of(const CoolTab& T, double lg) {
  int k = (int)floor((lg - T.lu0) * T.inv_dex);
  return k < 0 ? 0 : (k > T.K - 2 ? T.K - 2 : k);
}

// int from u_k to u of du / lam inside power-law bin k, l = ln(u / u_k)
__device__ inline double in_bin(const CoolTab& T, int k, double l) {
  const double oma = T.oma[k], co = T.co[k];
  return oma == 0.0 ? co * l : co * expm1(oma * l);
}

// u in power-law bin k with int from u_k to u of du / lam = g:
// ln(u / u_k) = g / c_k, or log1p(g (1 - a_k) / c_k) / (1 - a_k)
__device__ inline double in_bin_inverse(const CoolTab& T, int k, double g) {
  const double oma = T.oma[k], y = g / T.co[k];
  const double t = oma == 0.0 ? y : log1p(y) / oma;
  return exp(node_lnu(T, k) + t);
}

// lam > 0 in power-law bin k (c_k has the sign of lam_k)
__device__ inline bool bin_cools(const CoolTab& T, int k) {
  const double oma = T.oma[k], co = T.co[k];
  return (oma == 0.0 ? co : co * oma) > 0.0;
}

// Sign-change bin k: returns u and sets left (rho t still to integrate).
__device__ inline double equilibrium_bin(const CoolTab& T, int k, double u, double& left) {
  const double uk = node_u(T, k), uk1 = node_u(T, k + 1);
  const double lk = T.lam[k], lk1 = T.lam[k + 1];
  const double ueq = lk1 != lk ? uk - lk * (uk1 - uk) / (lk1 - lk) : uk;
  const double lin = lk + (lk1 - lk) * (u - uk) / (uk1 - uk);
  const double mag = fmax(fabs(lk), fabs(lk1));
  if (lin == 0.0 || mag == 0.0) {
    left = 0.0;
    return u;
  }
  const bool down = lin > 0.0;
  const bool toward = (ueq < u) == down;
  const double target = toward ? ueq : (down ? uk : uk1);
  const double dist = fabs(u - target);
  if (mag * left <= dist) {
    const double r = down ? u - mag * left : u + mag * left;
    left = 0.0;
    return r;
  }
  left = toward ? 0.0 : left - dist / mag;
  return target;
}

// One phase from the anchor u: the run of same-sign bins, or the sign-change bin.
__device__ inline double cool_phase(const CoolTab& T, double u, double& left) {
  const double lg = log10(u);
  const int k = bin_of(T, lg);
  const int2 run = T.run[k];
  if (run.x < 0) return equilibrium_bin(T, k, u, left);
  const bool cooling = bin_cools(T, k);
  // G(u^1) = G(u^0) - rho dt; G rises with u where lam > 0, falls where lam < 0
  const double l = kLn10 * (lg - T.lu0 - (double)k * T.dex);
  const double target = T.G[k] + in_bin(T, k, l) - left;
  // nodes of the run: run.x .. run.y + 1 (G = 0 at run.x); the motion runs
  // out of the run past its lowest (cooling) or highest (heating) node
  const int end_node = cooling ? run.x : run.y + 1;
  if (target < T.G[end_node]) {
    const double ue = node_u(T, end_node);
    left = T.G[end_node] - target;  // rho t left at that node
    const int nb = cooling ? end_node - 1 : end_node;  // the bin beyond the run
    if (nb < 0 || nb > T.K - 2) {
      left = 0.0;
      return ue;  // clamped at the end of the table
    }
    return equilibrium_bin(T, nb, ue, left);
  }
  // binary search among the run's nodes for the bin j holding the target:
  // cooling: G increasing in the node index, search in [run.x, k]; heating:
  // G decreasing, search in [k, run.y]
  int lo = cooling ? run.x : k, hi = cooling ? k : run.y;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const bool before = cooling ? T.G[mid] <= target : T.G[mid] >= target;
    if (before) lo = mid; else hi = mid - 1;
  }
  left = 0.0;
  return in_bin_inverse(T, lo, target - T.G[lo]);
}

template <class R>
__device__ inline void cool_one(const CoolTab& T, int64_t i, double dt, const R* rho, R* u) {
  double ui = (double)u[i];
  ui = ui < T.u_lo ? T.u_lo : (ui > T.u_hi ? T.u_hi : ui);
  double left = (double)rho[i] * dt;
  // an unstable zero sends u out of its bin once; each side ends in a run
  for (int phase = 0; phase < 3 && left > 0.0; ++phase) ui = cool_phase(T, ui, left);
  u[i] = (R)ui;
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_cool(CoolTab T, int64_t n, double dt,
                                                 const R* __restrict__ rho, R* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  cool_one(T, i, dt, rho, u);
}

// The same with the per-bin table copied into LDS once per block (persistent
// blocks striding over the particles): the bin lookup and the binary search
// read LDS instead of waiting on the L2 at every dependent step. The table
// takes 32 bytes per node (co, oma, G, run); lam, read only in sign-change
// bins, stays in global memory.
constexpr int kCoolBlock = 1024;

template <class R>
__global__ void __launch_bounds__(kCoolBlock) k_cool_lds(CoolTab Tg, int64_t n, double dt,
                                                         const R* __restrict__ rho,
                                                         R* __restrict__ u) {
  extern __shared__ double table[];
  const int K = Tg.K;
  double* co = table;
  double* oma = co + K;
  double* G = oma + K;
  int2* run = (int2*)(G + K);
  for (int k = threadIdx.x; k < K; k += kCoolBlock) {
    G[k] = Tg.G[k];
    if (k < K - 1) {
      co[k] = Tg.co[k];
      oma[k] = Tg.oma[k];
      run[k] = Tg.run[k];
    }
  }
  __syncthreads();
  CoolTab T = Tg;
  T.co = co;
  T.oma = oma;
  T.G = G;
  T.run = run;
  for (int64_t i = (int64_t)blockIdx.x * kCoolBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kCoolBlock)
    cool_one(T, i, dt, rho, u);
}

// Table preparation, one block: slope a_k and c_k = u_k / lam_k per bin, kept
// as oma_k = 1 - a_k and co_k, and the runs; then the prefix integrals within
// every run (run starts get G = 0).
__global__ void __launch_bounds__(kBlock) k_cool_prepare(int K, double lu0, double dex,
                                                         const double* __restrict__ lam,
                                                         double* __restrict__ oma,
                                                         double* __restrict__ co,
                                                         double* __restrict__ G,
                                                         int2* __restrict__ run,
                                                         double* __restrict__ binint) {
  CoolTab T{K, lu0, dex, 1.0 / dex, 0.0, 0.0, lam, co, oma, G, run};
  for (int k = threadIdx.x; k < K - 1; k += kBlock) {
    const double lk = lam[k], lk1 = lam[k + 1];
    if (lk * lk1 > 0.0) {
      const double om = 1.0 - log(lk1 / lk) / (kLn10 * dex);
      const double c = node_u(T, k) / lk;
      oma[k] = om;
      co[k] = om == 0.0 ? c : c / om;
    } else {
      oma[k] = 0.0;
      co[k] = 0.0;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K - 1; k += kBlock) {
    const bool pl = lam[k] * lam[k + 1] > 0.0;
    binint[k] = pl ? in_bin(T, k, kLn10 * dex) : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // prefix integrals, restarting after every sign-change bin
    int start = 0;
    G[0] = 0.0;
    for (int k = 0; k < K - 1; ++k) {
      if (lam[k] * lam[k + 1] > 0.0) {
        G[k + 1] = G[k] + binint[k];
        run[k] = make_int2(start, -1);
      } else {
        G[k + 1] = 0.0;
        run[k] = make_int2(-1, -1);
        start = k + 1;
      }
    }
    // the last bin of every run, from the top down
    int last = -1;
    for (int k = K - 2; k >= 0; --k) {
      if (run[k].x < 0) {
        last = -1;
        continue;
      }
      if (last < 0) last = k;
      run[k].y = last;
    }
  }
}

}  // namespace

void launch_cool_prepare(int K, double lu0, double dex, const double* lam, double* oma,
                         double* co, double* G, void* run, double* binint, hipStream_t s) {
  hipLaunchKernelGGL(k_cool_prepare, dim3(1), dim3(kBlock), 0, s, K, lu0, dex, lam, oma, co, G,
                     (int2*)run, binint);
}

template <class R>
void launch_cool(int K, double lu0, double dex, const double* lam, const double* co,
                 const double* oma, const double* G, const void* run, int64_t n, double dt,
                 const R* rho, R* u, hipStream_t s) {
  const double u_lo = std::pow(10.0, lu0), u_hi = std::pow(10.0, lu0 + (K - 1) * dex);
  CoolTab T{K, lu0, dex, 1.0 / dex, u_lo, u_hi, lam, co, oma, G, (const int2*)run};
  const size_t lds = 32 * (size_t)K;
  if (lds <= 65536) {
    // two blocks of 1024 per compute unit over the 256 units, or fewer
    const int64_t want = (n + kCoolBlock - 1) / kCoolBlock;
    const int64_t blocks = want < 512 ? want : 512;
    hipLaunchKernelGGL(k_cool_lds<R>, dim3((unsigned)blocks), dim3(kCoolBlock), lds, s, T, n, dt,
                       rho, u);
  } else {
    hipLaunchKernelGGL(k_cool<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, T, n, dt, rho, u);
  }
}

template void launch_cool<float>(int, double, double, const double*, const double*,
                                 const double*, const double*, const void*, int64_t, double,
                                 const float*, float*, hipStream_t);
template void launch_cool<double>(int, double, double, const double*, const double*,
                                  const double*, const double*, const void*, int64_t, double,
                                  const double*, double*, hipStream_t);

}  // namespace crk
