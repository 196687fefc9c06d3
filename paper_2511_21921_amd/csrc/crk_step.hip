// Time integration around the passes: the two kicks and the drift of one
// kick-drift-kick step on a single timestep level (App. A.4), and the open,
// drift, predict and close kernels of the power-of-two hierarchy, with the
// smoothing length advanced by the combined Thacker and continuity rate and
// its exponential update (App. A.3). Every array is in the caller's order;
// each thread owns one particle (HBM-bound elementwise work).
#include "crk_internal.h"
#include "crk_state.h"

namespace crk {
namespace {

// First half kick, drift and smoothing-length update of particle i:
//   v^1/2 = v + a dt / 2 (stored in v), u^1/2 = u + du dt / 2 (stored in u);
//   the evaluation at the end of the step takes v^1/2 + a dt / 2 and
//   u^1/2 + du dt / 2 (vp, up);
//   x <- x + v^1/2 dt in FP64, wrapped into [0, box);
//   Delta_N = n_h V^(1/3) / h, h^T = h (1 - lam + lam Delta_N),
//   hdot = (h^T - h) / dt + h div(v) / 3 and h <- h exp(hdot dt / h), whose
//   exponent is lam (Delta_N - 1) + div(v) dt / 3.
// V and grad v are those of the evaluation at the start of the step.
template <class R>
__global__ void __launch_bounds__(kBlock) k_kick_drift(int64_t n, double dt, double lam,
                                                       double n_h, double box,
                                                       double* __restrict__ x,
                                                       R* __restrict__ v, R* __restrict__ u,
                                                       R* __restrict__ h,
                                                       const R* __restrict__ V,
                                                       const R* __restrict__ gradv,
                                                       const double* __restrict__ accel,
                                                       const double* __restrict__ dudt,
                                                       R* __restrict__ vp, R* __restrict__ up) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double half = 0.5 * dt;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double acc = accel[a * n + i];
    const double vh = (double)v[a * n + i] + half * acc;
    v[a * n + i] = (R)vh;
    vp[a * n + i] = (R)(vh + half * acc);
    double t = x[a * n + i] + vh * dt;
    if (t >= box) t -= box;
    if (t < 0.0) t += box;
    x[a * n + i] = t;
  }
  const double du = dudt[i];
  const double uh = (double)u[i] + half * du;
  u[i] = (R)uh;
  up[i] = (R)(uh + half * du);
  const double hi = (double)h[i];
  const double div = (double)gradv[i] + (double)gradv[4 * n + i] + (double)gradv[8 * n + i];
  const double delta_n = n_h * cbrt((double)V[i]) / hi;
  h[i] = (R)(hi * exp(lam * (delta_n - 1.0) + div * dt / 3.0));
}

// Second half kick with the acceleration and du/dt at the end of the step.
template <class R>
__global__ void __launch_bounds__(kBlock) k_kick_close(int64_t n, double dt, R* __restrict__ v,
                                                       R* __restrict__ u,
                                                       const double* __restrict__ accel,
                                                       const double* __restrict__ dudt) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double half = 0.5 * dt;
#pragma unroll
  for (int a = 0; a < 3; ++a) v[a * n + i] = (R)((double)v[a * n + i] + half * accel[a * n + i]);
  u[i] = (R)((double)u[i] + half * dudt[i]);
}

// ------------------------------------------------ timestep hierarchy ----
// One big step dt on power-of-two levels (App. A.4): a particle of level L
// is active on intervals dt_a = dt / 2^L = 2^(lmax - L) dt_min and every
// particle drifts on dt_min = dt / 2^lmax. jend counts substep ends.

__device__ inline int64_t level_span(const int* levels, int lmax, int64_t i) {
  return (int64_t)1 << (lmax - levels[i]);  // substeps per active interval
}

// Opening of an interval for the particles whose interval starts at substep
// end jend (all at jend = 0): first half kick into vh, uh, and the combined
// Thacker and continuity rate (App. A.3)
//   hdot = (h^T - h) / dt_a + h div(v) / 3,  h^T = h (1 - lam + lam Delta_N),
// from the particle's latest evaluation (V, grad v).
template <class R>
__global__ void __launch_bounds__(kBlock) k_hier_open(
    int64_t n, const int* __restrict__ levels, int lmax, int64_t jend, double dt_min, double lam,
    double n_h, const R* __restrict__ v, const R* __restrict__ u, const R* __restrict__ h,
    const R* __restrict__ V, const R* __restrict__ gradv, const double* __restrict__ accel,
    const double* __restrict__ dudt, R* __restrict__ vh, R* __restrict__ uh,
    double* __restrict__ hdot) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t per = level_span(levels, lmax, i);
  if (jend & (per - 1)) return;
  const double dta = (double)per * dt_min;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    vh[a * n + i] = (R)((double)v[a * n + i] + 0.5 * dta * accel[a * n + i]);
  uh[i] = (R)((double)u[i] + 0.5 * dta * dudt[i]);
  const double hi = (double)h[i];
  const double div = (double)gradv[i] + (double)gradv[4 * n + i] + (double)gradv[8 * n + i];
  const double delta_n = n_h * cbrt((double)V[i]) / hi;
  const double h_thacker = hi * (1.0 - lam + lam * delta_n);
  hdot[i] = (h_thacker - hi) / dta + hi * div / 3.0;
}

// Timestep refinement at the start of substep j (App. A.5): a particle with
// refine_at = j moves to the finer level refine_level. Its interval opened
// at the last substep on the grid of its old level, e = (j - that) dt_min
// before; its velocity and energy advance under the constant a^0, du^0 to
// t_r = j dt_min (v <- v + a^0 e), and a new interval of the new level opens
// there as k_hier_open opens one (half kick and hdot from the particle's
// current h and stored V, grad v). j lies on the new level's grid (checked
// by the caller), so the new interval ends on it; the cycle thus ends with
// v^1 = v^0 + a^0 e + (a^0 + a^1) dt_c / 2, the piecewise-constant final
// kick, and the particle keeps the new level to the end of the big step.
template <class R>
__global__ void __launch_bounds__(kBlock) k_hier_refine(
    int64_t n, int64_t j, const int* __restrict__ refine_at, const int* __restrict__ refine_level,
    int* __restrict__ lvl, int lmax, double dt_min, double lam, double n_h, R* __restrict__ v,
    R* __restrict__ u, const R* __restrict__ h, const R* __restrict__ V,
    const R* __restrict__ gradv, const double* __restrict__ accel,
    const double* __restrict__ dudt, R* __restrict__ vh, R* __restrict__ uh,
    double* __restrict__ hdot) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || refine_at[i] != j) return;
  const int64_t per_old = level_span(lvl, lmax, i);
  const double e = (double)(j & (per_old - 1)) * dt_min;
  lvl[i] = refine_level[i];
  const double dtc = (double)level_span(lvl, lmax, i) * dt_min;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double vr = (double)v[a * n + i] + accel[a * n + i] * e;
    v[a * n + i] = (R)vr;
    vh[a * n + i] = (R)((double)(R)vr + 0.5 * dtc * accel[a * n + i]);
  }
  const double ur = (double)u[i] + dudt[i] * e;
  u[i] = (R)ur;
  uh[i] = (R)((double)(R)ur + 0.5 * dtc * dudt[i]);
  const double hi = (double)h[i];
  const double div = (double)gradv[i] + (double)gradv[4 * n + i] + (double)gradv[8 * n + i];
  const double delta_n = n_h * cbrt((double)V[i]) / hi;
  const double h_thacker = hi * (1.0 - lam + lam * delta_n);
  hdot[i] = (h_thacker - hi) / dtc + hi * div / 3.0;
}

// Drift of substep j for every particle: positions on the parabola of the
// particle's constant a^0, v_j = v^1/2 + a^0 (t_elapsed + (dt_min - dt_a) / 2)
// (FP64, wrapped into [0, box)); h <- h exp(hdot dt_min / h); the passive
// state V = (h / n_h)^3 and rho <- rho exp(-div(v) dt_min) (App. A.3), which
// the next evaluation recomputes for the particles it updates.
template <class R>
__global__ void __launch_bounds__(kBlock) k_hier_drift(
    int64_t n, const int* __restrict__ levels, int lmax, int64_t j, double dt_min, double n_h,
    double box, double* __restrict__ x, const R* __restrict__ vh,
    const double* __restrict__ accel, R* __restrict__ h, const double* __restrict__ hdot,
    R* __restrict__ V, R* __restrict__ rho, const R* __restrict__ gradv) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t per = level_span(levels, lmax, i);
  const int64_t start = j & ~(per - 1);
  const double dta = (double)per * dt_min;
  const double c = (double)(j - start) * dt_min + 0.5 * (dt_min - dta);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double vj = (double)vh[a * n + i] + accel[a * n + i] * c;
    double t = x[a * n + i] + vj * dt_min;
    if (t >= box) t -= box;
    if (t < 0.0) t += box;
    x[a * n + i] = t;
  }
  const double hi = (double)h[i];
  const double hn = hi * exp(hdot[i] * dt_min / hi);
  h[i] = (R)hn;
  const double q = hn / n_h;
  V[i] = (R)(q * q * q);
  const double div = (double)gradv[i] + (double)gradv[4 * n + i] + (double)gradv[8 * n + i];
  rho[i] = (R)((double)rho[i] * exp(-div * dt_min));
}

// Velocity and energy of every particle at substep end jend under its
// constant a^0 and du^0: v^1/2 + a^0 t, t = time since the centre of the
// particle's interval (the end-of-interval prediction of the active ones).
template <class R>
__global__ void __launch_bounds__(kBlock) k_hier_predict(
    int64_t n, const int* __restrict__ levels, int lmax, int64_t jend, double dt_min,
    const R* __restrict__ vh, const R* __restrict__ uh, const double* __restrict__ accel,
    const double* __restrict__ dudt, R* __restrict__ vp, R* __restrict__ up) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t per = level_span(levels, lmax, i);
  const int64_t start = (jend - 1) & ~(per - 1);
  const double t = (double)(jend - start) * dt_min - 0.5 * (double)per * dt_min;
#pragma unroll
  for (int a = 0; a < 3; ++a) vp[a * n + i] = (R)((double)vh[a * n + i] + accel[a * n + i] * t);
  up[i] = (R)((double)uh[i] + dudt[i] * t);
}

// Second half kick of the particles whose interval ends at jend; their new
// acceleration and du/dt become the stored a^0, du^0.
template <class R>
__global__ void __launch_bounds__(kBlock) k_hier_close(
    int64_t n, const int* __restrict__ levels, int lmax, int64_t jend, double dt_min,
    R* __restrict__ v, R* __restrict__ u, const R* __restrict__ vh, const R* __restrict__ uh,
    const double* __restrict__ acc1, const double* __restrict__ du1, double* __restrict__ accel,
    double* __restrict__ dudt) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t per = level_span(levels, lmax, i);
  if (jend & (per - 1)) return;
  const double half = 0.5 * (double)per * dt_min;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double acc = acc1[a * n + i];
    v[a * n + i] = (R)((double)vh[a * n + i] + half * acc);
    accel[a * n + i] = acc;
  }
  u[i] = (R)((double)uh[i] + half * du1[i]);
  dudt[i] = du1[i];
}

// Largest level (a max counter) over the levels and the refinement levels,
// and the count of levels outside [0, 30] or refinements not to a finer
// level (refine_at null: none).
__global__ void __launch_bounds__(kBlock) k_level_range(const int* __restrict__ levels,
                                                        const int* __restrict__ refine_at,
                                                        const int* __restrict__ refine_level,
                                                        int64_t n,
                                                        unsigned long long* __restrict__ cnt,
                                                        unsigned long long* __restrict__ hist) {
  __shared__ unsigned int bins[32];
  if (threadIdx.x < 32) bins[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  unsigned long long top = 0, bad = 0;
  if (i < n) {
    const int L = levels[i];
    if (L < 0 || L > 30) bad = 1; else top = (unsigned long long)L;
    if (L >= 0 && L <= 30) atomicAdd(&bins[L], 1u);
    if (refine_at && refine_at[i] >= 0) {
      const int Lr = refine_level[i];
      if (!(Lr > L && Lr <= 30)) bad = 1; else top = top > (unsigned long long)Lr ? top : Lr;
      atomicAdd(&bins[31], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x < 32 && bins[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)bins[threadIdx.x]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(top, o, 64);
    top = t > top ? t : top;
    bad += __shfl_xor(bad, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (top) atomicMax(cnt_at(cnt, CNT_H_ITER_MAX), top);
    if (bad) atomicAdd(cnt_at(cnt, CNT_BAD_INPUT), bad);
  }
}

// Refinements off the grid of their new level (refine_at not a multiple of
// 2^(lmax - refine_level)) or past the last substep, counted as bad input.
__global__ void __launch_bounds__(kBlock) k_refine_grid(const int* __restrict__ refine_at,
                                                        const int* __restrict__ refine_level,
                                                        int64_t n, int lmax,
                                                        unsigned long long* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  unsigned long long bad = 0;
  if (i < n && refine_at[i] >= 0) {
    const int64_t j = refine_at[i];
    const int64_t per = (int64_t)1 << (lmax - refine_level[i]);
    if (j >= ((int64_t)1 << lmax) || (j & (per - 1))) bad = 1;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, 64);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(cnt_at(cnt, CNT_BAD_INPUT), bad);
}

}  // namespace

template <class R>
void launch_hier_open(int64_t n, const int* levels, int lmax, int64_t jend, double dt_min,
                      double lam, double n_h, const R* v, const R* u, const R* h, const R* V,
                      const R* gradv, const double* accel, const double* dudt, R* vh, R* uh,
                      double* hdot, hipStream_t s) {
  hipLaunchKernelGGL(k_hier_open<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, levels, lmax, jend,
                     dt_min, lam, n_h, v, u, h, V, gradv, accel, dudt, vh, uh, hdot);
}

template <class R>
void launch_hier_drift(int64_t n, const int* levels, int lmax, int64_t j, double dt_min,
                       double n_h, double box, double* x, const R* vh, const double* accel, R* h,
                       const double* hdot, R* V, R* rho, const R* gradv, hipStream_t s) {
  hipLaunchKernelGGL(k_hier_drift<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, levels, lmax, j,
                     dt_min, n_h, box, x, vh, accel, h, hdot, V, rho, gradv);
}

template <class R>
void launch_hier_predict(int64_t n, const int* levels, int lmax, int64_t jend, double dt_min,
                         const R* vh, const R* uh, const double* accel, const double* dudt, R* vp,
                         R* up, hipStream_t s) {
  hipLaunchKernelGGL(k_hier_predict<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, levels, lmax,
                     jend, dt_min, vh, uh, accel, dudt, vp, up);
}

template <class R>
void launch_hier_close(int64_t n, const int* levels, int lmax, int64_t jend, double dt_min, R* v,
                       R* u, const R* vh, const R* uh, const double* acc1, const double* du1,
                       double* accel, double* dudt, hipStream_t s) {
  hipLaunchKernelGGL(k_hier_close<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, levels, lmax,
                     jend, dt_min, v, u, vh, uh, acc1, du1, accel, dudt);
}

void launch_level_range(const int* levels, const int* refine_at, const int* refine_level,
                        int64_t n, unsigned long long* cnt, unsigned long long* hist,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_level_range, dim3(grid_for(n)), dim3(kBlock), 0, s, levels, refine_at,
                     refine_level, n, cnt, hist);
}

void launch_refine_grid(const int* refine_at, const int* refine_level, int64_t n, int lmax,
                        unsigned long long* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_refine_grid, dim3(grid_for(n)), dim3(kBlock), 0, s, refine_at,
                     refine_level, n, lmax, cnt);
}

template <class R>
void launch_hier_refine(int64_t n, int64_t j, const int* refine_at, const int* refine_level,
                        int* lvl, int lmax, double dt_min, double lam, double n_h, R* v, R* u,
                        const R* h, const R* V, const R* gradv, const double* accel,
                        const double* dudt, R* vh, R* uh, double* hdot, hipStream_t s) {
  hipLaunchKernelGGL(k_hier_refine<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, j, refine_at,
                     refine_level, lvl, lmax, dt_min, lam, n_h, v, u, h, V, gradv, accel, dudt,
                     vh, uh, hdot);
}

template <class R>
void launch_kick_drift(int64_t n, double dt, double lam, double n_h, double box, double* x, R* v,
                       R* u, R* h, const R* V, const R* gradv, const double* accel,
                       const double* dudt, R* vp, R* up, hipStream_t s) {
  hipLaunchKernelGGL(k_kick_drift<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, dt, lam, n_h, box,
                     x, v, u, h, V, gradv, accel, dudt, vp, up);
}

template <class R>
void launch_kick_close(int64_t n, double dt, R* v, R* u, const double* accel, const double* dudt,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_kick_close<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, dt, v, u, accel,
                     dudt);
}

#define CRK_STEP_INSTANTIATE(R)                                                                  \
  template void launch_kick_drift<R>(int64_t, double, double, double, double, double*, R*, R*, \
                                     R*, const R*, const R*, const double*, const double*, R*,  \
                                     R*, hipStream_t);                                           \
  template void launch_kick_close<R>(int64_t, double, R*, R*, const double*, const double*,     \
                                     hipStream_t);                                               \
  template void launch_hier_open<R>(int64_t, const int*, int, int64_t, double, double, double,  \
                                    const R*, const R*, const R*, const R*, const R*,           \
                                    const double*, const double*, R*, R*, double*, hipStream_t); \
  template void launch_hier_drift<R>(int64_t, const int*, int, int64_t, double, double, double, \
                                     double*, const R*, const double*, R*, const double*, R*,   \
                                     R*, const R*, hipStream_t);                                 \
  template void launch_hier_predict<R>(int64_t, const int*, int, int64_t, double, const R*,     \
                                       const R*, const double*, const double*, R*, R*,          \
                                       hipStream_t);                                             \
  template void launch_hier_close<R>(int64_t, const int*, int, int64_t, double, R*, R*,         \
                                     const R*, const R*, const double*, const double*, double*, \
                                     double*, hipStream_t);                                      \
  template void launch_hier_refine<R>(int64_t, int64_t, const int*, const int*, int*, int,      \
                                      double, double, double, R*, R*, const R*, const R*,       \
                                      const R*, const double*, const double*, R*, R*, double*,  \
                                      hipStream_t);
CRK_STEP_INSTANTIATE(float)
CRK_STEP_INSTANTIATE(double)

}  // namespace crk
