// Time integration around the passes: the two kicks and the drift of one
// kick-drift-kick step on a single timestep level (App. A.4), with the
// smoothing length advanced by the combined Thacker and continuity rate and
// its exponential update (App. A.3). Every array is in the caller's order;
// each thread owns one particle (HBM-bound elementwise work).
#include "crk_internal.h"

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

}  // namespace

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
                                     hipStream_t);
CRK_STEP_INSTANTIATE(float)
CRK_STEP_INSTANTIATE(double)

}  // namespace crk
