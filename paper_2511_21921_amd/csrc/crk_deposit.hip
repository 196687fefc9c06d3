// Subgrid sources coupling to the gas: the source volume of App. A.2 eq.
// (Vsg) and the normalised SPH deposition of mass, metals, energy and
// momentum (eqs. windmetal, Anorm, starmetal, stellarmom, AGNE):
//   V_s^-1 = sum over gas j of W(|x_sj|, h_j) plus the self term W(0, h_s),
//     h_s = n_h,s V_s^(1/3), so V_s = (1 - C w(0) / n_h,s^3) / sum_j W(|x_sj|, h_j);
//   A_s^-1 = sum over eligible gas j of V_j W(|x_sj|, h_s);
//   gas j receives A_s V_j W(|x_sj|, h_s) of every source's mass, metal mass
//     and energy; the mass brings the source's momentum, the energy goes into
//     the internal energy of the grown particle.
// Deposition is gathered from the gas side (each gas particle sums over the
// sources that reach it), so no float atomics are used and results are
// reproducible. Searches run over uniform periodic grids of sorted points
// with cells at least the search radius (27-cell stencils; grids with fewer
// than 3 cells per side collapse to one cell). Arithmetic is FP64.
#include "crk_passes.h"

namespace crk {
namespace {

// a sorted point set on a periodic grid: perm maps sorted -> caller index
struct PointGrid {
  int G;
  double ell, box;
  const uint32_t* start;  // [G^3 + 1]
  const uint32_t* perm;   // [n]
};

__device__ inline int cell_of(double x, double box, int G) {
  double t = x - box * floor(x / box);
  int c = (int)(t * (double)G / box);
  return c < 0 ? 0 : (c >= G ? G - 1 : c);
}

template <int K>
__device__ inline double kernel_W(double r, double h) {
  double w, dw;
  Shape<K>::eval(r / h, w, dw);
  return Shape<K>::C * w / (h * h * h);
}

__device__ inline double min_image2(const double* xa, int64_t na, int64_t a, const double* xb,
                                    int64_t nb, int64_t b, double box) {
  double r2 = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double t = xb[d * nb + b] - xa[d * na + a];
    t -= box * rint(t / box);
    r2 += t * t;
  }
  return r2;
}

// visits every point of grid g in the 27 cells around position (x, y, z)
template <class F>
__device__ inline void for_near(const PointGrid& g, double x, double y, double z, F&& f) {
  const int G = g.G;
  const int cx = cell_of(x, g.box, G), cy = cell_of(y, g.box, G), cz = cell_of(z, g.box, G);
  const int r = G >= 3 ? 1 : 0;
  for (int dz = -r; dz <= r; ++dz)
    for (int dy = -r; dy <= r; ++dy)
      for (int dx = -r; dx <= r; ++dx) {
        const int c = ((cz + dz + G) % G * G + (cy + dy + G) % G) * G + (cx + dx + G) % G;
        for (uint32_t k = g.start[c]; k < g.start[c + 1]; ++k) f((int64_t)g.perm[k]);
      }
}

__global__ void __launch_bounds__(kBlock) k_point_keys(const double* __restrict__ x, int64_t n,
                                                       double box, int G,
                                                       uint32_t* __restrict__ keys,
                                                       uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int cx = cell_of(x[i], box, G), cy = cell_of(x[n + i], box, G),
            cz = cell_of(x[2 * n + i], box, G);
  keys[i] = ((uint32_t)cz * G + (uint32_t)cy) * G + (uint32_t)cx;
  vals[i] = (uint32_t)i;
}

// largest value of a positive array, as double bits into a counter slot
template <class R>
__global__ void __launch_bounds__(kBlock) k_max_bits(const R* __restrict__ a, int64_t n,
                                                     unsigned long long* __restrict__ cnt,
                                                     int slot) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  unsigned long long b = 0;
  if (i < n) {
    const double v = (double)a[i];
    // non-finite or non-positive values are reported as +infinity
    b = (v > 0.0 && v < 1e300) ? (unsigned long long)__double_as_longlong(v)
                                 : 0x7ff0000000000000ull;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(b, o, 64);
    b = t > b ? t : b;
  }
  if ((threadIdx.x & 63) == 0 && b) atomicMax(cnt_at(cnt, slot), b);
}

template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_dep_volume(PointGrid gas, const double* __restrict__ xg,
                                                       int64_t ng, const R* __restrict__ hg,
                                                       const double* __restrict__ xs, int64_t ns,
                                                       double self_frac, double n_h_s,
                                                       R* __restrict__ Vs, R* __restrict__ hs,
                                                       unsigned long long* __restrict__ cnt) {
  const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  unsigned long long hb = 0;
  if (s < ns) {
    double sum = 0.0;
    for_near(gas, xs[s], xs[ns + s], xs[2 * ns + s], [&](int64_t j) {
      const double r2 = min_image2(xs, ns, s, xg, ng, j, gas.box);
      const double h = (double)hg[j];
      if (r2 < h * h) sum += kernel_W<K>(sqrt(r2), h);
    });
    double V = 0.0, h = 0.0;
    if (sum > 0.0) {
      V = (1.0 - self_frac) / sum;
      h = n_h_s * cbrt(V);
    }
    Vs[s] = (R)V;
    hs[s] = (R)h;
    hb = (unsigned long long)__double_as_longlong(h);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(hb, o, 64);
    hb = t > hb ? t : hb;
  }
  if ((threadIdx.x & 63) == 0 && hb) atomicMax(cnt_at(cnt, CNT_HMAX_OUT_BITS), hb);
}

template <class R>
__device__ inline bool eligible(const R* m, const R* mZ, int64_t j, double z_max, double m_max) {
  const double mj = (double)m[j];
  return (double)mZ[j] <= z_max * mj && mj <= m_max;
}

template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_dep_norm(PointGrid gas, const double* __restrict__ xg,
                                                     int64_t ng, const R* __restrict__ Vg,
                                                     const R* __restrict__ mg,
                                                     const R* __restrict__ mZg,
                                                     const double* __restrict__ xs, int64_t ns,
                                                     const R* __restrict__ hs, double z_max,
                                                     double m_max, R* __restrict__ As) {
  const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (s >= ns) return;
  const double h = (double)hs[s];
  double sum = 0.0;
  if (h > 0.0)
    for_near(gas, xs[s], xs[ns + s], xs[2 * ns + s], [&](int64_t j) {
      const double r2 = min_image2(xs, ns, s, xg, ng, j, gas.box);
      if (r2 < h * h && eligible(mg, mZg, j, z_max, m_max))
        sum += (double)Vg[j] * kernel_W<K>(sqrt(r2), h);
    });
  As[s] = (R)(sum > 0.0 ? 1.0 / sum : 0.0);
}

template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_dep_gather(
    PointGrid src, const double* __restrict__ xg, int64_t ng, const R* __restrict__ Vg,
    R* __restrict__ mg, R* __restrict__ vg, R* __restrict__ mZg, R* __restrict__ ug,
    const double* __restrict__ xs, int64_t ns, const R* __restrict__ hs,
    const R* __restrict__ As, const R* __restrict__ dM, const R* __restrict__ dMZ,
    const R* __restrict__ dE, const R* __restrict__ vs, double z_max, double m_max) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= ng || !eligible(mg, mZg, j, z_max, m_max)) return;
  const double Vj = (double)Vg[j];
  double dm = 0.0, dmz = 0.0, de = 0.0, dp[3] = {0.0, 0.0, 0.0};
  for_near(src, xg[j], xg[ng + j], xg[2 * ng + j], [&](int64_t s) {
    const double a = (double)As[s];
    if (!(a > 0.0)) return;
    const double h = (double)hs[s];
    const double r2 = min_image2(xg, ng, j, xs, ns, s, src.box);
    if (!(r2 < h * h)) return;
    const double f = a * Vj * kernel_W<K>(sqrt(r2), h);
    const double fm = f * (double)dM[s];
    dm += fm;
    dmz += f * (double)dMZ[s];
    de += f * (double)dE[s];
#pragma unroll
    for (int d = 0; d < 3; ++d) dp[d] += fm * (double)vs[d * ns + s];
  });
  if (dm == 0.0 && dmz == 0.0 && de == 0.0) return;
  const double m0 = (double)mg[j], m1 = m0 + dm;
  mg[j] = (R)m1;
  mZg[j] = (R)((double)mZg[j] + dmz);
#pragma unroll
  for (int d = 0; d < 3; ++d) vg[d * ng + j] = (R)((m0 * (double)vg[d * ng + j] + dp[d]) / m1);
  ug[j] = (R)((m0 * (double)ug[j] + de) / m1);
}

}  // namespace

void launch_point_keys(const double* x, int64_t n, double box, int G, uint32_t* keys,
                       uint32_t* vals, hipStream_t s) {
  hipLaunchKernelGGL(k_point_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, x, n, box, G, keys,
                     vals);
}

template <class R>
void launch_max_bits(const R* a, int64_t n, unsigned long long* cnt, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_max_bits<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, a, n, cnt, slot);
}

#define CRK_DEP_DISPATCH(kernel, KFN, grid, ...)                                          \
  do {                                                                                    \
    if ((kernel) == 0)                                                                    \
      hipLaunchKernelGGL((KFN<R, 0>), dim3(grid_for(grid)), dim3(kBlock), 0, s, __VA_ARGS__); \
    else                                                                                  \
      hipLaunchKernelGGL((KFN<R, 1>), dim3(grid_for(grid)), dim3(kBlock), 0, s, __VA_ARGS__); \
  } while (0)

template <class R>
void launch_dep_volume(int kernel, int G, double ell, double box, const uint32_t* start,
                       const uint32_t* perm, const double* xg, int64_t ng, const R* hg,
                       const double* xs, int64_t ns, double self_frac, double n_h_s, R* Vs, R* hs,
                       unsigned long long* cnt, hipStream_t s) {
  PointGrid g{G, ell, box, start, perm};
  CRK_DEP_DISPATCH(kernel, k_dep_volume, ns, g, xg, ng, hg, xs, ns, self_frac, n_h_s, Vs, hs,
                   cnt);
}

template <class R>
void launch_dep_norm(int kernel, int G, double ell, double box, const uint32_t* start,
                     const uint32_t* perm, const double* xg, int64_t ng, const R* Vg, const R* mg,
                     const R* mZg, const double* xs, int64_t ns, const R* hs, double z_max,
                     double m_max, R* As, hipStream_t s) {
  PointGrid g{G, ell, box, start, perm};
  CRK_DEP_DISPATCH(kernel, k_dep_norm, ns, g, xg, ng, Vg, mg, mZg, xs, ns, hs, z_max, m_max, As);
}

template <class R>
void launch_dep_gather(int kernel, int G, double ell, double box, const uint32_t* start,
                       const uint32_t* perm, const double* xg, int64_t ng, const R* Vg, R* mg,
                       R* vg, R* mZg, R* ug, const double* xs, int64_t ns, const R* hs,
                       const R* As, const R* dM, const R* dMZ, const R* dE, const R* vs,
                       double z_max, double m_max, hipStream_t s) {
  PointGrid g{G, ell, box, start, perm};
  CRK_DEP_DISPATCH(kernel, k_dep_gather, ng, g, xg, ng, Vg, mg, vg, mZg, ug, xs, ns, hs, As, dM,
                   dMZ, dE, vs, z_max, m_max);
}

#define CRK_DEP_INSTANTIATE(R)                                                                \
  template void launch_max_bits<R>(const R*, int64_t, unsigned long long*, int, hipStream_t); \
  template void launch_dep_volume<R>(int, int, double, double, const uint32_t*,              \
                                     const uint32_t*, const double*, int64_t, const R*,      \
                                     const double*, int64_t, double, double, R*, R*,          \
                                     unsigned long long*, hipStream_t);                       \
  template void launch_dep_norm<R>(int, int, double, double, const uint32_t*, const uint32_t*, \
                                   const double*, int64_t, const R*, const R*, const R*,      \
                                   const double*, int64_t, const R*, double, double, R*,      \
                                   hipStream_t);                                              \
  template void launch_dep_gather<R>(int, int, double, double, const uint32_t*,              \
                                     const uint32_t*, const double*, int64_t, const R*, R*,  \
                                     R*, R*, R*, const double*, int64_t, const R*, const R*,  \
                                     const R*, const R*, const R*, const R*, double, double,  \
                                     hipStream_t);
CRK_DEP_INSTANTIATE(float)
CRK_DEP_INSTANTIATE(double)

}  // namespace crk
