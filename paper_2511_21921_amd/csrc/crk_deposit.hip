// Subgrid sources coupling to the gas: the source volume of App. A.2 eq.
// (Vsg) and the normalised SPH deposition of mass, metals, energy and
// momentum (eqs. windmetal, Anorm, starmetal, stellarmom, AGNE):
//   V_s^-1 = sum over gas j of W(|x_sj|, h_j) plus the self term W(0, h_s),
//     h_s = n_h,s V_s^(1/3), so V_s = (1 - C w(0) / n_h,s^3) / sum_j W(|x_sj|, h_j);
//   A_s^-1 = sum over eligible gas j of V_j W(|x_sj|, h_s);
//   gas j receives A_s V_j W(|x_sj|, h_s) of every source's mass, metal mass
//     and energy; the mass brings the source's momentum, the energy goes into
//     the internal energy of the grown particle.
// The gas is sorted into one periodic grid with cells at least the largest
// gas h wide, and packed in that order. Sources search it, one wave per
// source, over the cells that the sphere of the search radius touches (the
// largest gas h for the volume, h_s for the normalisation), so a source with
// a large h_s costs only itself. Cells along x are adjacent in the sorted
// order, so each row of the stencil is one or two contiguous ranges that
// the wave's lanes share. The normalisation pass counts each source's
// receivers and keeps the first 64 of them; the (gas, source) pairs are then
// written in source order (a source with more receivers walks its cells
// again), a stable sort by gas index groups them, and each gas particle sums
// its contributions in source order. No float atomics: results are
// reproducible. Arithmetic is FP64.
#include "crk_passes.h"

namespace crk {
namespace {

// the gas sorted into a periodic grid; perm maps sorted -> caller index and
// the packed arrays hold the gas in sorted order
struct PointGrid {
  int G;
  double box, inv_box;
  double hmax;            // the largest gas h
  const uint32_t* start;  // [G^3 + 1]
  const uint32_t* perm;   // [n]
  const double4* p4;      // [n] x, y, z, h
  const double2* pv;      // [n] V if eligible (else -1), 1 / h
};

__device__ inline int cell_of(double x, double box, int G) {
  const double t = x - box * floor(x / box);
  const int c = (int)(t * (double)G / box);
  return c < 0 ? 0 : (c >= G ? G - 1 : c);
}

// W(r, h) with 1 / h given (no divisions)
template <int K>
__device__ inline double kernel_W_inv(double r, double inv_h) {
  double w, dw;
  Shape<K>::eval(r * inv_h, w, dw);
  return Shape<K>::C * (inv_h * inv_h * inv_h) * w;
}

// nearest periodic image; the image choice can differ from rounding t / box
// only where both images lie half a box away, beyond every search radius
__device__ inline double min_image2(double ax, double ay, double az, double4 b,
                                    const PointGrid& g) {
  double tx = b.x - ax, ty = b.y - ay, tz = b.z - az;
  tx -= g.box * rint(tx * g.inv_box);
  ty -= g.box * rint(ty * g.inv_box);
  tz -= g.box * rint(tz * g.inv_box);
  return tx * tx + ty * ty + tz * tz;
}

// One wave visits every point of grid g within r of (x, y, z), and some
// beyond: the cells of a (2k+1)^3 stencil, k = ceil(r / cell), less the rows
// of cells (along x) whose gap to the point in y and z is at least r, each
// row cut to the cells whose gap in x is within what remains of r. Gaps are
// taken slightly short, so the pruning only ever keeps more. When the
// stencil would wrap onto itself (2k+1 >= G) the whole grid is visited, each
// cell once. Each lane sets up one row (one or two contiguous ranges of the
// sorted order, so the cell starts of 64 rows load at once); the wave then
// runs through the rows' candidates 64 at a time across row boundaries. All
// lanes call f(q, valid) together (q a sorted index), in the same order on
// every run.
template <class F>
__device__ inline void wave_near(const PointGrid& g, double x, double y, double z, double r,
                                 F&& f) {
  const int G = g.G;
  const int lane = threadIdx.x & 63;
  const double cw = g.box / G;  // cell width
  const double rc = r / cw * (1.0 + 1e-9);  // the radius in cells, with a margin
  const int k = (int)ceil(rc);
  if (2 * k + 1 >= G) {
    // the sorted order runs through all cells
    const uint32_t b = g.start[G * G * G];
    for (uint32_t q0 = 0; q0 < b; q0 += 64) {
      const uint32_t q = q0 + lane;
      f(q < b ? q : 0u, q < b);
    }
    return;
  }
  // the point in cell units: cell index and offset inside the cell
  auto locate = [&](double p, int& c, double& fr) {
    const double t = p - g.box * floor(p / g.box);
    const double u = t * (double)G / g.box;
    c = (int)u;
    c = c < 0 ? 0 : (c >= G ? G - 1 : c);
    fr = u - (double)c;
    fr = fr < 0.0 ? 0.0 : (fr > 1.0 ? 1.0 : fr);
  };
  int ix, iy, iz;
  double fx, fy, fz;
  locate(x, ix, fx);
  locate(y, iy, fy);
  locate(z, iz, fz);
  // gap (in cells) from the point to the cell d away along one axis
  auto gap = [](int d, double fr) {
    const double v = d > 0 ? (double)d - fr : (d < 0 ? (double)(-d - 1) + fr : 0.0);
    return v > 1e-9 ? v - 1e-9 : 0.0;
  };
  const double rc2 = rc * rc;
  const int side = 2 * k + 1, nrows = side * side;
  for (int r0 = 0; r0 < nrows; r0 += 64) {
    // this lane's row: dz, dy = row index / side, row index % side (minus k)
    uint32_t a1 = 0, n1 = 0, a2 = 0, n2 = 0;
    const int ri = r0 + lane;
    if (ri < nrows) {
      const int dz = ri / side - k, dy = ri % side - k;
      const double gz = gap(dz, fz), gy = gap(dy, fy);
      const double gyz = gy * gy + gz * gz;
      if (gyz < rc2) {
        const double rx = sqrt(rc2 - gyz);
        int dpos = (int)ceil(rx + fx + 1e-9) - 1;
        int dneg = (int)ceil(rx + 1.0 - fx + 1e-9) - 1;
        dpos = dpos > k ? k : (dpos < 0 ? 0 : dpos);
        dneg = dneg > k ? k : (dneg < 0 ? 0 : dneg);
        const int span = dneg + dpos + 1;
        const int row = ((iz + dz + G) % G * G + (iy + dy + G) % G) * G;
        const int x0 = (ix - dneg + G) % G;
        if (x0 + span <= G) {
          a1 = g.start[row + x0];
          n1 = g.start[row + x0 + span] - a1;
        } else {
          a1 = g.start[row + x0];
          n1 = g.start[row + G] - a1;
          a2 = g.start[row];
          n2 = g.start[row + x0 + span - G] - a2;
        }
      }
    }
    // exclusive prefix of the rows' candidate counts over the lanes
    const uint32_t len = n1 + n2;
    uint32_t pre = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(pre, o, 64);
      if (lane >= o) pre += t;
    }
    const uint32_t total = __shfl(pre, 63, 64);
    pre -= len;
    for (uint32_t c0 = 0; c0 < total; c0 += 64) {
      const uint32_t c = c0 + lane;
      // the row holding candidate c: the last lane whose prefix is <= c
      int lo = 0;
#pragma unroll
      for (int step = 32; step > 0; step >>= 1) {
        const uint32_t p = __shfl(pre, lo + step, 64);
        if (p <= c) lo += step;
      }
      const uint32_t o = c - __shfl(pre, lo, 64);
      const uint32_t b1 = __shfl(a1, lo, 64), m1 = __shfl(n1, lo, 64);
      const uint32_t b2 = __shfl(a2, lo, 64);
      const bool valid = c < total;
      f(valid ? (o < m1 ? b1 + o : b2 + (o - m1)) : 0u, valid);
    }
  }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
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
// (grid-stride: one atomic per block)
template <class R>
__global__ void __launch_bounds__(kBlock) k_max_bits(const R* __restrict__ a, int64_t n,
                                                     unsigned long long* __restrict__ cnt,
                                                     int slot) {
  unsigned long long b = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const double v = (double)a[i];
    // non-finite or non-positive values are reported as +infinity
    const unsigned long long t = (v > 0.0 && v < 1e300)
                                     ? (unsigned long long)__double_as_longlong(v)
                                     : 0x7ff0000000000000ull;
    b = t > b ? t : b;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(b, o, 64);
    b = t > b ? t : b;
  }
  __shared__ unsigned long long red[kBlock / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) b = red[w] > b ? red[w] : b;
    if (b) atomicMax(cnt_at(cnt, slot), b);
  }
}

// rank[perm[q]] = q: the sorted position of every caller index
__global__ void __launch_bounds__(kBlock) k_dep_rank(const uint32_t* __restrict__ perm, int64_t n,
                                                     uint32_t* __restrict__ rank) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q < n) rank[perm[q]] = (uint32_t)q;
}

// the gas in sorted order: x, y, z, h, the volume (-1 when the particle may
// not receive: metallicity above z_max or mass above m_max) and 1 / h; read
// in caller order, written at the sorted position
template <class R>
__global__ void __launch_bounds__(kBlock) k_dep_pack(const uint32_t* __restrict__ rank,
                                                     const double* __restrict__ xg, int64_t ng,
                                                     const R* __restrict__ hg,
                                                     const R* __restrict__ Vg,
                                                     const R* __restrict__ mg,
                                                     const R* __restrict__ mZg, double z_max,
                                                     double m_max, double4* __restrict__ p4,
                                                     double2* __restrict__ pv) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= ng) return;
  const int64_t q = rank[j];
  const double h = (double)hg[j];
  p4[q] = make_double4(xg[j], xg[ng + j], xg[2 * ng + j], h);
  const double m = (double)mg[j];
  const bool ok = (double)mZg[j] <= z_max * m && m <= m_max;
  pv[q] = make_double2(ok ? (double)Vg[j] : -1.0, 1.0 / h);
}

constexpr int kWaves = kBlock / 64;  // sources per block in the source passes
template <class R, int K>
__global__ void __launch_bounds__(kBlock)
    k_dep_volume(PointGrid gas, const double* __restrict__ xs,
                 int64_t ns, double self_frac, double n_h_s, R* __restrict__ Vs,
                 R* __restrict__ hs) {
  const int64_t s = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (s >= ns) return;  // whole waves
  double sum = 0.0;
  const double sx = xs[s], sy = xs[ns + s], sz = xs[2 * ns + s];
  // every gas particle that can reach the source lies within the largest gas h
  wave_near(gas, sx, sy, sz, gas.hmax, [&](uint32_t q, bool valid) {
    if (!valid) return;
    const double4 b = gas.p4[q];
    const double r2 = min_image2(sx, sy, sz, b, gas);
    if (r2 < b.w * b.w) sum += kernel_W_inv<K>(sqrt(r2), gas.pv[q].y);
  });
  sum = wave_sum(sum);
  double V = 0.0, h = 0.0;
  if (sum > 0.0) {
    V = (1.0 - self_frac) / sum;
    h = n_h_s * cbrt(V);
  }
  if ((threadIdx.x & 63) == 0) {
    Vs[s] = (R)V;
    hs[s] = (R)h;
  }
}

// receivers kept per source by the normalisation pass (more: the pair pass
// walks that source's cells again)
constexpr int kSlot = 64;

// A_s and the number of receivers of every source; the largest h_s (double
// bits, CNT_HMAX_OUT_BITS) and the total receiver count (CNT_PAIRS_GATHER).
// The first kSlot receivers (gas caller index) go to the source's slot, in
// traversal order.
template <class R, int K>
__global__ void __launch_bounds__(kBlock)
    k_dep_norm(PointGrid gas, const double* __restrict__ xs,
               int64_t ns, const R* __restrict__ hs, const R* __restrict__ dM,
               const R* __restrict__ dMZ, const R* __restrict__ dE, const R* __restrict__ vs,
               R* __restrict__ As, double4* __restrict__ sp, uint32_t* __restrict__ npair,
               uint32_t* __restrict__ slot, unsigned long long* __restrict__ cnt) {
  const int64_t s = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (s >= ns) return;  // whole waves
  const double h = (double)hs[s];
  const int lane = threadIdx.x & 63;
  double sum = 0.0;
  uint32_t c = 0;  // receivers so far (the same in every lane)
  uint32_t* my_slot = slot + s * kSlot;
  // beyond half the box the nearest image is not unique: the host rejects
  // the call, and the search here is skipped
  const double sx = xs[s], sy = xs[ns + s], sz = xs[2 * ns + s];
  const double inv_h = 1.0 / h;
  if (h > 0.0 && h < 0.5 * gas.box)
    wave_near(gas, sx, sy, sz, h, [&](uint32_t q, bool valid) {
      bool in = false;
      if (valid) {
        const double r2 = min_image2(sx, sy, sz, gas.p4[q], gas);
        const double V = gas.pv[q].x;
        in = r2 < h * h && V >= 0.0;
        if (in) sum += V * kernel_W_inv<K>(sqrt(r2), inv_h);
      }
      const unsigned long long m = __ballot(in);
      const uint32_t at = c + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      if (in && at < (uint32_t)kSlot) my_slot[at] = gas.perm[q];
      c += (uint32_t)__popcll(m);
    });
  sum = wave_sum(sum);
  if (lane == 0) {
    const bool on = sum > 0.0;
    const R A = (R)(on ? 1.0 / sum : 0.0);
    As[s] = A;
    npair[s] = on ? c : 0u;
    if (on) {
      // what every receiver reads: position and 1 / h_s; A_s times the mass,
      // metal mass and energy handed over; A_s dM times the velocity
      const double a = (double)A, am = a * (double)dM[s];
      sp[3 * s] = make_double4(sx, sy, sz, inv_h);
      sp[3 * s + 1] = make_double4(am, a * (double)dMZ[s], a * (double)dE[s], 0.0);
      sp[3 * s + 2] = make_double4(am * (double)vs[s], am * (double)vs[ns + s],
                                   am * (double)vs[2 * ns + s], 0.0);
    }
    unsigned long long hb = (unsigned long long)__double_as_longlong(h);
    if (hb) atomicMax(cnt_at(cnt, CNT_HMAX_OUT_BITS), hb);
    if (on) atomicAdd(cnt_at(cnt, CNT_PAIRS_GATHER), (unsigned long long)c);
  }
}

// writes each source's receivers (gas index, source index) at its offset, in
// the traversal order of k_dep_norm: copied from the source's slot, or, for
// a source with more than kSlot receivers, found by the same traversal
template <class R>
__global__ void __launch_bounds__(kBlock)
    k_dep_pairs(PointGrid gas, const double* __restrict__ xs,
                int64_t ns, const R* __restrict__ hs, const uint32_t* __restrict__ npair,
                const uint32_t* __restrict__ slot, const uint32_t* __restrict__ off,
                uint32_t* __restrict__ pj, uint32_t* __restrict__ ps) {
  const int64_t s = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (s >= ns) return;  // whole waves
  const uint32_t c = npair[s];
  if (c == 0) return;
  const uint32_t o = off[s];
  const int lane = threadIdx.x & 63;
  if (c <= (uint32_t)kSlot) {
    if ((uint32_t)lane < c) {
      pj[o + lane] = slot[s * kSlot + lane];
      ps[o + lane] = (uint32_t)s;
    }
    return;
  }
  const double h = (double)hs[s];
  uint32_t t = 0;  // pairs written so far (the same in every lane)
  const double sx = xs[s], sy = xs[ns + s], sz = xs[2 * ns + s];
  wave_near(gas, sx, sy, sz, h, [&](uint32_t q, bool valid) {
    bool in = false;
    if (valid) in = min_image2(sx, sy, sz, gas.p4[q], gas) < h * h && gas.pv[q].x >= 0.0;
    const unsigned long long m = __ballot(in);
    const uint32_t at = t + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (in && at < c) {
      pj[o + at] = gas.perm[q];
      ps[o + at] = (uint32_t)s;
    }
    t += (uint32_t)__popcll(m);
  });
}

// every gas particle sums its (source-ordered) contributions and grows
template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_dep_apply(
    const double* __restrict__ xg, int64_t ng, const R* __restrict__ Vg, R* __restrict__ mg,
    R* __restrict__ vg, R* __restrict__ mZg, R* __restrict__ ug, const double4* __restrict__ sp,
    const uint32_t* __restrict__ first, const uint32_t* __restrict__ ps, double box) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= ng) return;
  const uint32_t q0 = first[j], q1 = first[j + 1];
  if (q0 == q1) return;
  const double Vj = (double)Vg[j];
  const double xj = xg[j], yj = xg[ng + j], zj = xg[2 * ng + j], inv_box = 1.0 / box;
  double dm = 0.0, dmz = 0.0, de = 0.0, dp[3] = {0.0, 0.0, 0.0};
  for (uint32_t q = q0; q < q1; ++q) {
    const int64_t s = ps[q];
    const double4 a = sp[3 * s], b = sp[3 * s + 1], c = sp[3 * s + 2];
    double tx = a.x - xj, ty = a.y - yj, tz = a.z - zj;
    tx -= box * rint(tx * inv_box);
    ty -= box * rint(ty * inv_box);
    tz -= box * rint(tz * inv_box);
    const double f = Vj * kernel_W_inv<K>(sqrt(tx * tx + ty * ty + tz * tz), a.w);
    dm += f * b.x;
    dmz += f * b.y;
    de += f * b.z;
    dp[0] += f * c.x;
    dp[1] += f * c.y;
    dp[2] += f * c.z;
  }
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
  const int64_t blocks = std::min<int64_t>(grid_for(n), 2048);
  hipLaunchKernelGGL(k_max_bits<R>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a, n, cnt, slot);
}

#define CRK_DEP_DISPATCH(kernel, KFN, count, ...)                                           \
  do {                                                                                      \
    if ((kernel) == 0)                                                                      \
      hipLaunchKernelGGL((KFN<R, 0>), dim3(grid_for(count)), dim3(kBlock), 0, s, __VA_ARGS__); \
    else                                                                                    \
      hipLaunchKernelGGL((KFN<R, 1>), dim3(grid_for(count)), dim3(kBlock), 0, s, __VA_ARGS__); \
  } while (0)

template <class R>
void launch_dep_pack(const uint32_t* perm, uint32_t* rank, const double* xg, int64_t ng,
                     const R* hg, const R* Vg, const R* mg, const R* mZg, double z_max,
                     double m_max, void* p4, void* pv, hipStream_t s) {
  hipLaunchKernelGGL(k_dep_rank, dim3(grid_for(ng)), dim3(kBlock), 0, s, perm, ng, rank);
  hipLaunchKernelGGL(k_dep_pack<R>, dim3(grid_for(ng)), dim3(kBlock), 0, s, rank, xg, ng, hg, Vg,
                     mg, mZg, z_max, m_max, (double4*)p4, (double2*)pv);
}

template <class R>
void launch_dep_volume(int kernel, const DepGrid& d, const double* xs, int64_t ns, double self_frac, double n_h_s, R* Vs, R* hs, hipStream_t s) {
  PointGrid g{d.G, d.box, 1.0 / d.box, d.hmax, d.start, d.perm, (const double4*)d.p4,
              (const double2*)d.pv};
  CRK_DEP_DISPATCH(kernel, k_dep_volume, ns * 64, g, xs, ns, self_frac, n_h_s, Vs, hs);
}

template <class R>
void launch_dep_norm(int kernel, const DepGrid& d, const double* xs, int64_t ns, const R* hs,
                     const R* dM, const R* dMZ, const R* dE, const R* vs, R* As, void* sp,
                     uint32_t* npair, uint32_t* slot, unsigned long long* cnt, hipStream_t s) {
  PointGrid g{d.G, d.box, 1.0 / d.box, d.hmax, d.start, d.perm, (const double4*)d.p4,
              (const double2*)d.pv};
  CRK_DEP_DISPATCH(kernel, k_dep_norm, ns * 64, g, xs, ns, hs, dM, dMZ, dE, vs, As,
                   (double4*)sp, npair, slot, cnt);
}

template <class R>
void launch_dep_pairs(const DepGrid& d, const double* xs, int64_t ns, const R* hs,
                      const uint32_t* npair, const uint32_t* slot, const uint32_t* off,
                      uint32_t* pj, uint32_t* ps, hipStream_t s) {
  PointGrid g{d.G, d.box, 1.0 / d.box, d.hmax, d.start, d.perm, (const double4*)d.p4,
              (const double2*)d.pv};
  hipLaunchKernelGGL(k_dep_pairs<R>, dim3(grid_for(ns * 64)), dim3(kBlock), 0, s, g, xs, ns, hs,
                     npair, slot, off, pj, ps);
}

template <class R>
void launch_dep_apply(int kernel, const double* xg, int64_t ng, const R* Vg, R* mg, R* vg, R* mZg,
                      R* ug, const void* sp, const uint32_t* first, const uint32_t* ps, double box,
                      hipStream_t s) {
  CRK_DEP_DISPATCH(kernel, k_dep_apply, ng, xg, ng, Vg, mg, vg, mZg, ug, (const double4*)sp, first,
                   ps, box);
}

#define CRK_DEP_INSTANTIATE(R)                                                                 \
  template void launch_max_bits<R>(const R*, int64_t, unsigned long long*, int, hipStream_t);  \
  template void launch_dep_pack<R>(const uint32_t*, uint32_t*, const double*, int64_t,       \
                                   const R*, const R*, const R*, const R*, double, double,     \
                                   void*, void*, hipStream_t);                                 \
  template void launch_dep_volume<R>(int, const DepGrid&, const double*, int64_t, double,     \
                                     double, R*, R*, hipStream_t);                             \
  template void launch_dep_norm<R>(int, const DepGrid&, const double*, int64_t, const R*,     \
                                   const R*, const R*, const R*, const R*, R*, void*,          \
                                   uint32_t*, uint32_t*, unsigned long long*, hipStream_t);    \
  template void launch_dep_pairs<R>(const DepGrid&, const double*, int64_t, const R*,         \
                                    const uint32_t*, const uint32_t*, const uint32_t*,         \
                                    uint32_t*, uint32_t*, hipStream_t);                        \
  template void launch_dep_apply<R>(int, const double*, int64_t, const R*, R*, R*, R*, R*,    \
                                    const void*, const uint32_t*, const uint32_t*, double,     \
                                    hipStream_t);
CRK_DEP_INSTANTIATE(float)
CRK_DEP_INSTANTIATE(double)

}  // namespace crk
