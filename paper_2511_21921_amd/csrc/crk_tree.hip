// Neighbour search for strongly clustered particle sets.
//
// When smoothing lengths span orders of magnitude (gas clumps in a
// cosmological volume), a cell list sized to the largest h puts whole clumps
// into single cells. This path instead sorts the particles along a Morton
// curve over a 1024^3 lattice (positions are kept as lattice coordinates
// plus FP32/FP64 offsets from the lattice-cell centre), takes every wave of 64
// consecutive particles as a leaf, and builds an implicit binary tree of leaf
// boxes with the largest h below each node. A wave walks the tree without a
// stack (wave-uniform control flow) and reads each overlapping leaf as one
// coalesced 64-particle tile that is broadcast to its lanes, exactly as the
// cell-list path reads its row segments.
#include "crk_passes.h"

namespace crk {
namespace {

__device__ inline uint32_t spread10(uint32_t v) {
  v &= 1023u;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ inline double wrap01(double xa, double L) {
  double t = xa - L * floor(xa / L);
  if (t >= L) t -= L;
  if (t < 0.0) t = 0.0;
  return t;
}

__global__ void __launch_bounds__(kBlock) k_morton(const double* __restrict__ x, int64_t n,
                                                   double L, uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double inv = 1024.0 / L;
  uint32_t c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int k = (int)(wrap01(x[a * n + i], L) * inv);
    c[a] = (uint32_t)(k < 1024 ? k : 1023);
  }
  keys[i] = spread10(c[0]) | (spread10(c[1]) << 1) | (spread10(c[2]) << 2);
  vals[i] = (uint32_t)i;
}

// Leaf boxes (absolute positions, FP32) and the largest h of each leaf.
template <class R>
__global__ void __launch_bounds__(kBlock) k_leaf_boxes(State<R> S, const R* __restrict__ h) {
  const int64_t leaf = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int nleaf = S.lvl_cnt[0];
  if (leaf >= nleaf) return;
  const int64_t b = leaf * 64, e = (b + 64 < S.n) ? b + 64 : S.n;
  float lo[3] = {3e30f, 3e30f, 3e30f}, hi[3] = {-3e30f, -3e30f, -3e30f}, hm = 0.f;
  for (int64_t s = b; s < e; ++s) {
    const uint32_t c3 = S.cell3[s];
    const R4<R> p = S.pos4[s];
    const float c[3] = {(float)(c3 & 1023u), (float)((c3 >> 10) & 1023u), (float)(c3 >> 20)};
    const float xi[3] = {(float)p.x, (float)p.y, (float)p.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float v = (c[a] + 0.5f) * (float)S.ell + xi[a];
      lo[a] = fminf(lo[a], v);
      hi[a] = fmaxf(hi[a], v);
    }
    hm = fmaxf(hm, (float)h[s]);
  }
  S.nlo[leaf] = make_float4(lo[0], lo[1], lo[2], hm);
  S.nhi[leaf] = make_float4(hi[0], hi[1], hi[2], 0.f);
}

__global__ void __launch_bounds__(kBlock) k_tree_up(float4* nlo, float4* nhi, int off_c,
                                                    int cnt_c, int off_p, int cnt_p) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= cnt_p) return;
  float4 lo = nlo[off_c + 2 * k], hi = nhi[off_c + 2 * k];
  if (2 * k + 1 < cnt_c) {
    const float4 l2 = nlo[off_c + 2 * k + 1], h2 = nhi[off_c + 2 * k + 1];
    lo = make_float4(fminf(lo.x, l2.x), fminf(lo.y, l2.y), fminf(lo.z, l2.z), fmaxf(lo.w, l2.w));
    hi = make_float4(fmaxf(hi.x, h2.x), fmaxf(hi.y, h2.y), fmaxf(hi.z, h2.z), 0.f);
  }
  nlo[off_p + k] = lo;
  nhi[off_p + k] = hi;
}

// First candidate radius of every particle from the density of its leaf:
// h0 = n_h (leaf box volume / leaf count)^(1/3), and the fixed h when h is
// an input.
template <class R>
__global__ void __launch_bounds__(kBlock) k_init_radius(State<R> S, int h_mode) {
  const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (s >= S.n) return;
  R r;
  if (h_mode == 0) {
    r = S.hbuf[s];
  } else {
    const int64_t leaf = s >> 6;
    const float4 lo = S.nlo[leaf], hi = S.nhi[leaf];
    const int64_t cnt = ((leaf + 1) * 64 < S.n ? (leaf + 1) * 64 : S.n) - leaf * 64;
    const double pad = 0.5 * S.ell_d;  // a leaf of coincident lattice cells has no volume
    const double vol = ((double)(hi.x - lo.x) + pad) * ((double)(hi.y - lo.y) + pad) *
                       ((double)(hi.z - lo.z) + pad);
    const double h0 = cbrt(S.n_h3 * vol / (double)cnt);
    r = (R)fmin(h0, 0.45 * S.box);
  }
  S.rad[s] = r;
  S.rlo[s] = R(0);
  S.rhi[s] = R(0);
  S.todo[s] = 1;
}

__device__ inline float box_gap2(float4 alo, float4 ahi, float4 blo, float4 bhi, float L) {
  const float al[3] = {alo.x, alo.y, alo.z}, ah[3] = {ahi.x, ahi.y, ahi.z};
  const float bl[3] = {blo.x, blo.y, blo.z}, bh[3] = {bhi.x, bhi.y, bhi.z};
  float g2 = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float best = 3e30f;
#pragma unroll
    for (int k = -1; k <= 1; ++k) {
      const float sh = (float)k * L;
      const float g = fmaxf(0.f, fmaxf(bl[a] + sh - ah[a], al[a] - (bh[a] + sh)));
      best = fminf(best, g);
    }
    g2 += best * best;
  }
  return g2;
}

// Stackless walk of the implicit binary tree for the wave's own leaf. A node
// is entered when its box comes within radius of the leaf box, radius =
// max(qr, node h_max) when use_node_h, else qr. f(leaf) is called for every
// leaf reached. All control flow is wave-uniform.
template <class R, class F>
__device__ inline void tree_walk(const State<R>& S, int64_t wave, float qr, bool use_node_h,
                                 F&& f) {
  const float4 qlo = S.nlo[wave], qhi = S.nhi[wave];
  const float L = (float)S.box;
  const int top = S.nlevels - 1;
  int level = top, k = 0;
  while (true) {
    bool visit = false;
    if (k < S.lvl_cnt[level]) {
      const float4 lo = S.nlo[S.lvl_off[level] + k], hi = S.nhi[S.lvl_off[level] + k];
      float r = use_node_h ? fmaxf(qr, lo.w) : qr;
      r = r * 1.00001f + 4e-6f * L;  // conservative against FP32 rounding of the boxes
      visit = box_gap2(qlo, qhi, lo, hi, L) < r * r;
    }
    if (visit && level > 0) {
      --level;
      k = 2 * k;
      continue;
    }
    if (visit) f(k);
    while (level < top && (k & 1)) {
      k >>= 1;
      ++level;
    }
    if (level == top) break;
    ++k;
  }
}

// Lattice separation x_ij from the lane's (pi, ci) and a candidate (pj, cj).
template <class R>
__device__ inline void lattice_sep(const State<R>& S, const R4<R>& pi, uint32_t a,
                                   const R4<R>& pj, uint32_t b, R x[3]) {
  const int G = S.G, half = S.G >> 1;
  int d[3] = {(int)(a & 1023u) - (int)(b & 1023u),
              (int)((a >> 10) & 1023u) - (int)((b >> 10) & 1023u),
              (int)(a >> 20) - (int)(b >> 20)};
#pragma unroll
  for (int t = 0; t < 3; ++t) d[t] = d[t] < -half ? d[t] + G : (d[t] >= half ? d[t] - G : d[t]);
  x[0] = (pi.x - pj.x) + R(d[0]) * S.ell;
  x[1] = (pi.y - pj.y) + R(d[1]) * S.ell;
  x[2] = (pi.z - pj.z) + R(d[2]) * S.ell;
}

// Calls f(j, pj, mj, cj) for every particle of leaf k, broadcast to the wave.
template <class R, class F>
__device__ inline void leaf_tile(const State<R>& S, int64_t leaf, F&& f) {
  const int lane = threadIdx.x & 63;
  const int64_t b = leaf * 64;
  const int cnt = (int)((b + 64 < S.n ? b + 64 : S.n) - b);
  const int64_t jl = b + (lane < cnt ? lane : 0);
  const R4<R> pl = S.pos4[jl];
  const R ml = S.mass[jl];
  const int cl = (int)S.cell3[jl];
  for (int t = 0; t < cnt; ++t) {
    R4<R> pj;
    pj.x = bcast(pl.x, t);
    pj.y = bcast(pl.y, t);
    pj.z = bcast(pl.z, t);
    pj.w = bcast(pl.w, t);
    f((uint32_t)(b + t), pj, bcast(ml, t), (uint32_t)bcast(cl, t));
  }
}

// Candidates of every unsolved particle within its own radius ri. When they
// overflow the capacity, counts at seven smaller radii ri q^k (k = 1..7, down
// to the largest radius rlo known to be too small for the h root, else by
// 0.6 per step) give the largest radius that fits, which the next round uses.
// Only when nothing above rlo fits is the capacity itself too small: the
// count just above rlo is reported for the host to grow it.
template <class R>
__global__ void __launch_bounds__(kBlock) k_candidates_tree(State<R> S) {
  constexpr int kBins = 7;
  const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = s < S.n;
  const int64_t sc = active ? s : 0;
  const bool mine = active && S.todo[sc];
  const R ri = mine ? S.rad[sc] : R(0);
  float qr = (float)ri;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) qr = fmaxf(qr, __shfl_xor(qr, o, 64));
  qr = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(qr)));
  const int64_t wave = __builtin_amdgcn_readfirstlane((int)(s >> 6));
  unsigned long long retry = 0, ovf = 0;
  if (__ballot(mine) != 0ull) {
    const R4<R> pi = S.pos4[sc];
    const uint32_t ci = S.cell3[sc];
    const R mi_inv = R(1) / S.mass[sc];
    const R r2cap = ri * ri;
    const int64_t qs = scratch_slot(S, sc);
    const R lo = (mine && S.shrink) ? S.rlo[sc] : R(0);
    const double q = lo > R(0) ? pow((double)lo / (double)ri, 1.0 / (kBins + 1)) : 0.6;
    R rk[kBins], t2[kBins];
    int hk[kBins];
    {
      double r = (double)ri;
#pragma unroll
      for (int k = 0; k < kBins; ++k) {
        r *= q;
        rk[k] = (R)r;
        t2[k] = rk[k] * rk[k];
        hk[k] = 0;
      }
    }
    const int cap = S.scr_cap;
    int cnt = 0;
    Stage4<R> sr, sm;
    tree_walk(S, wave, qr, false, [&](int64_t leaf) {
      leaf_tile(S, leaf, [&](uint32_t j, const R4<R>& pj, R mj, uint32_t cj) {
        if (!mine || j == (uint32_t)s) return;
        R x[3];
        lattice_sep(S, pi, ci, pj, cj, x);
        const R r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        if (r2 < r2cap) {
          if (cnt < cap) {
            const int slot = cnt & 3;
            sr.put(slot, Sc<R>::sqrt(r2));
            sm.put(slot, mj * mi_inv);
            if (slot == 3) {
              sr.flush(S.scr_r, qs, cap, cnt);
              if (!S.equal_mass) sm.flush(S.scr_m, qs, cap, cnt);
            }
          }
          ++cnt;
#pragma unroll
          for (int k = 0; k < kBins; ++k) hk[k] += r2 < t2[k] ? 1 : 0;
        }
      });
    });
    if (mine) {
      if (cnt > cap && S.shrink) {
        int kfit = -1;
#pragma unroll
        for (int k = kBins - 1; k >= 0; --k)
          if (hk[k] <= cap) kfit = k;  // counts fall with k: the first fit is the largest
        if (kfit >= 0) {
          S.rad[s] = rk[kfit];
          S.rhi[s] = kfit == 0 ? ri : rk[kfit - 1];
        } else {
          const R last = rk[kBins - 1];
          S.rhi[s] = last;
          if (lo > R(0) && last < R(1.01) * lo) {
            S.rad[s] = last;  // fits once the capacity has grown
            ovf = (unsigned long long)hk[kBins - 1];
          } else {
            S.rad[s] = lo > R(0) ? Sc<R>::sqrt(lo * last) : R(0.6) * last;
          }
        }
        S.ccnt[s] = -1;
        retry = 1;
      } else if (cnt > cap) {
        S.ccnt[s] = cap;  // fixed h: the host grows the capacity and reruns
        ovf = (unsigned long long)cnt;
      } else {
        if (cnt & 3) {
          sr.flush(S.scr_r, qs, cap, cnt - 1);
          if (!S.equal_mass) sm.flush(S.scr_m, qs, cap, cnt - 1);
        }
        S.ccnt[s] = cnt;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    retry += __shfl_xor(retry, o, 64);
    const unsigned long long a = __shfl_xor(ovf, o, 64);
    ovf = a > ovf ? a : ovf;
  }
  if ((threadIdx.x & 63) == 0) {
    if (retry) atomicAdd(&S.cnt[CNT_RETRY], retry);
    if (ovf) atomicMax(&S.cnt[CNT_SCR_OVERFLOW], ovf);
  }
}

// Symmetric neighbour lists r_ij < max(h_i, h_j) by a walk with node radius
// max(own leaf h_max, node h_max). Two passes over the same walk: COUNT stores
// the list lengths and every wave's capacity in chunk rows (its longest list,
// rounded up to 4 entries); after a scan of those into S.grow / S.srow, FILL
// writes the entries. Both passes visit the same pairs in the same order.
template <class R, bool FILL>
__global__ void __launch_bounds__(kBlock) k_nlist_tree(State<R> S, uint32_t* __restrict__ wg,
                                                       uint32_t* __restrict__ ws) {
  const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if ((s & ~(int64_t)63) >= S.n) return;  // whole wave past the end: it has no leaf
  const bool active = s < S.n;
  const int64_t sc = active ? s : 0;
  const R4<R> pi = S.pos4[sc];
  const uint32_t ci = S.cell3[sc];
  const R hi2 = pi.w * pi.w;
  const int64_t wave = __builtin_amdgcn_readfirstlane((int)(s >> 6));
  const float qr = S.nlo[wave].w;  // largest h of the wave's own leaf
  int ng = 0, ns = 0, cap = 0, scap = 0;
  int64_t gb = 0, sb = 0;
  if (FILL) {
    cap = (int)(S.grow[wave + 1] - S.grow[wave]) * 4;
    scap = (int)(S.srow[wave + 1] - S.srow[wave]) * 4;
    gb = slot_base(S.grow[wave], s);
    sb = slot_base(S.srow[wave], s);
  }
  Stage4<uint32_t> sg, ss;
  tree_walk(S, wave, qr, true, [&](int64_t leaf) {
    leaf_tile(S, leaf, [&](uint32_t j, const R4<R>& pj, R mj, uint32_t cj) {
      (void)mj;
      if (!active || j == (uint32_t)s) return;
      R x[3];
      lattice_sep(S, pi, ci, pj, cj, x);
      const R r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      const uint32_t e = j << kCodeBits;
      if (r2 * hi2 < R(1)) {
        if (FILL && ng < cap) {
          sg.put(ng & 3, e);
          if ((ng & 3) == 3) sg.flush_at(S.nlist, gb, ng);
        }
        ++ng;
      } else if (r2 * (pj.w * pj.w) < R(1)) {
        if (FILL && ns < scap) {
          ss.put(ns & 3, e);
          if ((ns & 3) == 3) ss.flush_at(S.slist, sb, ns);
        }
        ++ns;
      }
    });
  });
  if (FILL) {
    if (active) {
      const int gst = ng < cap ? ng : cap, sst = ns < scap ? ns : scap;
      if (gst & 3) sg.flush_at(S.nlist, gb, gst - 1);
      if (sst & 3) ss.flush_at(S.slist, sb, sst - 1);
    }
    return;
  }
  unsigned long long g = 0, f = 0;
  int mg = 0, ms = 0;
  if (active) {
    S.ng[s] = ng;
    S.ns[s] = ns;
    g = (unsigned long long)ng;
    f = (unsigned long long)(ng + ns);
    mg = ng;
    ms = ns;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    g += __shfl_xor(g, o, 64);
    f += __shfl_xor(f, o, 64);
    mg = max(mg, __shfl_xor(mg, o, 64));
    ms = max(ms, __shfl_xor(ms, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    wg[wave] = (uint32_t)((mg + 3) >> 2);
    ws[wave] = (uint32_t)((ms + 3) >> 2);
    if (g) atomicAdd(&S.cnt[CNT_PAIRS_GATHER], g);
    if (f) atomicAdd(&S.cnt[CNT_PAIRS_FORCE], f);
  }
}

}  // namespace

void launch_morton(const double* x, int64_t n, double box, uint32_t* keys, uint32_t* vals,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_morton, dim3(grid_for(n)), dim3(kBlock), 0, s, x, n, box, keys, vals);
}

template <class R>
void launch_tree_build(const State<R>& S, const R* h, const int* host_off, const int* host_cnt,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_leaf_boxes<R>, dim3(grid_for(host_cnt[0])), dim3(kBlock), 0, s, S, h);
  for (int l = 0; l + 1 < S.nlevels; ++l)
    hipLaunchKernelGGL(k_tree_up, dim3(grid_for(host_cnt[l + 1])), dim3(kBlock), 0, s, S.nlo,
                       S.nhi, host_off[l], host_cnt[l], host_off[l + 1], host_cnt[l + 1]);
}

template <class R>
void launch_init_radius(const State<R>& S, int h_mode, hipStream_t s) {
  hipLaunchKernelGGL(k_init_radius<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S, h_mode);
}

template <class R>
void launch_candidates_tree(const State<R>& S, hipStream_t s) {
  hipLaunchKernelGGL(k_candidates_tree<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S);
}

template <class R>
void launch_nlist_tree(const State<R>& S, bool fill, uint32_t* wg, uint32_t* ws, hipStream_t s) {
  if (fill)
    hipLaunchKernelGGL((k_nlist_tree<R, true>), dim3(grid_for(S.n)), dim3(kBlock), 0, s, S, wg,
                       ws);
  else
    hipLaunchKernelGGL((k_nlist_tree<R, false>), dim3(grid_for(S.n)), dim3(kBlock), 0, s, S, wg,
                       ws);
}

#define CRK_INSTANTIATE_TREE(R)                                                               \
  template void launch_tree_build<R>(const State<R>&, const R*, const int*, const int*,      \
                                     hipStream_t);                                           \
  template void launch_init_radius<R>(const State<R>&, int, hipStream_t);                    \
  template void launch_candidates_tree<R>(const State<R>&, hipStream_t);                     \
  template void launch_nlist_tree<R>(const State<R>&, bool, uint32_t*, uint32_t*, hipStream_t);

CRK_INSTANTIATE_TREE(float)
CRK_INSTANTIATE_TREE(double)

}  // namespace crk
