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

__global__ void __launch_bounds__(kBlock) k_morton(const double* __restrict__ x, int64_t n,
                                                   double L, uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals) {
  const int64_t i = particle_id();
  if (i >= n) return;
  const double inv = 1024.0 / L;
  uint32_t c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c[a] = (uint32_t)cell_coord(wrap_pos(x[a * n + i], L), inv, 1024);
  }
  keys[i] = spread10(c[0]) | (spread10(c[1]) << 1) | (spread10(c[2]) << 2);
  vals[i] = (uint32_t)i;
}

// Leaf boxes (absolute positions, FP32) and the largest h of each leaf.
template <class R>
__global__ void __launch_bounds__(kBlock) k_leaf_boxes(State<R> S, const R* __restrict__ h) {
  const int64_t leaf = particle_id();
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

// Absolute position of a sorted particle (FP32, the rounding of the node
// boxes) from its lattice cell and its offset from the cell centre.
template <class R>
__device__ inline void abs_pos(const State<R>& S, uint32_t c3, const R4<R>& p, float a[3]) {
  const float ell = (float)S.ell;
  a[0] = ((float)(c3 & 1023u) + 0.5f) * ell + (float)p.x;
  a[1] = ((float)((c3 >> 10) & 1023u) + 0.5f) * ell + (float)p.y;
  a[2] = ((float)(c3 >> 20) + 0.5f) * ell + (float)p.z;
}

// Squared periodic distance from point a to the box [lo, hi] (both in the
// unit cell [0, L] up to rounding).
__device__ inline float point_gap2(const float a[3], float4 lo, float4 hi, float L) {
  const float l[3] = {lo.x, lo.y, lo.z}, h[3] = {hi.x, hi.y, hi.z};
  float g2 = 0.f;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const float d1 = l[t] - a[t], d2 = a[t] - h[t];
    float g = 0.f;
    if (d1 > 0.f) g = fminf(d1, a[t] + L - h[t]);       // left of the box, or its image
    else if (d2 > 0.f) g = fminf(d2, l[t] + L - a[t]);  // right of the box, or its image
    g2 += g * g;
  }
  return g2;
}

// Radius widened against the FP32 rounding of positions and node boxes.
__device__ inline float pad_radius(float r, float L) { return r * 1.00001f + 4e-6f * L; }

// Stackless walk of the implicit binary tree. A node is entered when
// need(lo, hi) holds for any lane of the wave (each lane tests its own
// sphere against the node box); f(leaf) is called for every leaf reached.
// All control flow is wave-uniform.
template <class R, class N, class F>
__device__ inline void tree_walk(const State<R>& S, N&& need, F&& f) {
  const int top = S.nlevels - 1;
  int level = top, k = 0;
  while (true) {
    bool visit = false;
    if (k < S.lvl_cnt[level]) {
      const int64_t node = S.lvl_off[level] + k;
      visit = __ballot(need(S.nlo[node], S.nhi[node])) != 0ull;
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

// First candidate radius of every particle, kept small so that the first
// walk stays cheap (particles whose h root lies beyond it grow it in later
// rounds): the least of the h that the target count would need at the
// density of the particle's 8 nearest leaf-mates, n_h r_8 (4 pi / 24)^(1/3),
// at the density of its leaf box, and 1.5x that of the mean density. The
// caller's h is kept instead (x1.05) when it lies within a factor 2 of that
// estimate (a previous step's h). With fixed h the radius is h.
template <class R>
__global__ void __launch_bounds__(kBlock) k_init_radius(State<R> S, int h_mode) {
  const int64_t s = particle_id();
  if ((s & ~(int64_t)63) >= S.n) return;
  const bool active = s < S.n;
  const int64_t sc = active ? s : 0;
  const int64_t leaf = sc >> 6;
  R r = S.hbuf[sc];
  if (h_mode != 0) {
    const R4<R> pi = S.pos4[sc];
    const uint32_t ci = S.cell3[sc];
    float d[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) d[t] = 3e30f;
    leaf_tile(S, leaf, [&](uint32_t j, const R4<R>& pj, R mj, uint32_t cj) {
      (void)mj;
      if (j == (uint32_t)sc) return;
      R x[3];
      lattice_sep(S, pi, ci, pj, cj, x);
      float v = (float)(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
#pragma unroll
      for (int t = 0; t < 8; ++t) {  // keep the 8 smallest, sorted
        const float lo = fminf(d[t], v);
        v = fmaxf(d[t], v);
        d[t] = lo;
      }
    });
    const int64_t b = leaf * 64;
    const int64_t cnt = (b + 64 < S.n ? b + 64 : S.n) - b;
    const float4 lo = S.nlo[leaf], hi = S.nhi[leaf];
    const double pad = 0.5 * S.ell_d;  // coincident lattice cells have no volume
    const double vol = ((double)(hi.x - lo.x) + pad) * ((double)(hi.y - lo.y) + pad) *
                       ((double)(hi.z - lo.z) + pad);
    double est = cbrt(S.n_h3 * vol / (double)cnt);
    if (cnt >= 9)  // (4 pi / 24)^(1/3)
      est = fmin(est, cbrt(S.n_h3) * sqrt((double)d[7]) * 0.80599597700823482);
    est = fmin(est, 1.5 * cbrt(S.n_h3 / (double)S.n) * S.box);
    const double g = (double)r;
    const double h0 = (g > 0.5 * est && g < 2.0 * est) ? 1.05 * g : est;
    r = (R)fmin(h0, 0.45 * S.box);
  }
  if (active) {
    S.rad[s] = r;
    S.need[s] = S.scr_cap;
    S.todo[s] = 1;
  }
}

// Candidates of every unsolved particle within its own radius ri, written to
// its scratch slot. A particle whose candidates overflow its capacity also
// gets, from the same walk, the counts and the h-root test
// f(r) = C (w(0) + sum_j (m_j/m_i) w(r_ij / r)) - n_h^3 > 0 at ri and at four
// smaller radii ri 0.75^k: the next round uses the smallest of these radii
// that holds the root, with exactly the capacity its count needs, or, when
// none does, a radius grown from the count. With fixed h only the capacity
// is raised. Sums over the candidates that did fit are taken afterwards from
// the scratch, so particles that fit pay only for the counts.
template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_candidates_tree(State<R> S) {
  constexpr int kBins = 4;
  const int64_t s = particle_id();
  const bool active = s < S.n;
  const int64_t sc = active ? s : 0;
  const bool mine = active && S.todo[sc];
  const R ri = mine ? S.rad[sc] : R(0);
  unsigned long long retry = 0;
  if (__ballot(mine) != 0ull) {
    const R4<R> pi = S.pos4[sc];
    const uint32_t ci = S.cell3[sc];
    const R mi_inv = R(1) / S.mass[sc];
    const R r2cap = ri * ri;
    int cap = 0;
    int64_t base = 0;
    if (mine) base = scratch_base(S, sc, cap);
    R rk[kBins], t2[kBins], ik[kBins], fk[kBins];
    int hk[kBins];
    {
      R r = ri;
#pragma unroll
      for (int k = 0; k < kBins; ++k) {
        r *= R(0.75);
        rk[k] = r;
        t2[k] = r * r;
        ik[k] = R(1) / r;
        fk[k] = R(Shape<K>::w0);
        hk[k] = 0;
      }
    }
    const R iri = mine ? R(1) / ri : R(0);
    R fi = R(Shape<K>::w0);
    // adds the f sums of one candidate at ri and at the smaller radii
    auto add_sums = [&](R r, R mr) {
      R w, dw;
      Shape<K>::eval(r * iri, w, dw);
      fi += mr * w;
#pragma unroll
      for (int k = 0; k < kBins; ++k) {
        Shape<K>::eval(r * ik[k], w, dw);
        fk[k] += mr * w;
      }
    };
    int cnt = 0;
    Stage4<R> sr, sm;
    float P[3];
    abs_pos(S, ci, pi, P);
    const float L = (float)S.box;
    const float rp = mine ? pad_radius((float)ri, L) : -1.f;
    const float rp2 = rp * rp;
    auto need = [&](float4 lo, float4 hi) { return mine && point_gap2(P, lo, hi, L) < rp2; };
    tree_walk(S, need, [&](int64_t leaf) {
      leaf_tile(S, leaf, [&](uint32_t j, const R4<R>& pj, R mj, uint32_t cj) {
        if (!mine || j == (uint32_t)s) return;
        R x[3];
        lattice_sep(S, pi, ci, pj, cj, x);
        const R r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        if (r2 < r2cap) {
          const R r = Sc<R>::sqrt(r2);
          const R mr = mj * mi_inv;
          if (cnt < cap) {
            const int slot = cnt & 3;
            sr.put(slot, r);
            sm.put(slot, mr);
            if (slot == 3) {
              sr.flush_group(S.scr_r, base, cnt);
              if (!S.equal_mass) sm.flush_group(S.scr_m, base, cnt);
            }
          } else if (S.shrink) {
            add_sums(r, mr);
          }
          ++cnt;
#pragma unroll
          for (int k = 0; k < kBins; ++k) hk[k] += r2 < t2[k] ? 1 : 0;
        }
      });
    });
    if (mine) {
      if (cnt > cap && S.shrink) {
        for (int k = 0; k < cap; ++k) {  // the candidates that fitted
          const int64_t e = group_at(base, k);
          add_sums(S.scr_r[e], S.equal_mass ? R(1) : S.scr_m[e]);
        }
        const R C = R(Shape<K>::C), n_h3 = R(S.n_h3);
        R rs = R(0);
        int ns = 0;
        if (C * fi - n_h3 > R(0)) {
          rs = ri;
          ns = cnt;
        }
#pragma unroll
        for (int k = 0; k < kBins; ++k)  // radii fall with k: keep the last one holding the root
          if (C * fk[k] - n_h3 > R(0)) {
            rs = rk[k];
            ns = hk[k];
          }
        if (rs > R(0)) {
          S.rad[s] = rs;
          S.need[s] = ((ns > 4 ? ns : 4) + 3) & ~3;
        } else {  // the root lies beyond ri
          const double g = grow_factor(S.n_h3, cnt);
          S.rad[s] = (R)((double)ri * g);
          S.need[s] = need_after_growth(cnt, g);
        }
        S.ccnt[s] = -1;
        retry = 1;
      } else if (cnt > cap) {
        S.need[s] = (cnt + 3) & ~3;  // fixed h: exactly the capacity it needs
        S.ccnt[s] = -1;
        retry = 1;
      } else {
        if (cnt & 3) {
          sr.flush_group(S.scr_r, base, cnt - 1);
          if (!S.equal_mass) sm.flush_group(S.scr_m, base, cnt - 1);
        }
        S.ccnt[s] = cnt;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) retry += __shfl_xor(retry, o, 64);
  if ((threadIdx.x & 63) == 0 && retry) atomicAdd(cnt_at(S.cnt, CNT_RETRY), retry);
}

// Capacity of every group of 64 scratch slots, in rows of 16-entry groups:
// the largest request of the unsolved particles ranked into it (rows zeroed
// beforehand).
template <class R>
__global__ void __launch_bounds__(kBlock) k_slot_rows(State<R> S, uint32_t* __restrict__ rows) {
  const int64_t s = particle_id();
  if (s >= S.n || !S.todo[s]) return;
  atomicMax(&rows[S.cslot[s] >> 6], (uint32_t)((S.need[s] + 15) >> 4));
}

// Gather lists r_ij < h_i by a walk with each lane's own h. Every wave's
// capacity (S.grow) comes from an upper bound of its counts; the counts are
// stored in full, so an overflow (the host checks the largest) can be
// rerun with exact capacities. Entries come in ascending j.
template <class R>
__global__ void __launch_bounds__(kBlock) k_gather_tree(State<R> S) {
  const int64_t s = particle_id();
  if ((s & ~(int64_t)63) >= S.n) return;  // whole wave past the end: it has no leaf
  const bool active = s < S.n;
  const int64_t sc = active ? s : 0;
  const R4<R> pi = S.pos4[sc];
  const uint32_t ci = S.cell3[sc];
  const R hi2 = pi.w * pi.w;
  const int64_t wave = sc >> 6;
  const int cap = (int)(S.grow[wave + 1] - S.grow[wave]) * 4;
  const int64_t gb = slot_base(S.grow[wave], sc);
  int ng = 0;
  Stage4<uint32_t> sg;
  float P[3];
  abs_pos(S, ci, pi, P);
  const float L = (float)S.box;
  const float rp = active ? pad_radius((float)(R(1) / pi.w), L) : -1.f;
  const float rp2 = rp * rp;
  auto need = [&](float4 lo, float4 hi) { return active && point_gap2(P, lo, hi, L) < rp2; };
  tree_walk(S, need, [&](int64_t leaf) {
    leaf_tile(S, leaf, [&](uint32_t j, const R4<R>& pj, R mj, uint32_t cj) {
      (void)mj;
      if (!active || j == (uint32_t)s) return;
      R x[3];
      lattice_sep(S, pi, ci, pj, cj, x);
      const R r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      if (r2 * hi2 < R(1)) {
        if (ng < cap) {
          sg.put(ng & 3, j << kCodeBits);
          if ((ng & 3) == 3) sg.flush_at(S.nlist, gb, ng);
        }
        ++ng;
      }
    });
  });
  unsigned long long g = 0, ovf = 0;
  if (active) {
    const int st = ng < cap ? ng : cap;
    if (st & 3) sg.flush_at(S.nlist, gb, st - 1);
    S.ng[s] = ng;
    g = (unsigned long long)ng;
    if (ng > cap) ovf = (unsigned long long)ng;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    g += __shfl_xor(g, o, 64);
    const unsigned long long a = __shfl_xor(ovf, o, 64);
    ovf = a > ovf ? a : ovf;
  }
  if ((threadIdx.x & 63) == 0) {
    if (g) atomicAdd(cnt_at(S.cnt, CNT_PAIRS_GATHER), g);
    if (ovf) atomicMax(cnt_at(S.cnt, CNT_LIST_OVERFLOW), ovf);
  }
}

// Per-wave capacity in chunk rows from per-particle counts: the largest of
// its lanes' cnt[s] + extra, rounded up to 4 entries.
__global__ void __launch_bounds__(kBlock) k_wave_rows(const int* __restrict__ cnt, int64_t n,
                                                      int extra, uint32_t* __restrict__ rows) {
  const int64_t s = particle_id();
  if ((s & ~(int64_t)63) >= n) return;
  int c = s < n ? cnt[s] + extra : 0;
  c = c > 0 ? c : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c = max(c, __shfl_xor(c, o, 64));
  if ((threadIdx.x & 63) == 0) rows[s >> 6] = (uint32_t)((c + 3) >> 2);
}

// Scatter-only part of the symmetric list by transposing the gather lists:
// j belongs to i's scatter-only list when i is in j's gather list
// (r_ij < h_j) but j is not in i's (r_ij >= h_i). The separation is the same
// expression with both signs flipped, so r_ij^2 is bit-identical from both
// sides. COUNT adds to ns[i]; FILL appends j at fillc[i] (unordered, sorted
// afterwards).
template <class R, bool FILL>
__global__ void __launch_bounds__(kBlock) k_scatter_tree(State<R> S, int* __restrict__ fillc) {
  const int64_t s = particle_id();
  if (s >= S.n) return;
  const R4<R> pj = S.pos4[s];
  const uint32_t cj = S.cell3[s];
  const int64_t w = s >> 6;
  const int ng = S.ng[s];
  const int64_t gb = slot_base(S.grow[w], s);
  for (int k = 0; k < ng; ++k) {
    const uint32_t i = S.nlist[slot_at(gb, k)] >> kCodeBits;
    const R4<R> pi = S.pos4[i];
    R x[3];
    lattice_sep(S, pi, S.cell3[i], pj, cj, x);
    const R r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    if (!(r2 * (pi.w * pi.w) < R(1))) {
      if (FILL) {
        const int t = atomicAdd(&fillc[i], 1);
        const int64_t wi = (int64_t)(i >> 6);
        const int scap = (int)(S.srow[wi + 1] - S.srow[wi]) * 4;
        if (t < scap) S.slist[slot_at(slot_base(S.srow[wi], i), t)] = (uint32_t)s << kCodeBits;
      } else {
        atomicAdd(&S.ns[i], 1);
      }
    }
  }
}

// Sorts every scatter-only list by j (insertion sort; the lists are short),
// giving the order a walk would produce and making runs reproducible; counts
// the force pairs.
template <class R>
__global__ void __launch_bounds__(kBlock) k_scatter_sort(State<R> S) {
  const int64_t s = particle_id();
  unsigned long long f = 0;
  if (s < S.n) {
    const int64_t w = s >> 6;
    const int scap = (int)(S.srow[w + 1] - S.srow[w]) * 4;
    const int ns = S.ns[s] < scap ? S.ns[s] : scap;
    const int64_t sb = slot_base(S.srow[w], s);
    for (int a = 1; a < ns; ++a) {
      const uint32_t v = S.slist[slot_at(sb, a)];
      int b = a - 1;
      while (b >= 0 && S.slist[slot_at(sb, b)] > v) {
        S.slist[slot_at(sb, b + 1)] = S.slist[slot_at(sb, b)];
        --b;
      }
      S.slist[slot_at(sb, b + 1)] = v;
    }
    f = (unsigned long long)(S.ng[s] + S.ns[s]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o, 64);
  if ((threadIdx.x & 63) == 0 && f) atomicAdd(cnt_at(S.cnt, CNT_PAIRS_FORCE), f);
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
void launch_candidates_tree(const State<R>& S, int kernel, hipStream_t s) {
  if (kernel == 0)
    hipLaunchKernelGGL((k_candidates_tree<R, 0>), dim3(grid_for(S.n)), dim3(kBlock), 0, s, S);
  else
    hipLaunchKernelGGL((k_candidates_tree<R, 1>), dim3(grid_for(S.n)), dim3(kBlock), 0, s, S);
}

template <class R>
void launch_slot_rows(const State<R>& S, uint32_t* rows, hipStream_t s) {
  hipLaunchKernelGGL(k_slot_rows<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S, rows);
}

template <class R>
void launch_gather_tree(const State<R>& S, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_tree<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S);
}

void launch_wave_rows(const int* cnt, int64_t n, int extra, uint32_t* rows, hipStream_t s) {
  hipLaunchKernelGGL(k_wave_rows, dim3(grid_for(n)), dim3(kBlock), 0, s, cnt, n, extra, rows);
}

template <class R>
void launch_scatter_tree(const State<R>& S, bool fill, int* fillc, hipStream_t s) {
  if (fill) {
    hipLaunchKernelGGL((k_scatter_tree<R, true>), dim3(grid_for(S.n)), dim3(kBlock), 0, s, S,
                       fillc);
    hipLaunchKernelGGL(k_scatter_sort<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S);
  } else {
    hipLaunchKernelGGL((k_scatter_tree<R, false>), dim3(grid_for(S.n)), dim3(kBlock), 0, s, S,
                       fillc);
  }
}

#define CRK_INSTANTIATE_TREE(R)                                                               \
  template void launch_tree_build<R>(const State<R>&, const R*, const int*, const int*,      \
                                     hipStream_t);                                           \
  template void launch_init_radius<R>(const State<R>&, int, hipStream_t);                    \
  template void launch_candidates_tree<R>(const State<R>&, int, hipStream_t);                \
  template void launch_slot_rows<R>(const State<R>&, uint32_t*, hipStream_t);               \
  template void launch_gather_tree<R>(const State<R>&, hipStream_t);                         \
  template void launch_scatter_tree<R>(const State<R>&, bool, int*, hipStream_t);

CRK_INSTANTIATE_TREE(float)
CRK_INSTANTIATE_TREE(double)

}  // namespace crk
