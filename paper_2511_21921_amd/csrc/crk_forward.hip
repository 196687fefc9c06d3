// Forward CRKSPH pair passes on gfx950.
//
// One lane owns one cell-sorted particle i; a 64-lane wave owns 64
// consecutive particles of the cell order, so the lanes of a wave share
// almost all of their neighbours and the gathered neighbour records stay in
// the vector L1 / L2. Pair arithmetic is in Real (FP32 or FP64); the 3x3
// second-moment solve and the force / energy accumulators are FP64.
//
// Passes (paper: arXiv:2511.21921):
//   k_hsolve   smoothing length from the Thacker fixed point Delta_N = 1
//              (App. A.3, eq. thacker) and the volume of App. A.2, eq. Vg;
//   k_volume   the volume alone for fixed h;
//   k_nlist    symmetric neighbour list r_ij < max(h_i, h_j);
//   k_moments  geometric moments and the corrections A, B, grad A, grad B of
//              W^R_ij = A_i (1 + B_i . x_ij) W_ij(h_i) (App. A.1, eq. RK);
//   k_density  density (Sec. 2.5.1, eq. rhow), velocity gradient
//              (App. A.1, eq. gradv), ideal-gas EOS and the relaxation flag
//              exp(|div v| dt) > 8 (App. A.1);
//   k_force    pairwise momentum and compatible energy with the limited
//              artificial viscosity (Sec. 2.1).
#include "crk_passes.h"

namespace crk {
namespace {

template <class R>
__device__ inline R dot3(const R a[3], const R b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// ------------------------------------------------------------- inputs ----

// Grid-stride over the inputs; each block reduces in LDS and issues one
// atomic per counter (per-wave atomics on four shared addresses serialise).
template <class R>
__global__ void __launch_bounds__(kBlock) k_check_inputs(const double* __restrict__ x,
                                                         const R* __restrict__ h,
                                                         const R* __restrict__ m,
                                                         const R* __restrict__ u, int64_t n,
                                                         unsigned long long* cnt) {
  unsigned long long hb = 0, bad = 0, mb = 0, ib = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const double hv = (double)h[i], mv = (double)m[i], uv = (double)u[i];
    const double x0 = fabs(x[i]), x1 = fabs(x[n + i]), x2 = fabs(x[2 * n + i]);
    const bool ok = hv > 0.0 && mv > 0.0 && uv > 0.0 && hv < 1e300 && uv < 1e300 && mv < 1e300 &&
                    x0 < 1e300 && x1 < 1e300 && x2 < 1e300;
    bad += ok ? 0 : 1;
    if (ok) {
      const unsigned long long a = dbits(hv), b = dbits(mv), c = dbits(1.0 / mv);
      hb = a > hb ? a : hb;  // positive doubles order as their bit patterns
      mb = b > mb ? b : mb;
      ib = c > ib ? c : ib;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    bad += __shfl_xor(bad, o, 64);
    unsigned long long t = __shfl_xor(hb, o, 64);
    hb = t > hb ? t : hb;
    t = __shfl_xor(mb, o, 64);
    mb = t > mb ? t : mb;
    t = __shfl_xor(ib, o, 64);
    ib = t > ib ? t : ib;
  }
  __shared__ unsigned long long part[kBlock / 64][4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[w][0] = hb;
    part[w][1] = bad;
    part[w][2] = mb;
    part[w][3] = ib;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kBlock / 64; ++k) {
      hb = part[k][0] > hb ? part[k][0] : hb;
      bad += part[k][1];
      mb = part[k][2] > mb ? part[k][2] : mb;
      ib = part[k][3] > ib ? part[k][3] : ib;
    }
    if (hb) atomicMax(cnt_at(cnt, CNT_HMAX_BITS), hb);
    if (bad) atomicAdd(cnt_at(cnt, CNT_BAD_INPUT), bad);
    if (mb) atomicMax(cnt_at(cnt, CNT_MMAX_BITS), mb);
    if (ib) atomicMax(cnt_at(cnt, CNT_MINVMAX_BITS), ib);
  }
}

__global__ void __launch_bounds__(kBlock) k_keys(const double* __restrict__ x, int64_t n,
                                                 double L, int G, uint32_t* __restrict__ keys,
                                                 uint32_t* __restrict__ vals) {
  const int64_t i = particle_id();
  if (i >= n) return;
  const double inv = (double)G / L;
  int c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c[a] = cell_coord(wrap_pos(x[a * n + i], L), inv, G);
  }
  keys[i] = ((uint32_t)c[2] * G + (uint32_t)c[1]) * G + (uint32_t)c[0];
  vals[i] = (uint32_t)i;
}

// The kept cell list against new positions: every sorted slot s recomputes
// the cell of its particle perm[s] and counts it in CNT_MOVED when that
// differs from keys[s] (the list then no longer sorts these positions).
__global__ void __launch_bounds__(kBlock) k_keys_check(const double* __restrict__ x, int64_t n,
                                                       double L, int G,
                                                       const uint32_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ perm,
                                                       unsigned long long* __restrict__ cnt) {
  const int64_t s = particle_id();
  if ((s & ~(int64_t)63) >= n) return;
  unsigned long long moved = 0;
  if (s < n) {
    const double inv = (double)G / L;
    const uint32_t p = perm[s];
    if (p < (uint32_t)n) {
      int c[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) c[a] = cell_coord(wrap_pos(x[a * n + p], L), inv, G);
      moved = ((uint32_t)c[2] * G + (uint32_t)c[1]) * G + (uint32_t)c[0] != keys[s] ? 1ull : 0ull;
    } else {
      moved = 1;  // not a permutation of these particles
    }
  }
  wave_add_u64(cnt_at(cnt, CNT_MOVED), moved);
}

// Hierarchy: the particles (caller order) active at the end of substep jend,
// counted in CNT_ACTIVE.
__global__ void __launch_bounds__(kBlock) k_count_active(const int* __restrict__ levels,
                                                         int64_t n, int lmax, int64_t jend,
                                                         unsigned long long* __restrict__ cnt) {
  const int64_t p = particle_id();
  if ((p & ~(int64_t)63) >= n) return;
  unsigned long long a = 0;
  if (p < n) a = (jend & ((1ll << (lmax - levels[p])) - 1)) == 0 ? 1ull : 0ull;
  wave_add_u64(cnt_at(cnt, CNT_ACTIVE), a);
}

// The sorted slots of the active particles, appended to list (a wave's at
// once; the order is not kept).
template <class R>
__global__ void __launch_bounds__(kBlock) k_active_list(State<R> S, uint32_t* __restrict__ list) {
  const int64_t s = particle_id();
  if ((s & ~(int64_t)63) >= S.n) return;
  const bool a = s < S.n && !is_passive(S, s);
  const uint64_t b = __ballot(a);
  if (b == 0ull) return;
  const int lane = threadIdx.x & 63;
  unsigned long long base = 0;
  if (lane == __ffsll((unsigned long long)b) - 1)
    base = atomicAdd(S.cnt + CNT_ACTLIST * kCntSpread, (unsigned long long)__popcll(b));
  base = __shfl(base, __ffsll((unsigned long long)b) - 1, 64);
  if (a) list[base + __popcll(b & ((1ull << lane) - 1ull))] = (uint32_t)s;
}

// cell_start[c] = first sorted position whose key is >= c, for c = 0..ncell
// (a binary search of the sorted keys per cell; no atomics). The largest
// occupancy start[c + 1] - start[c] is reduced per block into one atomic;
// a block whose largest occupancy exceeds occ_limit raises CNT_TOO_DENSE.
__global__ void __launch_bounds__(kBlock) k_cell_bounds(const uint32_t* __restrict__ keys,
                                                        int64_t n, int64_t ncell,
                                                        uint32_t* __restrict__ start,
                                                        unsigned long long occ_limit,
                                                        unsigned long long* __restrict__ cnt) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  auto lower = [&](int64_t v) {
    int64_t lo = 0, hi = n;  // keys[lo - 1] < v <= keys[hi]
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)keys[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  unsigned long long occ = 0;
  if (c <= ncell) {
    const int64_t b = lower(c);
    start[c] = (uint32_t)b;
    if (c < ncell) occ = (unsigned long long)(lower(c + 1) - b);
  }
  __shared__ unsigned long long red[kBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(occ, o, 64);
    occ = t > occ ? t : occ;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = occ;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int w = 0; w < kBlock / 64; ++w) m = red[w] > m ? red[w] : m;
    if (m) atomicMax(cnt_at(cnt, CNT_CELL_MAX), m);
    if (m > occ_limit) atomicMax(cnt_at(cnt, CNT_TOO_DENSE), 1ull);
  }
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_gather(State<R> S, const double* __restrict__ x,
                                                   const R* __restrict__ v,
                                                   const R* __restrict__ m,
                                                   const R* __restrict__ u,
                                                   const R* __restrict__ h) {
  const int64_t s = particle_id();
  if (s >= S.n) return;
  const int64_t n = S.n;
  const uint32_t p = S.perm[s];
  if (p >= (uint32_t)n) return;
  int c[3];
  R xi[3];
  const double inv = (double)S.G / S.box;
  // the cell list's own cell of the slot (on a kept list the particle may
  // have left it: its offset from that cell's centre is then beyond half a
  // side, but the walk stays consistent with the list)
  const uint32_t key = S.lattice ? 0u : S.keys[s];
  const uint32_t G = (uint32_t)S.G;
  const uint32_t kz = key / (G * G);
  const int kc[3] = {(int)(key % G), (int)((key / G) % G), (int)(kz < G ? kz : G - 1)};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double t = wrap_pos(x[a * n + p], S.box);
    c[a] = S.lattice ? cell_coord(t, inv, S.G) : kc[a];
    xi[a] = (R)(t - ((double)c[a] + 0.5) * S.ell_d);
  }
  R4<R> q;
  q.x = xi[0];
  q.y = xi[1];
  q.z = xi[2];
  q.w = R(c[0]);  // the cell's x index until the h solve is done (then 1/h)
  S.pos(s) = q;
  R4<R> w;
  w.x = v[p];
  w.y = v[n + p];
  w.z = v[2 * n + p];
  w.w = R(0);
  S.vel(s) = w;
  S.mass[s] = m[p];
  S.uu[s] = u[p];
  S.hbuf[s] = h[p];
  S.cell3[s] = (uint32_t)c[0] | ((uint32_t)c[1] << 10) | ((uint32_t)c[2] << 20);
}

// ---------------------------------------------------------- candidates ----
// One traversal of the stencil cells per particle collects every j != i
// with r_ij < rcap (rcap >= every h, at most two cell sides), storing the
// packed entry and (r, m_j / m_i). The h solve, the fixed-h volume and the
// neighbour list all read this list instead of walking the cells again.
// EM: all masses equal (m_j / m_i = 1 is not stored).

template <class R, bool EM>
__global__ void __launch_bounds__(kBlock) k_candidates(State<R> S) {
  // a speculative cell list found too dense (strong clustering): the host
  // discards this evaluation and takes the tree, so skip the quadratic walk
  if (__ballot(S.cnt[CNT_TOO_DENSE * kCntSpread + (threadIdx.x & 63)] != 0ull)) return;
  const int64_t s = particle_id();
  if (s >= S.n) return;
  if (is_passive(S, s)) {  // no sums of its own this substep
    S.ccnt[s] = 0;
    return;
  }
  if (S.act) return;  // a listed active particle: k_candidates_rows
  const R4<R> pi = S.pos(s);
  const R mi_inv = EM ? R(1) : R(1) / S.mass[s];
  const R rc2 = S.rcap * S.rcap;
  int cap;
  const int64_t base = scratch_base(S, s, cap);
  int cnt = 0;
  // Each lane walks the cells of its own 5x5x5 stencil that come within the
  // candidate radius of the particle (planes and rows beyond it are skipped).
  // In a row the cells within reach form one run of dx (the distance to a
  // cell is convex in dx), and consecutive cells of a row hold consecutive
  // particles, so the run is one contiguous range of particles (split where
  // the row wraps), read four at a time with the loads in flight together.
  // A particle's cell within the run comes from the x index kept in its position record's w.
  // Accepted candidates are shifted into four registers per array and
  // written as one 16-byte store per array every fourth one: the lanes of a
  // wave run their tests in step, so whatever the accept path costs, the
  // wave pays at almost every test (shifting needs no slot selects).
  const uint32_t c3 = S.cell3[s];
  const int G = S.G;
  const int cx = (int)(c3 & 1023u), cy = (int)((c3 >> 10) & 1023u), cz = (int)(c3 >> 20);
  const R ell = S.ell;
  const uint32_t n = (uint32_t)S.n;
  uint32_t e0 = 0, e1 = 0, e2 = 0, e3 = 0;
  R r0 = R(0), r1 = R(0), r2s = R(0), r3 = R(0);
  R m0 = R(0), m1 = R(0), m2 = R(0), m3 = R(0);
  auto flush = [&](int k) {  // the chunk of entries k & ~3 .. (k & ~3) + 3
    const int64_t q = group_at(base, k & ~3);
    *reinterpret_cast<uint4*>(S.cand + q) = make_uint4(e0, e1, e2, e3);
    R4<R> t;
    t.x = r0;
    t.y = r1;
    t.z = r2s;
    t.w = r3;
    *reinterpret_cast<R4<R>*>(S.scr_r + q) = t;
    if (!EM) {
      t.x = m0;
      t.y = m1;
      t.z = m2;
      t.w = m3;
      *reinterpret_cast<R4<R>*>(S.scr_m + q) = t;
    }
  };
  // squared distance from the particle to the slab of offset d along one axis
  auto gap2 = [&](R xi, int d) {
    const R lo = (R(d) - R(0.5)) * ell - xi, hi = xi - (R(d) + R(0.5)) * ell;
    const R g = lo > hi ? lo : hi;
    return g > R(0) ? g * g : R(0);
  };
  // cells dx = d0 .. d1 of the row, stored from cell c0 (x index x0) on; the
  // particle itself can only turn up in the row through its own cell
  auto walk = [&](uint32_t c0, int x0, int d0, int d1, int dy, int dz, auto own_row) {
    const uint32_t b = S.cell_start[c0];
    uint32_t e = S.cell_start[c0 + (uint32_t)(d1 - d0 + 1)];
    if (e > n) e = n;
    // x offset of cell x of the run: (x - x0 + d0) ell; stencil code likewise
    const int xoff = d0 - x0;
    const int code0 = (int)stencil_code(0, dy, dz);
    const R oy = R(dy) * ell, oz = R(dz) * ell;
    for (uint32_t j0 = b; j0 < e; j0 += 4) {
      R4<R> pj[4];
      R mj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t j = j0 + u < e ? j0 + u : e - 1;
        pj[u] = S.pos(j);
        if (!EM) mj[u] = S.mass[j];
      }
      __builtin_amdgcn_sched_barrier(0);  // keep the four loads ahead of their first use
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t j = j0 + u;
        const int dx = (int)pj[u].w + xoff;
        R x[3];
        x[0] = (pi.x - pj[u].x) - R(dx) * ell;
        x[1] = (pi.y - pj[u].y) - oy;
        x[2] = (pi.z - pj[u].z) - oz;
        const R r2 = dot3(x, x);
        bool ok = j < e && r2 < rc2;
        if (decltype(own_row)::value) ok = ok && !(j == (uint32_t)s && dx == 0);
        if (ok) {
          if (cnt < cap) {
            e0 = e1;
            e1 = e2;
            e2 = e3;
            e3 = (j << kCodeBits) | (uint32_t)(code0 + dx);
            r0 = r1;
            r1 = r2s;
            r2s = r3;
            r3 = Sc<R>::sqrt(r2);
            if (!EM) {
              m0 = m1;
              m1 = m2;
              m2 = m3;
              m3 = mj[u] * mi_inv;
            }
            if ((cnt & 3) == 3) flush(cnt);
          }
          ++cnt;
        }
      }
    }
  };
  for (int dz = -2; dz <= 2; ++dz) {
    const R gz = gap2(pi.z, dz);
    if (!(gz < rc2)) continue;
    const int z = wrap_cell(cz + dz, G);
    for (int dy = -2; dy <= 2; ++dy) {
      const R gyz = gz + gap2(pi.y, dy);
      if (!(gyz < rc2)) continue;
      const int y = wrap_cell(cy + dy, G);
      const uint32_t rowbase = ((uint32_t)z * G + (uint32_t)y) * G;
      int dlo = 3, dhi = -3;
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx)
        if (gyz + gap2(pi.x, dx) < rc2) {
          dlo = dx < dlo ? dx : dlo;
          dhi = dx;
        }
      // the run split where the row wraps (G >= 2): x < 0, 0 <= x < G, x >= G
      const int a1 = min(dhi, -cx - 1);
      const int b0 = max(dlo, -cx), b1 = min(dhi, G - 1 - cx);
      const int c0 = max(dlo, G - cx);
      auto row = [&](auto own_row) {
        if (dlo <= a1)
          walk(rowbase + (uint32_t)(cx + dlo + G), cx + dlo + G, dlo, a1, dy, dz, own_row);
        if (b0 <= b1) walk(rowbase + (uint32_t)(cx + b0), cx + b0, b0, b1, dy, dz, own_row);
        if (c0 <= dhi)
          walk(rowbase + (uint32_t)(cx + c0 - G), cx + c0 - G, c0, dhi, dy, dz, own_row);
      };
      if (dy == 0 && dz == 0)
        row(std::true_type());
      else
        row(std::false_type());
    }
  }
  {
    // the last partial chunk: its m entries are the newest m in the registers
    const int st = cnt < cap ? cnt : cap, m = st & 3;
    if (m) {
      if (m == 1) {
        e0 = e3;
        r0 = r3;
        m0 = m3;
      } else if (m == 2) {
        e0 = e2; e1 = e3;
        r0 = r2s; r1 = r3;
        m0 = m2; m1 = m3;
      } else {
        e0 = e1; e1 = e2; e2 = e3;
        r0 = r1; r1 = r2s; r2s = r3;
        m0 = m1; m1 = m2; m2 = m3;
      }
      flush(st - 1);
    }
  }
  // only the stored entries are ever read; the overflow makes the host grow
  // the capacity and run the candidate pass again
  S.ccnt[s] = cnt < cap ? cnt : cap;
  if (cnt > cap) atomicMax(cnt_at(S.cnt, CNT_SCR_OVERFLOW), (unsigned long long)cnt);
}

// sum_k (m_k/m_i) w(r_k / h) over the candidates plus the self term w(0), and
// dsum = sum_k (m_k/m_i) w'(q_k) q_k. The list is read a 16-entry group at a
// time, its loads issued together.
template <class R, int K>
__device__ inline R candidate_sum(const State<R>& S, int64_t base, int cnt, R h, R& dsum) {
  const R hinv = R(1) / h;
  R sum = R(Shape<K>::w0), ds = R(0);
  for (int k = 0; k < cnt; k += 16) {
    const int64_t e = group_at(base, k);
    R rr[16], mm[16];
    load_group(S.scr_r + e, rr);
    if (!S.equal_mass) load_group(S.scr_m + e, mm);
    const int left = cnt - k;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      // entries past the count are moved outside the support (w = w' = 0)
      const bool in = t < left;
      const R q = in ? rr[t] * hinv : R(2);
      R w, dw;
      Shape<K>::eval(q, w, dw);
      const R mt = S.equal_mass ? R(1) : (in ? mm[t] : R(0));
      sum += mt * w;
      ds += mt * dw * q;
    }
  }
  dsum = ds;
  return sum;
}

// ------------------------------------------------------------- h solve ----
// f(h) = C (w(0) + sum_{j != i} (m_j/m_i) w(r_ij / h)) - n_h^3, which is
// h^3 sum_j (m_j/m_i) W(r_ij, h) - n_h^3: zero exactly when Delta_N = 1.
// f is non-decreasing in h; safeguarded Newton inside a bisection bracket,
// stopping when a Newton step falls below the tolerance.

// Cell path: a thread per particle (the tree path solves with k_hsolve_rows).
template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_hsolve(State<R> S) {
  const int64_t s = particle_id();
  unsigned long long iters = 0, unconv = 0, capped = 0, hbits = 0;
  if (s < S.n) {
    int scap;
    const int64_t q = scratch_base(S, s, scap);
    const int cnt = S.ccnt[s] < scap ? S.ccnt[s] : scap;
    const R C = R(Shape<K>::C);
    const R n_h3 = R(S.n_h3);
    const R Rcap = S.rcap;
    const R rtol = R(S.rtol);
    R h = first_h(S.hbuf[s], Rcap, cnt, S.n_h3);
    R dsum, sum = candidate_sum<R, K>(S, q, cnt, h, dsum);
    R f = C * sum - n_h3;
    // the bracket [0, Rcap] holds the root only if f(Rcap) > 0; that needs
    // its own pass, taken only when the starting h is below the root
    bool cap_hit = false;
    if (!(f > R(0))) {
      R ds2;
      cap_hit = !(C * candidate_sum<R, K>(S, q, cnt, Rcap, ds2) - n_h3 > R(0));
    }
    if (cap_hit) {
      capped = 1;  // the root lies beyond the candidate radius
    } else {
      R lo = R(0), hi = Rcap;
      bool conv = false;
      int it = 0;
      R hn = h;
      for (;;) {
        const R fp = -C * dsum / h;
        if (f > R(0)) hi = h; else lo = h;
        hn = R(0.5) * (lo + hi);
        if (fp > R(0)) {
          const R nt = h - f / fp;
          const R step = nt > h ? nt - h : h - nt;
          if (step <= rtol * h) {
            hn = nt < lo ? lo : (nt > hi ? hi : nt);
            conv = true;
            break;
          }
          if (nt > lo && nt < hi) hn = nt;
        }
        if (hi - lo <= rtol * hn) {
          conv = true;
          break;
        }
        if (++it >= S.max_iter) break;
        h = hn;
        sum = candidate_sum<R, K>(S, q, cnt, h, dsum);
        f = C * sum - n_h3;
      }
      iters = (unsigned long long)(it + 1);
      unconv = conv ? 0 : 1;
      // V at the final h from the last sums: the step is below the
      // tolerance, so the first-order term leaves an error of order rtol^2
      // (an unconverged h gets its own pass)
      const R sum_f = conv ? sum - dsum / h * (hn - h) : candidate_sum<R, K>(S, q, cnt, hn, dsum);
      S.hbuf[s] = hn;
      S.Vbuf[s] = hn * hn * hn / (C * sum_f);
      hbits = dbits((double)hn);
    }
  }
  wave_max_u64(cnt_at(S.cnt, CNT_H_ITER_MAX), iters);
  wave_add_u64(cnt_at(S.cnt, CNT_H_UNCONV), unconv);
  wave_add_u64(cnt_at(S.cnt, CNT_H_CAPPED), capped);
  wave_max_u64(cnt_at(S.cnt, CNT_HMAX_OUT_BITS), hbits);
}

// Fixed h: V_i = m_i / sum_j m_j W(r_ij, h_i), self term included.
template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_volume(State<R> S) {
  const int64_t s = particle_id();
  if (s >= S.n) return;
  if (is_passive(S, s)) return;  // V comes from the stored state (k_pack)
  if (S.act) return;             // a listed active particle: k_volume_rows
  const R h = S.hbuf[s];
  int scap;
  const int64_t base = scratch_base(S, s, scap);
  R dsum;
  const R sum = candidate_sum<R, K>(S, base, S.ccnt[s] < scap ? S.ccnt[s] : scap, h, dsum);
  S.Vbuf[s] = h * h * h / (R(Shape<K>::C) * sum);
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_pack(State<R> S, R* __restrict__ h_out,
                                                 R* __restrict__ V_out) {
  const int64_t s = particle_id();
  if (s >= S.n) return;
  const uint32_t p = S.perm[s];
  const bool pas = is_passive(S, s);
  const R h = S.hbuf[s], V = pas ? S.pV[p] : S.Vbuf[s];
  S.pos(s).w = R(1) / h;
  S.vel(s).w = V;
  if (!h_out || pas) return;  // an input still (a speculative forward), or stored
  h_out[p] = h;
  V_out[p] = V;
}

// --------------------------------------------------------- neighbour list --

template <class R>
__global__ void __launch_bounds__(kBlock) k_nlist(State<R> S) {
  const int64_t s = particle_id();
  unsigned long long g = 0, f = 0, ovf = 0, sovf = 0, cands = 0;
  // (a listed active particle: k_nlist_rows)
  if (s < S.n && !(S.act && !is_passive(S, s))) {
    // Classified by the stored candidate distance r: it is the same value
    // from both sides of a pair (the separation is computed with both signs
    // flipped), so j lands in i's scatter-only list exactly when i is in j's
    // gather list, and only h_j has to be gathered.
    const R hi = S.hbuf[s];
    int ng = 0, ns = 0;
    const int cap = S.list_cap, scap = S.slist_cap;
    Stage4<uint32_t> sg, ss;
    int ccap;
    const int64_t base = scratch_base(S, s, ccap);
    // passive particles keep no lists (their force is not summed)
    const int cc = is_passive(S, s) ? 0 : (S.ccnt[s] < ccap ? S.ccnt[s] : ccap);
    cands = (unsigned long long)cc;
    for (int k = 0; k < cc; k += 16) {
      const int64_t c = group_at(base, k);
      uint32_t ee[16];
      R rr[16], hj[16];
      load_group(S.cand + c, ee);
      load_group(S.scr_r + c, rr);
      // h_j only where the pair is not a gather pair of i, all loads at once
#pragma unroll
      for (int t = 0; t < 16; ++t)
        hj[t] = (k + t < cc && !(rr[t] < hi)) ? S.hbuf[ee[t] >> kCodeBits] : R(0);
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const bool in = k + t < cc;
        const uint32_t e = ee[t];
        if (in && rr[t] < hi) {
          if (ng < cap) {
            sg.put(ng & 3, e);
            if ((ng & 3) == 3) sg.flush(S.nlist, s, cap, ng);
          }
          ++ng;
          if (S.needed) S.needed[e >> kCodeBits] = 1;
        } else if (in && rr[t] < hj[t]) {
          if (ns < scap) {
            ss.put(ns & 3, e);
            if ((ns & 3) == 3) ss.flush(S.slist, s, scap, ns);
          }
          ++ns;
          if (S.needed) S.needed[e >> kCodeBits] = 1;
        }
      }
    }
    const int gst = ng < cap ? ng : cap, sst = ns < scap ? ns : scap;
    if (gst & 3) sg.flush(S.nlist, s, cap, gst - 1);
    if (sst & 3) ss.flush(S.slist, s, scap, sst - 1);
    S.ng[s] = ng;
    S.ns[s] = ns;
    g = (unsigned long long)ng;
    f = (unsigned long long)(ng + ns);
    if (ng > cap) ovf = (unsigned long long)ng;
    if (ns > scap) sovf = (unsigned long long)ns;
  }
  wave_add_u64(cnt_at(S.cnt, CNT_PAIRS_GATHER), g);
  wave_add_u64(cnt_at(S.cnt, CNT_PAIRS_FORCE), f);
  wave_add_u64(cnt_at(S.cnt, CNT_CANDIDATES), cands);
  wave_max_u64(cnt_at(S.cnt, CNT_LIST_OVERFLOW), ovf);
  wave_max_u64(cnt_at(S.cnt, CNT_SLIST_OVERFLOW), sovf);
}

// ------------------------------------------------ moments + corrections ----
// Moments over j with r_ij < h_i, self included (V_j, h_i fixed; d_g is
// the derivative with respect to the evaluation point x_i):
//   m0 = sum V W, m1_a = sum V x_a W, m2_ab = sum V x_a x_b W,
//   d_g m0 = sum V d_g W, d_g m1_a = delta_ag m0 + sum V x_a d_g W,
//   d_g m2_ab = delta_ag m1_b + delta_bg m1_a + sum V x_a x_b d_g W.
// Corrections from sum V W^R = 1 and sum V x W^R = 0:
//   B = -m2^-1 m1, A = 1 / (m0 + B.m1),
//   d_g B = -m2^-1 (d_g m1 + d_g m2 B), d_g A = -A^2 (d_g m0 + d_g B.m1 + B.d_g m1).

// Symmetric-pair index of (a, b) in (xx, xy, xz, yy, yz, zz).
__device__ inline constexpr int sym6(int a, int b) {
  return a <= b ? (a == 0 ? b : (a == 1 ? 2 + b : 5)) : (b == 0 ? a : (b == 1 ? 2 + a : 5));
}

template <class R>
struct Moments {
  R m0, m1[3], m2[6], dm0[3], X1[9], X2[18];
};

// The sums start from the self term (m0 = V_i W(0)) or from zero.
template <class R, int K>
__device__ __forceinline__ void moments_start(const State<R>& S, int64_t s, bool self,
                                              Moments<R>& M) {
  const R hinv = S.pos(s).w;
  const R C3 = R(Shape<K>::C) * hinv * hinv * hinv;
  M.m0 = self ? S.vel(s).w * C3 * R(Shape<K>::w0) : R(0);
#pragma unroll
  for (int t = 0; t < 3; ++t) M.m1[t] = M.dm0[t] = R(0);
#pragma unroll
  for (int t = 0; t < 6; ++t) M.m2[t] = R(0);
#pragma unroll
  for (int t = 0; t < 9; ++t) M.X1[t] = R(0);
#pragma unroll
  for (int t = 0; t < 18; ++t) M.X2[t] = R(0);
}

// Adds neighbour entry e of particle s (position pi, 1/h hinv, C h^-3 and
// C h^-4) to the sums.
template <class R, int K>
__device__ __forceinline__ void moment_term(const State<R>& S, int64_t s, const R4<R>& pi,
                                            R hinv, R C3, R C4, uint32_t e, Moments<R>& M) {
  const uint32_t j = e >> kCodeBits;
  const R4<R> pj = S.pos(j);
  const R Vj = S.vel(j).w;
  R x[3];
  pair_x(S, s, pi, pj, e, x);
  const R r2 = dot3(x, x);
  const R rinv = Sc<R>::rsqrt(r2);
  const R q = r2 * rinv * hinv;
  R w, dw;
  Shape<K>::eval(q, w, dw);
  const R VW = Vj * C3 * w;
  const R fg = Vj * C4 * dw * rinv;
  const R Vg[3] = {fg * x[0], fg * x[1], fg * x[2]};
  const R p6[6] = {x[0] * x[0], x[0] * x[1], x[0] * x[2], x[1] * x[1], x[1] * x[2], x[2] * x[2]};
  M.m0 += VW;
#pragma unroll
  for (int a = 0; a < 3; ++a) M.m1[a] += x[a] * VW;
#pragma unroll
  for (int t = 0; t < 6; ++t) M.m2[t] += p6[t] * VW;
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    M.dm0[g] += Vg[g];
#pragma unroll
    for (int a = 0; a < 3; ++a) M.X1[g * 3 + a] += x[a] * Vg[g];
#pragma unroll
    for (int t = 0; t < 6; ++t) M.X2[g * 6 + t] += p6[t] * Vg[g];
  }
}

template <class R, int K>
__device__ inline void accumulate_moments(const State<R>& S, int64_t s, Moments<R>& M) {
  const R4<R> pi = S.pos(s);
  const R hinv = pi.w;
  const R C3 = R(Shape<K>::C) * hinv * hinv * hinv;
  const R C4 = C3 * hinv;
  moments_start<R, K>(S, s, true, M);
  const NbrRef nb = nbr_ref(S, s);
  uint4 ebuf;
  const int ng = nb.ng;
  for (int k = 0; k < ng; ++k)
    moment_term<R, K>(S, s, pi, hinv, C3, C4, gather_entry(S, nb, k, ebuf), M);
}

// Sums of a 16-lane row, each lane taking the entries k = sub mod 16, then
// summed over the row (every lane ends with the row's sums).
template <class R, int K>
__device__ inline void accumulate_moments_row(const State<R>& S, int64_t s, int sub,
                                              Moments<R>& M) {
  const R4<R> pi = S.pos(s);
  const R hinv = pi.w;
  const R C3 = R(Shape<K>::C) * hinv * hinv * hinv;
  const R C4 = C3 * hinv;
  moments_start<R, K>(S, s, sub == 0, M);
  const NbrRef nb = nbr_ref(S, s);
  for (int k = sub; k < nb.ng; k += 16)
    moment_term<R, K>(S, s, pi, hinv, C3, C4, S.nlist[slot_at(nb.gb, k)], M);
  R* v = reinterpret_cast<R*>(&M);
#pragma unroll
  for (int t = 0; t < 40; ++t)
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) v[t] += __shfl_xor(v[t], o, 16);
}

// Full moment set (40 values, FP64) from the accumulated sums.
struct Mom64 {
  double m0, m1[3], m2[9], dm0[3], dm1[9], dm2[27];
};

template <class R>
__device__ inline void expand_moments(const Moments<R>& M, Mom64& D) {
  D.m0 = (double)M.m0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    D.m1[a] = (double)M.m1[a];
    D.dm0[a] = (double)M.dm0[a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) D.m2[a * 3 + b] = (double)M.m2[sym6(a, b)];
#pragma unroll
  for (int g = 0; g < 3; ++g)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      D.dm1[g * 3 + a] = (double)M.X1[g * 3 + a] + (a == g ? D.m0 : 0.0);
#pragma unroll
      for (int b = 0; b < 3; ++b)
        D.dm2[(g * 3 + a) * 3 + b] = (double)M.X2[g * 6 + sym6(a, b)] +
                                     (a == g ? D.m1[b] : 0.0) + (b == g ? D.m1[a] : 0.0);
    }
}

struct Corr64 {
  double A, B[3], dA[3], dB[9], inv[9];
  bool singular;
};

template <class R>
__device__ inline void solve_corrections(const Mom64& D, Corr64& o) {
  const double* m2 = D.m2;
  double cof[9];
  cof[0] = m2[4] * m2[8] - m2[5] * m2[7];
  cof[1] = m2[2] * m2[7] - m2[1] * m2[8];
  cof[2] = m2[1] * m2[5] - m2[2] * m2[4];
  cof[3] = m2[5] * m2[6] - m2[3] * m2[8];
  cof[4] = m2[0] * m2[8] - m2[2] * m2[6];
  cof[5] = m2[2] * m2[3] - m2[0] * m2[5];
  cof[6] = m2[3] * m2[7] - m2[4] * m2[6];
  cof[7] = m2[1] * m2[6] - m2[0] * m2[7];
  cof[8] = m2[0] * m2[4] - m2[1] * m2[3];
  const double det = m2[0] * cof[0] + m2[1] * cof[3] + m2[2] * cof[6];
  const double tr = fabs(m2[0]) + fabs(m2[4]) + fabs(m2[8]);
  o.singular = !(fabs(det) > SingularTol<R>::v * tr * tr * tr);
  if (o.singular) {
    o.A = 1.0;
#pragma unroll
    for (int t = 0; t < 3; ++t) o.B[t] = o.dA[t] = 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) o.dB[t] = o.inv[t] = 0.0;
    return;
  }
  const double id = 1.0 / det;
#pragma unroll
  for (int t = 0; t < 9; ++t) o.inv[t] = cof[t] * id;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    o.B[a] = -(o.inv[a * 3 + 0] * D.m1[0] + o.inv[a * 3 + 1] * D.m1[1] + o.inv[a * 3 + 2] * D.m1[2]);
  o.A = 1.0 / (D.m0 + o.B[0] * D.m1[0] + o.B[1] * D.m1[1] + o.B[2] * D.m1[2]);
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    double rhs[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      rhs[b] = D.dm1[g * 3 + b];
#pragma unroll
      for (int e = 0; e < 3; ++e) rhs[b] += D.dm2[(g * 3 + b) * 3 + e] * o.B[e];
    }
    double t = D.dm0[g];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      o.dB[g * 3 + a] = -(o.inv[a * 3 + 0] * rhs[0] + o.inv[a * 3 + 1] * rhs[1] +
                          o.inv[a * 3 + 2] * rhs[2]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) t += o.dB[g * 3 + a] * D.m1[a] + o.B[a] * D.dm1[g * 3 + a];
    o.dA[g] = -(o.A * o.A) * t;
  }
}

template <class R>
__device__ inline void store_kc(const State<R>& S, int64_t s, const Corr64& c) {
  // packed form: a = A, b = A B, c_g = dA_g + A B_g, M_ga = dA_g B_a + A dB_ga
  R v[16];
  v[0] = (R)c.A;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    v[1 + t] = (R)(c.A * c.B[t]);
    v[4 + t] = (R)(c.dA[t] + c.A * c.B[t]);
  }
#pragma unroll
  for (int g = 0; g < 3; ++g)
#pragma unroll
    for (int a = 0; a < 3; ++a) v[7 + g * 3 + a] = (R)(c.dA[g] * c.B[a] + c.A * c.dB[g * 3 + a]);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    R4<R> q;
    q.x = v[4 * t];
    q.y = v[4 * t + 1];
    q.z = v[4 * t + 2];
    q.w = v[4 * t + 3];
    S.kc4[4 * s + t] = q;
  }
}

// Corrections from the sums of particle s: stored (moments when kept,
// packed corrections) and written in caller order; 1 when the second moment
// was singular.
template <class R>
__device__ inline unsigned long long moments_finish(const State<R>& S, int64_t s,
                                                    const Moments<R>& M, CorrOut o) {
  Mom64 D;
  expand_moments(M, D);
  if (S.mom) {
    const int64_t n = S.n;
    S.mom[s] = (R)D.m0;
#pragma unroll
    for (int t = 0; t < 3; ++t) S.mom[(1 + t) * n + s] = M.m1[t];
#pragma unroll
    for (int t = 0; t < 6; ++t) S.mom[(4 + t) * n + s] = M.m2[t];
#pragma unroll
    for (int t = 0; t < 3; ++t) S.mom[(10 + t) * n + s] = M.dm0[t];
#pragma unroll
    for (int t = 0; t < 9; ++t) S.mom[(13 + t) * n + s] = M.X1[t];
#pragma unroll
    for (int t = 0; t < 18; ++t) S.mom[(22 + t) * n + s] = M.X2[t];
  }
  Corr64 c;
  solve_corrections<R>(D, c);
  store_kc(S, s, c);
  const int64_t n = S.n;
  const uint32_t p = S.perm[s];
  R* A = (R*)o.A;
  R* B = (R*)o.B;
  R* gA = (R*)o.gradA;
  R* gB = (R*)o.gradB;
  A[p] = (R)c.A;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    B[t * n + p] = (R)c.B[t];
    gA[t * n + p] = (R)c.dA[t];
  }
#pragma unroll
  for (int t = 0; t < 9; ++t) gB[t * n + p] = (R)c.dB[t];
  return c.singular ? 1ull : 0ull;
}

template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_moments(State<R> S, CorrOut o) {
  const int64_t s = particle_id();
  unsigned long long sing = 0;
  if (s < S.n && is_passive(S, s)) {
    if (!S.needed || S.needed[s]) {
      // the corrections of the particle's last evaluation, where a force
      // pair of an active particle reads them
      const int64_t n = S.n;
      const uint32_t p = S.perm[s];
      Corr64 c;
      c.A = (double)S.pA[p];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        c.B[t] = (double)S.pB[t * n + p];
        c.dA[t] = (double)S.pgA[t * n + p];
      }
#pragma unroll
      for (int t = 0; t < 9; ++t) c.dB[t] = (double)S.pgB[t * n + p];
      store_kc(S, s, c);
    }
  } else if (s < S.n && !S.act) {  // (a list of active particles: k_moments_rows)
    Moments<R> M;
    accumulate_moments<R, K>(S, s, M);
    sing = moments_finish<R>(S, s, M, o);
  }
  wave_add_u64(cnt_at(S.cnt, CNT_SINGULAR), sing);
}

// The active particles of a hierarchy substep listed in act (nact of them),
// a 16-lane row each.
template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_moments_rows(State<R> S, CorrOut o) {
  const int64_t r = particle_id() >> 4;
  const int sub = threadIdx.x & 15;
  unsigned long long sing = 0;
  if (r < (int64_t)S.cnt[CNT_ACTLIST * kCntSpread]) {
    const int64_t s = S.act[r];
    Moments<R> M;
    accumulate_moments_row<R, K>(S, s, sub, M);
    if (sub == 0) sing = moments_finish<R>(S, s, M, o);
  }
  if (sing) atomicAdd(cnt_at(S.cnt, CNT_SINGULAR), sing);
}

// ------------------------------------------------ density, grad v, EOS ----

template <class R>
__device__ inline void load_kc(const State<R>& S, int64_t j, KC<R>& k) {
  const R4<R> q0 = S.kc4[4 * j], q1 = S.kc4[4 * j + 1], q2 = S.kc4[4 * j + 2],
              q3 = S.kc4[4 * j + 3];
  k.a = q0.x;
  k.b[0] = q0.y;
  k.b[1] = q0.z;
  k.b[2] = q0.w;
  k.c[0] = q1.x;
  k.c[1] = q1.y;
  k.c[2] = q1.z;
  k.M[0] = q1.w;
  k.M[1] = q2.x;
  k.M[2] = q2.y;
  k.M[3] = q2.z;
  k.M[4] = q2.w;
  k.M[5] = q3.x;
  k.M[6] = q3.y;
  k.M[7] = q3.z;
  k.M[8] = q3.w;
}

template <class R>
__device__ inline void load_gv(const State<R>& S, int64_t j, R gv[9], R& relaxed) {
  const R4<R> q0 = S.gv4[3 * j], q1 = S.gv4[3 * j + 1], q2 = S.gv4[3 * j + 2];
  gv[0] = q0.x;
  gv[1] = q0.y;
  gv[2] = q0.z;
  gv[3] = q0.w;
  gv[4] = q1.x;
  gv[5] = q1.y;
  gv[6] = q1.z;
  gv[7] = q1.w;
  gv[8] = q2.x;
  relaxed = q2.y;
}

// The density sums of particle s over its gather entries k = k0, k0 + DK, ...
// (the self term with k0 = 0): Num, Den and the nine grad v sums.
template <class R, int K, int DK>
__device__ inline void density_sums(const State<R>& S, int64_t s, int k0, R sums[11]) {
  const R4<R> pi = S.pos(s);
  const R4<R> vi = S.vel(s);
  const R hinv = pi.w;
  const R C3 = R(Shape<K>::C) * hinv * hinv * hinv;
  const R C4 = C3 * hinv;
  KC<R> ki;
  load_kc(S, s, ki);
  // self term: x = 0, W^R_ii = A_i W(0)
  const R W0 = C3 * R(Shape<K>::w0);
  R num = k0 == 0 ? S.mass[s] * vi.w * ki.a * W0 : R(0);
  R den = k0 == 0 ? vi.w * vi.w * ki.a * W0 : R(0);
  R gv[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) gv[t] = R(0);
  const NbrRef nb = nbr_ref(S, s);
  uint4 ebuf;
  const int ng = nb.ng;
  for (int k = k0; k < ng; k += DK) {
    const uint32_t e = DK == 1 ? gather_entry(S, nb, k, ebuf) : S.nlist[slot_at(nb.gb, k)];
    const uint32_t j = e >> kCodeBits;
    const R4<R> pj = S.pos(j);
    const R4<R> vj = S.vel(j);
    const R mj = S.mass[j];
    R x[3];
    pair_x(S, s, pi, pj, e, x);
    const R r2 = dot3(x, x);
    const R rinv = Sc<R>::rsqrt(r2);
    R w, dw;
    Shape<K>::eval(r2 * rinv * hinv, w, dw);
    const R W = C3 * w;
    const R fg = C4 * dw * rinv;
    const R gW[3] = {fg * x[0], fg * x[1], fg * x[2]};
    R WR, gWR[3];
    kc_apply(ki, x, W, gW, WR, gWR);
    num += mj * vj.w * WR;
    den += vj.w * vj.w * WR;
    const R dv[3] = {vi.x - vj.x, vi.y - vj.y, vi.z - vj.z};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int g = 0; g < 3; ++g) gv[a * 3 + g] -= vj.w * dv[a] * gWR[g];
  }
  sums[0] = num;
  sums[1] = den;
#pragma unroll
  for (int t = 0; t < 9; ++t) sums[2 + t] = gv[t];
}

// rho, P, c and the relaxation flag from the sums of particle s, stored and
// written in caller order; 1 when relaxed.
template <class R>
__device__ inline unsigned long long density_finish(const State<R>& S, int64_t s,
                                                    const R sums[11], R* rho_out,
                                                    R* gradv_out) {
  unsigned long long nrel = 0;
  {
    const R num = sums[0], den = sums[1];
    R gv[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) gv[t] = sums[2 + t];
    const R rho = num / den;
    const R u = S.uu[s];
    const R gam = R(S.gamma);
    const R P = (gam - R(1)) * rho * u;
    const R c = Sc<R>::sqrt(gam * (gam - R(1)) * u);
    R relaxed = R(0);
    if (S.dt_relax > 0.0) {
      const double div = (double)gv[0] + (double)gv[4] + (double)gv[8];
      // exp(|div v| dt) > 8  <=>  |div v| dt > ln 8
      if (fabs(div) * S.dt_relax > 2.0794415416798357) {
        relaxed = R(1);
        nrel = 1;
      }
    }
    R4<R> st;
    st.x = rho;
    st.y = P;
    st.z = c;
    st.w = den;
    S.st4[s] = st;
    R4<R> g0, g1, g2;
    g0.x = gv[0]; g0.y = gv[1]; g0.z = gv[2]; g0.w = gv[3];
    g1.x = gv[4]; g1.y = gv[5]; g1.z = gv[6]; g1.w = gv[7];
    g2.x = gv[8]; g2.y = relaxed; g2.z = R(0); g2.w = R(0);
    S.gv4[3 * s] = g0;
    S.gv4[3 * s + 1] = g1;
    S.gv4[3 * s + 2] = g2;
    const int64_t n = S.n;
    const uint32_t p = S.perm[s];
    rho_out[p] = rho;
#pragma unroll
    for (int t = 0; t < 9; ++t) gradv_out[t * n + p] = gv[t];
  }
  return nrel;
}

template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_density(State<R> S, R* __restrict__ rho_out,
                                                    R* __restrict__ gradv_out) {
  const int64_t s = particle_id();
  unsigned long long nrel = 0;
  const bool pas = s < S.n && is_passive(S, s);
  if (pas && S.needed && !S.needed[s]) {
    // a passive particle no active one reads this substep: nothing to pack
  } else if (pas) {
    // the carried density and the gradient of the last evaluation; P and c
    // from that density and the particle's u
    const int64_t n = S.n;
    const uint32_t p = S.perm[s];
    const R rho = S.prho[p];
    R gv[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) gv[t] = S.pgv[t * n + p];
    const R u = S.uu[s];
    const R gam = R(S.gamma);
    R relaxed = R(0);
    if (S.dt_relax > 0.0) {
      const double div = (double)gv[0] + (double)gv[4] + (double)gv[8];
      if (fabs(div) * S.dt_relax > 2.0794415416798357) relaxed = R(1);
    }
    R4<R> st;
    st.x = rho;
    st.y = (gam - R(1)) * rho * u;
    st.z = Sc<R>::sqrt(gam * (gam - R(1)) * u);
    st.w = R(0);
    S.st4[s] = st;
    R4<R> g0, g1, g2;
    g0.x = gv[0]; g0.y = gv[1]; g0.z = gv[2]; g0.w = gv[3];
    g1.x = gv[4]; g1.y = gv[5]; g1.z = gv[6]; g1.w = gv[7];
    g2.x = gv[8]; g2.y = relaxed; g2.z = R(0); g2.w = R(0);
    S.gv4[3 * s] = g0;
    S.gv4[3 * s + 1] = g1;
    S.gv4[3 * s + 2] = g2;
  } else if (s < S.n && !S.act) {  // (a list of active particles: k_density_rows)
    R sums[11];
    density_sums<R, K, 1>(S, s, 0, sums);
    nrel = density_finish<R>(S, s, sums, rho_out, gradv_out);
  }
  wave_add_u64(cnt_at(S.cnt, CNT_RELAXED), nrel);
}

// The active particles of a hierarchy substep listed in act, a 16-lane row
// each.
template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_density_rows(State<R> S, R* __restrict__ rho_out,
                                                         R* __restrict__ gradv_out) {
  const int64_t r = particle_id() >> 4;
  const int sub = threadIdx.x & 15;
  unsigned long long nrel = 0;
  if (r < (int64_t)S.cnt[CNT_ACTLIST * kCntSpread]) {
    const int64_t s = S.act[r];
    R sums[11];
    density_sums<R, K, 16>(S, s, sub, sums);
#pragma unroll
    for (int t = 0; t < 11; ++t)
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) sums[t] += __shfl_xor(sums[t], o, 16);
    if (sub == 0) nrel = density_finish<R>(S, s, sums, rho_out, gradv_out);
  }
  if (nrel) atomicAdd(cnt_at(S.cnt, CNT_RELAXED), nrel);
}


// ------------------------------------------------------ force and du/dt ----
// For j != i with r_ij < max(h_i, h_j):
//   G_ij = grad_i W^R_ij - grad_j W^R_ji (uncorrected on both sides when
//   either particle is relaxed),
//   limiter phi = clamp(4 n d / (n + d)^2, 0, 1) with n = x.(grad v_i x),
//   d = x.(grad v_j x); midpoint velocity jump
//   v' = (v_i - phi/2 grad v_i x) - (v_j + phi/2 grad v_j x);
//   mu_k = min(0, v'.x h_k / (r^2 + eps2 h_k^2)), Q_k = rho_k (-alpha c_k mu_k + beta mu_k^2);
//   F_ij = -1/2 V_i V_j (P_i + P_j + Q_i + Q_j) G_ij;
//   a_i = sum F_ij / m_i, du_i/dt = -1/(2 m_i) sum (v_i - v_j).F_ij.

template <class R, int K>
__device__ inline void side_grad(const KC<R>& k, const R x[3], R r2, R rinv, R hinv,
                                 R out[3]) {
  const R C3 = R(Shape<K>::C) * hinv * hinv * hinv;
  R w, dw;
  Shape<K>::eval(r2 * rinv * hinv, w, dw);
  const R W = C3 * w;
  const R fg = C3 * hinv * dw * rinv;
  const R gW[3] = {fg * x[0], fg * x[1], fg * x[2]};
  R WR;
  kc_apply(k, x, W, gW, WR, out);
}

// Adds the force pair of particle s with neighbour entry e (i's position,
// velocity, state, corrections, velocity gradient and relaxation flag, its
// h, and the viscosity parameters) to acc and du.
template <class R, int K>
__device__ __forceinline__ void force_term(const State<R>& S, int64_t s, const R4<R>& pi,
                                           const R4<R>& vi, const R4<R>& si, const KC<R>& ki,
                                           const R gvi[9], R reli, R hi, bool relax_on,
                                           R alpha, R beta, R eps2, uint32_t e, double acc[3],
                                           double& du) {
  const uint32_t j = e >> kCodeBits;
  const R4<R> pj = S.pos(j);
  const R4<R> vj = S.vel(j);
  const R4<R> sj = S.st4[j];
  KC<R> kj;
  load_kc(S, j, kj);
  R gvj[9], relj;
  load_gv(S, j, gvj, relj);
  R x[3];
  pair_x(S, s, pi, pj, e, x);
  const R r2 = dot3(x, x);
  const R rinv = Sc<R>::rsqrt(r2);
  KC<R> kiu = ki;
  if (relax_on && (reli != R(0) || relj != R(0))) {
    kc_plain(kiu);
    kc_plain(kj);
  }
  R Gi[3], Gj[3];
  side_grad<R, K>(kiu, x, r2, rinv, pi.w, Gi);
  const R xm[3] = {-x[0], -x[1], -x[2]};
  side_grad<R, K>(kj, xm, r2, rinv, pj.w, Gj);
  R G[3] = {Gi[0] - Gj[0], Gi[1] - Gj[1], Gi[2] - Gj[2]};
  // limited artificial viscosity
  R gix[3], gjx[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    gix[a] = gvi[a * 3] * x[0] + gvi[a * 3 + 1] * x[1] + gvi[a * 3 + 2] * x[2];
    gjx[a] = gvj[a * 3] * x[0] + gvj[a * 3 + 1] * x[1] + gvj[a * 3 + 2] * x[2];
  }
  const R nn = dot3(x, gix), dd = dot3(x, gjx);
  const R sum = nn + dd;
  const R s2 = sum * sum;
  R phi = R(0);
  if (s2 > R(0)) {
    phi = Sc<R>::div(R(4) * nn * dd, s2);
    phi = phi < R(0) ? R(0) : (phi > R(1) ? R(1) : phi);
  }
  const R hp = R(0.5) * phi;
  const R vp[3] = {(vi.x - vj.x) - hp * (gix[0] + gjx[0]), (vi.y - vj.y) - hp * (gix[1] + gjx[1]),
                   (vi.z - vj.z) - hp * (gix[2] + gjx[2])};
  const R vpx = dot3(vp, x);
  const R hj = Sc<R>::rcp(pj.w);
  R mui = Sc<R>::div(vpx * hi, r2 + eps2 * hi * hi);
  R muj = Sc<R>::div(vpx * hj, r2 + eps2 * hj * hj);
  mui = mui < R(0) ? mui : R(0);
  muj = muj < R(0) ? muj : R(0);
  const R Qi = si.x * (-alpha * si.z * mui + beta * mui * mui);
  const R Qj = sj.x * (-alpha * sj.z * muj + beta * muj * muj);
  const R sfac = R(-0.5) * vi.w * vj.w * (si.y + sj.y + Qi + Qj);
  const R F[3] = {sfac * G[0], sfac * G[1], sfac * G[2]};
  const R work = (vi.x - vj.x) * F[0] + (vi.y - vj.y) * F[1] + (vi.z - vj.z) * F[2];
  acc[0] += (double)F[0];
  acc[1] += (double)F[1];
  acc[2] += (double)F[2];
  du += (double)work;
}

// HIER: a substep of the timestep hierarchy (the passive particles keep their
// acceleration: nothing to sum or write); a separate instance, so that the
// ordinary forward's code is not shaped by the extra branch
template <class R, int K, bool HIER>
__global__ void __launch_bounds__(kBlock) k_force(State<R> S, double* __restrict__ accel,
                                                  double* __restrict__ dudt) {
  const int64_t s = particle_id();
  if (s >= S.n) return;
  if (HIER && (is_passive(S, s) || S.act)) return;  // (a list of active: k_force_rows)
  const R4<R> pi = S.pos(s);
  const R4<R> vi = S.vel(s);
  const R4<R> si = S.st4[s];
  KC<R> ki;
  load_kc(S, s, ki);
  R gvi[9], reli;
  load_gv(S, s, gvi, reli);
  const bool relax_on = S.dt_relax > 0.0;
  const R alpha = R(S.alpha), beta = R(S.beta), eps2 = R(S.eps2);
  const R hi = R(1) / pi.w;
  double acc[3] = {0.0, 0.0, 0.0}, du = 0.0;
  const NbrRef nb = nbr_ref(S, s);
  uint4 ebuf;  // at 3 waves per SIMD this beats 4 waves with the chunk in LDS
  const int ng = nb.ng, ns = nb.ns;
  const int total = ng + ns;
  for (int t = 0; t < total; ++t)
    force_term<R, K>(S, s, pi, vi, si, ki, gvi, reli, hi, relax_on, alpha, beta, eps2,
                     nbr_entry(S, nb, t, ebuf), acc, du);
  const int64_t n = S.n;
  const uint32_t p = S.perm[s];
  const double minv = 1.0 / (double)S.mass[s];
  accel[p] = acc[0] * minv;
  accel[n + p] = acc[1] * minv;
  accel[2 * n + p] = acc[2] * minv;
  dudt[p] = -0.5 * du * minv;
}

// The active particles of a hierarchy substep listed in act, a 16-lane row
// each: lane sub takes the pairs t = sub mod 16, the row sums in FP64.
template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_force_rows(State<R> S, double* __restrict__ accel,
                                                       double* __restrict__ dudt) {
  const int64_t r = particle_id() >> 4;
  const int sub = threadIdx.x & 15;
  if (r >= (int64_t)S.cnt[CNT_ACTLIST * kCntSpread]) return;  // the whole row
  const int64_t s = S.act[r];
  const R4<R> pi = S.pos(s);
  const R4<R> vi = S.vel(s);
  const R4<R> si = S.st4[s];
  KC<R> ki;
  load_kc(S, s, ki);
  R gvi[9], reli;
  load_gv(S, s, gvi, reli);
  const bool relax_on = S.dt_relax > 0.0;
  const R alpha = R(S.alpha), beta = R(S.beta), eps2 = R(S.eps2);
  const R hi = R(1) / pi.w;
  double acc[3] = {0.0, 0.0, 0.0}, du = 0.0;
  const NbrRef nb = nbr_ref(S, s);
  const int total = nb.ng + nb.ns;
  for (int t = sub; t < total; t += 16)
    force_term<R, K>(S, s, pi, vi, si, ki, gvi, reli, hi, relax_on, alpha, beta, eps2,
                     nbr_entry1(S, nb, t), acc, du);
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a] += __shfl_xor(acc[a], o, 16);
    du += __shfl_xor(du, o, 16);
  }
  if (sub == 0) {
    const int64_t n = S.n;
    const uint32_t p = S.perm[s];
    const double minv = 1.0 / (double)S.mass[s];
    accel[p] = acc[0] * minv;
    accel[n + p] = acc[1] * minv;
    accel[2 * n + p] = acc[2] * minv;
    dudt[p] = -0.5 * du * minv;
  }
}

// ------------------------------------------------------------ checks -----

template <class R>
__global__ void __launch_bounds__(kBlock) k_nonfinite(const R* __restrict__ a, int64_t na,
                                                      unsigned long long* cnt) {
  const int64_t i = particle_id();
  unsigned long long bad = 0;
  if (i < na) {
    const double v = (double)a[i];
    bad = (v - v == 0.0) ? 0 : 1;
  }
  wave_add_u64(cnt_at(cnt, CNT_NONFINITE), bad);
}


// ---------------------------------------------- rows for few active ones --
// A hierarchy substep with few active particles (listed in act) gives each a
// 16-lane row in the candidate, volume and neighbour-list passes as well;
// the rows keep the entry order and values of the thread kernels.

// The stencil walk of k_candidates by a row: its lanes test 16 consecutive
// particles of a cell run at a time and append the accepted ones in order.
template <class R, bool EM>
__global__ void __launch_bounds__(kBlock) k_candidates_rows(State<R> S) {
  if (__ballot(S.cnt[CNT_TOO_DENSE * kCntSpread + (threadIdx.x & 63)] != 0ull)) return;
  const int64_t r = particle_id() >> 4;
  if (r >= (int64_t)S.cnt[CNT_ACTLIST * kCntSpread]) return;  // the whole row
  const int lane = threadIdx.x & 63, sub = lane & 15;
  const uint64_t rowbits = 0xFFFFull << (lane & 48);
  const uint64_t below = rowbits & ((1ull << lane) - 1ull);
  const int64_t s = S.act[r];
  const R4<R> pi = S.pos(s);
  const R mi_inv = EM ? R(1) : R(1) / S.mass[s];
  const R rc2 = S.rcap * S.rcap;
  int cap;
  const int64_t base = scratch_base(S, s, cap);
  int cnt = 0;  // uniform over the row
  const uint32_t c3 = S.cell3[s];
  const int G = S.G;
  const int cx = (int)(c3 & 1023u), cy = (int)((c3 >> 10) & 1023u), cz = (int)(c3 >> 20);
  const R ell = S.ell;
  const uint32_t n = (uint32_t)S.n;
  auto gap2 = [&](R xi, int d) {
    const R lo = (R(d) - R(0.5)) * ell - xi, hi = xi - (R(d) + R(0.5)) * ell;
    const R g = lo > hi ? lo : hi;
    return g > R(0) ? g * g : R(0);
  };
  auto walk = [&](uint32_t c0, int x0, int d0, int d1, int dy, int dz, bool own_row) {
    const uint32_t b = S.cell_start[c0];
    uint32_t e = S.cell_start[c0 + (uint32_t)(d1 - d0 + 1)];
    if (e > n) e = n;
    const int xoff = d0 - x0;
    const int code0 = (int)stencil_code(0, dy, dz);
    const R oy = R(dy) * ell, oz = R(dz) * ell;
    for (uint32_t j0 = b; j0 < e; j0 += 16) {
      const uint32_t j = j0 + (uint32_t)sub;
      const bool valid = j < e;
      const R4<R> pj = S.pos(valid ? j : e - 1);
      const int dx = (int)pj.w + xoff;
      R x[3];
      x[0] = (pi.x - pj.x) - R(dx) * ell;
      x[1] = (pi.y - pj.y) - oy;
      x[2] = (pi.z - pj.z) - oz;
      const R r2 = dot3(x, x);
      bool ok = valid && r2 < rc2;
      if (own_row) ok = ok && !(j == (uint32_t)s && dx == 0);
      const uint64_t bm = __ballot(ok) & rowbits;
      const int at = cnt + __popcll(bm & below);
      if (ok && at < cap) {
        const int64_t q = group_at(base, at);
        S.cand[q] = (j << kCodeBits) | (uint32_t)(code0 + dx);
        S.scr_r[q] = Sc<R>::sqrt(r2);
        if (!EM) S.scr_m[q] = S.mass[j] * mi_inv;
      }
      cnt += __popcll(bm);
    }
  };
  for (int dz = -2; dz <= 2; ++dz) {
    const R gz = gap2(pi.z, dz);
    if (!(gz < rc2)) continue;
    const int z = wrap_cell(cz + dz, G);
    for (int dy = -2; dy <= 2; ++dy) {
      const R gyz = gz + gap2(pi.y, dy);
      if (!(gyz < rc2)) continue;
      const int y = wrap_cell(cy + dy, G);
      const uint32_t rowbase = ((uint32_t)z * G + (uint32_t)y) * G;
      int dlo = 3, dhi = -3;
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx)
        if (gyz + gap2(pi.x, dx) < rc2) {
          dlo = dx < dlo ? dx : dlo;
          dhi = dx;
        }
      const int a1 = min(dhi, -cx - 1);
      const int b0 = max(dlo, -cx), b1 = min(dhi, G - 1 - cx);
      const int c0 = max(dlo, G - cx);
      const bool own = dy == 0 && dz == 0;
      if (dlo <= a1) walk(rowbase + (uint32_t)(cx + dlo + G), cx + dlo + G, dlo, a1, dy, dz, own);
      if (b0 <= b1) walk(rowbase + (uint32_t)(cx + b0), cx + b0, b0, b1, dy, dz, own);
      if (c0 <= dhi) walk(rowbase + (uint32_t)(cx + c0 - G), cx + c0 - G, c0, dhi, dy, dz, own);
    }
  }
  if (sub == 0) {
    S.ccnt[s] = cnt < cap ? cnt : cap;
    if (cnt > cap) atomicMax(cnt_at(S.cnt, CNT_SCR_OVERFLOW), (unsigned long long)cnt);
  }
}

// The fixed-h volume of k_volume by a row (the self term in lane 0).
template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_volume_rows(State<R> S) {
  const int64_t r = particle_id() >> 4;
  if (r >= (int64_t)S.cnt[CNT_ACTLIST * kCntSpread]) return;
  const int sub = threadIdx.x & 15;
  const int64_t s = S.act[r];
  const R h = S.hbuf[s];
  const R hinv = R(1) / h;
  int scap;
  const int64_t base = scratch_base(S, s, scap);
  const int cnt = S.ccnt[s] < scap ? S.ccnt[s] : scap;
  R sum = sub == 0 ? R(Shape<K>::w0) : R(0);
  for (int k = sub; k < cnt; k += 16) {
    const int64_t e = group_at(base, k);
    R w, dw;
    Shape<K>::eval(S.scr_r[e] * hinv, w, dw);
    sum += (S.equal_mass ? R(1) : S.scr_m[e]) * w;
  }
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 16);
  if (sub == 0) S.Vbuf[s] = h * h * h / (R(Shape<K>::C) * sum);
}

// The neighbour lists of k_nlist by a row: 16 candidates at a time, the
// gather and scatter-only entries appended in candidate order.
template <class R>
__global__ void __launch_bounds__(kBlock) k_nlist_rows(State<R> S) {
  const int64_t r = particle_id() >> 4;
  if (r >= (int64_t)S.cnt[CNT_ACTLIST * kCntSpread]) return;
  const int lane = threadIdx.x & 63, sub = lane & 15;
  const uint64_t rowbits = 0xFFFFull << (lane & 48);
  const uint64_t below = rowbits & ((1ull << lane) - 1ull);
  const int64_t s = S.act[r];
  const R hi = S.hbuf[s];
  int ccap;
  const int64_t base = scratch_base(S, s, ccap);
  const int cc = S.ccnt[s] < ccap ? S.ccnt[s] : ccap;
  const int cap = S.list_cap, scap = S.slist_cap;
  int ng = 0, ns = 0;  // uniform over the row
  for (int k = 0; k < cc; k += 16) {
    const int t = k + sub;
    const bool in = t < cc;
    const int64_t c = group_at(base, in ? t : 0);
    const uint32_t e = S.cand[c];
    const R rr = S.scr_r[c];
    const bool g = in && rr < hi;
    const bool sc = in && !g && rr < S.hbuf[e >> kCodeBits];
    const uint64_t gm = __ballot(g) & rowbits, sm = __ballot(sc) & rowbits;
    if (g) {
      const int at = ng + __popcll(gm & below);
      if (at < cap) S.nlist[list_index(s, cap, at)] = e;
    }
    if (sc) {
      const int at = ns + __popcll(sm & below);
      if (at < scap) S.slist[list_index(s, scap, at)] = e;
    }
    if (S.needed && (g || sc)) S.needed[e >> kCodeBits] = 1;
    ng += __popcll(gm);
    ns += __popcll(sm);
  }
  if (sub == 0) {
    S.ng[s] = ng;
    S.ns[s] = ns;
    atomicAdd(cnt_at(S.cnt, CNT_PAIRS_GATHER), (unsigned long long)ng);
    atomicAdd(cnt_at(S.cnt, CNT_PAIRS_FORCE), (unsigned long long)(ng + ns));
    atomicAdd(cnt_at(S.cnt, CNT_CANDIDATES), (unsigned long long)cc);
    if (ng > cap) atomicMax(cnt_at(S.cnt, CNT_LIST_OVERFLOW), (unsigned long long)ng);
    if (ns > scap) atomicMax(cnt_at(S.cnt, CNT_SLIST_OVERFLOW), (unsigned long long)ns);
  }
}
}  // namespace

// ----------------------------------------------------------- launchers ----

template <class R>
void launch_check_inputs(const double* x, const R* h, const R* m, const R* u, int64_t n,
                         unsigned long long* cnt, hipStream_t s) {
  const unsigned blocks = grid_for(n) < 1024u ? grid_for(n) : 1024u;
  hipLaunchKernelGGL(k_check_inputs<R>, dim3(blocks > 0 ? blocks : 1), dim3(kBlock), 0, s, x, h,
                     m, u, n, cnt);
}

void launch_keys(const double* x, int64_t n, double box, int G, uint32_t* keys, uint32_t* vals,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, x, n, box, G, keys, vals);
}

void launch_keys_check(const double* x, int64_t n, double box, int G, const uint32_t* keys,
                       const uint32_t* perm, unsigned long long* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_keys_check, dim3(grid_for(n)), dim3(kBlock), 0, s, x, n, box, G, keys,
                     perm, cnt);
}

void launch_count_active(const int* levels, int64_t n, int lmax, int64_t jend,
                         unsigned long long* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_count_active, dim3(grid_for(n)), dim3(kBlock), 0, s, levels, n, lmax, jend,
                     cnt);
}
template <class R>
void launch_active_list(const State<R>& S, uint32_t* list, hipStream_t s) {
  hipLaunchKernelGGL(k_active_list<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S, list);
}

void launch_cell_bounds(const uint32_t* keys, int64_t n, int64_t ncell, uint32_t* start,
                        unsigned long long occ_limit, unsigned long long* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_bounds, dim3((unsigned)((ncell + kBlock) / kBlock)), dim3(kBlock), 0,
                     s, keys, n, ncell, start, occ_limit, cnt);
}

template <class R>
void launch_gather(const State<R>& S, const double* x, const R* v, const R* m, const R* u,
                   const R* h, hipStream_t s) {
  hipLaunchKernelGGL(k_gather<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S, x, v, m, u, h);
}

#define CRK_DISPATCH_K(kernel, KFN, ...)                                                 \
  do {                                                                                   \
    if ((kernel) == 0)                                                                   \
      hipLaunchKernelGGL((KFN<R, 0>), dim3(grid_for(S.n)), dim3(kBlock), 0, s, __VA_ARGS__); \
    else                                                                                 \
      hipLaunchKernelGGL((KFN<R, 1>), dim3(grid_for(S.n)), dim3(kBlock), 0, s, __VA_ARGS__); \
  } while (0)

template <class R>
void launch_candidates(const State<R>& S, hipStream_t s) {
  if (S.equal_mass)
    hipLaunchKernelGGL((k_candidates<R, true>), dim3(grid_for(S.n)), dim3(kBlock), 0, s, S);
  else
    hipLaunchKernelGGL((k_candidates<R, false>), dim3(grid_for(S.n)), dim3(kBlock), 0, s, S);
  if (S.act && S.nact > 0) {
    const dim3 rg(grid_for(16 * S.nact));
    if (S.equal_mass)
      hipLaunchKernelGGL((k_candidates_rows<R, true>), rg, dim3(kBlock), 0, s, S);
    else
      hipLaunchKernelGGL((k_candidates_rows<R, false>), rg, dim3(kBlock), 0, s, S);
  }
}
template <class R>
void launch_hsolve(const State<R>& S, int kernel, hipStream_t s) {
  if (S.n == 0) return;
  const dim3 g(grid_for(S.n)), b(kBlock);
  if (kernel == 0) hipLaunchKernelGGL((k_hsolve<R, 0>), g, b, 0, s, S);
  else hipLaunchKernelGGL((k_hsolve<R, 1>), g, b, 0, s, S);
}
template <class R>
void launch_volume(const State<R>& S, int kernel, hipStream_t s) {
  if (S.n == 0) return;
  const dim3 g(grid_for(S.n)), b(kBlock);
  if (kernel == 0) hipLaunchKernelGGL((k_volume<R, 0>), g, b, 0, s, S);
  else hipLaunchKernelGGL((k_volume<R, 1>), g, b, 0, s, S);
  if (S.act && S.nact > 0) {
    const dim3 rg(grid_for(16 * S.nact));
    if (kernel == 0) hipLaunchKernelGGL((k_volume_rows<R, 0>), rg, b, 0, s, S);
    else hipLaunchKernelGGL((k_volume_rows<R, 1>), rg, b, 0, s, S);
  }
}
template <class R>
void launch_pack(const State<R>& S, R* h_out, R* V_out, hipStream_t s) {
  hipLaunchKernelGGL(k_pack<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S, h_out, V_out);
}
template <class R>
void launch_nlist(const State<R>& S, hipStream_t s) {
  hipLaunchKernelGGL(k_nlist<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S);
  if (S.act && S.nact > 0)
    hipLaunchKernelGGL(k_nlist_rows<R>, dim3(grid_for(16 * S.nact)), dim3(kBlock), 0, s, S);
}
// a 16-lane row per listed active particle
#define CRK_DISPATCH_ROWS(kernel, KFN, ...)                                                 \
  do {                                                                                      \
    const dim3 rg(grid_for(16 * S.nact));                                                   \
    if ((kernel) == 0)                                                                      \
      hipLaunchKernelGGL((KFN<R, 0>), rg, dim3(kBlock), 0, s, __VA_ARGS__);                 \
    else                                                                                    \
      hipLaunchKernelGGL((KFN<R, 1>), rg, dim3(kBlock), 0, s, __VA_ARGS__);                 \
  } while (0)

template <class R>
void launch_moments(const State<R>& S, int kernel, CorrOut o, hipStream_t s) {
  CRK_DISPATCH_K(kernel, k_moments, S, o);
  if (S.act && S.nact > 0) CRK_DISPATCH_ROWS(kernel, k_moments_rows, S, o);
}
template <class R>
void launch_density(const State<R>& S, int kernel, R* rho_out, R* gradv_out, hipStream_t s) {
  CRK_DISPATCH_K(kernel, k_density, S, rho_out, gradv_out);
  if (S.act && S.nact > 0) CRK_DISPATCH_ROWS(kernel, k_density_rows, S, rho_out, gradv_out);
}
template <class R>
void launch_force(const State<R>& S, int kernel, double* accel, double* dudt, hipStream_t s) {
  const dim3 grid(grid_for(S.n)), block(kBlock);
  if (S.act) {  // the passive particles need nothing: only the rows
    if (S.nact > 0) CRK_DISPATCH_ROWS(kernel, k_force_rows, S, accel, dudt);
  } else if (S.levels) {
    if (kernel == 0)
      hipLaunchKernelGGL((k_force<R, 0, true>), grid, block, 0, s, S, accel, dudt);
    else
      hipLaunchKernelGGL((k_force<R, 1, true>), grid, block, 0, s, S, accel, dudt);
  } else {
    if (kernel == 0)
      hipLaunchKernelGGL((k_force<R, 0, false>), grid, block, 0, s, S, accel, dudt);
    else
      hipLaunchKernelGGL((k_force<R, 1, false>), grid, block, 0, s, S, accel, dudt);
  }
}
template <class R>
void launch_count_nonfinite(const R* a, int64_t na, unsigned long long* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite<R>, dim3(grid_for(na)), dim3(kBlock), 0, s, a, na, cnt);
}
void launch_count_nonfinite_f64(const double* a, int64_t na, unsigned long long* cnt,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite<double>, dim3(grid_for(na)), dim3(kBlock), 0, s, a, na, cnt);
}

#define CRK_INSTANTIATE(R)                                                                   \
  template void launch_check_inputs<R>(const double*, const R*, const R*, const R*, int64_t, \
                                       unsigned long long*, hipStream_t);                    \
  template void launch_gather<R>(const State<R>&, const double*, const R*, const R*,         \
                                 const R*, const R*, hipStream_t);                           \
  template void launch_candidates<R>(const State<R>&, hipStream_t);                          \
  template void launch_hsolve<R>(const State<R>&, int, hipStream_t); \
  template void launch_volume<R>(const State<R>&, int, hipStream_t); \
  template void launch_pack<R>(const State<R>&, R*, R*, hipStream_t);                        \
  template void launch_nlist<R>(const State<R>&, hipStream_t);                               \
  template void launch_moments<R>(const State<R>&, int, CorrOut, hipStream_t);               \
  template void launch_density<R>(const State<R>&, int, R*, R*, hipStream_t);                \
  template void launch_force<R>(const State<R>&, int, double*, double*, hipStream_t);        \
  template void launch_active_list<R>(const State<R>&, uint32_t*, hipStream_t);              \
  template void launch_count_nonfinite<R>(const R*, int64_t, unsigned long long*, hipStream_t);

CRK_INSTANTIATE(float)
CRK_INSTANTIATE(double)

}  // namespace crk
