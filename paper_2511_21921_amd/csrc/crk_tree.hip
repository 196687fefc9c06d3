// Neighbour search for strongly clustered particle sets.
//
// When smoothing lengths span orders of magnitude (gas clumps in a
// cosmological volume), a cell list sized to the largest h puts whole clumps
// into single cells. This path instead sorts the particles along a Morton
// curve over a 1024^3 lattice (positions are kept as lattice coordinates
// plus FP32/FP64 offsets from the lattice-cell centre), takes every run of
// kLeaf = 16 consecutive particles as a search leaf, and builds an implicit
// tree of leaf boxes with kFan = 8 children per node (a node is named by its
// level and index; its children are the kFan nodes that follow kFan times
// its index one level down). A particle's 16-lane row walks the tree for its
// sphere: a step tests the children of one node (one per lane) and keeps, as
// bits of one 64-bit word, the children still to visit at each level, so the
// walk needs no stack (the four rows of a wave, consecutive particles, walk
// the levels above the leaves together, breadth first, on all 64 lanes). The
// particles of a reached leaf are tested one per lane. Candidates within a particle's (padded) radius are kept as indices, each
// particle's contiguous in one pool: the h solve recomputes their distances,
// and the gather list is the candidates within the solved h.
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
  for (int a = 0; a < 3; ++a) c[a] = (uint32_t)cell_coord(wrap_pos(x[a * n + i], L), inv, 1024);
  keys[i] = spread10(c[0]) | (spread10(c[1]) << 1) | (spread10(c[2]) << 2);
  vals[i] = (uint32_t)i;
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

// Leaf boxes (absolute positions, FP32) and the largest h of each leaf; the
// absolute positions themselves go to absp (the search's leaf tests).
template <class R>
__global__ void __launch_bounds__(kBlock) k_leaf_boxes(State<R> S, const R* __restrict__ h,
                                                       float4* __restrict__ absp) {
  const int64_t leaf = particle_id();
  const int nleaf = S.lvl_off[kMaxLevels];  // level 0 count
  if (leaf >= nleaf) return;
  const int64_t b = leaf * kLeaf, e = (b + kLeaf < S.n) ? b + kLeaf : S.n;
  float lo[3] = {3e30f, 3e30f, 3e30f}, hi[3] = {-3e30f, -3e30f, -3e30f}, hm = 0.f;
  for (int64_t s = b; s < e; ++s) {
    float v[3];
    abs_pos(S, S.cell3[s], S.pos(s), v);
    absp[s] = make_float4(v[0], v[1], v[2], 0.f);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], v[a]);
      hi[a] = fmaxf(hi[a], v[a]);
    }
    hm = fmaxf(hm, (float)h[s]);
  }
  S.ncen[leaf] = make_float4(lo[0], lo[1], lo[2], hm);  // corners until k_box_centres
  S.nhw[leaf] = make_float4(hi[0], hi[1], hi[2], 0.f);
}

// Node k of a level from its (up to kFan) children k kFan + c one level down.
__global__ void __launch_bounds__(kBlock) k_tree_up(float4* nlo, float4* nhi, int off_c,
                                                    int cnt_c, int off_p, int cnt_p) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= cnt_p) return;
  float4 lo = nlo[off_c + kFan * k], hi = nhi[off_c + kFan * k];
  for (int c = 1; c < kFan && kFan * k + c < cnt_c; ++c) {
    const float4 l2 = nlo[off_c + kFan * k + c], h2 = nhi[off_c + kFan * k + c];
    lo = make_float4(fminf(lo.x, l2.x), fminf(lo.y, l2.y), fminf(lo.z, l2.z), fmaxf(lo.w, l2.w));
    hi = make_float4(fmaxf(hi.x, h2.x), fmaxf(hi.y, h2.y), fmaxf(hi.z, h2.z), 0.f);
  }
  nlo[off_p + k] = lo;
  nhi[off_p + k] = hi;
}

// Every node box from its corners to (centre, h_max) and (half-widths, 0).
__global__ void __launch_bounds__(kBlock) k_box_centres(float4* __restrict__ lo_c,
                                                        float4* __restrict__ hi_w, int nnode) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= nnode) return;
  const float4 lo = lo_c[k], hi = hi_w[k];
  lo_c[k] = make_float4(0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z), lo.w);
  hi_w[k] = make_float4(0.5f * (hi.x - lo.x), 0.5f * (hi.y - lo.y), 0.5f * (hi.z - lo.z), 0.f);
}

// Radius widened against the FP32 rounding of positions and node boxes.
__device__ inline float pad_radius(float r, float L) { return r * 1.00001f + 4e-6f * L; }

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

// The level offsets and counts of the implicit tree, copied to LDS (a row's
// walk indexes them by its own level).
struct Levels {
  int off[kMaxLevels], cnt[kMaxLevels];
};

// First candidate radius of every particle, kept small so that the first
// walk stays cheap (particles whose h root lies beyond it grow it in later
// rounds): the least of the h that the target count would need at the
// density of the particle's 8 nearest wave-mates (the 64 particles of its
// wave), n_h r_8 (4 pi / 24)^(1/3), at the density of the wave's box, and
// 1.5x that of the mean density (the estimate lies a fifth above the root
// for the median particle and below it for a few percent). When the caller's
// h lies within [0.75, 1.33] of the estimate (a previous step's h), 1.05 h is
// taken where it is larger. With fixed h the radius is h.
template <class R>
__global__ void __launch_bounds__(kBlock) k_init_radius(State<R> S, int h_mode) {
  const int64_t s = particle_id();
  if ((s & ~(int64_t)63) >= S.n) return;
  const bool active = s < S.n;
  const int64_t sc = active ? s : 0;
  const int64_t wave = sc >> 6;
  R r = S.hbuf[sc];
  if (h_mode != 0) {
    const int lane = threadIdx.x & 63;
    const R4<R> pi = S.pos(sc);
    const uint32_t ci = S.cell3[sc];
    const int64_t b = wave * 64;
    const int cnt = (int)((b + 64 < S.n ? b + 64 : S.n) - b);
    // the wave's particles, broadcast to its lanes one at a time
    const int64_t jl = b + (lane < cnt ? lane : 0);
    const R4<R> pl = S.pos(jl);
    const int cl = (int)S.cell3[jl];
    float d[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) d[t] = 3e30f;
    for (int t = 0; t < cnt; ++t) {
      R4<R> pj;
      pj.x = bcast(pl.x, t);
      pj.y = bcast(pl.y, t);
      pj.z = bcast(pl.z, t);
      pj.w = R(0);
      const uint32_t cj = (uint32_t)bcast(cl, t);
      if (b + t == sc) continue;
      R x[3];
      lattice_sep(S, pi, ci, pj, cj, x);
      float v = (float)(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
#pragma unroll
      for (int q = 0; q < 8; ++q) {  // keep the 8 smallest, sorted
        const float lo = fminf(d[q], v);
        v = fmaxf(d[q], v);
        d[q] = lo;
      }
    }
    // the wave's box: the union of its (up to four) leaves
    const int nleaf = S.lvl_off[kMaxLevels];
    float lo[3] = {3e30f, 3e30f, 3e30f}, hi[3] = {-3e30f, -3e30f, -3e30f};
    for (int q = 0; q < 4 && wave * 4 + q < nleaf; ++q) {
      const float4 c = S.ncen[wave * 4 + q], w = S.nhw[wave * 4 + q];
      const float cc[3] = {c.x, c.y, c.z}, ww[3] = {w.x, w.y, w.z};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(lo[a], cc[a] - ww[a]);
        hi[a] = fmaxf(hi[a], cc[a] + ww[a]);
      }
    }
    const double pad = 0.5 * S.ell_d;  // coincident lattice cells have no volume
    const double vol = ((double)(hi[0] - lo[0]) + pad) * ((double)(hi[1] - lo[1]) + pad) *
                       ((double)(hi[2] - lo[2]) + pad);
    // (a wave of fewer than nine particles, the ragged last one, tells
    // nothing of the density: the mean density's h then)
    double est = cnt >= 9 ? cbrt(S.n_h3 * vol / (double)cnt) : cbrt(S.n_h3 / (double)S.n) * S.box;
    if (cnt >= 9)  // (4 pi / 24)^(1/3)
      est = fmin(est, cbrt(S.n_h3) * sqrt((double)d[7]) * 0.80599597700823482);
    est = fmin(est, 1.5 * cbrt(S.n_h3 / (double)S.n) * S.box);
    const double g = (double)r;
    const double h0 = (g > 0.75 * est && g < 1.33 * est) ? fmax(1.05 * g, est) : est;
    r = (R)fmin(h0, 0.45 * S.box);
  }
  if (active) {
    S.rad[s] = r;
    S.rad[S.n + s] = R(0);  // no radius known below the root yet
    S.need[s] = S.scr_cap;
    S.todo[s] = 1;
  }
}

// The h solve of k_hsolve (or the volume of k_volume for fixed h) with a
// 16-lane row per particle: lane sub takes the kept candidates 16 it + sub,
// recomputing their distances from the positions (the candidate pass keeps
// only the indices), holding those of the first kRegGroups groups in
// registers and recomputing any further ones at every evaluation. The sums over the row are butterfly
// reductions, which leave the same value in every lane, so the solve is
// uniform over the row and its lane 0 writes the results. The spread over
// the row keeps a particle with thousands of candidates (a sphere that
// takes in a dense clump core) from holding a wave for thousands of serial
// steps per evaluation. order null: row t takes particle t; else order[t].
constexpr int kRegGroups = 16;
template <class R, int K, bool EM>
__global__ void __launch_bounds__(kBlock) k_hsolve_rows(State<R> S,
                                                        const uint32_t* __restrict__ order,
                                                        int64_t nt) {
  const int64_t tid = particle_id();
  if (((tid & ~(int64_t)63) >> 4) >= nt) return;  // the wave's four rows past the end
  const int64_t t = tid >> 4;
  const int sub = threadIdx.x & 15;
  const int64_t s = t < nt ? (order ? (int64_t)order[t] : t) : S.n;
  // particles still to solve whose candidate pass fitted (uniform over the row)
  const bool work = s < S.n && S.todo[s] && S.ccnt[s] >= 0;
  unsigned long long iters = 0, unconv = 0, capped = 0, hbits = 0;
  if (__ballot(work) != 0ull) {
    int cnt = 0;
    int64_t base = 0;
    if (work) {
      base = 4 * (int64_t)S.cpos[s];
      cnt = S.ccnt[s];
    }
    const int ngroups = (cnt + 15) >> 4;
    // the distance and mass ratio of kept entry e, from the exact
    // separation (lattice offsets, as every later pass computes it)
    const int64_t sc = s < S.n ? s : 0;
    const R4<R> pi = S.pos(sc);
    const uint32_t ci = S.cell3[sc];
    const R mi_inv = EM ? R(1) : R(1) / S.mass[sc];
    // Lanes past the count load entry 0 of the row, or of the pool when the
    // row has no entry (the word at its position is then another row's or
    // was never written); the index is clamped below n, so that whatever
    // such a lane loaded addresses a particle (its terms are discarded).
    const int64_t at0 = cnt > 0 ? base : 0;
    const uint32_t jmax = (uint32_t)(S.n - 1);
    auto entry = [&](int e, R& r, R& mr) {
      const uint32_t w = S.cand[e < cnt ? base + e : at0] >> kCodeBits;
      const uint32_t j = w < jmax ? w : jmax;
      R x[3];
      lattice_sep(S, pi, ci, S.pos(j), S.cell3[j], x);
      r = Sc<R>::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
      mr = EM ? R(1) : S.mass[j] * mi_inv;
    };
    R rk[kRegGroups], mk[kRegGroups];
    // all slots at once, without branches, so that their loads are in
    // flight together (slots past the count stay unused)
#pragma unroll
    for (int it = 0; it < kRegGroups; ++it) entry(16 * it + sub, rk[it], mk[it]);
    auto sums = [&](R h, R& dsum) {
      const R hinv = R(1) / h;
      R sum = R(0), ds = R(0);
      auto add = [&](int e, R r, R mr) {
        // entries past the count are moved outside the support (w = w' = 0)
        const bool in = e < cnt;
        const R q = in ? r * hinv : R(2);
        R w, dw;
        Shape<K>::eval(q, w, dw);
        const R mt = EM ? R(1) : (in ? mr : R(0));
        sum += mt * w;
        ds += mt * dw * q;
      };
#pragma unroll
      for (int it = 0; it < kRegGroups; ++it)
        if (it < ngroups) add(16 * it + sub, rk[it], mk[it]);
      for (int it = kRegGroups; it < ngroups; ++it) {
        R r, mr;
        entry(16 * it + sub, r, mr);
        add(16 * it + sub, r, mr);
      }
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o, 16);
        ds += __shfl_xor(ds, o, 16);
      }
      dsum = ds;
      return sum + R(Shape<K>::w0);
    };
    const R C = R(Shape<K>::C);
    if (work && !S.shrink) {
      // fixed h: V_i = m_i / sum_j m_j W(r_ij, h_i), self term included
      const R h = S.hbuf[s];
      R dsum;
      const R sum = sums(h, dsum);
      if (sub == 0) {
        S.todo[s] = 0;
        if (!is_passive(S, s)) S.Vbuf[s] = h * h * h / (C * sum);
      }
    } else if (work) {
      // f(h) = C (w(0) + sum_j (m_j/m_i) w(r_ij / h)) - n_h^3, non-decreasing
      // in h: safeguarded Newton inside a bisection bracket, as k_hsolve
      const R Rcap = S.rad[s];
      const R n_h3 = R(S.n_h3);
      const R rtol = R(S.rtol);
      R h = first_h(S.hbuf[s], Rcap, cnt, S.n_h3);
      R dsum, sum = sums(h, dsum);
      R f = C * sum - n_h3;
      // the bracket [0, Rcap] holds the root only if f(Rcap) > 0
      bool cap_hit = false;
      if (!(f > R(0))) {
        R ds2;
        cap_hit = !(C * sums(Rcap, ds2) - n_h3 > R(0));
      }
      if (cap_hit) {
        // the root lies beyond the radius: grow it by what the candidate
        // count suggests; the particle is taken again in the next round
        if (sub == 0) {
          capped = 1;
          const double g = grow_factor(S.n_h3, cnt);
          S.rad[S.n + s] = Rcap;
          S.rad[s] = (R)((double)Rcap * g);
          S.need[s] = max(S.need[s], need_after_growth(cnt, g));
        }
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
            const R nt_ = h - f / fp;
            const R step = nt_ > h ? nt_ - h : h - nt_;
            if (step <= rtol * h) {
              hn = nt_ < lo ? lo : (nt_ > hi ? hi : nt_);
              conv = true;
              break;
            }
            if (nt_ > lo && nt_ < hi) hn = nt_;
          }
          if (hi - lo <= rtol * hn) {
            conv = true;
            break;
          }
          if (++it >= S.max_iter) break;
          h = hn;
          sum = sums(h, dsum);
          f = C * sum - n_h3;
        }
        // V at the final h from the last sums (first order in the step, which
        // is below the tolerance; an unconverged h gets its own pass)
        const R sum_f = conv ? sum - dsum / h * (hn - h) : sums(hn, dsum);
        if (sub == 0) {
          iters = (unsigned long long)(it + 1);
          unconv = conv ? 0 : 1;
          S.hbuf[s] = hn;
          S.Vbuf[s] = hn * hn * hn / (C * sum_f);
          hbits = dbits((double)hn);
          S.todo[s] = 0;
        }
      }
    }
  }
  wave_max_u64(cnt_at(S.cnt, CNT_H_ITER_MAX), iters);
  wave_add_u64(cnt_at(S.cnt, CNT_H_UNCONV), unconv);
  wave_add_u64(cnt_at(S.cnt, CNT_H_CAPPED), capped);
  wave_max_u64(cnt_at(S.cnt, CNT_HMAX_OUT_BITS), hbits);
}

// LDS staging capacity of a row, in entries: 16 KB a block of 16 rows, which
// leaves room in the LDS for the eight blocks per CU the registers allow
// (320 entries gave six, and the search took 68.9 ms at clumps256 against
// 66.4 with 256 and the retries of its larger overflow)
constexpr int kStage = 256;

// Candidates of every unsolved particle: the j != s whose FP32 absolute
// position lies within its radius ri padded beyond the FP32 rounding (their
// indices, in ascending j), kept contiguous in the candidate pool from entry
// 4 cpos[s]. They hold every j with r_ij < ri and at most a thin shell
// beyond it, which adds nothing to the sums or lists of any h <= ri: the h
// solve and the list filter compute the exact separations themselves. A
// 16-lane row takes one particle (order null: row t takes particle t; else
// order[t], the unsolved particles of a retry round in rank order). It works
// in the row's room (room_for(need[s]) entries at pool_base4 + coff4[s]), or
// (STAGE) in the row's LDS stage of scr_cap entries, after which every block
// takes the room its rows' candidates need from the pool's bump counter and
// copies them there (a block that finds the pool full leaves its particles
// to the next round, with room of their own).
//    The four rows of a wave walk the levels above level 1 together, breadth
//     first, for a sphere holding their four (see shared_walk below), and
//     each row then tests the leaves of the level-1 nodes its own sphere
//     reaches. Rows far apart walk alone: a step tests the kFan children of
//     the current node one per lane (a child is entered when the sphere,
//     padded beyond the FP32 rounding, reaches its box), records the reached
//     children as bits of pend (8 bits per level) and moves to the deepest
//     pending one, so the walk needs no stack. Either way reached leaves are
//     queued per row in LDS and tested by all rows of the wave in step, two
//     a step (a row's q-th and (q+1)-th queued leaves at step q / 2), so that
//     the wave's leaf tests take as many steps as its longest queue rather
//     than, step by step of the walk, the most leaves any row reached. A
//     leaf's 16 particles are tested one per lane against the padded sphere
//     as absolute FP32 positions; the passed indices are appended in order
//     (prefix counts over the row's ballot).
// A particle whose passed indices overflow its capacity is counted: the next
// round takes the radius that would hold 1.3 (4 pi / 3) n_h^3 of them at the
// density seen (at least half of ri), with capacity for 1.3 times what that
// density gives there; a radius that then falls short of the h root is grown
// by the h solve, and once that has happened radii only grow (an overflow
// keeps the radius and raises the capacity), so the rounds end. With fixed h
// the capacity is raised.
// A row per particle rather than 16 particles sharing a walk: rows of
// neighbouring particles test every lane against the union of 16 spheres
// (about eight times the particles of one sphere, most of them rejected),
// and the retry rounds' rows of scattered particles the union of 16
// disjoint neighbourhoods.
template <class R, int K, bool EM, bool STAGE>
__global__ void __launch_bounds__(kBlock) k_candidates_tree(State<R> S,
                                                            const float4* __restrict__ absp,
                                                            const uint32_t* __restrict__ order,
                                                            int64_t nt) {
  __shared__ Levels lv;
  for (int t = threadIdx.x; t < S.nlevels; t += kBlock) {
    lv.off[t] = S.lvl_off[t];
    lv.cnt[t] = S.lvl_off[kMaxLevels + t];
  }
  __syncthreads();
  constexpr int kRowBuf = 40;  // leaves a row queues between drains (the block then takes 20 KB of LDS: eight blocks per CU)
  __shared__ uint32_t lbuf[kBlock / 16][kRowBuf];
  // STAGE: every row's passed indices (its candidates), in LDS
  __shared__ uint4 stage4[STAGE ? kBlock / 16 : 1][STAGE ? kStage / 4 : 1];
  __shared__ uint32_t rcnt[kBlock / 16];
  __shared__ unsigned long long rbase[kBlock / 16];
  // each wave's frontiers of the shared walk (the level being expanded and
  // the next one)
  constexpr int kFront = 32;
  constexpr float kSharedReach = 4.0f;  // largest common radius over the rows' largest
  __shared__ uint32_t front[kBlock / 64][2][kFront];
  static_assert(kFan == 8, "the shared walk takes 8 frontier nodes of 8 children a step");
  const int64_t tid = particle_id();
  // a wave whose four rows are past the end leaves at once, unless the
  // block's barriers below still need it
  if (!STAGE && ((tid & ~(int64_t)63) >> 4) >= nt) return;
  const int64_t t = tid >> 4;                      // this row's rank in the round
  const int lane = threadIdx.x & 63, sub = lane & 15, rowid = lane >> 4;
  const uint64_t rowbits = 0xFFFFull << (16 * rowid);
  const uint64_t below = rowbits & ((1ull << lane) - 1ull);  // row lanes before this one
  uint32_t* rbuf = lbuf[threadIdx.x >> 4];
  uint32_t* srow = reinterpret_cast<uint32_t*>(stage4[STAGE ? threadIdx.x >> 4 : 0]);
  const bool active = t < nt;
  const int64_t s = active ? (order ? (int64_t)order[t] : t) : S.n;
  const int64_t sc = active ? s : 0;
  const bool mine = active && S.todo[sc];  // uniform over the row
  unsigned long long retry = 0, kept = 0;
  bool fits = false;  // uniform over the row: the passed indices fitted
  int np = 0, cnt = 0;  // uniform over the row
  if (__ballot(mine) != 0ull) {
    const R ri = mine ? S.rad[sc] : R(0);
    const R4<R> pi = S.pos(sc);
    const uint32_t ci = S.cell3[sc];
    int cap = 0;
    int64_t base = 0;
    if (mine) {
      if constexpr (STAGE) {
        cap = S.scr_cap;  // at most kStage
      } else {
        cap = room_for(S.need[sc], order != nullptr);  // order: a retry round
        base = 4 * (S.pool_base4 + (int64_t)S.coff4[sc]);
      }
    }
    auto put = [&](int at, uint32_t v) {
      if constexpr (STAGE)
        srow[at] = v;
      else
        S.cand[base + at] = v;
    };
    float P[3];
    abs_pos(S, ci, pi, P);
    const float L = (float)S.box;
    const float inv_L = 1.0f / L;
    const float rp = mine ? pad_radius((float)ri, L) : -1.f;
    const float rp2 = mine ? rp * rp : -1.f;
    const uint32_t n32 = (uint32_t)S.n, s32 = (uint32_t)s;
    // ---- the walk and the padded tests, passed indices in order ----
    // A sphere that stays a padded radius away from every face of the box
    // reaches no periodic image (box centres and positions lie in the box),
    // so its tests need no nearest-image shift; rows whose sphere crosses a
    // face take it (wave-uniform choice).
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) inside = inside && P[a] > rp + 1e-5f * L && P[a] < L - rp - 1e-5f * L;
    auto phase1 = [&](auto wrap_t) {
      constexpr bool WRAP = decltype(wrap_t)::value;
      auto box2 = [&](float4 c, float4 w) {  // squared gap to the box of centre c
        const float cc[3] = {c.x, c.y, c.z}, ww[3] = {w.x, w.y, w.z};
        float g2 = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          float d = cc[a] - P[a];
          if constexpr (WRAP) d -= L * rintf(d * inv_L);
          const float g = fmaxf(fabsf(d) - ww[a], 0.f);
          g2 += g * g;
        }
        return g2;
      };
      auto gap_at = [&](float4 c, float4 w, const float* Q) {  // box2 from point Q
        const float cc[3] = {c.x, c.y, c.z}, ww[3] = {w.x, w.y, w.z};
        float g2 = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          float d = cc[a] - Q[a];
          if constexpr (WRAP) d -= L * rintf(d * inv_L);
          const float g = fmaxf(fabsf(d) - ww[a], 0.f);
          g2 += g * g;
        }
        return g2;
      };
      auto point2 = [&](float4 c) {  // squared distance to point c
        const float cc[3] = {c.x, c.y, c.z};
        float d2 = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          float d = cc[a] - P[a];
          if constexpr (WRAP) d -= L * rintf(d * inv_L);
          d2 += d * d;
        }
        return d2;
      };
      // (32-bit indices: the tree path takes fewer than 2^25 particles; absp
      // has a whole number of waves of entries, so the last leaf's padding
      // is loaded too, and its tests discarded, without a branch)
      // (the test of particle j at position a; on: the lane has a leaf)
      auto test_at = [&](bool on, uint32_t j, float4 a) {
        const bool pass = on & (j < n32) & (j != s32) & (point2(a) < rp2);
        const uint64_t b = __ballot(pass) & rowbits;
        const int at = np + __popcll(b & below);
        if (pass && at < cap) put(at, j << kCodeBits);
        np += __popc((uint32_t)(b >> (lane & 48)));
      };
      // Reached leaves are queued per row in LDS and tested by all rows in
      // step (a row's q-th queued leaf at step q), so that a wave's leaf tests
      // take as many steps as its longest queue rather than, step by step of
      // the walk, the most leaves any row reached.
      int nbuf = 0;  // uniform over the row
      auto drain = [&]() {
        // the entries the row's lanes wrote are read by the whole row: keep
        // the wave's LDS accesses in program order
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // two queued leaves a step, their position loads in flight together
        // (a row past its queue takes leaf 0 and discards its tests)
        for (int q = 0; __ballot(q < nbuf) != 0ull; q += 2) {
          const bool on0 = q < nbuf, on1 = q + 1 < nbuf;
          const uint32_t j0 = (on0 ? rbuf[q] : 0u) * (uint32_t)kLeaf + (uint32_t)sub;
          const uint32_t j1 = (on1 ? rbuf[q + 1] : 0u) * (uint32_t)kLeaf + (uint32_t)sub;
          const float4 a0 = absp[j0], a1 = absp[j1];
          test_at(on0, j0, a0);
          test_at(on1, j1, a1);
        }
        __builtin_amdgcn_wave_barrier();  // the reads above before the next writes
        nbuf = 0;
      };
      const int top = S.nlevels - 1;
      auto wave_sync = [&]() {  // the wave's LDS writes before its reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      };
      // The four rows of a wave walk the levels above the leaves together,
      // breadth first, for one sphere that holds their four (centre C on
      // their mean, radius Ru): a step tests the children of up to eight
      // frontier nodes, one per lane, and compacts the reached ones, in
      // order, into the next level's frontier. A box that a row's sphere
      // reaches is reached by this sphere (triangle inequality, padded beyond
      // the FP32 rounding), and so are all the boxes above it, which hold
      // it. The level-1 children of the reached level-2 nodes are kept when
      // one of the rows' own spheres reaches them, and each row tests the
      // leaves of the kept ones against its own sphere (two nodes a step, a
      // leaf per lane) and queues the reached leaves: the leaves and the
      // order of its own walk, in far fewer steps (the rows' walks take one
      // node a step, on half of their lanes, and the wave as many steps as
      // its longest walk). Taken while the common sphere stays within
      // kSharedReach times the rows' largest radius (consecutive particles
      // of the first round lie well within it); rows further apart, or a
      // frontier that outgrows its buffer before any leaf is queued, walk
      // alone.
      auto shared_walk = [&]() -> bool {
        float C[3] = {0.f, 0.f, 0.f}, Q0[3];
        float rq[4], off[4][3];
        int f = -1, nm = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          rq[r] = __shfl(rp, 16 * r);  // -1 for a row without a particle
          if (rq[r] > 0.f && f < 0) f = r;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) Q0[a] = __shfl(P[a], 16 * (f < 0 ? 0 : f));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            float d = __shfl(P[a], 16 * r) - Q0[a];
            if constexpr (WRAP) d -= L * rintf(d * inv_L);
            off[r][a] = rq[r] > 0.f ? d : 0.f;
            C[a] += off[r][a];
          }
          nm += rq[r] > 0.f ? 1 : 0;
        }
        float Ru = 0.f, rmax = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) C[a] /= (float)(nm > 0 ? nm : 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float e2 = 0.f;
#pragma unroll
          for (int a = 0; a < 3; ++a) e2 += (off[r][a] - C[a]) * (off[r][a] - C[a]);
          if (rq[r] > 0.f) {
            Ru = fmaxf(Ru, sqrtf(e2) + rq[r]);
            rmax = fmaxf(rmax, rq[r]);
          }
        }
        if (!(nm > 0 && Ru <= kSharedReach * rmax)) return false;
        Ru = Ru * 1.00001f + 4e-6f * L;
        const float Ru2 = Ru * Ru;
#pragma unroll
        for (int a = 0; a < 3; ++a) C[a] += Q0[a];
        auto boxu = [&](float4 c, float4 w) {  // squared gap from C to the box
          const float cc[3] = {c.x, c.y, c.z}, ww[3] = {w.x, w.y, w.z};
          float g2 = 0.f;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            float d = cc[a] - C[a];
            if constexpr (WRAP) d -= L * rintf(d * inv_L);
            const float g = fmaxf(fabsf(d) - ww[a], 0.f);
            g2 += g * g;
          }
          return g2;
        };
        const uint64_t lt = (1ull << lane) - 1ull;  // the wave's lanes before this one
        uint32_t* fa_buf = front[threadIdx.x >> 6][0];
        uint32_t* fb_buf = front[threadIdx.x >> 6][1];
        // the reached children (level cl) of frontier nodes k0 .. k0 + 7,
        // lane 8 k + c taking child c of node k0 + k; node index per lane
        auto expand = [&](int k0, int fa, int cl, uint32_t& ch) -> bool {
          const int k = k0 + (lane >> 3);
          const bool vk = k < fa;
          ch = fa_buf[vk ? k : 0] * (uint32_t)kFan + (uint32_t)(lane & 7);
          const bool valid = vk && ch < (uint32_t)lv.cnt[cl];
          const int node = lv.off[cl] + (valid ? (int)ch : 0);
          return valid && boxu(S.ncen[node], S.nhw[node]) < Ru2;
        };
        int fa = 1;  // the root
        if (lane == 0) fa_buf[0] = 0u;
        wave_sync();
        for (int lvl = top; lvl > 2; --lvl) {
          int fb = 0;
          for (int k0 = 0; k0 < fa; k0 += 8) {
            uint32_t ch;
            const bool reach = expand(k0, fa, lvl - 1, ch);
            const uint64_t m = __ballot(reach);
            const int at = fb + __popcll(m & lt);
            if (reach && at < kFront) fb_buf[at] = ch;
            fb += __popcll(m);
          }
          wave_sync();
          if (fb > kFront) return false;
          uint32_t* t = fa_buf;
          fa_buf = fb_buf;
          fb_buf = t;
          fa = fb;
        }
        // fa_buf: the reached level-2 nodes, ascending. Their children (the
        // level-1 nodes), one per lane, are kept when a row's own sphere
        // reaches them (the bits of m); every row then tests the leaves of
        // the kept nodes against its own sphere, two nodes a step (lanes
        // 8-15 take the second), a leaf per lane.
        for (int k0 = 0; k0 < fa; k0 += 8) {
          const int k = k0 + (lane >> 3);
          const bool vk = k < fa;
          const uint32_t ch = fa_buf[vk ? k : 0] * (uint32_t)kFan + (uint32_t)(lane & 7);
          const bool valid = vk && ch < (uint32_t)lv.cnt[1];
          const int node = lv.off[1] + (valid ? (int)ch : 0);
          const float4 bc = S.ncen[node], bw = S.nhw[node];
          bool any = false;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float Qr[3] = {__shfl(P[0], 16 * r), __shfl(P[1], 16 * r),
                                 __shfl(P[2], 16 * r)};
            const float rr = __shfl(rp, 16 * r);
            any = any || (rr > 0.f && gap_at(bc, bw, Qr) < rr * rr);
          }
          uint64_t m = __ballot(valid && any);
          while (m != 0ull) {
            const int b1 = __builtin_ctzll(m);
            m &= m - 1;
            const int b2 = m != 0ull ? __builtin_ctzll(m) : 64;
            if (m != 0ull) m &= m - 1;
            const int bb = sub < 8 ? b1 : b2;
            const int bs = bb < 64 ? bb : b1;
            const uint32_t l1 = fa_buf[k0 + (bs >> 3)] * (uint32_t)kFan + (uint32_t)(bs & 7);
            const uint32_t leaf = l1 * (uint32_t)kFan + (uint32_t)(sub & 7);
            const bool ok = mine && bb < 64 && leaf < (uint32_t)lv.cnt[0];
            const int ln = lv.off[0] + (ok ? (int)leaf : 0);
            const bool h = ok && box2(S.ncen[ln], S.nhw[ln]) < rp2;
            const uint64_t hb = __ballot(h) & rowbits;
            if (h) rbuf[nbuf + __popcll(hb & below)] = leaf;
            nbuf += __popcll(hb);
            if (__ballot(nbuf > kRowBuf - 16) != 0ull) drain();
          }
        }
        return true;
      };
      const bool shared = top >= 2 && shared_walk();
      int cur = 0, cur_level = top;  // the node whose children are tested next
      uint64_t pend = 0;             // children still to visit, bit 8 l + c at level l
      bool walking = !shared && mine && top > 0;
      if (mine && top == 0) {
        if (sub == 0) rbuf[0] = 0;
        nbuf = 1;
      }
      while (__ballot(walking) != 0ull) {
        if (walking) {
          const int cl = cur_level - 1;
          const int c0 = cur * kFan;
          const int m = min(kFan, lv.cnt[cl] - c0);
          const int node = lv.off[cl] + c0 + (sub < m ? sub : m - 1);
          const bool h = sub < m && box2(S.ncen[node], S.nhw[node]) < rp2;
          const uint64_t hb = __ballot(h) & rowbits;
          const uint32_t mask = (uint32_t)(hb >> (16 * rowid));
          if (cl == 0) {  // the reached leaves, in order, to the row's queue
            if (h) rbuf[nbuf + __popcll(hb & below)] = (uint32_t)(c0 + sub);
            nbuf += __popc(mask);
          } else {
            pend |= (uint64_t)mask << (8 * cl);
          }
          if (pend == 0ull) {
            walking = false;
          } else {  // the deepest pending child; its parent is an ancestor of cur
            const int b = __builtin_ctzll(pend);
            pend &= pend - 1;
            const int lvl = b >> 3;
            cur = ((cur >> (3 * (lvl + 1 - cur_level))) << 3) + (b & 7);
            cur_level = lvl;
          }
        }
        if (__ballot(nbuf > kRowBuf - kFan) != 0ull) drain();  // a queue that could overflow
      }
      drain();
    };
    if (__ballot(!inside) == 0ull)
      phase1(std::false_type());
    else
      phase1(std::true_type());
    // every passed index fitted the row's room: they are its candidates
    fits = mine && np <= cap;
    if (fits) cnt = np;
    if (mine && sub == 0) {
      if (np > cap && S.shrink && S.rad[S.n + s] == R(0)) {
        const double want = 1.3 * 4.18879020478639098 * S.n_h3;
        const double f = fmax(cbrt(want / (double)np), 0.5);
        S.rad[s] = (R)((double)ri * f);
        const int ns = (int)(1.3 * (double)np * f * f * f) + 1;
        S.need[s] = ((ns > 4 ? ns : 4) + 3) & ~3;
        S.ccnt[s] = -1;
        retry = 1;
      } else if (np > cap) {
        S.need[s] = (np + 3) & ~3;
        S.ccnt[s] = -1;
        retry = 1;
      } else if (!STAGE) {
        S.ccnt[s] = cnt;
        S.cpos[s] = (uint32_t)(base >> 2);
        kept = (unsigned long long)cnt;
      }
    }
  }
  if constexpr (STAGE) {
    // the block's kept candidates go to the pool in one piece: each row's
    // count rounded up to 4 entries, their sum taken from the bump counter
    const int row = threadIdx.x >> 4;
    const int c4 = fits ? (cnt + 3) & ~3 : 0;
    if (sub == 0) rcnt[row] = (uint32_t)c4;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long tot = 0;
      for (int q = 0; q < kBlock / 16; ++q) tot += rcnt[q];
      unsigned long long b = tot ? atomicAdd(S.cnt + CNT_POOL * kCntSpread, tot) : 0ull;
      for (int q = 0; q < kBlock / 16; ++q) {
        rbase[q] = b;
        b += rcnt[q];
      }
    }
    __syncthreads();
    if (fits) {
      const unsigned long long b = rbase[row];
      if (b + (unsigned long long)c4 <= (unsigned long long)S.pool_cap) {
        for (int k = 4 * sub; k < c4; k += 64)
          *reinterpret_cast<uint4*>(S.cand + b + k) = *reinterpret_cast<const uint4*>(srow + k);
        if (sub == 0) {
          S.ccnt[s] = cnt;
          S.cpos[s] = (uint32_t)(b >> 2);
          kept = (unsigned long long)cnt;
        }
      } else if (sub == 0) {
        // the pool is full: the next round gives the particle room of its own
        S.need[s] = (np + 3) & ~3;
        S.ccnt[s] = -1;
        retry = 1;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    retry += __shfl_xor(retry, o, 64);
    kept += __shfl_xor(kept, o, 64);
  }
  if (lane == 0 && retry) atomicAdd(cnt_at(S.cnt, CNT_RETRY), retry);
  if (lane == 0 && kept) atomicAdd(cnt_at(S.cnt, CNT_CANDIDATES), kept);
}

// The room every unsolved particle gets in a retry round, in 4-entry units
// (zero for the solved ones; need4[n] = 0 closes the exclusive sums).
template <class R>
__global__ void __launch_bounds__(kBlock) k_need4(State<R> S, uint32_t* __restrict__ need4,
                                                  bool retry) {
  const int64_t s = particle_id();
  if (s < S.n) need4[s] = S.todo[s] ? (uint32_t)(room_for(S.need[s], retry) >> 2) : 0u;
  if (s == 0) need4[S.n] = 0u;
}

// The unsolved particles in rank order.
template <class R>
__global__ void __launch_bounds__(kBlock) k_rank_order(State<R> S, uint32_t* __restrict__ order) {
  const int64_t s = particle_id();
  if (s < S.n && S.todo[s]) order[S.cslot[s]] = (uint32_t)s;
}

// Neighbour lists from the stored candidates of every particle (the
// candidates hold every j with r_ij below the particle's radius, which is at
// least its solved h): the gather list (r_ij < h_i, in candidate order, which
// is ascending j) and the particle's share in the scatter-only lists, the
// transpose: i belongs to j's scatter-only list when i gathers j
// (r_ij < h_i) but j does not gather i (r_ij >= h_j). The separation is
// recomputed as the candidate walk computed it, from i's side; from j's side
// it is the exact negation (lattice offsets and differences negate exactly),
// so j's own gather filter and this test decide alike. COUNT stores the gather lengths and adds to the scatter-only counts
// ns[j]; WRITE (with per-wave capacities from those counts) writes the gather
// entries and appends i at fillc[j] (unordered; sorted afterwards).
// A 16-lane row per particle: the row takes 16 candidates at a time, one per
// lane, and appends the gather entries in order (prefix counts over the
// row's ballot), so that a particle's hundreds of recomputed separations are
// in flight together rather than one after another.
template <class R, bool WRITE>
__global__ void __launch_bounds__(kBlock) k_filter_tree(State<R> S, int* __restrict__ fillc) {
  const int64_t tid = particle_id();
  if (((tid & ~(int64_t)63) >> 4) >= S.n) return;  // the wave's four rows past the end
  const int64_t s = tid >> 4;
  const int lane = threadIdx.x & 63, sub = lane & 15;
  const uint64_t rowbits = 0xFFFFull << (lane & 48);
  const uint64_t below = rowbits & ((1ull << lane) - 1ull);
  const bool active = s < S.n;
  const int64_t sc = active ? s : 0;
  const int cnt = active ? S.ccnt[sc] : 0;  // uniform over the row
  const int64_t base = 4 * (int64_t)S.cpos[sc];
  const R h = S.hbuf[sc];
  const R4<R> pi = S.pos(sc);
  const uint32_t ci = S.cell3[sc];
  int64_t gb = 0;
  if (WRITE) gb = slot_base(S.grow[sc >> 6], sc);
  int ng = 0;  // uniform over the row
  // one group of 16 entries, one per lane, from its loaded records
  auto group = [&](bool in, uint32_t ent, uint32_t j, const R4<R>& pj, uint32_t cj, R hj) {
    R x[3];
    lattice_sep(S, pi, ci, pj, cj, x);
    const R r = Sc<R>::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const bool g = in && r < h;
    const uint64_t b = __ballot(g) & rowbits;
    if (WRITE && g) S.nlist[slot_at(gb, ng + __popcll(b & below))] = ent;
    ng += __popcll(b);
    if (g && !(r < hj)) {  // this particle is in j's scatter-only list
      if (WRITE) {
        const int u = atomicAdd(&fillc[j], 1);
        const int64_t wj = (int64_t)(j >> 6);
        const int scap = (int)(S.srow[wj + 1] - S.srow[wj]) * 4;
        if (u < scap) S.slist[slot_at(slot_base(S.srow[wj], j), u)] = (uint32_t)s << kCodeBits;
      } else {
        atomicAdd(&S.ns[j], 1);
      }
    }
  };
  // two groups a step, every load of both issued before either is used
  // (lanes past the count take entry 0 of the row, whose records they
  // load and discard: the row has an entry whenever the loop runs)
  for (int k = 0; k < cnt; k += 32) {
    const int e0 = k + sub, e1 = k + 16 + sub;
    const bool in0 = e0 < cnt, in1 = e1 < cnt;
    const uint32_t ent0 = S.cand[base + (in0 ? e0 : 0)];
    const uint32_t ent1 = S.cand[base + (in1 ? e1 : 0)];
    const uint32_t j0 = ent0 >> kCodeBits, j1 = ent1 >> kCodeBits;
    const R4<R> p0 = S.pos(j0), p1 = S.pos(j1);
    const uint32_t c0 = S.cell3[j0], c1 = S.cell3[j1];
    const R h0 = S.hbuf[j0], h1 = S.hbuf[j1];
    group(in0, ent0, j0, p0, c0, h0);
    group(in1, ent1, j1, p1, c1, h1);
  }
  unsigned long long gsum = 0;
  if (active && sub == 0) {
    if (WRITE)
      gsum = (unsigned long long)ng;
    else
      S.ng[s] = ng;
  }
  if (WRITE) wave_add_u64(cnt_at(S.cnt, CNT_PAIRS_GATHER), gsum);
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

// Ascending bitonic sorting network over N values held in registers (every
// index is a compile-time constant once the loops unroll).
template <int N>
__device__ inline void bitonic_sort(uint32_t (&a)[N]) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const uint32_t lo = min(a[i], a[l]), hi = max(a[i], a[l]);
          a[i] = (i & k) == 0 ? lo : hi;
          a[l] = (i & k) == 0 ? hi : lo;
        }
      }
    }
  }
}

// One lane's list of ns <= N entries, read as 16-byte chunks, padded with
// 0xffffffff, sorted in registers and written back chunk by chunk.
template <int N>
__device__ inline void sort_list_regs(uint32_t* __restrict__ list, int64_t sb, int ns) {
  uint32_t a[N];
#pragma unroll
  for (int c = 0; c < N / 4; ++c) {
    uint4 q = make_uint4(0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu);
    if (4 * c < ns) q = *reinterpret_cast<const uint4*>(list + slot_at(sb, 4 * c));
    a[4 * c] = 4 * c < ns ? q.x : 0xffffffffu;
    a[4 * c + 1] = 4 * c + 1 < ns ? q.y : 0xffffffffu;
    a[4 * c + 2] = 4 * c + 2 < ns ? q.z : 0xffffffffu;
    a[4 * c + 3] = 4 * c + 3 < ns ? q.w : 0xffffffffu;
  }
  bitonic_sort<N>(a);
#pragma unroll
  for (int c = 0; c < N / 4; ++c)
    if (4 * c < ns)
      *reinterpret_cast<uint4*>(list + slot_at(sb, 4 * c)) =
          make_uint4(a[4 * c], a[4 * c + 1], a[4 * c + 2], a[4 * c + 3]);
}

// Sorts every scatter-only list by j, giving the order a walk would produce
// and making runs reproducible; counts the force pairs. Lists of at most 32
// entries are sorted in their lane's registers (a network of the wave's size
// class); longer ones are queued (queue[], their number in the slot 0 of
// CNT_LONG_LISTS) for k_sort_long.
constexpr int kShortList = 32;
template <class R>
__global__ void __launch_bounds__(kBlock) k_scatter_sort(State<R> S, uint32_t* __restrict__ queue) {
  const int64_t s = particle_id();
  if ((s & ~(int64_t)63) >= S.n) return;
  unsigned long long f = 0;
  int ns = 0;
  int64_t sb = 0;
  if (s < S.n) {
    const int64_t w = s >> 6;
    const int scap = (int)(S.srow[w + 1] - S.srow[w]) * 4;
    ns = S.ns[s] < scap ? S.ns[s] : scap;
    sb = slot_base(S.srow[w], s);
    f = (unsigned long long)(S.ng[s] + S.ns[s]);
  }
  if (ns > kShortList) {
    queue[atomicAdd(S.cnt + CNT_LONG_LISTS * kCntSpread, 1ull)] = (uint32_t)s;
    ns = 0;
  }
  int big = ns;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) big = max(big, __shfl_xor(big, o, 64));
  if (big > 16) {
    sort_list_regs<32>(S.slist, sb, ns);
  } else if (big > 8) {
    sort_list_regs<16>(S.slist, sb, ns);
  } else if (big > 1) {
    sort_list_regs<8>(S.slist, sb, ns);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o, 64);
  if ((threadIdx.x & 63) == 0 && f) atomicAdd(cnt_at(S.cnt, CNT_PAIRS_FORCE), f);
}

// The queued long scatter-only lists, one per single-wave block in turn: up
// to kLongSort entries are padded to a power of two with 0xffffffff and
// sorted by a bitonic network in LDS (each compare-exchange owned by the lane
// of its lower index, a barrier between steps); a longer list takes an
// insertion sort in memory by one lane.
constexpr int kLongSort = 4096;
template <class R>
__global__ void __launch_bounds__(64) k_sort_long(State<R> S, const uint32_t* __restrict__ queue) {
  __shared__ uint32_t buf[kLongSort];
  const unsigned long long nq = S.cnt[CNT_LONG_LISTS * kCntSpread];
  const int lane = threadIdx.x;
  for (unsigned long long q = blockIdx.x; q < nq; q += gridDim.x) {
    const int64_t s = queue[q];
    const int64_t w = s >> 6;
    const int scap = (int)(S.srow[w + 1] - S.srow[w]) * 4;
    const int ns = S.ns[s] < scap ? S.ns[s] : scap;
    const int64_t sb = slot_base(S.srow[w], s);
    if (ns > kLongSort) {
      if (lane == 0) {
        for (int a = 1; a < ns; ++a) {
          const uint32_t v = S.slist[slot_at(sb, a)];
          int b = a - 1;
          while (b >= 0 && S.slist[slot_at(sb, b)] > v) {
            S.slist[slot_at(sb, b + 1)] = S.slist[slot_at(sb, b)];
            --b;
          }
          S.slist[slot_at(sb, b + 1)] = v;
        }
      }
      continue;
    }
    int P = 64;
    while (P < ns) P <<= 1;
    for (int k = lane; k < P; k += 64) buf[k] = k < ns ? S.slist[slot_at(sb, k)] : 0xffffffffu;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = lane; i < P; i += 64) {
          const int l = i ^ j;
          if (l > i) {
            const uint32_t a = buf[i], b = buf[l];
            if ((a > b) == ((i & k) == 0)) {
              buf[i] = b;
              buf[l] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int k = lane; k < ns; k += 64) S.slist[slot_at(sb, k)] = buf[k];
    __syncthreads();  // the reads above before the next list's writes
  }
}

}  // namespace

void launch_morton(const double* x, int64_t n, double box, uint32_t* keys, uint32_t* vals,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_morton, dim3(grid_for(n)), dim3(kBlock), 0, s, x, n, box, keys, vals);
}

template <class R>
void launch_tree_build(const State<R>& S, const R* h, float4* absp, const int* host_off,
                       const int* host_cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_leaf_boxes<R>, dim3(grid_for(host_cnt[0])), dim3(kBlock), 0, s, S, h,
                     absp);
  for (int l = 0; l + 1 < S.nlevels; ++l)
    hipLaunchKernelGGL(k_tree_up, dim3(grid_for(host_cnt[l + 1])), dim3(kBlock), 0, s, S.ncen,
                       S.nhw, host_off[l], host_cnt[l], host_off[l + 1], host_cnt[l + 1]);
  const int nnode = host_off[S.nlevels - 1] + host_cnt[S.nlevels - 1];
  hipLaunchKernelGGL(k_box_centres, dim3(grid_for(nnode)), dim3(kBlock), 0, s, S.ncen, S.nhw,
                     nnode);
}

template <class R>
void launch_init_radius(const State<R>& S, int h_mode, hipStream_t s) {
  hipLaunchKernelGGL(k_init_radius<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S, h_mode);
}

template <class R>
void launch_rank_order(const State<R>& S, uint32_t* order, hipStream_t s) {
  hipLaunchKernelGGL(k_rank_order<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S, order);
}

template <class R>
void launch_candidates_tree(const State<R>& S, const float4* absp, int kernel, bool stage,
                            const uint32_t* order, int64_t nt, hipStream_t s) {
  if (nt <= 0) return;
  const dim3 g(grid_for(16 * nt)), b(kBlock);  // a 16-lane row per particle
  auto go = [&](auto em, auto st) {
    constexpr bool EM = decltype(em)::value, ST = decltype(st)::value;
    if (kernel == 0)
      hipLaunchKernelGGL((k_candidates_tree<R, 0, EM, ST>), g, b, 0, s, S, absp, order, nt);
    else
      hipLaunchKernelGGL((k_candidates_tree<R, 1, EM, ST>), g, b, 0, s, S, absp, order, nt);
  };
  if (S.equal_mass) {
    if (stage)
      go(std::true_type(), std::true_type());
    else
      go(std::true_type(), std::false_type());
  } else {
    if (stage)
      go(std::false_type(), std::true_type());
    else
      go(std::false_type(), std::false_type());
  }
}

bool stage_fits(int scr_cap) { return scr_cap <= kStage; }

template <class R>
void launch_hsolve_tree(const State<R>& S, int kernel, const uint32_t* order, int64_t nt,
                        hipStream_t s) {
  if (nt <= 0) return;
  const dim3 g(grid_for(16 * nt)), b(kBlock);  // a 16-lane row per particle
  if (S.equal_mass) {
    if (kernel == 0)
      hipLaunchKernelGGL((k_hsolve_rows<R, 0, true>), g, b, 0, s, S, order, nt);
    else
      hipLaunchKernelGGL((k_hsolve_rows<R, 1, true>), g, b, 0, s, S, order, nt);
  } else {
    if (kernel == 0)
      hipLaunchKernelGGL((k_hsolve_rows<R, 0, false>), g, b, 0, s, S, order, nt);
    else
      hipLaunchKernelGGL((k_hsolve_rows<R, 1, false>), g, b, 0, s, S, order, nt);
  }
}

template <class R>
void launch_need4(const State<R>& S, uint32_t* need4, bool retry, hipStream_t s) {
  hipLaunchKernelGGL(k_need4<R>, dim3(grid_for(S.n + 1)), dim3(kBlock), 0, s, S, need4, retry);
}

template <class R>
void launch_filter_tree(const State<R>& S, bool write, int* fillc, uint32_t* queue,
                        hipStream_t s) {
  if (write) {
    hipLaunchKernelGGL((k_filter_tree<R, true>), dim3(grid_for(16 * S.n)), dim3(kBlock), 0, s,
                       S, fillc);
    hipLaunchKernelGGL(k_scatter_sort<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S, queue);
    hipLaunchKernelGGL(k_sort_long<R>, dim3(1024), dim3(64), 0, s, S, (const uint32_t*)queue);
  } else {
    hipLaunchKernelGGL((k_filter_tree<R, false>), dim3(grid_for(16 * S.n)), dim3(kBlock), 0, s,
                       S, fillc);
  }
}

void launch_wave_rows(const int* cnt, int64_t n, int extra, uint32_t* rows, hipStream_t s) {
  hipLaunchKernelGGL(k_wave_rows, dim3(grid_for(n)), dim3(kBlock), 0, s, cnt, n, extra, rows);
}

#define CRK_INSTANTIATE_TREE(R)                                                               \
  template void launch_tree_build<R>(const State<R>&, const R*, float4*, const int*, const int*,      \
                                     hipStream_t);                                           \
  template void launch_init_radius<R>(const State<R>&, int, hipStream_t);                    \
  template void launch_rank_order<R>(const State<R>&, uint32_t*, hipStream_t);              \
  template void launch_candidates_tree<R>(const State<R>&, const float4*, int, bool,         \
                                          const uint32_t*, int64_t, hipStream_t);            \
  template void launch_hsolve_tree<R>(const State<R>&, int, const uint32_t*, int64_t,       \
                                      hipStream_t);                                          \
  template void launch_need4<R>(const State<R>&, uint32_t*, bool, hipStream_t);               \
  template void launch_filter_tree<R>(const State<R>&, bool, int*, uint32_t*, hipStream_t);

CRK_INSTANTIATE_TREE(float)
CRK_INSTANTIATE_TREE(double)

}  // namespace crk
