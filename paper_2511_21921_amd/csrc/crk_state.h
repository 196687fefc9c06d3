// Device state of one evaluation: the cell list and the cell-sorted
// structure-of-arrays intermediates, passed by value to every pass kernel.
#pragma once

#include "crk_device.h"

namespace crk {

constexpr int kLeaf = 16;        // tree path: particles per search leaf (a Morton run)
constexpr int kFan = 8;          // tree path: children per tree node
constexpr int kMaxLevels = 40;   // tree path: largest number of tree levels

// Counters of one evaluation (unsigned long long, kCntSpread slots each).
enum Counter {
  CNT_HMAX_BITS = 0,   // max input h as double bits
  CNT_BAD_INPUT,       // h <= 0, m <= 0 or u <= 0
  CNT_PAIRS_GATHER,
  CNT_PAIRS_FORCE,
  CNT_H_ITER_MAX,
  CNT_H_UNCONV,
  CNT_H_CAPPED,
  CNT_SCR_OVERFLOW,    // largest candidate count beyond the candidate capacity
  CNT_LIST_OVERFLOW,   // largest gather count beyond the list capacity
  CNT_SLIST_OVERFLOW,  // largest scatter-only count beyond its capacity
  CNT_MMAX_BITS,       // max mass as double bits
  CNT_MINVMAX_BITS,    // max 1/mass as double bits
  CNT_RETRY,           // particles that need another candidate round (tree path)
  CNT_SINGULAR,
  CNT_RELAXED,
  CNT_NONFINITE,
  CNT_HMAX_OUT_BITS,   // max solved h as double bits
  CNT_CELL_MAX,        // largest cell occupancy of the cell list
  CNT_TOO_DENSE,       // a cell beyond the occupancy limit of a speculative cell list
  CNT_CANDIDATES,      // candidates kept by the neighbour search (all its passes)
  CNT_LONG_LISTS,      // tree path: scatter-only lists queued for the wave sort (slot 0 only)
  CNT_POOL,            // tree path: candidate pool entries taken by staged blocks (slot 0 only)
  CNT_MOVED,           // particles whose cell differs from the kept cell list's
  CNT_ACTIVE,          // hierarchy: particles active at the substep's end
  CNT_ACTLIST,         // hierarchy: length of the active list (slot 0 only)
  CNT_COUNT
};

// Every counter lives in kCntSpread slots; a block adds to the slot of its
// index modulo kCntSpread and the host folds the slots (sum, or max for the
// maxima). Atomics on one address serialise in the memory-side atomic unit,
// and a per-wave counter of a kernel whose waves all end together would
// queue thousands of them behind its last wave.
constexpr int kCntSpread = 64;
__device__ inline unsigned long long* cnt_at(unsigned long long* cnt, int c) {
  return cnt + c * kCntSpread + (blockIdx.x & (kCntSpread - 1));
}

// A wave's sum (or maximum) of v, added (or maxed) into *dst by its lane 0.
__device__ inline void wave_add_u64(unsigned long long* dst, unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
}
__device__ inline void wave_max_u64(unsigned long long* dst, unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long t = __shfl_xor(v, o, 64);
    v = t > v ? t : v;
  }
  if ((threadIdx.x & 63) == 0 && v) atomicMax(dst, v);
}

// Bits of a non-negative double, ordered as the value (counter maxima).
__device__ inline unsigned long long dbits(double d) {
  return (unsigned long long)__double_as_longlong(d);
}

template <class R>
struct State {
  int64_t n;
  int G;              // cells per side (lattice cells per side when lattice = 1)
  int lattice;        // 0: cell list with stencil codes; 1: tree over a fine lattice
  double box, ell_d;  // box side and cell side (FP64)
  R ell;              // cell side in Real
  // cell list
  const uint32_t* perm;        // sorted -> caller index
  const uint32_t* keys;        // sorted cell keys
  const uint32_t* cell_start;  // [G^3 + 1]
  uint32_t* cell3;             // packed cell coordinates x | y << 10 | z << 20
  // sorted particle data: position and velocity records side by side, so
  // that a neighbour's pair (one aligned 2 x Real4) is one fetch
  R4<R>* pv;    // [2 i]: (xi_x, xi_y, xi_z, 1/h); [2 i + 1]: (v_x, v_y, v_z, V)
  __device__ R4<R>& pos(int64_t i) const { return pv[2 * i]; }
  __device__ R4<R>& vel(int64_t i) const { return pv[2 * i + 1]; }
  R* mass;
  R* uu;
  R* hbuf;      // h (in: input or guess)
  R* Vbuf;
  R4<R>* st4;   // (rho, P, c, den) with den = sum V_j^2 W^R_ij
  R4<R>* gv4;   // 3 per particle: grad v rows, then (gv_22, relaxed, 0, 0)
  R4<R>* kc4;   // 4 per particle: packed corrected-kernel coefficients
  R* mom;       // [40][n] moments kept for the adjoint (may be null)
  // neighbour lists (chunked SELL): gather entries (r < h_i) and
  // scatter-only entries (h_i <= r < h_j)
  uint32_t* nlist;
  uint32_t* slist;
  int* ng;
  int* ns;
  int list_cap;
  int slist_cap;
  // per-wave capacities (tree path): chunk-row offset of every wave's gather
  // and scatter-only lists, one entry per wave plus the total; null when
  // every wave has list_cap / slist_cap
  const uint32_t* grow;
  const uint32_t* srow;
  // candidates within rcap of each particle (16-entry groups, group_base):
  // packed entries, r, and m_j/m_i (the last only when the masses differ);
  // scr_cap is a multiple of 16
  uint32_t* cand;
  R* scr_r;
  R* scr_m;
  int* ccnt;
  int scr_cap;
  int equal_mass;
  R rcap;
  R* rad;             // per-particle candidate radius (tree path) or null; followed
                      // (at rad + n) by the largest radius known to lie below the root
  int* need;          // per-particle candidate capacity request (tree path) or null
  int* todo;          // per-particle "h not solved yet" flag (tree path) or null
  // tree path: rank of each particle among the unsolved ones; null on the
  // cell path
  const uint32_t* cslot;
  // tree path candidate pool (cand), every particle's candidates contiguous
  // from entry 4 cpos[s]: a round that stages them in LDS (the first, when
  // the capacity fits) appends each block's at a bump counter (the slot 0 of
  // CNT_POOL) below pool_cap entries; the other rounds give particle s the
  // room need[s] at 4 (pool_base4 + coff4[s]) (coff4: exclusive sums of the
  // requests of the round, in 4-entry units)
  const uint32_t* coff4;
  int64_t pool_base4;
  int64_t pool_cap;
  int shrink;         // tree path: adapt the radius of an overflowing particle
  // tree over leaves of kLeaf Morton-sorted particles (tree path): node boxes,
  // built as (x, y, z, h_max) low and (x, y, z, -) high corners, then kept as
  // (centre, h_max) in ncen and (half-widths, -) in nhw
  float4* ncen;
  float4* nhw;
  const int* lvl_off;  // [2 kMaxLevels]: node offset of each level (level 0 =
                       // leaves), then the node count of each level
  int nlevels;
  // tree path: where each particle's candidates start, in 4-entry units
  uint32_t* cpos;
  unsigned long long* cnt;
  // parameters
  double n_h3, gamma, alpha, beta, eps2, dt_relax, rtol;
  int max_iter;
  // timestep hierarchy (App. A.3, A.4; levels null: every particle active).
  // A particle of level L is passive at the end of substep jend unless
  // 2^(lev_max - L) divides jend. Passive particles collect no candidates or
  // lists, skip the volume, moment, density and force sums and take V, rho,
  // grad v and the corrections A, B, grad A, grad B from these caller-order
  // arrays (their state of the last evaluation, V and rho updated while
  // passive) when an active particle's force pair reads them.
  const int* levels;
  int lev_max;
  int jend;  // substep end, at most 2^30
  const R* pV;
  const R* prho;
  const R* pgv;
  const R* pA;
  const R* pB;
  const R* pgA;
  const R* pgB;
  // per sorted particle, set by the neighbour-list pass for the active
  // particles and their list partners: the passive particles whose stored
  // state a force pair reads (null: every particle's state is packed)
  uint8_t* needed;
  // a substep with few active particles: their sorted slots (as many as the
  // slot 0 of CNT_ACTLIST counts, in no particular order); the pair passes
  // then give each a 16-lane row, in grids of nact rows, a bound on that
  // number (act null: a thread per particle)
  const uint32_t* act;
  int64_t nact;
};

// whether sorted particle s is passive (reads nothing without a hierarchy)
template <class R>
__device__ inline bool is_passive(const State<R>& S, int64_t s) {
  if (!S.levels) return false;
  const long long per = 1ll << (S.lev_max - S.levels[S.perm[s]]);
  return ((long long)S.jend & (per - 1)) != 0;
}

__device__ inline int wrap_cell(int c, int G) { return c < 0 ? c + G : (c >= G ? c - G : c); }

// Wave broadcast of lane k's value (k wave-uniform).
__device__ inline float bcast(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ inline double bcast(double v, int k) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
  return __hiloint2double(hi, lo);
}
__device__ inline int bcast(int v, int k) { return __builtin_amdgcn_readlane(v, k); }

// Periodic separation x_ij = x_i - x_j. Cell-list path: from the stencil
// code of the list entry. Lattice path: from both particles' lattice
// coordinates, the difference wrapped to the nearest periodic image.
template <class R>
__device__ inline void pair_x(const State<R>& S, int64_t s, const R4<R>& pi, const R4<R>& pj,
                              uint32_t e, R x[3]) {
  if (!S.lattice) {
    pair_sep<R>(pi, pj, e & kCodeMask, S.ell, x);
    return;
  }
  const uint32_t a = S.cell3[s], b = S.cell3[e >> kCodeBits];
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

// Index of this thread's particle, with the block index remapped so that
// each of the 8 XCDs (which receive blocks round-robin, block b on XCD
// b mod 8) processes one contiguous eighth of the blocks: particles that
// are close in the sorted order, and so share neighbours, then share that
// XCD's L2 instead of being fetched by all eight.
__device__ inline int64_t particle_id() {
  const int64_t B = gridDim.x, b = blockIdx.x;
  const int64_t q = B >> 3, r = B & 7, x = b & 7, i = b >> 3;
  const int64_t blk = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
  return blk * kBlock + threadIdx.x;
}

// Tree path radius growth when the h root lies beyond the radius: by the
// factor that would bring the candidate count to the target (4 pi / 3) n_h^3
// at the density seen, x1.1, kept within [1.25, 4].
__device__ inline double grow_factor(double n_h3, int cnt) {
  const double g = 1.1 * cbrt(4.18879020478639098 * n_h3 / (double)(cnt > 1 ? cnt : 1));
  return g < 1.25 ? 1.25 : (g > 4.0 ? 4.0 : g);
}

// First h of the solve: the h at which cnt candidates within Rcap would be
// (4 pi / 3) n_h^3 at uniform density, Rcap (target / cnt)^(1/3), unless the
// caller's h lies within a factor 1.5 of it (a previous step's h); always
// inside (0, Rcap). The root does not depend on it, only the iterations do.
template <class R>
__device__ inline R first_h(R h_in, R Rcap, int cnt, double n_h3) {
  const double est = (double)Rcap * cbrt(4.18879020478639098 * n_h3 / (double)(cnt > 1 ? cnt : 1));
  double h = (double)h_in;
  if (!(h > est / 1.5 && h < est * 1.5)) h = est;
  if (!(h > 0.0 && h < (double)Rcap)) h = 0.5 * (double)Rcap;
  return (R)h;
}

// Capacity to request for the grown radius: the count scaled by the volume,
// with 30% room, in whole 4-entry chunks.
__device__ inline int need_after_growth(int cnt, double g) {
  const double v = 1.3 * (double)(cnt > 1 ? cnt : 1) * g * g * g;
  const int c = v < 1e8 ? (int)v : 100000000;
  return (c + 3) & ~3;
}

// Tree path: the room a round gives a particle that asks for need entries,
// in whole 4-entry chunks: in a retry round half as much again (an overflow
// of the estimate costs another round); in the first, where every particle
// asks for the uniform capacity, just that.
__device__ inline int room_for(int need, bool retry) {
  return (need + (retry ? need >> 1 : 0) + 3) & ~3;
}

// First word and capacity of particle s's candidate scratch on the cell
// path: slot s with the uniform capacity.
template <class R>
__device__ inline int64_t scratch_base(const State<R>& S, int64_t s, int& cap) {
  cap = S.scr_cap;
  return group_base((s >> 6) * (int64_t)(S.scr_cap >> 4), s);
}

// Where particle s's symmetric neighbour list lives: the gather part
// (r < h_s) and the scatter-only part (h_s <= r < h_j), with their lengths.
struct NbrRef {
  int64_t gb, sb;
  int ng, ns;
};

template <class R>
__device__ inline NbrRef nbr_ref(const State<R>& S, int64_t s) {
  const int64_t w = s >> 6;
  int64_t g0, s0;
  int gcap, scap;
  if (S.grow) {
    g0 = S.grow[w];
    s0 = S.srow[w];
    gcap = (int)(S.grow[w + 1] - S.grow[w]) * 4;
    scap = (int)(S.srow[w + 1] - S.srow[w]) * 4;
  } else {
    g0 = w * (S.list_cap >> 2);
    s0 = w * (S.slist_cap >> 2);
    gcap = S.list_cap;
    scap = S.slist_cap;
  }
  NbrRef r;
  r.gb = slot_base(g0, s);
  r.sb = slot_base(s0, s);
  r.ng = S.ng[s] < gcap ? S.ng[s] : gcap;
  r.ns = S.ns[s] < scap ? S.ns[s] : scap;
  return r;
}

// Entry t of the symmetric list, gather part first, for t = 0, 1, 2, ... in
// order: each 4-entry chunk is read with one 16-byte load into buf.
template <class R>
__device__ inline uint32_t nbr_entry(const State<R>& S, const NbrRef& r, int t, uint4& buf) {
  const bool g = t < r.ng;
  const int k = g ? t : t - r.ng;
  if ((k & 3) == 0)
    buf = *reinterpret_cast<const uint4*>(g ? S.nlist + slot_at(r.gb, k)
                                            : S.slist + slot_at(r.sb, k));
  const int q = k & 3;
  return q == 0 ? buf.x : (q == 1 ? buf.y : (q == 2 ? buf.z : buf.w));
}

// Entry t of the symmetric list, reading each 4-entry chunk with one 16-byte
// load into the lane's own LDS slot (no barrier: a lane touches only its
// slot). The chunk then holds no registers across the pair computation.
template <class R>
__device__ inline uint32_t nbr_entry_lds(const State<R>& S, const NbrRef& r, int t, uint4* slot) {
  const bool g = t < r.ng;
  const int k = g ? t : t - r.ng;
  if ((k & 3) == 0)
    *slot = *reinterpret_cast<const uint4*>(g ? S.nlist + slot_at(r.gb, k)
                                              : S.slist + slot_at(r.sb, k));
  return reinterpret_cast<const uint32_t*>(slot)[k & 3];
}

// Entry t of the symmetric list with a 4-byte load of its own (for kernels
// that cannot spare the registers of the chunk buffer).
template <class R>
__device__ inline uint32_t nbr_entry1(const State<R>& S, const NbrRef& r, int t) {
  return t < r.ng ? S.nlist[slot_at(r.gb, t)] : S.slist[slot_at(r.sb, t - r.ng)];
}

// Entry k of the gather list alone, for k = 0, 1, 2, ... in order.
template <class R>
__device__ inline uint32_t gather_entry(const State<R>& S, const NbrRef& r, int k, uint4& buf) {
  if ((k & 3) == 0) buf = *reinterpret_cast<const uint4*>(S.nlist + slot_at(r.gb, k));
  const int q = k & 3;
  return q == 0 ? buf.x : (q == 1 ? buf.y : (q == 2 ? buf.z : buf.w));
}

}  // namespace crk
