// Launch wrappers of the forward and adjoint pass kernels (host side).
#pragma once

#include "crk_internal.h"
#include "crk_state.h"

namespace crk {

// Max of positive h (as double bits) and a count of bad inputs.
template <class R>
void launch_check_inputs(const double* x, const R* h, const R* m, const R* u, int64_t n,
                         unsigned long long* cnt, hipStream_t s);

// Cell keys of wrapped positions, identity values, and per-cell counts.
void launch_keys(const double* x, int64_t n, double box, int G, uint32_t* keys, uint32_t* vals,
                 hipStream_t s);
void launch_cell_bounds(const uint32_t* keys, int64_t n, int64_t ncell, uint32_t* start,
                        unsigned long long occ_limit, unsigned long long* cnt, hipStream_t s);
// Counts in CNT_MOVED the sorted slots whose particle's cell (from x) is no
// longer keys[s]: zero means the kept cell list still sorts x.
void launch_keys_check(const double* x, int64_t n, double box, int G, const uint32_t* keys,
                       const uint32_t* perm, unsigned long long* cnt, hipStream_t s);

// Morton keys over the 1024^3 lattice (tree path) and identity values.
void launch_morton(const double* x, int64_t n, double box, uint32_t* keys, uint32_t* vals,
                   hipStream_t s);
// Leaf boxes (with the largest h of each leaf, from h) and the node levels.
template <class R>
void launch_tree_build(const State<R>& S, const R* h, float4* absp, const int* host_off,
                       const int* host_cnt, hipStream_t s);
template <class R>
void launch_init_radius(const State<R>& S, int h_mode, hipStream_t s);
// The particles still to solve in rank order: order[cslot[s]] = s.
template <class R>
void launch_rank_order(const State<R>& S, uint32_t* order, hipStream_t s);
// Candidates of the unsolved particles, a 16-lane row per particle: row t
// takes particle t (order null) or order[t], for t < nt. stage: the rows
// work in LDS (capacity scr_cap, at most what stage_fits allows) and the
// blocks append to the pool at the CNT_POOL counter, below pool_cap; else
// each particle works in its room of need[s] at pool_base4 + coff4[s].
template <class R>
void launch_candidates_tree(const State<R>& S, const float4* absp, int kernel, bool stage,
                            const uint32_t* order, int64_t nt, hipStream_t s);
bool stage_fits(int scr_cap);
// The h solve (solved h) or the volume (fixed h) of the particles whose
// candidates the round kept, a 16-lane row per particle (order as above).
template <class R>
void launch_hsolve_tree(const State<R>& S, int kernel, const uint32_t* order, int64_t nt,
                        hipStream_t s);
// need4[s]: the room unsolved particle s gets (room_for), in 4-entry units (0
// when solved), and need4[n] = 0; retry: a round after the first
template <class R>
void launch_need4(const State<R>& S, uint32_t* need4, bool retry, hipStream_t s);
// Gather lists and the scatter-only lists (their transpose) from the kept
// candidates: lengths and scatter-only counts (write = false), then entries,
// the scatter-only ones appended at fillc and then sorted (queue: room for n
// particle indices, the lists too long to sort in registers; the counter
// CNT_LONG_LISTS must start at zero).
template <class R>
void launch_filter_tree(const State<R>& S, bool write, int* fillc, uint32_t* queue,
                        hipStream_t s);
void launch_wave_rows(const int* cnt, int64_t n, int extra, uint32_t* rows, hipStream_t s);

// Hierarchy: CNT_ACTIVE counts the particles active at the end of substep
// jend; the active sorted slots appended to list (CNT_ACTLIST, slot 0, must
// start at zero).
void launch_count_active(const int* levels, int64_t n, int lmax, int64_t jend,
                         unsigned long long* cnt, hipStream_t s);
template <class R>
void launch_active_list(const State<R>& S, uint32_t* list, hipStream_t s);

// Gather caller arrays into cell-sorted SoA with cell-centre offsets.
template <class R>
void launch_gather(const State<R>& S, const double* x, const R* v, const R* m, const R* u,
                   const R* h, hipStream_t s);

// Candidates within rcap (every j != i that any later pass can need).
template <class R>
void launch_candidates(const State<R>& S, hipStream_t s);
template <class R>
void launch_hsolve(const State<R>& S, int kernel, hipStream_t s);
template <class R>
void launch_volume(const State<R>& S, int kernel, hipStream_t s);
// Stores 1/h and V into the packed records and writes h, V in caller order.
template <class R>
void launch_pack(const State<R>& S, R* h_out, R* V_out, hipStream_t s);
template <class R>
void launch_nlist(const State<R>& S, hipStream_t s);

struct CorrOut {
  void *A, *B, *gradA, *gradB;
};
template <class R>
void launch_moments(const State<R>& S, int kernel, CorrOut o, hipStream_t s);
template <class R>
void launch_density(const State<R>& S, int kernel, R* rho_out, R* gradv_out, hipStream_t s);
template <class R>
void launch_force(const State<R>& S, int kernel, double* accel, double* dudt, hipStream_t s);

// Non-finite output count over a Real array and a double array.
template <class R>
void launch_count_nonfinite(const R* a, int64_t na, unsigned long long* cnt, hipStream_t s);
void launch_count_nonfinite_f64(const double* a, int64_t na, unsigned long long* cnt,
                                hipStream_t s);

// ---- adjoint ------------------------------------------------------------
template <class R>
struct AdjState {
  // per-particle adjoint accumulators (sorted order, FP64)
  double* gx;    // [3][n] position adjoint
  double* gv;    // [3][n] velocity adjoint
  double* gu;    // [n] internal-energy adjoint
  double* gh;    // [n] smoothing-length adjoint (direct terms)
  double* gV;    // [n] volume adjoint
  double* gkc;   // [16][n] adjoint of the packed corrections (a, b, c, M)
  double* gab;   // [2][blocks] per-block alpha, beta partial sums
  // records gathered from neighbours, packed per particle in Real:
  R4<R>* wgt4;   // (w_a / m, w_u / (2 m)) loss weights over the mass, sorted order
  R4<R>* gvc4;   // 3 per particle: grad v adjoint (9), Num bar, Den bar, 0
  R4<R>* mom4;   // 10 per particle: adjoint of the 40 raw moment sums
  R* kap;        // [n] volume / smoothing-length coefficient kappa
  const double* w_a;  // [3][n] loss weights on accel, caller order
  const double* w_u;  // [n] loss weights on du/dt, caller order
};

// Writes zeros to a[0 .. na) with a kernel (no memset node in a captured graph).
void launch_zero_f64(double* a, int64_t na, hipStream_t s);

template <class R>
void launch_bwd_prep(const State<R>& S, const AdjState<R>& G, hipStream_t s);
template <class R>
void launch_bwd_force(const State<R>& S, const AdjState<R>& G, int kernel, hipStream_t s);
template <class R>
void launch_bwd_density(const State<R>& S, const AdjState<R>& G, int kernel, hipStream_t s);
template <class R>
void launch_bwd_corr(const State<R>& S, const AdjState<R>& G, int kernel, hipStream_t s);
template <class R>
void launch_bwd_moments(const State<R>& S, const AdjState<R>& G, int kernel, int h_mode,
                        hipStream_t s);
template <class R>
void launch_bwd_volume(const State<R>& S, const AdjState<R>& G, int kernel, hipStream_t s);
template <class R>
void launch_bwd_finish(const State<R>& S, const AdjState<R>& G, double* g_x, double* g_v,
                       double* g_u, double* g_ab, hipStream_t s);

// time step (caller order, elementwise)
template <class R>
void launch_kick_drift(int64_t n, double dt, double lam, double n_h, double box, double* x, R* v,
                       R* u, R* h, const R* V, const R* gradv, const double* accel,
                       const double* dudt, R* vp, R* up, hipStream_t s);
template <class R>
void launch_kick_close(int64_t n, double dt, R* v, R* u, const double* accel, const double* dudt,
                       hipStream_t s);

// timestep hierarchy (caller order, elementwise)
template <class R>
void launch_hier_open(int64_t n, const int* levels, int lmax, int64_t jend, double dt_min,
                      double lam, double n_h, const R* v, const R* u, const R* h, const R* V,
                      const R* gradv, const double* accel, const double* dudt, R* vh, R* uh,
                      double* hdot, hipStream_t s);
template <class R>
void launch_hier_drift(int64_t n, const int* levels, int lmax, int64_t j, double dt_min,
                       double n_h, double box, double* x, const R* vh, const double* accel, R* h,
                       const double* hdot, R* V, R* rho, const R* gradv, hipStream_t s);
template <class R>
void launch_hier_predict(int64_t n, const int* levels, int lmax, int64_t jend, double dt_min,
                         const R* vh, const R* uh, const double* accel, const double* dudt, R* vp,
                         R* up, hipStream_t s);
template <class R>
void launch_hier_close(int64_t n, const int* levels, int lmax, int64_t jend, double dt_min, R* v,
                       R* u, const R* vh, const R* uh, const double* acc1, const double* du1,
                       double* accel, double* dudt, hipStream_t s);
// timestep refinement (App. A.5): re-synchronise and reopen the particles
// refined at substep j on their finer level (lvl: the current levels)
template <class R>
void launch_hier_refine(int64_t n, int64_t j, const int* refine_at, const int* refine_level,
                        int* lvl, int lmax, double dt_min, double lam, double n_h, R* v, R* u,
                        const R* h, const R* V, const R* gradv, const double* accel,
                        const double* dudt, R* vh, R* uh, double* hdot, hipStream_t s);
// largest level and bad levels or refinements (refine_at null: none), the
// particles per level (hist[L], L <= 30) and the refined ones (hist[31]; hist
// must start at zero), then refinements off their level's grid for the
// largest level lmax
void launch_level_range(const int* levels, const int* refine_at, const int* refine_level,
                        int64_t n, unsigned long long* cnt, unsigned long long* hist,
                        hipStream_t s);
void launch_refine_grid(const int* refine_at, const int* refine_level, int64_t n, int lmax,
                        unsigned long long* cnt, hipStream_t s);

// subgrid deposition: the gas grid, the source passes, the pair list and
// the per-gas sums (caller order)
void launch_point_keys(const double* x, int64_t n, double box, int G, uint32_t* keys,
                       uint32_t* vals, hipStream_t s);
template <class R>
void launch_max_bits(const R* a, int64_t n, unsigned long long* cnt, int slot, hipStream_t s);
// the sorted gas of one deposition call (p4: double4 x, y, z, h per gas)
struct DepGrid {
  int G;
  double box;
  double hmax;            // the largest gas h
  const uint32_t* start;  // [G^3 + 1]
  const uint32_t* perm;   // [n] sorted -> caller index
  const void* p4;         // [n] double4
  const void* pv;         // [n] double2: V (-1 where the gas may not receive), 1 / h
};
template <class R>
void launch_dep_pack(const uint32_t* perm, uint32_t* rank, const double* xg, int64_t ng,
                     const R* hg, const R* Vg, const R* mg, const R* mZg, double z_max,
                     double m_max, void* p4, void* pv, hipStream_t s);
template <class R>
void launch_dep_volume(int kernel, const DepGrid& d, const double* xs, int64_t ns, double self_frac, double n_h_s, R* Vs, R* hs, hipStream_t s);
template <class R>
void launch_dep_norm(int kernel, const DepGrid& d, const double* xs, int64_t ns, const R* hs,
                     const R* dM, const R* dMZ, const R* dE, const R* vs, R* As, void* sp,
                     uint32_t* npair, uint32_t* slot, unsigned long long* cnt, hipStream_t s);
template <class R>
void launch_dep_pairs(const DepGrid& d, const double* xs, int64_t ns, const R* hs,
                      const uint32_t* npair, const uint32_t* slot, const uint32_t* off,
                      uint32_t* pj, uint32_t* ps, hipStream_t s);
template <class R>
void launch_dep_apply(int kernel, const double* xg, int64_t ng, const R* Vg, R* mg, R* vg, R* mZg,
                      R* ug, const void* sp, const uint32_t* first, const uint32_t* ps, double box,
                      hipStream_t s);

// exact-integration cooling (caller order, elementwise); run holds int2 per bin
void launch_cool_prepare(int K, double lu0, double dex, const double* lam, double* oma,
                         double* co, double* G, void* run, double* binint, hipStream_t s);
template <class R>
void launch_cool(int K, double lu0, double dex, const double* lam, const double* co,
                 const double* oma, const double* G, const void* run, int64_t n, double dt,
                 const R* rho, R* u, hipStream_t s);

}  // namespace crk
