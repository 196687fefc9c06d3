// Context, workspace and the C ABI of libcrk.so (declared in crk.h).
//
// A forward call: (1) reads the largest input h and picks the cell grid;
// (2) builds the cell list (cell keys, stable radix sort, cell starts);
// (3) gathers the particles into cell-sorted SoA records with FP32/FP64
// offsets from their cell centre; (4) solves h (or takes it as given) and
// the volume; (5) builds the symmetric neighbour list; (6) runs the moment,
// correction, density and force passes. All work is enqueued on the
// caller's stream; the host reads back three small control words (the
// largest h, the h-solve status, the list-capacity check).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "crk.h"
#include "crk_passes.h"

namespace {

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

namespace {
enum Pass {
  P_CELLS = 0, P_CAND, P_HSOLVE, P_NLIST, P_MOMENTS, P_DENSITY, P_FORCE,
  P_BWD_FORCE, P_BWD_DENSITY, P_BWD_CORR, P_BWD_MOMENTS, P_BWD_VOLUME, P_BWD_OTHER, P_STEP,
  P_COOL, P_DEPOSIT, P_NPASS
};
const char* kPassNames[P_NPASS] = {"cells",     "candidates",  "hsolve",      "nlist",
                                   "moments",   "density",     "force",       "bwd_force",
                                   "bwd_density", "bwd_corr",  "bwd_moments", "bwd_volume",
                                   "bwd_other", "step", "cool",
                                   "deposit"};
}  // namespace

struct crk_ctx {
  crk_params p;
  // per-pass timing
  hipEvent_t ev0[P_NPASS] = {}, ev1[P_NPASS] = {};
  bool pending[P_NPASS] = {};
  double ms_total[P_NPASS] = {};
  long long ms_calls[P_NPASS] = {};
  bool events_ready = false;
  std::string err;
  // workspace
  Buf keys_a, keys_b, vals_a, vals_b, cell_start, sort_tmp, scan_tmp;
  Buf pv, mass, uu, hbuf, Vbuf, st4, gv4, kc4, mom, nlist, slist, ng, ns, scr_r, scr_m,
      cand, ccnt, cell3;
  Buf cnt;
  // tree path
  Buf rad, need, todo, tslot, nlo, nhi, lvl, wrow, lrow, cpos, torder, absp, hl_lvl, need4, coff;
  // tree path candidate pool: entries the last forward's rounds took, and the
  // placement of the current round (see State::pool_base4)
  size_t pool_hint = 0;
  size_t adj_bytes = 0;  // the adjoint workspace carved from the pool (last backward)
  int64_t pool_base4 = 0;
  int64_t pool_cap = 0;
  uint32_t host_rows[2] = {};
  int lvl_off[crk::kMaxLevels] = {}, lvl_cnt[crk::kMaxLevels] = {};
  int nlevels = 0;
  int lattice = 0;
  // (the adjoint workspace is carved from the candidate scratch or pool)
  // time step: the velocity and energy predicted for the end-of-step evaluation
  Buf vpred, upred;
  // timestep hierarchy: half-kicked velocity and energy, hdot, and the
  // evaluation of the substep (its accel and du/dt before the close)
  Buf hl_vh, hl_uh, hl_hdot, hl_acc, hl_du, hl_need, hl_act;
  // a substep with few active particles lists them (hl_act) for the row
  // passes: hl_rows, and their number
  bool hl_rows = false;
  long long hl_nact = 0;
  // per big step: the particles per level and the refined ones (read once),
  // and for the current substep a bound on its active particles from them
  Buf hl_hist;
  unsigned long long hl_hist_host[32] = {};
  long long hl_bound = 0;
  // levels and stored state seen by the passes during a hierarchical
  // substep (null levels: every particle active)
  const int* hl_levels = nullptr;
  int hl_lmax = 0;
  long long hl_jend = 0;
  const void *hl_V = nullptr, *hl_rho = nullptr, *hl_gv = nullptr, *hl_A = nullptr,
             *hl_B = nullptr, *hl_gA = nullptr, *hl_gB = nullptr;
  // cooling table: lam at the nodes, per-bin slope, prefix integrals within
  // each run of same-sign bins, each bin's run (int2), per-bin integrals
  Buf cool_lam, cool_oma, cool_co, cool_G, cool_run, cool_binint;
  int cool_K = 0;
  double cool_lu0 = 0.0, cool_dex = 0.0;
  // subgrid deposition: one sorted point grid at a time and its counters
  Buf dep_keys_a, dep_keys_b, dep_vals_a, dep_vals_b, dep_start, dep_tmp, dep_cnt;
  Buf dep_npair, dep_off, dep_first, dep_pj_a, dep_pj_b, dep_ps_a, dep_ps_b, dep_ptmp, dep_p4,
      dep_pv, dep_sp, dep_slot;
  unsigned long long host_cnt[crk::CNT_COUNT] = {};  // folded counters
  unsigned long long* host_raw = nullptr;  // the device slots (pinned)
  int list_cap = 128;
  int slist_cap = 32;
  int scr_cap = 192;
  int equal_mass = 0;
  // state of the last forward
  long long n_last = -1;
  long long searched = 0;  // particles the last forward's neighbour searches took
  int G = 0;
  double ell = 0.0;
  double rcap = 0.0;
  int precision_last = -1;
  bool reserved_fixed = false;
  // Cell-list geometry of the last forward that settled on its first
  // attempt; the next forward with the same n and precision launches every
  // pass with it and checks once at the end that it still holds.
  // the sorted cell keys and permutation of the last cell-list build (grid
  // cells_G, cells_n particles; cells_G = 0 once they are overwritten)
  int cells_G = 0;
  long long cells_n = -1;
  // whether the last check of a kept cell list found no particle moved: the
  // next speculative forward then keeps the list without reading the check
  // first (a move found at the end rejects that forward)
  bool cells_stable = false;
  bool spec_ok = false;
  long long spec_n = -1;
  int spec_prec = -1;
  int spec_G = 0;
  double spec_rcap = 0.0;
  int spec_em = 0;
};

namespace {

using namespace crk;

crk_status fail(crk_ctx* c, crk_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

crk_status hip_fail(crk_ctx* c, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? CRK_ENOMEM : CRK_EHIP, m);
}

#define CRK_HIP(call, where)                          \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
  } while (0)

hipError_t ensure(Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return hipSuccess;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    if (e != hipSuccess) return e;
    b.p = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return e;
  }
  b.bytes = bytes;
  return hipSuccess;
}

void release(Buf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

// Grows b to at least bytes, keeping its first keep bytes: copied on stream
// s, which is synchronised before the old block is freed.
hipError_t ensure_keep(Buf& b, size_t bytes, size_t keep, hipStream_t s) {
  if (b.bytes >= bytes) return hipSuccess;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return e;
  if (b.p && keep) {
    e = hipMemcpyAsync(p, b.p, std::min(keep, b.bytes), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      (void)hipFree(p);
      return e;
    }
  }
  release(b);
  b.p = p;
  b.bytes = bytes;
  return hipSuccess;
}

crk_status check_params(crk_ctx* ctx, const crk_params* p) {
  if (!p) return fail(ctx, CRK_EINVAL, "params is NULL");
  if (!(p->box > 0.0) || !std::isfinite(p->box)) return fail(ctx, CRK_EINVAL, "box must be > 0");
  if (!(p->n_h > 0.0)) return fail(ctx, CRK_EINVAL, "n_h must be > 0");
  if (!(p->gamma > 1.0)) return fail(ctx, CRK_EINVAL, "gamma must be > 1");
  if (p->kernel != CRK_CUBIC_SPLINE && p->kernel != CRK_WENDLAND_C4)
    return fail(ctx, CRK_EINVAL, "unknown kernel");
  if (p->precision != CRK_FP32 && p->precision != CRK_FP64)
    return fail(ctx, CRK_EINVAL, "unknown precision");
  if (p->h_mode != 0 && p->h_mode != 1) return fail(ctx, CRK_EINVAL, "h_mode must be 0 or 1");
  if (p->h_max_iter < 1) return fail(ctx, CRK_EINVAL, "h_max_iter must be >= 1");
  if (p->search < 0 || p->search > 2) return fail(ctx, CRK_EINVAL, "search must be 0, 1 or 2");
  if (!(p->h_rtol > 0.0)) return fail(ctx, CRK_EINVAL, "h_rtol must be > 0");
  if (!(p->eps2 >= 0.0) || !(p->dt_relax >= 0.0))
    return fail(ctx, CRK_EINVAL, "eps2 and dt_relax must be >= 0");
  // the shape with only the self term must fall short of n_h^3
  const double c0 = p->kernel == 0 ? 8.0 / kPi : 495.0 / (32.0 * kPi);
  if (!(p->n_h * p->n_h * p->n_h > c0))
    return fail(ctx, CRK_EINVAL, "n_h too small: the self term alone meets the neighbour target");
  return CRK_OK;
}

size_t real_size(int precision) { return precision == CRK_FP64 ? 8 : 4; }

// Per-particle workspace (independent of the neighbour-list capacity).
hipError_t ensure_particles(crk_ctx* c, int64_t n) {
  const size_t R = real_size(c->p.precision);
  const int64_t npad = ((n + 63) / 64) * 64;
  hipError_t e;
  // grown key or permutation buffers lose the kept cell list
  if (c->keys_a.bytes < 4 * (size_t)npad || c->vals_a.bytes < 4 * (size_t)npad) c->cells_G = 0;
#define ENS(b, bytes) \
  if ((e = ensure(c->b, (size_t)(bytes))) != hipSuccess) return e
  ENS(keys_a, 4 * npad);
  ENS(keys_b, 4 * npad);
  ENS(vals_a, 4 * npad);
  ENS(vals_b, 4 * npad);
  ENS(sort_tmp, 4 * (size_t)radix_tmp_words(n));
  ENS(pv, 8 * R * npad);
  ENS(mass, R * npad);
  ENS(uu, R * npad);
  ENS(hbuf, R * npad);
  ENS(Vbuf, R * npad);
  ENS(st4, 4 * R * npad);
  ENS(gv4, 12 * R * npad);
  ENS(kc4, 16 * R * npad);
  ENS(ng, 4 * npad);
  ENS(ns, 4 * npad);
  ENS(ccnt, 4 * npad);
  ENS(cell3, 4 * npad);
  ENS(cnt, 8 * CNT_COUNT * kCntSpread);
  if (c->p.store_corrections) ENS(mom, 40 * R * npad);
#undef ENS
  return hipSuccess;
}

template <class R>
State<R> make_state(crk_ctx* c, int64_t n) {
  State<R> S;
  S.n = n;
  S.G = c->G;
  S.box = c->p.box;
  S.ell_d = c->ell;
  S.ell = (R)c->ell;
  S.perm = (const uint32_t*)c->vals_a.p;
  S.keys = (const uint32_t*)c->keys_a.p;
  S.cell_start = (const uint32_t*)c->cell_start.p;
  S.cell3 = (uint32_t*)c->cell3.p;
  S.pv = (R4<R>*)c->pv.p;
  S.mass = (R*)c->mass.p;
  S.uu = (R*)c->uu.p;
  S.hbuf = (R*)c->hbuf.p;
  S.Vbuf = (R*)c->Vbuf.p;
  S.st4 = (R4<R>*)c->st4.p;
  S.gv4 = (R4<R>*)c->gv4.p;
  S.kc4 = (R4<R>*)c->kc4.p;
  S.mom = c->p.store_corrections ? (R*)c->mom.p : nullptr;
  S.nlist = (uint32_t*)c->nlist.p;
  S.slist = (uint32_t*)c->slist.p;
  S.ng = (int*)c->ng.p;
  S.ns = (int*)c->ns.p;
  S.list_cap = c->list_cap;
  S.slist_cap = c->slist_cap;
  S.cand = (uint32_t*)c->cand.p;
  S.scr_r = (R*)c->scr_r.p;
  S.scr_m = c->equal_mass ? (R*)c->scr_r.p : (R*)c->scr_m.p;  // never read when equal
  S.ccnt = (int*)c->ccnt.p;
  S.scr_cap = c->scr_cap;
  S.equal_mass = c->equal_mass;
  S.lattice = c->lattice;
  S.rad = c->lattice ? (R*)c->rad.p : nullptr;
  S.need = c->lattice ? (int*)c->need.p : nullptr;
  S.todo = c->lattice ? (int*)c->todo.p : nullptr;
  S.cslot = c->lattice ? (const uint32_t*)c->tslot.p : nullptr;
  S.coff4 = c->lattice ? (const uint32_t*)c->coff.p : nullptr;
  S.pool_base4 = c->pool_base4;
  S.pool_cap = c->pool_cap;
  S.shrink = c->p.h_mode == 1 ? 1 : 0;
  S.ncen = (float4*)c->nlo.p;
  S.nhw = (float4*)c->nhi.p;
  S.grow = c->lattice ? (const uint32_t*)c->lrow.p : nullptr;
  S.srow = c->lattice ? (const uint32_t*)c->lrow.p + (n + 63) / 64 + 1 : nullptr;
  S.lvl_off = (const int*)c->lvl.p;
  S.nlevels = c->nlevels;
  S.cpos = c->lattice ? (uint32_t*)c->cpos.p : nullptr;
  S.rcap = (R)c->rcap;
  S.cnt = (unsigned long long*)c->cnt.p;
  S.n_h3 = c->p.n_h * c->p.n_h * c->p.n_h;
  S.gamma = c->p.gamma;
  S.alpha = c->p.alpha;
  S.beta = c->p.beta;
  S.eps2 = c->p.eps2;
  S.dt_relax = c->p.dt_relax;
  S.rtol = c->p.h_rtol;
  S.max_iter = c->p.h_max_iter;
  S.levels = c->hl_levels;
  S.lev_max = c->hl_lmax;
  S.jend = (int)c->hl_jend;
  S.pV = (const R*)c->hl_V;
  S.prho = (const R*)c->hl_rho;
  S.pgv = (const R*)c->hl_gv;
  S.pA = (const R*)c->hl_A;
  S.pB = (const R*)c->hl_B;
  S.pgA = (const R*)c->hl_gA;
  S.pgB = (const R*)c->hl_gB;
  S.needed = c->hl_levels && !c->lattice ? (uint8_t*)c->hl_need.p : nullptr;
  const bool rows = c->hl_levels && c->hl_rows && !c->lattice;
  S.act = rows ? (const uint32_t*)c->hl_act.p : nullptr;
  S.nact = rows ? c->hl_nact : 0;
  return S;
}

hipError_t harvest(crk_ctx* c, int k) {
  if (!c->pending[k]) return hipSuccess;
  hipError_t e = hipEventSynchronize(c->ev1[k]);
  if (e != hipSuccess) return e;
  float ms = 0.f;
  e = hipEventElapsedTime(&ms, c->ev0[k], c->ev1[k]);
  if (e != hipSuccess) return e;
  c->ms_total[k] += ms;
  c->ms_calls[k] += 1;
  c->pending[k] = false;
  return hipSuccess;
}

hipError_t tbegin(crk_ctx* c, int k, hipStream_t s) {
  if (!c->p.timing) return hipSuccess;
  hipError_t e;
  if (!c->events_ready) {
    for (int i = 0; i < P_NPASS; ++i) {
      if ((e = hipEventCreate(&c->ev0[i])) != hipSuccess) return e;
      if ((e = hipEventCreate(&c->ev1[i])) != hipSuccess) return e;
    }
    c->events_ready = true;
  }
  if ((e = harvest(c, k)) != hipSuccess) return e;
  return hipEventRecord(c->ev0[k], s);
}

hipError_t tend(crk_ctx* c, int k, hipStream_t s) {
  if (!c->p.timing) return hipSuccess;
  c->pending[k] = true;
  return hipEventRecord(c->ev1[k], s);
}

// Copies the counter slots to the host and folds each counter's slots.
hipError_t read_counters(crk_ctx* c, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(c->host_raw, c->cnt.p, 8 * CNT_COUNT * kCntSpread,
                                hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  for (int k = 0; k < CNT_COUNT; ++k) {
    const bool is_max = k == CNT_HMAX_BITS || k == CNT_H_ITER_MAX || k == CNT_SCR_OVERFLOW ||
                        k == CNT_LIST_OVERFLOW || k == CNT_SLIST_OVERFLOW ||
                        k == CNT_MMAX_BITS || k == CNT_MINVMAX_BITS ||
                        k == CNT_HMAX_OUT_BITS || k == CNT_CELL_MAX ||
                        k == CNT_TOO_DENSE;
    unsigned long long v = 0;
    for (int t = 0; t < kCntSpread; ++t) {
      const unsigned long long x = c->host_raw[k * kCntSpread + t];
      v = is_max ? (x > v ? x : v) : v + x;
    }
    c->host_cnt[k] = v;
  }
  return hipSuccess;
}

// Hierarchy substeps with at most this many active particles (and not all)
// give each a 16-lane row in the pair passes.
constexpr long long kRowsMax = 32768;

// Whether this substep lists its active particles for the row passes, from
// na, their number or a bound on it (the row grids are sized by it; the row
// kernels take the list's own length).
void set_rows(crk_ctx* ctx, int64_t n, long long na) {
  ctx->hl_nact = na;
  // (the list has room for every particle: the hierarchy step sizes it)
  ctx->hl_rows = ctx->hl_levels && na <= kRowsMax && na < n && ctx->hl_act.bytes >= 4 * (size_t)n;
}

double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, 8);
  return d;
}

// Largest grid with cell side >= R, at most ~2 cells per particle and
// at most 1023 cells per side (10-bit packed coordinates).
int choose_grid(double box, double R, int64_t n) {
  double g = std::floor(box / R);
  if (!(g >= 1.0)) g = 1.0;
  g = std::min(g, 1023.0);
  while (g > 1.0 && g * g * g > 2.0 * (double)n + 8.0) g -= 1.0;
  return (int)g;
}

template <class R>
crk_status build_cells(crk_ctx* ctx, hipStream_t s, int64_t n, const double* x,
                       unsigned long long occ_limit) {
  const int64_t ncell = (int64_t)ctx->G * ctx->G * ctx->G;
  CRK_HIP(ensure(ctx->cell_start, 4 * (size_t)(ncell + 1)), "alloc cell starts");
  launch_keys(x, n, ctx->p.box, ctx->G, (uint32_t*)ctx->keys_a.p, (uint32_t*)ctx->vals_a.p, s);
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < ncell) ++bits;
  CRK_HIP(radix_sort_pairs((uint32_t*)ctx->keys_a.p, (uint32_t*)ctx->vals_a.p,
                           (uint32_t*)ctx->keys_b.p, (uint32_t*)ctx->vals_b.p, n, bits,
                           (uint32_t*)ctx->sort_tmp.p, s),
          "radix sort");
  launch_cell_bounds((const uint32_t*)ctx->keys_a.p, n, ncell, (uint32_t*)ctx->cell_start.p,
                     occ_limit, (unsigned long long*)ctx->cnt.p, s);
  CRK_HIP(hipGetLastError(), "cell bounds launch");
  ctx->cells_G = ctx->G;
  ctx->cells_n = n;
  return CRK_OK;
}

// Tree path: Morton order over the 1024^3 lattice, search leaves of kLeaf
// particles, per-particle candidate radii adapted until every h is bracketed;
// the candidates of every particle are kept (rounds append to the candidate
// pool) and its gather list is filtered from them.
template <class R>
crk_status tree_solve(crk_ctx* ctx, hipStream_t s, int64_t n, const double* x, const R* v,
                      const R* m, const R* u, const R* h) {
  const crk_params& P = ctx->p;
  unsigned long long* dcnt = (unsigned long long*)ctx->cnt.p;
  const int64_t npad = ((n + 63) / 64) * 64;
  ctx->lattice = 1;
  ctx->G = 1024;
  ctx->ell = P.box / 1024.0;
  ctx->cells_G = 0;  // the Morton sort below takes the key buffers
  {
    // room for ~4x the expected neighbour count (4 pi / 3) n_h^3 before a
    // radius shrinks (the cell path's capacity is its own: it is set again
    // there)
    const double expect = 4.18879 * P.n_h * P.n_h * P.n_h;
    ctx->scr_cap = std::max(256, (int)((4.0 * expect + 31.0) / 32.0) * 32);
  }
  // levels of the implicit tree over the leaves
  const int nleaf = (int)((n + kLeaf - 1) / kLeaf);
  ctx->nlevels = 0;
  int off = 0;
  for (int c = nleaf;; c = (c + kFan - 1) / kFan) {
    // the walk keeps 8 bits per level below the top in 64 bits
    if (ctx->nlevels == 8) return fail(ctx, CRK_EINVAL, "tree too deep");
    ctx->lvl_off[ctx->nlevels] = off;
    ctx->lvl_cnt[ctx->nlevels] = c;
    off += c;
    ++ctx->nlevels;
    if (c == 1) break;
  }
  CRK_HIP(ensure(ctx->nlo, 16 * (size_t)off), "alloc tree");
  CRK_HIP(ensure(ctx->nhi, 16 * (size_t)off), "alloc tree");
  CRK_HIP(ensure(ctx->lvl, 4 * 2 * kMaxLevels), "alloc tree");
  CRK_HIP(ensure(ctx->rad, real_size(P.precision) * 2 * (size_t)npad), "alloc tree");
  CRK_HIP(ensure(ctx->todo, 4 * (size_t)(npad + 1)), "alloc tree");
  CRK_HIP(ensure(ctx->tslot, 4 * (size_t)(npad + 1)), "alloc tree");
  CRK_HIP(ensure(ctx->need, 4 * (size_t)npad), "alloc tree");
  CRK_HIP(ensure(ctx->cpos, 4 * (size_t)npad), "alloc tree");
  CRK_HIP(ensure(ctx->torder, 4 * (size_t)npad), "alloc tree");
  CRK_HIP(ensure(ctx->absp, 16 * (size_t)npad), "alloc tree");
  CRK_HIP(ensure(ctx->need4, 4 * (size_t)(npad + 1)), "alloc tree");
  CRK_HIP(ensure(ctx->coff, 4 * (size_t)(npad + 1)), "alloc tree");
  CRK_HIP(ensure(ctx->scan_tmp, 4 * (size_t)scan_tmp_words(n + 1)), "alloc scan");
  int lv[2 * kMaxLevels];
  for (int t = 0; t < kMaxLevels; ++t) {
    lv[t] = ctx->lvl_off[t];
    lv[kMaxLevels + t] = ctx->lvl_cnt[t];
  }
  CRK_HIP(hipMemcpyAsync(ctx->lvl.p, lv, sizeof(lv), hipMemcpyHostToDevice, s), "tree levels");
  CRK_HIP(hipMemsetAsync(dcnt, 0, 8 * CNT_COUNT * kCntSpread, s), "memset");
  CRK_HIP(tbegin(ctx, P_CELLS, s), "event");
  launch_morton(x, n, P.box, (uint32_t*)ctx->keys_a.p, (uint32_t*)ctx->vals_a.p, s);
  CRK_HIP(radix_sort_pairs((uint32_t*)ctx->keys_a.p, (uint32_t*)ctx->vals_a.p,
                           (uint32_t*)ctx->keys_b.p, (uint32_t*)ctx->vals_b.p, n, 30,
                           (uint32_t*)ctx->sort_tmp.p, s),
          "radix sort");
  {
    State<R> S = make_state<R>(ctx, n);
    launch_gather<R>(S, x, v, m, u, h, s);
    launch_tree_build<R>(S, S.hbuf, (float4*)ctx->absp.p, ctx->lvl_off, ctx->lvl_cnt, s);
    launch_init_radius<R>(S, P.h_mode, s);
  }
  CRK_HIP(tend(ctx, P_CELLS, s), "event");
  // Rounds over the particles still unsolved. Each round ranks them (scan of
  // the todo flags, todo[n] = 0), runs the candidate walk and the h solve (or
  // the volume for fixed h) on them, and stops when none is left. The first
  // two rounds stage every row in LDS when its capacity fits there, and the
  // blocks append the candidates to the pool (the second after what the
  // first took; a row of the second whose candidates outgrow its stage, as
  // one whose radius was grown may, is left to the third); the later rounds
  // give each particle the room it asks for after what the earlier rounds
  // took (the solved particles keep their candidates where they are).
  int* todo = (int*)ctx->todo.p;
  uint32_t* slot = (uint32_t*)ctx->tslot.p;
  uint32_t* need4 = (uint32_t*)ctx->need4.p;
  uint32_t* coff = (uint32_t*)ctx->coff.p;
  CRK_HIP(hipMemsetAsync(todo + n, 0, 4, s), "memset");
  const double expect = 4.18879 * P.n_h * P.n_h * P.n_h;
  int64_t used4 = 0;  // pool entries the earlier rounds took, in 4-entry units
  bool staged = false;
  unsigned long long pool_taken = 0;
  bool solved = false;
  for (int round = 0; round < 40; ++round) {
    const bool stage = stage_fits(ctx->scr_cap) && (round == 0 || (round == 1 && ctx->pool_cap > 0));
    CRK_HIP(exclusive_scan_u32((const uint32_t*)todo, slot, n + 1, (uint32_t*)ctx->scan_tmp.p,
                               s),
            "scan");
    CRK_HIP(hipMemcpyAsync(&ctx->host_rows[0], slot + n, 4, hipMemcpyDeviceToHost, s), "rows");
    if (!stage) {
      State<R> S = make_state<R>(ctx, n);
      launch_need4<R>(S, need4, round > 0, s);
      CRK_HIP(exclusive_scan_u32(need4, coff, n + 1, (uint32_t*)ctx->scan_tmp.p, s), "scan");
      CRK_HIP(hipMemcpyAsync(&ctx->host_rows[1], coff + n, 4, hipMemcpyDeviceToHost, s), "rows");
    }
    if (staged)
      CRK_HIP(hipMemcpyAsync(&pool_taken, dcnt + CNT_POOL * kCntSpread, 8, hipMemcpyDeviceToHost,
                             s),
              "pool");
    CRK_HIP(hipStreamSynchronize(s), "scan");
    if (staged) {
      used4 = (int64_t)(std::min<unsigned long long>(pool_taken, (unsigned long long)ctx->pool_cap) / 4);
      staged = false;
    }
    if (ctx->host_rows[0] == 0) {
      solved = true;
      break;
    }
    if (stage && round > 0) {
      staged = true;  // the pool and its counter go on from the first round
    } else if (stage) {
      // room for every round, from what the last forward's rounds took (at
      // first 2.5 times the expected neighbour count per particle, which
      // leaves the retry rounds room enough not to grow the pool), and for
      // the adjoint workspace carved from it; a pool an eighth or more
      // larger than that is given back first
      size_t want = ctx->pool_hint ? ctx->pool_hint : (size_t)((double)n * 2.5 * expect) + 4096;
      want = std::max(want, (ctx->adj_bytes + 3) / 4);
      if (ctx->cand.bytes > 4 * (want + want / 8)) release(ctx->cand);
      CRK_HIP(ensure(ctx->cand, 4 * want), "alloc candidates");
      CRK_HIP(hipMemsetAsync(dcnt + CNT_POOL * kCntSpread, 0, 8 * kCntSpread, s), "memset");
      ctx->pool_base4 = 0;
      // (candidate positions are kept in 4-entry units in 32 bits: a larger
      // pool leaves the rest to the retry rounds, which check their sizes)
      ctx->pool_cap = std::min<int64_t>((int64_t)(ctx->cand.bytes / 4), ((int64_t)1 << 34) - 4) &
                      ~(int64_t)3;
      staged = true;
    } else {
      const int64_t add4 = ctx->host_rows[1];
      if (used4 + add4 >= ((int64_t)1 << 32))
        return fail(ctx, CRK_ENOMEM, "candidate pool beyond 2^34 entries");
      CRK_HIP(ensure_keep(ctx->cand, 16 * (size_t)(used4 + add4), 16 * (size_t)used4, s),
              "alloc candidates");
      ctx->pool_base4 = used4;
      ctx->pool_cap = 0;
      used4 += add4;
    }
    CRK_HIP(hipMemsetAsync(dcnt + CNT_H_CAPPED * kCntSpread, 0, 8 * kCntSpread, s), "memset");
    CRK_HIP(hipMemsetAsync(dcnt + CNT_RETRY * kCntSpread, 0, 8 * kCntSpread, s), "memset");
    State<R> S = make_state<R>(ctx, n);
    // the first round takes every particle in place; later ones only the
    // unsolved, packed in rank order (the walk knows a retry round by order)
    const int64_t nt = ctx->host_rows[0];
    const uint32_t* order = nullptr;
    if (round > 0) {
      launch_rank_order<R>(S, (uint32_t*)ctx->torder.p, s);
      order = (const uint32_t*)ctx->torder.p;
    }
    CRK_HIP(tbegin(ctx, P_CAND, s), "event");
    launch_candidates_tree<R>(S, (const float4*)ctx->absp.p, P.kernel, stage, order, nt, s);
    CRK_HIP(tend(ctx, P_CAND, s), "event");
    ctx->searched += nt;
    CRK_HIP(tbegin(ctx, P_HSOLVE, s), "event");
    launch_hsolve_tree<R>(S, P.kernel, order, nt, s);
    CRK_HIP(tend(ctx, P_HSOLVE, s), "event");
    CRK_HIP(hipGetLastError(), "h solve launch");
  }
  // the next forward reserves what this one took, and a twentieth more
  ctx->pool_hint = (size_t)(4.2 * (double)used4) + 4096;
  CRK_HIP(read_counters(ctx, s), "h solve");
  if (!solved) return fail(ctx, CRK_EHIP, "tree h solve did not settle");
  return CRK_OK;
}

// Tree path neighbour lists with per-wave capacities. Gather lists filtered
// from the kept candidates (lengths, per-wave offsets, entries); scatter-only
// lists by transposing the gather lists: count, per-wave offsets, fill, sort.
template <class R>
crk_status tree_lists(crk_ctx* ctx, hipStream_t s, int64_t n) {
  unsigned long long* dcnt = (unsigned long long*)ctx->cnt.p;
  const int64_t nw = (n + 63) / 64;
  CRK_HIP(ensure(ctx->wrow, 4 * 2 * (size_t)(nw + 1)), "alloc neighbour list");
  CRK_HIP(ensure(ctx->lrow, 4 * 2 * (size_t)(nw + 1)), "alloc neighbour list");
  CRK_HIP(ensure(ctx->scan_tmp, 4 * (size_t)scan_tmp_words(nw + 1)), "alloc scan");
  uint32_t* wg = (uint32_t*)ctx->wrow.p;
  uint32_t* ws = wg + nw + 1;
  uint32_t* lg = (uint32_t*)ctx->lrow.p;
  uint32_t* ls = lg + nw + 1;
  int* ng = (int*)ctx->ng.p;
  int* ns = (int*)ctx->ns.p;
  int* fillc = (int*)ctx->need.p;  // free once h is solved
  // chunk rows per wave -> offsets -> host total; a row is 4 entries of 64 lanes
  auto offsets = [&](const int* c, int extra, uint32_t* rows, uint32_t* off,
                     uint32_t* host) -> hipError_t {
    hipError_t e = hipMemsetAsync(rows + nw, 0, 4, s);
    if (e != hipSuccess) return e;
    launch_wave_rows(c, n, extra, rows, s);
    e = exclusive_scan_u32(rows, off, nw + 1, (uint32_t*)ctx->scan_tmp.p, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(host, off + nw, 4, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
  };
  CRK_HIP(tbegin(ctx, P_NLIST, s), "event");
  CRK_HIP(hipMemsetAsync(ns, 0, 4 * (size_t)nw * 64, s), "memset");
  {
    State<R> S = make_state<R>(ctx, n);
    launch_filter_tree<R>(S, false, fillc, nullptr, s);
  }
  CRK_HIP(offsets(ng, 0, wg, lg, &ctx->host_rows[0]), "list rows");
  CRK_HIP(offsets(ns, 0, ws, ls, &ctx->host_rows[1]), "list rows");
  CRK_HIP(ensure(ctx->nlist, 4 * 256 * (size_t)ctx->host_rows[0]), "alloc neighbour list");
  CRK_HIP(ensure(ctx->slist, 4 * 256 * (size_t)ctx->host_rows[1]), "alloc neighbour list");
  CRK_HIP(hipMemsetAsync(dcnt + CNT_PAIRS_GATHER * kCntSpread, 0, 8 * 2 * kCntSpread, s), "memset");
  CRK_HIP(hipMemsetAsync(fillc, 0, 4 * (size_t)nw * 64, s), "memset");
  CRK_HIP(hipMemsetAsync(dcnt + CNT_LONG_LISTS * kCntSpread, 0, 8 * kCntSpread, s), "memset");
  {
    // the rank order of the search rounds is free: the queue of long lists
    State<R> S = make_state<R>(ctx, n);
    launch_filter_tree<R>(S, true, fillc, (uint32_t*)ctx->torder.p, s);
  }
  CRK_HIP(tend(ctx, P_NLIST, s), "event");
  CRK_HIP(hipGetLastError(), "neighbour list launch");
  return CRK_OK;
}

// One forward on the cell list with the geometry of the previous one (grid,
// candidate radius, equal-mass form, capacities): every pass is launched
// with no host read in between, and a single read of the counters at the
// end checks that the careful path would have taken exactly this attempt
// (same grid from this input's largest h, same mass form, no cell beyond
// the clustering limit, no candidate or list overflow, no capped h root).
// Then the results are the careful path's, bit for bit; otherwise
// *accepted stays false and the caller runs the careful path. When the last
// cell-list build is still at hand (same grid and count), one read first
// tells whether any particle has changed cell: if none has, the list is kept
// (its sorted order and cell starts are those a new sort of these positions
// gives), else it is built again.
template <class R>
crk_status forward_fast(crk_ctx* ctx, hipStream_t s, int64_t n, const double* x, const R* v,
                        const R* m, const R* u, R* h, R* V, R* rho, void* A, void* B,
                        void* gradA, void* gradB, R* gradv, double* accel, double* dudt,
                        bool* accepted) {
  const crk_params& P = ctx->p;
  *accepted = false;
  unsigned long long* dcnt = (unsigned long long*)ctx->cnt.p;
  CRK_HIP(hipMemsetAsync(dcnt, 0, 8 * CNT_COUNT * kCntSpread, s), "memset");
  launch_check_inputs<R>(x, h, m, u, n, dcnt, s);
  ctx->G = ctx->spec_G;
  ctx->ell = P.box / ctx->G;
  ctx->lattice = 0;
  ctx->rcap = ctx->spec_rcap;
  ctx->equal_mass = ctx->spec_em;
  const int64_t npad = ((n + 63) / 64) * 64;
  const double ncell = (double)ctx->G * ctx->G * ctx->G;
  const double occ_rule = std::max(1024.0, 16.0 * (double)n / ncell);
  CRK_HIP(tbegin(ctx, P_CELLS, s), "event");
  // the kept cell list: checked against these positions whenever it is at
  // hand; kept without waiting for the check when the last check found it
  // still sorted, else built again (the check then tells the next forward)
  const bool at_hand = ctx->cells_G == ctx->G && ctx->cells_n == n;
  if (at_hand)
    launch_keys_check(x, n, P.box, ctx->G, (const uint32_t*)ctx->keys_a.p,
                      (const uint32_t*)ctx->vals_a.p, dcnt, s);
  const bool kept = at_hand && ctx->cells_stable;
  if (!kept) {
    crk_status st = build_cells<R>(ctx, s, n, x,
                                   P.search == 0 ? (unsigned long long)occ_rule : ~0ull);
    if (st != CRK_OK) return st;
  }
  set_rows(ctx, n, ctx->hl_bound);
  {
    State<R> S = make_state<R>(ctx, n);
    launch_gather<R>(S, x, v, m, u, h, s);
    if (ctx->hl_rows) launch_active_list<R>(S, (uint32_t*)ctx->hl_act.p, s);
  }
  CRK_HIP(tend(ctx, P_CELLS, s), "event");
  CRK_HIP(ensure(ctx->cand, 4 * (size_t)npad * ctx->scr_cap), "alloc candidates");
  CRK_HIP(ensure(ctx->scr_r, real_size(P.precision) * (size_t)npad * ctx->scr_cap),
          "alloc candidates");
  if (!ctx->equal_mass)
    CRK_HIP(ensure(ctx->scr_m, real_size(P.precision) * (size_t)npad * ctx->scr_cap),
            "alloc candidates");
  CRK_HIP(ensure(ctx->nlist, 4 * (size_t)npad * ctx->list_cap), "alloc neighbour list");
  CRK_HIP(ensure(ctx->slist, 4 * (size_t)npad * ctx->slist_cap), "alloc neighbour list");
  State<R> S = make_state<R>(ctx, n);
  CRK_HIP(tbegin(ctx, P_CAND, s), "event");
  launch_candidates<R>(S, s);
  CRK_HIP(tend(ctx, P_CAND, s), "event");
  ctx->searched += n;
  CRK_HIP(tbegin(ctx, P_HSOLVE, s), "event");
  if (P.h_mode == 0)
    launch_volume<R>(S, P.kernel, s);
  else
    launch_hsolve<R>(S, P.kernel, s);
  CRK_HIP(tend(ctx, P_HSOLVE, s), "event");
  // the caller's h is an input until this evaluation is accepted: h and V
  // are written to the caller only then
  launch_pack<R>(S, (R*)nullptr, (R*)nullptr, s);
  CRK_HIP(tbegin(ctx, P_NLIST, s), "event");
  launch_nlist<R>(S, s);
  CRK_HIP(tend(ctx, P_NLIST, s), "event");
  CorrOut co{A, B, gradA, gradB};
  CRK_HIP(tbegin(ctx, P_MOMENTS, s), "event");
  launch_moments<R>(S, P.kernel, co, s);
  CRK_HIP(tend(ctx, P_MOMENTS, s), "event");
  CRK_HIP(tbegin(ctx, P_DENSITY, s), "event");
  launch_density<R>(S, P.kernel, rho, gradv, s);
  CRK_HIP(tend(ctx, P_DENSITY, s), "event");
  CRK_HIP(tbegin(ctx, P_FORCE, s), "event");
  launch_force<R>(S, P.kernel, accel, dudt, s);
  CRK_HIP(tend(ctx, P_FORCE, s), "event");
  if (P.check_finite) {
    launch_count_nonfinite_f64(accel, 3 * n, dcnt, s);
    launch_count_nonfinite_f64(dudt, n, dcnt, s);
    launch_count_nonfinite<R>(rho, n, dcnt, s);
    launch_count_nonfinite<R>(h, n, dcnt, s);
  }
  CRK_HIP(hipGetLastError(), "pass launch");
  CRK_HIP(read_counters(ctx, s), "speculative forward");
  const unsigned long long* hc = ctx->host_cnt;
  if (at_hand) ctx->cells_stable = hc[CNT_MOVED] == 0;
  if (kept && hc[CNT_MOVED]) {
    ctx->cells_G = 0;  // a particle left its cell: the list no longer sorts x
    return CRK_OK;
  }
  if (hc[CNT_BAD_INPUT]) return CRK_OK;  // the careful path reports it
  const double h0max = bits_to_double(hc[CNT_HMAX_BITS]);
  if (!(h0max < 0.5 * P.box)) return CRK_OK;
  const double reach = P.h_mode == 1 ? 1.25 * h0max : h0max;
  if (choose_grid(P.box, 0.5 * reach, n) != ctx->G) return CRK_OK;
  // fixed h: any radius >= this input's largest h gives the same sums
  if (P.h_mode == 0 && !(h0max <= ctx->rcap)) return CRK_OK;
  const double mmax = bits_to_double(hc[CNT_MMAX_BITS]);
  const double iinv = bits_to_double(hc[CNT_MINVMAX_BITS]);
  if ((std::fabs(mmax * iinv - 1.0) <= 4e-16 ? 1 : 0) != ctx->equal_mass) return CRK_OK;
  if (hc[CNT_TOO_DENSE] || hc[CNT_SCR_OVERFLOW] || hc[CNT_LIST_OVERFLOW] ||
      hc[CNT_SLIST_OVERFLOW])
    return CRK_OK;
  if (P.search == 0 && (double)hc[CNT_CELL_MAX] > occ_rule) return CRK_OK;
  if (P.h_mode == 1) {
    if (hc[CNT_H_CAPPED]) return CRK_OK;
    if (!(bits_to_double(hc[CNT_HMAX_OUT_BITS]) < 0.5 * P.box)) return CRK_OK;
  }
  launch_pack<R>(S, h, V, s);
  CRK_HIP(hipGetLastError(), "pack launch");
  *accepted = true;
  return CRK_OK;
}

template <class R>
crk_status forward_impl(crk_ctx* ctx, hipStream_t s, int64_t n, const double* x, const R* v,
                        const R* m, const R* u, R* h, R* V, R* rho, void* A, void* B,
                        void* gradA, void* gradB, R* gradv, double* accel, double* dudt,
                        crk_stats* stats) {
  const crk_params& P = ctx->p;
  ctx->n_last = -1;
  ctx->searched = 0;
  CRK_HIP(ensure_particles(ctx, n), "workspace allocation");
  unsigned long long* dcnt = (unsigned long long*)ctx->cnt.p;
  bool accepted = false;
  if (ctx->spec_ok && ctx->spec_n == n && ctx->spec_prec == P.precision && P.search != 2) {
    crk_status st = forward_fast<R>(ctx, s, n, x, v, m, u, h, V, rho, A, B, gradA, gradB, gradv,
                                    accel, dudt, &accepted);
    if (st != CRK_OK) return st;
  }
  ctx->spec_ok = false;
  if (!accepted) {
    CRK_HIP(hipMemsetAsync(dcnt, 0, 8 * CNT_COUNT * kCntSpread, s), "memset");
    launch_check_inputs<R>(x, h, m, u, n, dcnt, s);
    if (ctx->hl_levels)
      launch_count_active(ctx->hl_levels, n, ctx->hl_lmax, ctx->hl_jend, dcnt, s);
    CRK_HIP(hipGetLastError(), "input check launch");
    CRK_HIP(read_counters(ctx, s), "input check");
    set_rows(ctx, n, (long long)ctx->host_cnt[CNT_ACTIVE]);
    if (ctx->host_cnt[CNT_BAD_INPUT])
      return fail(ctx, CRK_EINVAL, "x must be finite; h, m and u finite and > 0");
    const double h0max = bits_to_double(ctx->host_cnt[CNT_HMAX_BITS]);
    {
      // all masses equal (to rounding) => m_j / m_i = 1 needs no storage
      const double mmax = bits_to_double(ctx->host_cnt[CNT_MMAX_BITS]);
      const double iinv = bits_to_double(ctx->host_cnt[CNT_MINVMAX_BITS]);
      ctx->equal_mass = std::fabs(mmax * iinv - 1.0) <= 4e-16 ? 1 : 0;
    }
    if (!(h0max < 0.5 * P.box))
      return fail(ctx, CRK_EDOMAIN, "smoothing length must stay below half the box");

    // candidates reach two cell sides (a 5x5x5 stencil walked with culling)
    double reach = P.h_mode == 1 ? 1.25 * h0max : h0max;
    ctx->G = choose_grid(P.box, 0.5 * reach, n);
    const int G0 = ctx->G;
    ctx->ell = P.box / ctx->G;
    ctx->lattice = 0;
    const int64_t npad = ((n + 63) / 64) * 64;
    bool solved = false;
    bool use_tree = P.search == 2;
    for (int attempt = 0; attempt < 12 && !solved && !use_tree; ++attempt) {
      // candidates reach two cell sides when h is solved; with fixed h 10 %
      // beyond the largest h (within two cell sides), so that the next
      // forward may speculate on this geometry while h grows a little
      ctx->rcap = P.h_mode == 1 ? 2.0 * ctx->ell : std::min(2.0 * ctx->ell, 1.1 * h0max);
      CRK_HIP(hipMemsetAsync(dcnt, 0, 8 * CNT_COUNT * kCntSpread, s), "memset");
      CRK_HIP(tbegin(ctx, P_CELLS, s), "event");
      crk_status st = build_cells<R>(ctx, s, n, x, ~0ull);
      if (st != CRK_OK) return st;
      if (P.search == 0 && attempt == 0) {
        // a cell holding more than 1024 particles and 16x the mean occupancy
        // means strong clustering: the cell list would need huge candidate
        // lists there (a high resolution alone raises every cell alike)
        CRK_HIP(read_counters(ctx, s), "cell occupancy");
        const double mean_occ = (double)n / ((double)ctx->G * ctx->G * ctx->G);
        if ((double)ctx->host_cnt[CNT_CELL_MAX] > std::max(1024.0, 16.0 * mean_occ)) {
          use_tree = true;
          CRK_HIP(tend(ctx, P_CELLS, s), "event");
          break;
        }
      }
      {
        State<R> S = make_state<R>(ctx, n);
        launch_gather<R>(S, x, v, m, u, h, s);
        if (ctx->hl_rows) launch_active_list<R>(S, (uint32_t*)ctx->hl_act.p, s);
      }
      CRK_HIP(tend(ctx, P_CELLS, s), "event");
      CRK_HIP(ensure(ctx->cand, 4 * (size_t)npad * ctx->scr_cap), "alloc candidates");
      CRK_HIP(ensure(ctx->scr_r, real_size(P.precision) * (size_t)npad * ctx->scr_cap),
              "alloc candidates");
      if (!ctx->equal_mass)
        CRK_HIP(ensure(ctx->scr_m, real_size(P.precision) * (size_t)npad * ctx->scr_cap),
                "alloc candidates");
      State<R> S = make_state<R>(ctx, n);
      CRK_HIP(tbegin(ctx, P_CAND, s), "event");
      launch_candidates<R>(S, s);
      CRK_HIP(tend(ctx, P_CAND, s), "event");
      ctx->searched += n;
      CRK_HIP(tbegin(ctx, P_HSOLVE, s), "event");
      if (P.h_mode == 0)
        launch_volume<R>(S, P.kernel, s);
      else
        launch_hsolve<R>(S, P.kernel, s);
      CRK_HIP(tend(ctx, P_HSOLVE, s), "event");
      CRK_HIP(hipGetLastError(), "h solve launch");
      CRK_HIP(read_counters(ctx, s), "h solve");
      if (ctx->host_cnt[CNT_SCR_OVERFLOW]) {
        // clustered: some particle has far more candidates than the mean
        // density gives within the candidate radius (rcap <= ell)
        const double expect = 4.18879 * ctx->rcap * ctx->rcap * ctx->rcap * (double)n /
                              (P.box * P.box * P.box);
        if (P.search == 0 &&
            (double)ctx->host_cnt[CNT_SCR_OVERFLOW] > std::max(1024.0, 16.0 * expect)) {
          use_tree = true;
          break;
        }
        ctx->scr_cap = (int)(((ctx->host_cnt[CNT_SCR_OVERFLOW] * 5) / 4 + 31) / 32 * 32);
        continue;  // same grid, larger candidate capacity
      }
      if (P.h_mode == 1 && ctx->host_cnt[CNT_H_CAPPED]) {
        // a root beyond a candidate radius of half the box breaks h < box / 2
        if (ctx->rcap >= 0.5 * P.box)
          return fail(ctx, CRK_EDOMAIN, "h solve needs h beyond half the box");
        // cells too small for some root: widen them (to no fewer than 2 per
        // side, which the row wrap of the stencil walk assumes) and solve again
        ctx->G = std::max(2, std::min(ctx->G - 1, (int)std::floor(ctx->G / 1.5)));
        ctx->ell = P.box / ctx->G;
        continue;
      }
      solved = true;
    }
    if (use_tree) {
      crk_status st = tree_solve<R>(ctx, s, n, x, v, m, u, h);
      if (st != CRK_OK) return st;
      solved = true;
    }
    if (!solved) return fail(ctx, CRK_EHIP, "h solve: grid adaptation did not settle");
    if (!ctx->lattice && ctx->G == G0) {
      // settled on the first grid: the next forward may speculate with it
      ctx->spec_ok = true;
      ctx->spec_n = n;
      ctx->spec_prec = P.precision;
      ctx->spec_G = ctx->G;
      ctx->spec_rcap = ctx->rcap;
      ctx->spec_em = ctx->equal_mass;
    }
    if (P.h_mode == 1) {
      const double hmax = bits_to_double(ctx->host_cnt[CNT_HMAX_OUT_BITS]);
      if (!(hmax < 0.5 * P.box))
        return fail(ctx, CRK_EDOMAIN, "solved smoothing length reaches half the box");
    }
    {
      State<R> S = make_state<R>(ctx, n);
      launch_pack<R>(S, h, V, s);
    }
    if (ctx->lattice) {
      crk_status st = tree_lists<R>(ctx, s, n);
      if (st != CRK_OK) return st;
  } else {
    // neighbour lists, grown until they fit
    for (int attempt = 0; attempt < 8; ++attempt) {
      CRK_HIP(ensure(ctx->nlist, 4 * (size_t)npad * ctx->list_cap), "alloc neighbour list");
      CRK_HIP(ensure(ctx->slist, 4 * (size_t)npad * ctx->slist_cap), "alloc neighbour list");
      State<R> S = make_state<R>(ctx, n);
      CRK_HIP(hipMemsetAsync(dcnt + CNT_PAIRS_GATHER * kCntSpread, 0, 8 * 2 * kCntSpread, s), "memset");
      CRK_HIP(hipMemsetAsync(dcnt + CNT_LIST_OVERFLOW * kCntSpread, 0, 8 * 2 * kCntSpread, s), "memset");
      CRK_HIP(hipMemsetAsync(dcnt + CNT_CANDIDATES * kCntSpread, 0, 8 * kCntSpread, s), "memset");
      CRK_HIP(tbegin(ctx, P_NLIST, s), "event");
      launch_nlist<R>(S, s);
      CRK_HIP(tend(ctx, P_NLIST, s), "event");
      CRK_HIP(hipGetLastError(), "neighbour list launch");
      CRK_HIP(read_counters(ctx, s), "neighbour list");
      const unsigned long long need = ctx->host_cnt[CNT_LIST_OVERFLOW];
      const unsigned long long sneed = ctx->host_cnt[CNT_SLIST_OVERFLOW];
      if (!need && !sneed) break;
      if (need) ctx->list_cap = (int)((need * 5 / 4 + 31) / 32 * 32);
      if (sneed) ctx->slist_cap = (int)((sneed * 5 / 4 + 31) / 32 * 32);
      if (attempt == 7) return fail(ctx, CRK_EHIP, "neighbour list did not fit");
    }
  }
  State<R> S = make_state<R>(ctx, n);
  CorrOut co{A, B, gradA, gradB};
  CRK_HIP(tbegin(ctx, P_MOMENTS, s), "event");
  launch_moments<R>(S, P.kernel, co, s);
  CRK_HIP(tend(ctx, P_MOMENTS, s), "event");
  CRK_HIP(tbegin(ctx, P_DENSITY, s), "event");
  launch_density<R>(S, P.kernel, rho, gradv, s);
  CRK_HIP(tend(ctx, P_DENSITY, s), "event");
  CRK_HIP(tbegin(ctx, P_FORCE, s), "event");
  launch_force<R>(S, P.kernel, accel, dudt, s);
  CRK_HIP(tend(ctx, P_FORCE, s), "event");
  CRK_HIP(hipGetLastError(), "pass launch");
  if (P.check_finite) {
    launch_count_nonfinite_f64(accel, 3 * n, dcnt, s);
    launch_count_nonfinite_f64(dudt, n, dcnt, s);
    launch_count_nonfinite<R>(rho, n, dcnt, s);
    launch_count_nonfinite<R>(h, n, dcnt, s);
    CRK_HIP(hipGetLastError(), "finite check launch");
  }
  if (stats || P.check_finite) CRK_HIP(read_counters(ctx, s), "stats");
  } else {
    // the speculative forward was accepted; its read holds every counter
    ctx->spec_ok = true;
  }
  ctx->n_last = n;
  ctx->precision_last = P.precision;
  crk_status result = CRK_OK;
  {
    // the h-solve counters are always on the host (read after the solve, or
    // by the speculative forward's end-of-call read)
    const unsigned long long* hc = ctx->host_cnt;
    if (stats) {
      stats->n_pairs_gather = (long long)hc[CNT_PAIRS_GATHER];
      stats->n_pairs_force = (long long)hc[CNT_PAIRS_FORCE];
      stats->h_iter_max = (int)hc[CNT_H_ITER_MAX];
      stats->h_unconverged = (int)hc[CNT_H_UNCONV];
      stats->m2_singular = (int)hc[CNT_SINGULAR];
      stats->relaxed = (int)hc[CNT_RELAXED];
      stats->nonfinite = (int)hc[CNT_NONFINITE];
      stats->grid = ctx->G;
      stats->speculative = accepted ? 1 : 0;
      stats->n_candidates = (long long)hc[CNT_CANDIDATES];
      stats->n_searched = ctx->searched;
    }
    if (hc[CNT_H_UNCONV]) {
      result = CRK_ENOTCONV;
      ctx->err = "h solve reached the iteration cap for some particles";
    }
    if (P.check_finite && hc[CNT_NONFINITE]) {
      result = CRK_ENONFINITE;
      ctx->err = "non-finite outputs";
    }
  }
  return result;
}

// The adjoint workspace of n particles (Real of RS bytes): the arrays of
// AdjState in declaration order (gx, gv, gu, gh, gV, gkc, gab, wgt4, gvc4,
// mom4, kap), each 256-byte aligned. Writes the offsets, returns the total.
constexpr int kAdjArrays = 11;
constexpr size_t adj_layout(int64_t n, size_t RS, size_t* off) {
  const size_t N = (size_t)(((n + 63) / 64) * 64);
  const size_t blocks = (size_t)((n + kBlock - 1) / kBlock);
  const size_t bytes[kAdjArrays] = {8 * 3 * N,  8 * 3 * N,  8 * N,       8 * N,
                                    8 * N,      8 * 16 * N, 8 * 2 * blocks, 4 * RS * N,
                                    12 * RS * N, 40 * RS * N, RS * N};
  size_t t = 0;
  for (int k = 0; k < kAdjArrays; ++k) {
    if (off) off[k] = t;
    t += (bytes[k] + 255) & ~(size_t)255;
  }
  return t;
}

template <class R>
void adj_pointers(AdjState<R>& G, void* const* p) {
  G.gx = (double*)p[0];
  G.gv = (double*)p[1];
  G.gu = (double*)p[2];
  G.gh = (double*)p[3];
  G.gV = (double*)p[4];
  G.gkc = (double*)p[5];
  G.gab = (double*)p[6];
  G.wgt4 = (R4<R>*)p[7];
  G.gvc4 = (R4<R>*)p[8];
  G.mom4 = (R4<R>*)p[9];
  G.kap = (R*)p[10];
}

// The adjoint of the last forward. The workspace is carved from arena when
// given (at least adj_layout(n) bytes), with no allocation, else from the
// candidate scratch, grown to that size if smaller: the scratch is dead once
// the forward has built its neighbour lists, and the next forward rebuilds
// it from nothing. Every workspace array is written before it is read:
// nothing needs to start at zero.
template <class R>
crk_status backward_impl(crk_ctx* ctx, hipStream_t s, int64_t n, const double* g_accel,
                         const double* g_dudt, double* g_x, double* g_v, double* g_u,
                         double* g_ab, unsigned char* arena = nullptr) {
  const crk_params& P = ctx->p;
  const size_t RS = real_size(P.precision);
  size_t off[kAdjArrays];
  const size_t total = adj_layout(n, RS, off);
  void* ptr[kAdjArrays];
  unsigned char* base = arena;
  if (!base) {
    CRK_HIP(ensure(ctx->cand, total), "adjoint workspace");
    base = (unsigned char*)ctx->cand.p;
    ctx->adj_bytes = total;
  }
  for (int k = 0; k < kAdjArrays; ++k) ptr[k] = base + off[k];
  // no timing events on the allocation-free path (creating them allocates)
  auto tb = [&](int k, hipStream_t st) { return arena ? hipSuccess : tbegin(ctx, k, st); };
  auto te = [&](int k, hipStream_t st) { return arena ? hipSuccess : tend(ctx, k, st); };
  State<R> S = make_state<R>(ctx, n);
  AdjState<R> G;
  adj_pointers(G, ptr);
  G.w_a = g_accel;
  G.w_u = g_dudt;
  launch_bwd_prep<R>(S, G, s);
  CRK_HIP(tb(P_BWD_FORCE, s), "event");
  launch_bwd_force<R>(S, G, P.kernel, s);
  CRK_HIP(te(P_BWD_FORCE, s), "event");
  CRK_HIP(tb(P_BWD_DENSITY, s), "event");
  launch_bwd_density<R>(S, G, P.kernel, s);
  CRK_HIP(te(P_BWD_DENSITY, s), "event");
  CRK_HIP(tb(P_BWD_CORR, s), "event");
  launch_bwd_corr<R>(S, G, P.kernel, s);
  CRK_HIP(te(P_BWD_CORR, s), "event");
  CRK_HIP(tb(P_BWD_MOMENTS, s), "event");
  launch_bwd_moments<R>(S, G, P.kernel, P.h_mode, s);
  CRK_HIP(te(P_BWD_MOMENTS, s), "event");
  CRK_HIP(tb(P_BWD_VOLUME, s), "event");
  launch_bwd_volume<R>(S, G, P.kernel, s);
  CRK_HIP(te(P_BWD_VOLUME, s), "event");
  CRK_HIP(tb(P_BWD_OTHER, s), "event");
  launch_bwd_finish<R>(S, G, g_x, g_v, g_u, g_ab, s);
  CRK_HIP(te(P_BWD_OTHER, s), "event");
  CRK_HIP(hipGetLastError(), "adjoint launch");
  return CRK_OK;
}

// One kick-drift-kick step (App. A.4) with the Thacker/continuity smoothing
// length (App. A.3): first kick, drift and h update, the forward at the new
// state with the predicted velocity and energy, second kick.
template <class R>
crk_status step_impl(crk_ctx* ctx, hipStream_t s, int64_t n, double dt, double lam, double* x,
                     R* v, const R* m, R* u, R* h, R* V, R* rho, void* A, void* B, void* gradA,
                     void* gradB, R* gradv, double* accel, double* dudt, crk_stats* stats) {
  const crk_params& P = ctx->p;
  const size_t N = (size_t)n;
  CRK_HIP(ensure(ctx->vpred, sizeof(R) * 3 * N), "step workspace");
  CRK_HIP(ensure(ctx->upred, sizeof(R) * N), "step workspace");
  R* vp = (R*)ctx->vpred.p;
  R* up = (R*)ctx->upred.p;
  CRK_HIP(tbegin(ctx, P_STEP, s), "event");
  launch_kick_drift<R>(n, dt, lam, P.n_h, P.box, x, v, u, h, V, gradv, accel, dudt, vp, up, s);
  CRK_HIP(tend(ctx, P_STEP, s), "event");
  CRK_HIP(hipGetLastError(), "kick-drift launch");
  crk_status st = forward_impl<R>(ctx, s, n, x, vp, m, up, h, V, rho, A, B, gradA, gradB, gradv,
                                  accel, dudt, stats);
  if (st != CRK_OK && st != CRK_ENOTCONV && st != CRK_ENONFINITE) return st;
  CRK_HIP(tbegin(ctx, P_STEP, s), "event");
  launch_kick_close<R>(n, dt, v, u, accel, dudt, s);
  CRK_HIP(tend(ctx, P_STEP, s), "event");
  CRK_HIP(hipGetLastError(), "kick launch");
  return st;
}

// One big step of the power-of-two timestep hierarchy (App. A.4; App. A.3
// for h, V and rho): open every interval, then per substep drift all
// particles, predict their velocity and energy, evaluate with the particles
// whose interval does not end passive (they keep their stored state), close
// the active ones and open their next interval.
template <class R>
crk_status hstep_impl(crk_ctx* ctx, hipStream_t s, int64_t n, double dt, double lam,
                      const int* levels, const int* refine_at, const int* refine_level,
                      double* x, R* v, const R* m, R* u, R* h, R* V, R* rho, void* A, void* B,
                      void* gradA, void* gradB, R* gradv, double* accel, double* dudt,
                      crk_stats* stats) {
  const crk_params& P = ctx->p;
  const size_t N = (size_t)n;
  CRK_HIP(ensure_particles(ctx, n), "workspace allocation");
  unsigned long long* dcnt = (unsigned long long*)ctx->cnt.p;
  CRK_HIP(hipMemsetAsync(dcnt, 0, 8 * CNT_COUNT * kCntSpread, s), "memset");
  CRK_HIP(ensure(ctx->hl_hist, 8 * 32), "step workspace");
  CRK_HIP(hipMemsetAsync(ctx->hl_hist.p, 0, 8 * 32, s), "memset");
  launch_level_range(levels, refine_at, refine_level, n, dcnt,
                     (unsigned long long*)ctx->hl_hist.p, s);
  CRK_HIP(hipGetLastError(), "level launch");
  CRK_HIP(hipMemcpyAsync(ctx->hl_hist_host, ctx->hl_hist.p, 8 * 32, hipMemcpyDeviceToHost, s),
          "levels");
  CRK_HIP(read_counters(ctx, s), "levels");
  if (ctx->host_cnt[CNT_BAD_INPUT])
    return fail(ctx, CRK_EINVAL,
                "levels must lie in [0, 30], refinements on a finer level in [1, 30]");
  const int lmax = (int)ctx->host_cnt[CNT_H_ITER_MAX];
  if (refine_at) {
    CRK_HIP(hipMemsetAsync(dcnt, 0, 8 * CNT_COUNT * kCntSpread, s), "memset");
    launch_refine_grid(refine_at, refine_level, n, lmax, dcnt, s);
    CRK_HIP(hipGetLastError(), "level launch");
    CRK_HIP(read_counters(ctx, s), "refinements");
    if (ctx->host_cnt[CNT_BAD_INPUT])
      return fail(ctx, CRK_EINVAL,
                  "a refinement starts before the last substep, on the grid of its new level");
  }
  const int64_t nsub = (int64_t)1 << lmax;
  const double dt_min = dt / (double)nsub;
  // the current level of every particle (refinements change it)
  CRK_HIP(ensure(ctx->hl_lvl, 4 * N), "step workspace");
  int* lvl = (int*)ctx->hl_lvl.p;
  CRK_HIP(hipMemcpyAsync(lvl, levels, 4 * N, hipMemcpyDeviceToDevice, s), "levels");
  CRK_HIP(ensure(ctx->vpred, sizeof(R) * 3 * N), "step workspace");
  CRK_HIP(ensure(ctx->upred, sizeof(R) * N), "step workspace");
  CRK_HIP(ensure(ctx->hl_vh, sizeof(R) * 3 * N), "step workspace");
  CRK_HIP(ensure(ctx->hl_uh, sizeof(R) * N), "step workspace");
  CRK_HIP(ensure(ctx->hl_hdot, 8 * N), "step workspace");
  CRK_HIP(ensure(ctx->hl_acc, 8 * 3 * N), "step workspace");
  CRK_HIP(ensure(ctx->hl_du, 8 * N), "step workspace");
  CRK_HIP(ensure(ctx->hl_need, N), "step workspace");
  CRK_HIP(ensure(ctx->hl_act, 4 * N), "step workspace");
  R* vp = (R*)ctx->vpred.p;
  R* up = (R*)ctx->upred.p;
  R* vh = (R*)ctx->hl_vh.p;
  R* uh = (R*)ctx->hl_uh.p;
  double* hdot = (double*)ctx->hl_hdot.p;
  double* acc1 = (double*)ctx->hl_acc.p;
  double* du1 = (double*)ctx->hl_du.p;
  CRK_HIP(tbegin(ctx, P_STEP, s), "event");
  launch_hier_open<R>(n, lvl, lmax, 0, dt_min, lam, P.n_h, v, u, h, V, gradv, accel, dudt, vh,
                      uh, hdot, s);
  CRK_HIP(tend(ctx, P_STEP, s), "event");
  crk_status result = CRK_OK;
  for (int64_t j = 0; j < nsub; ++j) {
    const int64_t jend = j + 1;
    CRK_HIP(tbegin(ctx, P_STEP, s), "event");
    if (refine_at)
      launch_hier_refine<R>(n, j, refine_at, refine_level, lvl, lmax, dt_min, lam, P.n_h, v, u,
                            h, V, gradv, accel, dudt, vh, uh, hdot, s);
    launch_hier_drift<R>(n, lvl, lmax, j, dt_min, P.n_h, P.box, x, vh, accel, h, hdot, V, rho,
                         gradv, s);
    launch_hier_predict<R>(n, lvl, lmax, jend, dt_min, vh, uh, accel, dudt, vp, up, s);
    CRK_HIP(tend(ctx, P_STEP, s), "event");
    CRK_HIP(hipGetLastError(), "hierarchy launch");
    // the neighbour-list pass marks the passive partners of active particles
    CRK_HIP(hipMemsetAsync(ctx->hl_need.p, 0, N, s), "memset");
    // the particles of the levels whose interval ends here, and every refined
    // one, bound those active at this substep's end
    {
      long long bound = (long long)ctx->hl_hist_host[31];
      for (int L = 0; L <= lmax; ++L)
        if ((jend & (((int64_t)1 << (lmax - L)) - 1)) == 0) bound += (long long)ctx->hl_hist_host[L];
      ctx->hl_bound = std::min<long long>(bound, n);
    }
    // the passes see the levels and the stored state during this forward only
    ctx->hl_levels = lvl;
    ctx->hl_lmax = lmax;
    ctx->hl_jend = jend;
    ctx->hl_V = V;
    ctx->hl_rho = rho;
    ctx->hl_gv = gradv;
    ctx->hl_A = A;
    ctx->hl_B = B;
    ctx->hl_gA = gradA;
    ctx->hl_gB = gradB;
    crk_status st = forward_impl<R>(ctx, s, n, x, vp, m, up, h, V, rho, A, B, gradA, gradB,
                                    gradv, acc1, du1, stats);
    ctx->hl_levels = nullptr;
    if (st != CRK_OK && st != CRK_ENOTCONV && st != CRK_ENONFINITE) return st;
    if (st != CRK_OK) result = st;
    CRK_HIP(tbegin(ctx, P_STEP, s), "event");
    launch_hier_close<R>(n, lvl, lmax, jend, dt_min, v, u, vh, uh, acc1, du1, accel, dudt, s);
    if (jend < nsub)
      launch_hier_open<R>(n, lvl, lmax, jend, dt_min, lam, P.n_h, v, u, h, V, gradv, accel, dudt,
                          vh, uh, hdot, s);
    CRK_HIP(tend(ctx, P_STEP, s), "event");
    CRK_HIP(hipGetLastError(), "hierarchy launch");
  }
  // the last evaluation had passive particles (unless lmax = 0): no adjoint
  if (lmax > 0) ctx->n_last = -1;
  return result;
}

// Subgrid deposition (App. A.2 eq. (Vsg); eqs. (windmetal), (Anorm),
// (starmetal), (stellarmom), (AGNE)): folds the deposition counters (max
// slots for the *_BITS counters, sums otherwise) after a read-back.
crk_status dep_read(crk_ctx* ctx, hipStream_t s, unsigned long long* out) {
  CRK_HIP(hipMemcpyAsync(ctx->host_raw, ctx->dep_cnt.p, 8 * CNT_COUNT * kCntSpread,
                         hipMemcpyDeviceToHost, s),
          "deposition counters");
  CRK_HIP(hipStreamSynchronize(s), "deposition counters");
  for (int k = 0; k < CNT_COUNT; ++k) {
    const bool is_max = k == CNT_HMAX_BITS || k == CNT_HMAX_OUT_BITS;
    unsigned long long v = 0;
    for (int t = 0; t < kCntSpread; ++t) {
      const unsigned long long x = ctx->host_raw[k * kCntSpread + t];
      v = is_max ? (x > v ? x : v) : v + x;
    }
    out[k] = v;
  }
  return CRK_OK;
}

int bits_for(int64_t n) {
  int b = 1;
  while (b < 31 && ((int64_t)1 << b) < n) ++b;
  return b;
}

template <class R>
crk_status deposit_impl(crk_ctx* ctx, hipStream_t s, int64_t ng, const double* xg, const R* hg,
                        const R* Vg, R* mg, R* vg, R* mZg, R* ug, int64_t ns, const double* xs,
                        const R* dM, const R* dMZ, const R* dE, const R* vs, double n_h_s,
                        double z_max, double m_max, R* Vs, R* hs, R* As) {
  const crk_params& P = ctx->p;
  const double box = P.box;
  const double w0 = P.kernel == CRK_CUBIC_SPLINE ? Shape<0>::C * Shape<0>::w0
                                                 : Shape<1>::C * Shape<1>::w0;
  const double self_frac = w0 / (n_h_s * n_h_s * n_h_s);
  if (!(self_frac < 1.0))
    return fail(ctx, CRK_EINVAL, "n_h,s^3 must exceed C w(0): the self term alone exceeds 1/V_s");
  if (ns == 0) return CRK_OK;
  if (ng == 0) {
    CRK_HIP(hipMemsetAsync(Vs, 0, sizeof(R) * ns, s), "deposition");
    CRK_HIP(hipMemsetAsync(hs, 0, sizeof(R) * ns, s), "deposition");
    CRK_HIP(hipMemsetAsync(As, 0, sizeof(R) * ns, s), "deposition");
    return CRK_OK;
  }
  CRK_HIP(ensure(ctx->dep_keys_a, 4 * (size_t)ng), "deposition workspace");
  CRK_HIP(ensure(ctx->dep_keys_b, 4 * (size_t)ng), "deposition workspace");
  CRK_HIP(ensure(ctx->dep_vals_a, 4 * (size_t)ng), "deposition workspace");
  CRK_HIP(ensure(ctx->dep_vals_b, 4 * (size_t)ng), "deposition workspace");
  CRK_HIP(ensure(ctx->dep_first, 4 * (size_t)(ng + 1)), "deposition workspace");
  CRK_HIP(ensure(ctx->dep_npair, 4 * (size_t)ns), "deposition workspace");
  CRK_HIP(ensure(ctx->dep_off, 4 * (size_t)ns), "deposition workspace");
  CRK_HIP(ensure(ctx->dep_tmp, 4 * (size_t)std::max(radix_tmp_words(ng), scan_tmp_words(ns))),
          "deposition workspace");
  CRK_HIP(ensure(ctx->dep_cnt, 8 * CNT_COUNT * (size_t)kCntSpread), "deposition workspace");
  unsigned long long* cnt = (unsigned long long*)ctx->dep_cnt.p;
  unsigned long long folded[CNT_COUNT];
  CRK_HIP(tbegin(ctx, P_DEPOSIT, s), "event");
  CRK_HIP(hipMemsetAsync(cnt, 0, 8 * CNT_COUNT * (size_t)kCntSpread, s), "deposition");
  // the gas search radius of eq. (Vsg): the largest gas h
  launch_max_bits<R>(hg, ng, cnt, CNT_HMAX_BITS, s);
  CRK_HIP(hipGetLastError(), "deposition launch");
  if (crk_status st = dep_read(ctx, s, folded)) return st;
  const double hmax = bits_to_double(folded[CNT_HMAX_BITS]);
  if (!std::isfinite(hmax)) return fail(ctx, CRK_EINVAL, "gas h must be finite and > 0");
  if (!(hmax < 0.5 * box))
    return fail(ctx, CRK_EDOMAIN, "gas smoothing length must stay below half the box");
  // the gas grid: cells at least the largest gas h
  const int G = choose_grid(box, hmax * (1.0 + 1e-9), ng);
  const int64_t ncell = (int64_t)G * G * G;
  CRK_HIP(ensure(ctx->dep_start, 4 * (size_t)(ncell + 1)), "deposition grid");
  launch_point_keys(xg, ng, box, G, (uint32_t*)ctx->dep_keys_a.p, (uint32_t*)ctx->dep_vals_a.p,
                    s);
  CRK_HIP(radix_sort_pairs((uint32_t*)ctx->dep_keys_a.p, (uint32_t*)ctx->dep_vals_a.p,
                           (uint32_t*)ctx->dep_keys_b.p, (uint32_t*)ctx->dep_vals_b.p, ng,
                           bits_for(ncell), (uint32_t*)ctx->dep_tmp.p, s),
          "deposition sort");
  launch_cell_bounds((const uint32_t*)ctx->dep_keys_a.p, ng, ncell, (uint32_t*)ctx->dep_start.p,
                     ~0ull, cnt, s);
  CRK_HIP(ensure(ctx->dep_p4, 32 * (size_t)ng), "deposition workspace");
  CRK_HIP(ensure(ctx->dep_pv, 16 * (size_t)ng), "deposition workspace");
  // the sort's second key buffer is free again: it holds the ranks
  launch_dep_pack<R>((const uint32_t*)ctx->dep_vals_a.p, (uint32_t*)ctx->dep_keys_b.p, xg, ng, hg,
                     Vg, mg, mZg, z_max, m_max, ctx->dep_p4.p, ctx->dep_pv.p, s);
  const DepGrid grid{G, box, hmax, (const uint32_t*)ctx->dep_start.p,
                     (const uint32_t*)ctx->dep_vals_a.p, ctx->dep_p4.p, ctx->dep_pv.p};
  launch_dep_volume<R>(P.kernel, grid, xs, ns, self_frac, n_h_s, Vs, hs, s);
  uint32_t* npair = (uint32_t*)ctx->dep_npair.p;
  CRK_HIP(ensure(ctx->dep_sp, 96 * (size_t)ns), "deposition workspace");
  CRK_HIP(ensure(ctx->dep_slot, 4 * 64 * (size_t)ns), "deposition workspace");
  launch_dep_norm<R>(P.kernel, grid, xs, ns, hs, dM, dMZ, dE, vs, As, ctx->dep_sp.p, npair,
                     (uint32_t*)ctx->dep_slot.p, cnt, s);
  CRK_HIP(hipGetLastError(), "deposition launch");
  if (crk_status st = dep_read(ctx, s, folded)) return st;
  const double hsmax = bits_to_double(folded[CNT_HMAX_OUT_BITS]);
  const unsigned long long npairs = folded[CNT_PAIRS_GATHER];
  if (!std::isfinite(hsmax)) return fail(ctx, CRK_ENONFINITE, "source volume is not finite");
  if (!(hsmax < 0.5 * box))
    return fail(ctx, CRK_EDOMAIN, "source smoothing length must stay below half the box");
  if (npairs > 0x7fffffffull) return fail(ctx, CRK_ENOMEM, "more than 2^31 source-gas pairs");
  if (npairs > 0) {
    // receivers of every source at its offset, grouped by gas index (stable:
    // source order within a gas particle), then one sum per gas particle
    const int64_t np = (int64_t)npairs;
    CRK_HIP(ensure(ctx->dep_pj_a, 4 * (size_t)np), "deposition pairs");
    CRK_HIP(ensure(ctx->dep_pj_b, 4 * (size_t)np), "deposition pairs");
    CRK_HIP(ensure(ctx->dep_ps_a, 4 * (size_t)np), "deposition pairs");
    CRK_HIP(ensure(ctx->dep_ps_b, 4 * (size_t)np), "deposition pairs");
    CRK_HIP(ensure(ctx->dep_ptmp, 4 * (size_t)radix_tmp_words(np)), "deposition pairs");
    CRK_HIP(exclusive_scan_u32(npair, (uint32_t*)ctx->dep_off.p, ns, (uint32_t*)ctx->dep_tmp.p,
                               s),
            "deposition scan");
    launch_dep_pairs<R>(grid, xs, ns, hs, npair, (const uint32_t*)ctx->dep_slot.p,
                        (const uint32_t*)ctx->dep_off.p, (uint32_t*)ctx->dep_pj_a.p,
                        (uint32_t*)ctx->dep_ps_a.p, s);
    CRK_HIP(radix_sort_pairs((uint32_t*)ctx->dep_pj_a.p, (uint32_t*)ctx->dep_ps_a.p,
                             (uint32_t*)ctx->dep_pj_b.p, (uint32_t*)ctx->dep_ps_b.p, np,
                             bits_for(ng), (uint32_t*)ctx->dep_ptmp.p, s),
            "deposition pair sort");
    launch_cell_bounds((const uint32_t*)ctx->dep_pj_a.p, np, ng, (uint32_t*)ctx->dep_first.p,
                       ~0ull, cnt, s);
    launch_dep_apply<R>(P.kernel, xg, ng, Vg, mg, vg, mZg, ug, ctx->dep_sp.p,
                        (const uint32_t*)ctx->dep_first.p, (const uint32_t*)ctx->dep_ps_a.p, box,
                        s);
    CRK_HIP(hipGetLastError(), "deposition launch");
  }
  CRK_HIP(tend(ctx, P_DEPOSIT, s), "event");
  return CRK_OK;
}

// ---- crk_backward_noalloc: the adjoint's workspace in a static array ----
// One copy of this array lives on every GPU the library runs on, for the
// life of the process. Host code never uses its name as an address: the
// address on each device comes from hipGetSymbolAddress, taken once per
// device with that device current, and is what the kernels receive.
constexpr long long kNoAllocMaxN = 65536;
constexpr size_t kNoAllocBytes = adj_layout(kNoAllocMaxN, 8, nullptr);  // 41 MiB (FP64 sizes)
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// This device's copy of scratch (address taken on its first use).
hipError_t scratch_address(unsigned char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = (unsigned char*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

void crk_default_params(crk_params* p, int precision) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->box = 1.0;
  p->gamma = 5.0 / 3.0;
  p->alpha = 1.0;
  p->beta = 2.0;
  p->eps2 = 0.01;
  p->n_h = 2.4814;
  p->kernel = CRK_CUBIC_SPLINE;
  p->precision = precision;
  p->h_mode = 1;
  p->h_max_iter = 60;
  p->h_rtol = precision == CRK_FP64 ? 1e-13 : 1e-6;
  p->dt_relax = 0.0;
  p->store_corrections = 0;
  p->check_finite = 0;
}

crk_status crk_create(crk_ctx** out, const crk_params* p) {
  if (!out) return CRK_EINVAL;
  *out = nullptr;
  crk_status st = check_params(nullptr, p);
  if (st != CRK_OK) return st;
  crk_ctx* c = new crk_ctx();
  c->p = *p;
  if (hipHostMalloc((void**)&c->host_raw, 8 * CNT_COUNT * kCntSpread, hipHostMallocDefault) !=
      hipSuccess) {
    delete c;
    return CRK_ENOMEM;
  }
  std::memset(c->host_raw, 0, 8 * CNT_COUNT * kCntSpread);
  *out = c;
  return CRK_OK;
}

crk_status crk_set_params(crk_ctx* ctx, const crk_params* p) {
  if (!ctx) return CRK_EINVAL;
  crk_status st = check_params(ctx, p);
  if (st != CRK_OK) return st;
  const crk_params o = ctx->p;
  ctx->p = *p;
  // the cell-list geometry depends on these; the kept forward state on every
  // parameter the passes or the adjoint read (all but timing and the check)
  const bool geometry = o.box != p->box || o.n_h != p->n_h || o.kernel != p->kernel ||
                        o.precision != p->precision || o.h_mode != p->h_mode ||
                        o.h_max_iter != p->h_max_iter || o.h_rtol != p->h_rtol ||
                        o.search != p->search;
  const bool state = geometry || o.gamma != p->gamma || o.alpha != p->alpha ||
                     o.beta != p->beta || o.eps2 != p->eps2 || o.dt_relax != p->dt_relax ||
                     o.store_corrections != p->store_corrections;
  if (geometry) ctx->spec_ok = false;
  if (state) ctx->n_last = -1;  // crk_backward needs a forward with these parameters
  return CRK_OK;
}

crk_status crk_reserve(crk_ctx* ctx, long long n_max) {
  if (!ctx || n_max < 0) return fail(ctx, CRK_EINVAL, "bad reserve size");
  if (n_max == 0) return CRK_OK;
  // a buffer that grows is reallocated: the state kept for crk_backward is
  // then gone
  const void* before[] = {ctx->pv.p, ctx->st4.p, ctx->kc4.p, ctx->gv4.p,
                          ctx->mom.p, ctx->nlist.p, ctx->slist.p, ctx->ng.p, ctx->ns.p,
                          ctx->vals_a.p, ctx->cell3.p, ctx->mass.p, ctx->uu.p, ctx->hbuf.p,
                          ctx->Vbuf.p};
  hipError_t e = ensure_particles(ctx, n_max);
  const int64_t npad = ((n_max + 63) / 64) * 64;
  if (e == hipSuccess) e = ensure(ctx->nlist, 4 * (size_t)npad * ctx->list_cap);
  if (e == hipSuccess) e = ensure(ctx->slist, 4 * (size_t)npad * ctx->slist_cap);
  if (e == hipSuccess)
    e = ensure(ctx->scr_r, real_size(ctx->p.precision) * (size_t)npad * ctx->scr_cap);
  if (e == hipSuccess) e = ensure(ctx->cand, 4 * (size_t)npad * ctx->scr_cap);
  const void* after[] = {ctx->pv.p, ctx->st4.p, ctx->kc4.p, ctx->gv4.p,
                         ctx->mom.p, ctx->nlist.p, ctx->slist.p, ctx->ng.p, ctx->ns.p,
                         ctx->vals_a.p, ctx->cell3.p, ctx->mass.p, ctx->uu.p, ctx->hbuf.p,
                         ctx->Vbuf.p};
  for (size_t k = 0; k < sizeof(before) / sizeof(before[0]); ++k)
    if (before[k] != after[k]) ctx->n_last = -1;
  if (e != hipSuccess) {
    ctx->n_last = -1;
    return hip_fail(ctx, e, "reserve");
  }
  return CRK_OK;
}

crk_status crk_destroy(crk_ctx* c) {
  if (!c) return CRK_OK;
  Buf* all[] = {&c->keys_a, &c->keys_b, &c->vals_a, &c->vals_b, &c->cell_start,
                &c->sort_tmp, &c->scan_tmp, &c->pv, &c->mass, &c->uu, &c->hbuf,
                &c->Vbuf, &c->st4, &c->gv4, &c->kc4, &c->mom, &c->nlist, &c->slist, &c->ng, &c->ns,
                &c->scr_r, &c->scr_m, &c->cand, &c->ccnt, &c->cell3, &c->cnt, &c->vpred, &c->upred,
                &c->hl_vh, &c->hl_uh, &c->hl_hdot, &c->hl_acc, &c->hl_du, &c->hl_need, &c->hl_act, &c->hl_hist,
                &c->cool_lam, &c->cool_oma, &c->cool_co, &c->cool_G, &c->cool_run, &c->cool_binint,
                &c->dep_keys_a, &c->dep_keys_b, &c->dep_vals_a, &c->dep_vals_b, &c->dep_start,
                &c->dep_tmp, &c->dep_cnt, &c->dep_npair, &c->dep_off, &c->dep_first,
                &c->dep_pj_a, &c->dep_pj_b, &c->dep_ps_a, &c->dep_ps_b, &c->dep_ptmp,
                &c->dep_p4, &c->dep_pv, &c->dep_sp, &c->dep_slot,
                &c->rad, &c->need, &c->todo, &c->tslot, &c->nlo, &c->nhi, &c->lvl, &c->wrow, &c->lrow,
                &c->cpos, &c->torder, &c->absp, &c->hl_lvl, &c->need4, &c->coff};
  for (Buf* b : all) release(*b);
  if (c->host_raw) (void)hipHostFree(c->host_raw);
  if (c->events_ready)
    for (int i = 0; i < P_NPASS; ++i) {
      (void)hipEventDestroy(c->ev0[i]);
      (void)hipEventDestroy(c->ev1[i]);
    }
  delete c;
  return CRK_OK;
}

const char* crk_last_error(const crk_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int crk_pass_count(void) { return P_NPASS; }

const char* crk_pass_name(int k) { return (k >= 0 && k < P_NPASS) ? kPassNames[k] : nullptr; }

crk_status crk_pass_times(crk_ctx* ctx, double* ms, long long* calls, int reset) {
  if (!ctx) return CRK_EINVAL;
  for (int k = 0; k < P_NPASS; ++k) {
    hipError_t e = harvest(ctx, k);
    if (e != hipSuccess) return hip_fail(ctx, e, "pass timing");
    if (ms) ms[k] = ctx->ms_total[k];
    if (calls) calls[k] = ctx->ms_calls[k];
    if (reset) {
      ctx->ms_total[k] = 0.0;
      ctx->ms_calls[k] = 0;
    }
  }
  return CRK_OK;
}

crk_status crk_forward(crk_ctx* ctx, void* hip_stream, long long n, const double* x,
                       const void* v, const void* m, const void* u, void* h, void* V, void* rho,
                       void* A, void* B, void* gradA, void* gradB, void* gradv, double* accel,
                       double* dudt, crk_stats* stats) {
  if (!ctx) return CRK_EINVAL;
  ctx->err.clear();
  if (n < 0) return fail(ctx, CRK_EINVAL, "n must be >= 0");
  if (n == 0) {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    ctx->n_last = 0;
    return CRK_OK;
  }
  if (n > (1ll << 25) - 1) return fail(ctx, CRK_EINVAL, "n exceeds 2^25 - 1 particles");
  if (!x || !v || !m || !u || !h || !V || !rho || !A || !B || !gradA || !gradB || !gradv ||
      !accel || !dudt)
    return fail(ctx, CRK_EINVAL, "null array argument");
  hipStream_t s = (hipStream_t)hip_stream;
  if (ctx->p.precision == CRK_FP64)
    return forward_impl<double>(ctx, s, n, x, (const double*)v, (const double*)m,
                                (const double*)u, (double*)h, (double*)V, (double*)rho, A, B,
                                gradA, gradB, (double*)gradv, accel, dudt, stats);
  return forward_impl<float>(ctx, s, n, x, (const float*)v, (const float*)m, (const float*)u,
                             (float*)h, (float*)V, (float*)rho, A, B, gradA, gradB,
                             (float*)gradv, accel, dudt, stats);
}

crk_status crk_backward(crk_ctx* ctx, void* hip_stream, long long n, const double* g_accel,
                        const double* g_dudt, double* g_x, double* g_v, double* g_u,
                        double* g_alpha_beta) {
  if (!ctx) return CRK_EINVAL;
  ctx->err.clear();
  if (n < 0 || n != ctx->n_last)
    return fail(ctx, CRK_EINVAL, "no forward with this n on the context");
  if (ctx->precision_last != ctx->p.precision)
    return fail(ctx, CRK_EINVAL, "precision changed since the forward");
  if (!g_alpha_beta) return fail(ctx, CRK_EINVAL, "null array argument");
  hipStream_t s = (hipStream_t)hip_stream;
  if (n == 0) {
    launch_zero_f64(g_alpha_beta, 2, s);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? CRK_OK : hip_fail(ctx, e, "zero fill");
  }
  if (!g_accel || !g_dudt || !g_x || !g_v || !g_u)
    return fail(ctx, CRK_EINVAL, "null array argument");
  if (ctx->p.precision == CRK_FP64)
    return backward_impl<double>(ctx, s, n, g_accel, g_dudt, g_x, g_v, g_u, g_alpha_beta);
  return backward_impl<float>(ctx, s, n, g_accel, g_dudt, g_x, g_v, g_u, g_alpha_beta);
}

crk_status crk_backward_noalloc(crk_ctx* ctx, void* hip_stream, long long n,
                                const double* g_accel, const double* g_dudt, double* g_x,
                                double* g_v, double* g_u, double* g_alpha_beta) {
  if (!ctx) return CRK_EINVAL;
  ctx->err.clear();
  if (n > kNoAllocMaxN)
    return fail(ctx, CRK_EINVAL, "crk_backward_noalloc takes at most 65536 particles");
  if (n < 0 || n != ctx->n_last)
    return fail(ctx, CRK_EINVAL, "no forward with this n on the context");
  if (ctx->precision_last != ctx->p.precision)
    return fail(ctx, CRK_EINVAL, "precision changed since the forward");
  if (!g_alpha_beta) return fail(ctx, CRK_EINVAL, "null array argument");
  hipStream_t s = (hipStream_t)hip_stream;
  if (n == 0) {
    launch_zero_f64(g_alpha_beta, 2, s);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? CRK_OK : hip_fail(ctx, e, "zero fill");
  }
  if (!g_accel || !g_dudt || !g_x || !g_v || !g_u)
    return fail(ctx, CRK_EINVAL, "null array argument");
  unsigned char* arena = nullptr;
  CRK_HIP(scratch_address(&arena), "static workspace address");
  if (adj_layout(n, real_size(ctx->p.precision), nullptr) > kNoAllocBytes)
    return fail(ctx, CRK_EINVAL, "static workspace too small");  // not reached for n <= max
  if (ctx->p.precision == CRK_FP64)
    return backward_impl<double>(ctx, s, n, g_accel, g_dudt, g_x, g_v, g_u, g_alpha_beta,
                                 arena);
  return backward_impl<float>(ctx, s, n, g_accel, g_dudt, g_x, g_v, g_u, g_alpha_beta, arena);
}

crk_status crk_kdk_step(crk_ctx* ctx, void* hip_stream, long long n, double dt,
                        double thacker_lambda, double* x, void* v, const void* m, void* u,
                        void* h, void* V, void* rho, void* A, void* B, void* gradA, void* gradB,
                        void* gradv, double* accel, double* dudt, crk_stats* stats) {
  if (!ctx) return CRK_EINVAL;
  ctx->err.clear();
  if (ctx->p.h_mode != 0)
    return fail(ctx, CRK_EINVAL, "the time step integrates h: the context needs h_mode 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, CRK_EINVAL, "dt must be finite and > 0");
  if (!(thacker_lambda >= 0.0 && thacker_lambda <= 1.0))
    return fail(ctx, CRK_EINVAL, "thacker_lambda must lie in [0, 1]");
  if (n < 0) return fail(ctx, CRK_EINVAL, "n must be >= 0");
  if (n == 0) {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    ctx->n_last = 0;
    return CRK_OK;
  }
  if (n > (1ll << 25) - 1) return fail(ctx, CRK_EINVAL, "n exceeds 2^25 - 1 particles");
  if (!x || !v || !m || !u || !h || !V || !rho || !A || !B || !gradA || !gradB || !gradv ||
      !accel || !dudt)
    return fail(ctx, CRK_EINVAL, "null array argument");
  hipStream_t s = (hipStream_t)hip_stream;
  if (ctx->p.precision == CRK_FP64)
    return step_impl<double>(ctx, s, n, dt, thacker_lambda, x, (double*)v, (const double*)m,
                             (double*)u, (double*)h, (double*)V, (double*)rho, A, B, gradA, gradB,
                             (double*)gradv, accel, dudt, stats);
  return step_impl<float>(ctx, s, n, dt, thacker_lambda, x, (float*)v, (const float*)m, (float*)u,
                          (float*)h, (float*)V, (float*)rho, A, B, gradA, gradB, (float*)gradv,
                          accel, dudt, stats);
}

crk_status crk_hkdk_step(crk_ctx* ctx, void* hip_stream, long long n, double dt,
                         double thacker_lambda, const int* levels, const int* refine_at,
                         const int* refine_level, double* x, void* v, const void* m, void* u,
                         void* h, void* V, void* rho, void* A, void* B, void* gradA, void* gradB,
                         void* gradv, double* accel, double* dudt, crk_stats* stats) {
  if (!ctx) return CRK_EINVAL;
  ctx->err.clear();
  if (ctx->p.h_mode != 0)
    return fail(ctx, CRK_EINVAL, "the time step integrates h: the context needs h_mode 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, CRK_EINVAL, "dt must be finite and > 0");
  if (!(thacker_lambda >= 0.0 && thacker_lambda <= 1.0))
    return fail(ctx, CRK_EINVAL, "thacker_lambda must lie in [0, 1]");
  if (n < 0) return fail(ctx, CRK_EINVAL, "n must be >= 0");
  if (n == 0) {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    ctx->n_last = 0;
    return CRK_OK;
  }
  if (n > (1ll << 25) - 1) return fail(ctx, CRK_EINVAL, "n exceeds 2^25 - 1 particles");
  if (!levels || !x || !v || !m || !u || !h || !V || !rho || !A || !B || !gradA || !gradB ||
      !gradv || !accel || !dudt || (refine_at && !refine_level))
    return fail(ctx, CRK_EINVAL, "null array argument");
  hipStream_t s = (hipStream_t)hip_stream;
  if (ctx->p.precision == CRK_FP64)
    return hstep_impl<double>(ctx, s, n, dt, thacker_lambda, levels, refine_at, refine_level, x,
                              (double*)v, (const double*)m, (double*)u, (double*)h, (double*)V,
                              (double*)rho, A, B, gradA, gradB, (double*)gradv, accel, dudt,
                              stats);
  return hstep_impl<float>(ctx, s, n, dt, thacker_lambda, levels, refine_at, refine_level, x,
                           (float*)v, (const float*)m, (float*)u, (float*)h, (float*)V,
                           (float*)rho, A, B, gradA, gradB, (float*)gradv, accel, dudt, stats);
}

crk_status crk_cooling_table(crk_ctx* ctx, void* hip_stream, int K, double log10_u0, double dex,
                             const double* lam) {
  if (!ctx) return CRK_EINVAL;
  ctx->err.clear();
  if (K < 2 || !lam) return fail(ctx, CRK_EINVAL, "a cooling table needs K >= 2 values");
  if (!(dex > 0.0) || !std::isfinite(dex) || !std::isfinite(log10_u0))
    return fail(ctx, CRK_EINVAL, "cooling table spacing must be finite and > 0");
  for (int k = 0; k < K; ++k)
    if (!std::isfinite(lam[k])) return fail(ctx, CRK_EINVAL, "cooling table values must be finite");
  if (!std::isfinite(log10_u0 + (K - 1) * dex) || std::fabs(log10_u0) > 300.0 ||
      std::fabs(log10_u0 + (K - 1) * dex) > 300.0)
    return fail(ctx, CRK_EINVAL, "cooling table energies out of the double range");
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t kk = (size_t)K;
  CRK_HIP(ensure(ctx->cool_lam, 8 * kk), "cooling table");
  CRK_HIP(ensure(ctx->cool_oma, 8 * kk), "cooling table");
  CRK_HIP(ensure(ctx->cool_G, 8 * kk), "cooling table");
  CRK_HIP(ensure(ctx->cool_run, 8 * kk), "cooling table");
  CRK_HIP(ensure(ctx->cool_binint, 8 * kk), "cooling table");
  CRK_HIP(ensure(ctx->cool_co, 8 * kk), "cooling table");
  CRK_HIP(hipMemcpyAsync(ctx->cool_lam.p, lam, 8 * kk, hipMemcpyHostToDevice, s), "cooling table");
  launch_cool_prepare(K, log10_u0, dex, (const double*)ctx->cool_lam.p, (double*)ctx->cool_oma.p,
                      (double*)ctx->cool_co.p, (double*)ctx->cool_G.p, ctx->cool_run.p,
                      (double*)ctx->cool_binint.p, s);
  CRK_HIP(hipGetLastError(), "cooling table launch");
  // the host copy of lam is read by the copy above: finish it before returning
  CRK_HIP(hipStreamSynchronize(s), "cooling table");
  ctx->cool_K = K;
  ctx->cool_lu0 = log10_u0;
  ctx->cool_dex = dex;
  return CRK_OK;
}

crk_status crk_cool(crk_ctx* ctx, void* hip_stream, long long n, double dt, const void* rho,
                    void* u) {
  if (!ctx) return CRK_EINVAL;
  ctx->err.clear();
  if (ctx->cool_K < 2) return fail(ctx, CRK_EINVAL, "no cooling table on the context");
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(ctx, CRK_EINVAL, "dt must be finite and >= 0");
  if (n < 0) return fail(ctx, CRK_EINVAL, "n must be >= 0");
  if (n == 0) return CRK_OK;
  if (!rho || !u) return fail(ctx, CRK_EINVAL, "null array argument");
  hipStream_t s = (hipStream_t)hip_stream;
  CRK_HIP(tbegin(ctx, P_COOL, s), "event");
  if (ctx->p.precision == CRK_FP64)
    launch_cool<double>(ctx->cool_K, ctx->cool_lu0, ctx->cool_dex, (const double*)ctx->cool_lam.p,
                        (const double*)ctx->cool_co.p, (const double*)ctx->cool_oma.p,
                        (const double*)ctx->cool_G.p, ctx->cool_run.p, n, dt, (const double*)rho,
                        (double*)u, s);
  else
    launch_cool<float>(ctx->cool_K, ctx->cool_lu0, ctx->cool_dex, (const double*)ctx->cool_lam.p,
                       (const double*)ctx->cool_co.p, (const double*)ctx->cool_oma.p,
                       (const double*)ctx->cool_G.p, ctx->cool_run.p, n, dt, (const float*)rho,
                       (float*)u, s);
  CRK_HIP(tend(ctx, P_COOL, s), "event");
  CRK_HIP(hipGetLastError(), "cooling launch");
  return CRK_OK;
}

crk_status crk_deposit(crk_ctx* ctx, void* hip_stream, long long n_gas, const double* x_gas,
                       const void* h_gas, const void* V_gas, void* m_gas, void* v_gas,
                       void* mZ_gas, void* u_gas, long long n_src, const double* x_src,
                       const void* dM, const void* dMZ, const void* dE, const void* v_src,
                       double n_h_src, double z_max, double m_max, void* V_src, void* h_src,
                       void* A_src) {
  if (!ctx) return CRK_EINVAL;
  ctx->err.clear();
  if (n_gas < 0 || n_src < 0) return fail(ctx, CRK_EINVAL, "counts must be >= 0");
  if (n_gas > 0xffffffffLL || n_src > 0xffffffffLL)
    return fail(ctx, CRK_EINVAL, "counts must fit 32-bit indices");
  if (!(n_h_src > 0.0) || !std::isfinite(n_h_src))
    return fail(ctx, CRK_EINVAL, "n_h_src must be finite and > 0");
  if (std::isnan(z_max) || std::isnan(m_max))
    return fail(ctx, CRK_EINVAL, "z_max and m_max must not be NaN");
  if (n_src > 0 && (!x_src || !dM || !dMZ || !dE || !v_src || !V_src || !h_src || !A_src))
    return fail(ctx, CRK_EINVAL, "null source array");
  if (n_src > 0 && n_gas > 0 &&
      (!x_gas || !h_gas || !V_gas || !m_gas || !v_gas || !mZ_gas || !u_gas))
    return fail(ctx, CRK_EINVAL, "null gas array");
  hipStream_t s = (hipStream_t)hip_stream;
  if (ctx->p.precision == CRK_FP64)
    return deposit_impl<double>(ctx, s, n_gas, x_gas, (const double*)h_gas, (const double*)V_gas,
                                (double*)m_gas, (double*)v_gas, (double*)mZ_gas, (double*)u_gas,
                                n_src, x_src, (const double*)dM, (const double*)dMZ,
                                (const double*)dE, (const double*)v_src, n_h_src, z_max, m_max,
                                (double*)V_src, (double*)h_src, (double*)A_src);
  return deposit_impl<float>(ctx, s, n_gas, x_gas, (const float*)h_gas, (const float*)V_gas,
                             (float*)m_gas, (float*)v_gas, (float*)mZ_gas, (float*)u_gas, n_src,
                             x_src, (const float*)dM, (const float*)dMZ, (const float*)dE,
                             (const float*)v_src, n_h_src, z_max, m_max, (float*)V_src,
                             (float*)h_src, (float*)A_src);
}

}  // extern "C"
