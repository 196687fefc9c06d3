// Adjoint (reverse-mode) CRKSPH passes on gfx950, in gather form.
//
// For the loss L = sum_i gA_i . a_i + sum_i gU_i du_i/dt, each pass gives
// every particle the derivatives of L with respect to its own quantities:
//   k_bwd_force    pairwise momentum/energy with viscosity -> x, v, h, V,
//                  packed corrections, rho, P, c, grad v, alpha, beta;
//                  the EOS adjoint (P, c -> rho, u) closes the kernel;
//   k_bwd_density  density and velocity gradient (own sums and the
//                  particle's share in its neighbours' sums) -> x, v, h, V,
//                  packed corrections;
//   k_bwd_corr     corrections -> the 40 moment sums through the FP64 solve
//                  (moments recomputed, or read when the forward kept them);
//   k_bwd_moments  moments -> x, h, V (own and neighbours' sums), then the
//                  volume / smoothing-length coefficient kappa;
//   k_bwd_volume   V_i = m_i / sum_j m_j W(r_ij, h_i) and, for solved h, the
//                  implicit-function term of the Thacker fixed point
//                  (App. A.3) -> x;
//   k_bwd_finish   caller order and the alpha, beta totals.
// Pair arithmetic in Real, accumulators in FP64; no float atomics.
#include "crk_adjoint.h"
#include "crk_passes.h"

namespace crk {
namespace {

template <class R>
__device__ inline R dot3b(const R a[3], const R b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

template <class R>
__device__ inline void load_kc4(const State<R>& S, int64_t j, KC<R>& k) {
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
__device__ inline void load_gv4(const State<R>& S, int64_t j, R gv[9], R& relaxed) {
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

template <class R>
__device__ inline void load_side(const State<R>& S, const AdjState<R>& G, int64_t j,
                                 PairSide<R>& o, R& relaxed) {
  const R4<R> p = S.pos(j);
  const R4<R> v = S.vel(j);
  const R4<R> st = S.st4[j];
  const R4<R> w = G.wgt4[j];
  load_kc4(S, j, o.kc);
  load_gv4(S, j, o.gv, relaxed);
  o.hinv = p.w;
  o.h = Sc<R>::rcp(p.w);
  o.V = v.w;
  o.rho = st.x;
  o.P = st.y;
  o.c = st.z;
  o.v[0] = v.x;
  o.v[1] = v.y;
  o.v[2] = v.z;
  o.wam[0] = w.x;
  o.wam[1] = w.y;
  o.wam[2] = w.z;
  o.wum = w.w;
}

template <class R>
__device__ inline void load_gvc(const AdjState<R>& G, int64_t j, R gvb[9], R& Numb, R& Denb) {
  const R4<R> q0 = G.gvc4[3 * j], q1 = G.gvc4[3 * j + 1], q2 = G.gvc4[3 * j + 2];
  gvb[0] = q0.x;
  gvb[1] = q0.y;
  gvb[2] = q0.z;
  gvb[3] = q0.w;
  gvb[4] = q1.x;
  gvb[5] = q1.y;
  gvb[6] = q1.z;
  gvb[7] = q1.w;
  gvb[8] = q2.x;
  Numb = q2.y;
  Denb = q2.z;
}

template <class R>
__device__ inline void load_mom(const AdjState<R>& G, int64_t j, R mb[40]) {
#pragma unroll
  for (int t = 0; t < 10; ++t) {
    const R4<R> q = G.mom4[10 * j + t];
    mb[4 * t] = q.x;
    mb[4 * t + 1] = q.y;
    mb[4 * t + 2] = q.z;
    mb[4 * t + 3] = q.w;
  }
}

// Loss weights gathered into sorted order.
template <class R>
__global__ void __launch_bounds__(kBlock) k_bwd_prep(State<R> S, AdjState<R> G) {
  const int64_t s = particle_id();
  if (s >= S.n) return;
  const int64_t n = S.n;
  const uint32_t q = S.perm[s];
  // the force adjoint uses the weights only as w_a / m and w_u / (2 m)
  const R m = S.mass[s];
  R4<R> w;
  w.x = (R)G.w_a[q] / m;
  w.y = (R)G.w_a[n + q] / m;
  w.z = (R)G.w_a[2 * n + q] / m;
  w.w = (R)G.w_u[q] / (R(2) * m);
  G.wgt4[s] = w;
}

// ------------------------------------------------------------------ B1+B2 --
template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_bwd_force(State<R> S, AdjState<R> G) {
  const int64_t s = particle_id();
  double pa = 0.0, pb = 0.0;
  if (s < S.n) {
    const int64_t n = S.n;
    PairSide<R> I, J;
    R reli, relj;
    load_side(S, G, s, I, reli);
    const KC<R> kci = I.kc;
    const bool relax_on = S.dt_relax > 0.0;
    const R alpha = R(S.alpha), beta = R(S.beta), eps2 = R(S.eps2);
    // x, v, h, V and the EOS adjoints accumulate in FP64; the 16 correction
    // and 9 velocity-gradient adjoint sums (one term per pair) in the
    // working precision, like the density adjoint's own correction sums
    ForceBar<double, R> ob;
    ob.zero();
    __shared__ uint4 eslot[kBlock];  // the lane's list chunk (registers are scarce here)
    const NbrRef nb = nbr_ref(S, s);
    const int ng = nb.ng, ns = nb.ns;
    const R4<R> pi = S.pos(s);
    for (int t = 0; t < ng + ns; ++t) {
      const uint32_t e = nbr_entry_lds(S, nb, t, &eslot[threadIdx.x]);
      const uint32_t j = e >> kCodeBits;
      load_side(S, G, j, J, relj);
      R x[3];
      pair_x(S, s, pi, S.pos(j), e, x);
      const bool plain = relax_on && (reli != R(0) || relj != R(0));
      if (plain) {
        kc_plain(I.kc);
        kc_plain(J.kc);
      } else {
        I.kc = kci;
      }
      force_pair_adj<R, double, R, K>(I, J, x, alpha, beta, eps2, !plain, ob);
    }
    // equation of state: P = (gamma - 1) rho u, c = sqrt(gamma (gamma - 1) u)
    const double gam = S.gamma;
    const double u = (double)S.uu[s];
    const double rhob = ob.rho + ob.P * (gam - 1.0) * u;
    const double ub = ob.P * (gam - 1.0) * (double)I.rho +
                      ob.c * gam * (gam - 1.0) / (2.0 * (double)I.c);
    for (int a = 0; a < 3; ++a) {
      G.gx[a * n + s] = ob.x[a];
      G.gv[a * n + s] = ob.v[a];
    }
    G.gh[s] = ob.h;
    G.gV[s] = ob.V;
    G.gu[s] = ub;
    G.gkc[s] = ob.kc.a;
    for (int t = 0; t < 3; ++t) {
      G.gkc[(1 + t) * n + s] = ob.kc.b[t];
      G.gkc[(4 + t) * n + s] = ob.kc.c[t];
    }
    for (int t = 0; t < 9; ++t) G.gkc[(7 + t) * n + s] = ob.kc.M[t];
    // density adjoint coefficients: rho = Num / Den
    const double den = (double)S.st4[s].w;
    R4<R> q0, q1, q2;
    q0.x = (R)ob.gv[0]; q0.y = (R)ob.gv[1]; q0.z = (R)ob.gv[2]; q0.w = (R)ob.gv[3];
    q1.x = (R)ob.gv[4]; q1.y = (R)ob.gv[5]; q1.z = (R)ob.gv[6]; q1.w = (R)ob.gv[7];
    q2.x = (R)ob.gv[8];
    q2.y = (R)(rhob / den);                       // Num bar
    q2.z = (R)(-rhob * (double)I.rho / den);      // Den bar
    q2.w = R(0);
    G.gvc4[3 * s] = q0;
    G.gvc4[3 * s + 1] = q1;
    G.gvc4[3 * s + 2] = q2;
    pa = ob.alpha;
    pb = ob.beta;
  }
  // per-block alpha, beta partial sums (fixed tree: deterministic)
  __shared__ double sa[kBlock], sb[kBlock];
  sa[threadIdx.x] = pa;
  sb[threadIdx.x] = pb;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    G.gab[2 * blockIdx.x] = sa[0];
    G.gab[2 * blockIdx.x + 1] = sb[0];
  }
}

// --------------------------------------------------------------------- B3 --
template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_bwd_density(State<R> S, AdjState<R> G) {
  const int64_t s = particle_id();
  if (s >= S.n) return;
  const int64_t n = S.n;
  const R4<R> pi = S.pos(s);
  const R4<R> vi = S.vel(s);
  const R mi = S.mass[s];
  KC<R> ki;
  load_kc4(S, s, ki);
  R gvb[9], Numb, Denb;
  load_gvc(G, s, gvb, Numb, Denb);
  // the 16 correction adjoints of the own sums accumulate in the working
  // precision (64 gather pairs; they feed the FP64 correction adjoint), which
  // keeps this kernel at 4 waves per SIMD in FP32
  KCBar<R> kb;
  kb.zero();
  double xb[3] = {0, 0, 0}, vb[3] = {0, 0, 0}, hb = 0, Vb = 0;
  R W0, dW0;
  kernel_self<R, K>(pi.w, W0, dW0);
  density_self_adj<R, double, R>(ki.a, mi, vi.w, W0, dW0, Numb, Denb, &kb, Vb, hb);
  const NbrRef nb = nbr_ref(S, s);
  uint4 ebuf;
  const int ng = nb.ng, ns = nb.ns;
  // Two passes over the list so that the particle's own corrections and
  // accumulators and the neighbour's records are not live together: own
  // sums (gather part), then the particle's share in its neighbours' sums
  // (every j with r < h_j).
  for (int t = 0; t < ng; ++t) {
    const uint32_t e = gather_entry(S, nb, t, ebuf);
    const uint32_t j = e >> kCodeBits;
    const R4<R> pj = S.pos(j);
    const R4<R> vj = S.vel(j);
    R x[3];
    pair_x(S, s, pi, pj, e, x);
    const R r2 = dot3b(x, x);
    const R rinv = Sc<R>::rsqrt(r2);
    const R r = r2 * rinv;
    const R vij[3] = {vi.x - vj.x, vi.y - vj.y, vi.z - vj.z};
    KEval<R> ev;
    kernel_eval<R, K>(r, rinv, pi.w, ev);
    density_own_adj<R, double, R>(ki, x, r, rinv, ev, S.mass[j], vj.w, vij, Numb, Denb, gvb,
                                  &kb, xb, hb, vb);
  }
  G.gh[s] += hb;
  G.gkc[s] += (double)kb.a;
  for (int q = 0; q < 3; ++q) {
    G.gkc[(1 + q) * n + s] += (double)kb.b[q];
    G.gkc[(4 + q) * n + s] += (double)kb.c[q];
  }
  for (int q = 0; q < 9; ++q) G.gkc[(7 + q) * n + s] += (double)kb.M[q];
  for (int t = 0; t < ng + ns; ++t) {
    const uint32_t e = nbr_entry(S, nb, t, ebuf);
    const uint32_t j = e >> kCodeBits;
    const R4<R> pj = S.pos(j);
    R x[3];
    pair_x(S, s, pi, pj, e, x);
    const R r2 = dot3b(x, x);
    if (!(r2 * (pj.w * pj.w) < R(1))) continue;
    const R rinv = Sc<R>::rsqrt(r2);
    const R r = r2 * rinv;
    const R4<R> vj = S.vel(j);
    const R vij[3] = {vi.x - vj.x, vi.y - vj.y, vi.z - vj.z};
    KC<R> kj;
    load_kc4(S, j, kj);
    R gvbj[9], Numbj, Denbj;
    load_gvc(G, j, gvbj, Numbj, Denbj);
    KEval<R> ej;
    kernel_eval<R, K>(r, rinv, pj.w, ej);
    density_rev_adj<R, double>(kj, x, r, rinv, ej, mi, vi.w, vij, Numbj, Denbj, gvbj, xb, Vb,
                               vb);
  }
  for (int a = 0; a < 3; ++a) {
    G.gx[a * n + s] += xb[a];
    G.gv[a * n + s] += vb[a];
  }
  G.gV[s] += Vb;
}

// --------------------------------------------------------------------- B4 --
// Raw moment sums of particle s (the forward's k_moments accumulation).
template <class R, int K>
__device__ inline void moments_raw(const State<R>& S, int64_t s, double raw[40]) {
  const R4<R> pi = S.pos(s);
  const R hinv = pi.w;
  R acc[40];
  for (int t = 0; t < 40; ++t) acc[t] = R(0);
  R W0, dW0;
  kernel_self<R, K>(hinv, W0, dW0);
  acc[0] = S.vel(s).w * W0;
  const NbrRef nb = nbr_ref(S, s);
  uint4 ebuf;
  const int ng = nb.ng;
  for (int k = 0; k < ng; ++k) {
    const uint32_t e = gather_entry(S, nb, k, ebuf);
    const uint32_t j = e >> kCodeBits;
    const R Vj = S.vel(j).w;
    R x[3];
    pair_x(S, s, pi, S.pos(j), e, x);
    const R r2 = dot3b(x, x);
    const R rinv = Sc<R>::rsqrt(r2);
    R w, dw;
    Shape<K>::eval(r2 * rinv * hinv, w, dw);
    const R C3 = R(Shape<K>::C) * hinv * hinv * hinv;
    const R VW = Vj * C3 * w;
    const R fg = Vj * C3 * hinv * dw * rinv;
    const R p6[6] = {x[0] * x[0], x[0] * x[1], x[0] * x[2], x[1] * x[1], x[1] * x[2], x[2] * x[2]};
    acc[0] += VW;
    for (int a = 0; a < 3; ++a) acc[1 + a] += x[a] * VW;
    for (int q = 0; q < 6; ++q) acc[4 + q] += p6[q] * VW;
    for (int g = 0; g < 3; ++g) {
      const R Vg = fg * x[g];
      acc[10 + g] += Vg;
      for (int a = 0; a < 3; ++a) acc[13 + g * 3 + a] += x[a] * Vg;
      for (int q = 0; q < 6; ++q) acc[22 + g * 6 + q] += p6[q] * Vg;
    }
  }
  for (int t = 0; t < 40; ++t) raw[t] = (double)acc[t];
}

// At least three waves per SIMD (168 VGPRs, a few spilled): measured at
// clumps256 10.5 -> 8.7 ms against the two the register count gives otherwise.
template <class R, int K>
__global__ void __launch_bounds__(kBlock, 3) k_bwd_corr(State<R> S, AdjState<R> G) {
  const int64_t s = particle_id();
  if (s >= S.n) return;
  const int64_t n = S.n;
  double raw[40];
  if (S.mom) {
    for (int t = 0; t < 40; ++t) raw[t] = (double)S.mom[t * n + s];
  } else {
    moments_raw<R, K>(S, s, raw);
  }
  double kcb[16];
  for (int t = 0; t < 16; ++t) kcb[t] = G.gkc[t * n + s];
  double out[40];
  corr_solve_adj(raw, kcb, out, SingularTol<R>::v);
#pragma unroll
  for (int t = 0; t < 10; ++t) {
    R4<R> q;
    q.x = (R)out[4 * t];
    q.y = (R)out[4 * t + 1];
    q.z = (R)out[4 * t + 2];
    q.w = (R)out[4 * t + 3];
    G.mom4[10 * s + t] = q;
  }
}

// ------------------------------------------------------------------ B5+B6 --
template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_bwd_moments(State<R> S, AdjState<R> G, int h_mode) {
  const int64_t s = particle_id();
  if (s >= S.n) return;
  const int64_t n = S.n;
  const R4<R> pi = S.pos(s);
  const R Vi = S.vel(s).w;
  const R mi = S.mass[s];
  R mb[40];
  load_mom(G, s, mb);
  R W0, dW0;
  kernel_self<R, K>(pi.w, W0, dW0);
  double Vb = (double)(mb[0] * W0), hb = (double)(mb[0] * Vi * dW0);
  double sh = (double)(mi * dW0);
  double xb[3] = {0, 0, 0};
  const NbrRef nb = nbr_ref(S, s);
  uint4 ebuf;
  const int ng = nb.ng, ns = nb.ns;
  // Own moment sums first (gather part), then the particle's share in its
  // neighbours' sums: the two sets of 40 moment adjoints are never live
  // together.
  for (int t = 0; t < ng; ++t) {
    const uint32_t e = gather_entry(S, nb, t, ebuf);
    const uint32_t j = e >> kCodeBits;
    const R4<R> pj = S.pos(j);
    R x[3];
    pair_x(S, s, pi, pj, e, x);
    const R r2 = dot3b(x, x);
    const R rinv = Sc<R>::rsqrt(r2);
    const R r = r2 * rinv;
    KEval<R> ev;
    kernel_eval<R, K>(r, rinv, pi.w, ev);
    R gx[3], gh;
    mom_pair_adj<R>(mb, x, rinv, ev, gx, gh);
    const R Vj = S.vel(j).w;
    for (int a = 0; a < 3; ++a) xb[a] += (double)(Vj * gx[a]);
    hb += (double)(Vj * gh);
    sh += (double)(S.mass[j] * ev.dWdh);
  }
  for (int t = 0; t < ng + ns; ++t) {
    const uint32_t e = nbr_entry(S, nb, t, ebuf);
    const uint32_t j = e >> kCodeBits;
    const R4<R> pj = S.pos(j);
    R x[3];
    pair_x(S, s, pi, pj, e, x);
    const R r2 = dot3b(x, x);
    if (!(r2 * (pj.w * pj.w) < R(1))) continue;
    const R rinv = Sc<R>::rsqrt(r2);
    const R r = r2 * rinv;
    R mbj[40];
    load_mom(G, j, mbj);
    KEval<R> ej;
    kernel_eval<R, K>(r, rinv, pj.w, ej);
    const R xm[3] = {-x[0], -x[1], -x[2]};
    R gx[3], gh;
    const R l = mom_pair_adj<R>(mbj, xm, rinv, ej, gx, gh);
    Vb += (double)l;
    for (int a = 0; a < 3; ++a) xb[a] -= (double)(Vi * gx[a]);
  }
  for (int a = 0; a < 3; ++a) G.gx[a * n + s] += xb[a];
  const double hbt = G.gh[s] + hb;
  const double Vbt = G.gV[s] + Vb;
  // volume and smoothing-length coefficient (V = m / S, S = sum m_j W(r, h))
  const double V = (double)Vi, m = (double)mi;
  const double Ssum = m / V;
  double kappa = -Vbt * V / Ssum;
  if (h_mode == 1) {
    const double h = (double)S.hbuf[s];
    const double dVdh = -V * sh / Ssum;
    const double htot = hbt + Vbt * dVdh;
    const double dFdh = 3.0 * h * h * Ssum / m + h * h * h * sh / m;
    kappa += -htot * (h * h * h / m) / dFdh;
  }
  G.kap[s] = (R)kappa;
}

// --------------------------------------------------------------------- B7 --
template <class R, int K>
__global__ void __launch_bounds__(kBlock) k_bwd_volume(State<R> S, AdjState<R> G) {
  const int64_t s = particle_id();
  if (s >= S.n) return;
  const int64_t n = S.n;
  const R4<R> pi = S.pos(s);
  const R mi = S.mass[s];
  const R ki = G.kap[s];
  double xb[3] = {0, 0, 0};
  const NbrRef nb = nbr_ref(S, s);
  uint4 ebuf;
  const int ng = nb.ng, ns = nb.ns;
  for (int t = 0; t < ng + ns; ++t) {
    const uint32_t e = nbr_entry(S, nb, t, ebuf);
    const uint32_t j = e >> kCodeBits;
    const R4<R> pj = S.pos(j);
    R x[3];
    pair_x(S, s, pi, pj, e, x);
    const R r2 = dot3b(x, x);
    const R rinv = Sc<R>::rsqrt(r2);
    const R r = r2 * rinv;
    R c = R(0);
    if (t < ng) {
      KEval<R> ev;
      kernel_eval<R, K>(r, rinv, pi.w, ev);
      c += ki * S.mass[j] * ev.f;
    }
    if (r2 * (pj.w * pj.w) < R(1)) {
      KEval<R> ej;
      kernel_eval<R, K>(r, rinv, pj.w, ej);
      c += G.kap[j] * mi * ej.f;
    }
    for (int a = 0; a < 3; ++a) xb[a] += (double)(c * x[a]);
  }
  for (int a = 0; a < 3; ++a) G.gx[a * n + s] += xb[a];
}

// ----------------------------------------------------------------- finish --
template <class R>
__global__ void __launch_bounds__(kBlock) k_bwd_unpermute(State<R> S, AdjState<R> G,
                                                          double* __restrict__ g_x,
                                                          double* __restrict__ g_v,
                                                          double* __restrict__ g_u) {
  const int64_t s = particle_id();
  if (s >= S.n) return;
  const int64_t n = S.n;
  const uint32_t p = S.perm[s];
  for (int a = 0; a < 3; ++a) {
    g_x[a * n + p] = G.gx[a * n + s];
    g_v[a * n + p] = G.gv[a * n + s];
  }
  g_u[p] = G.gu[s];
}

// Deterministic sum of the per-block alpha, beta partials: one block,
// fixed strided order, fixed tree.
__global__ void __launch_bounds__(kBlock) k_bwd_reduce_ab(const double* __restrict__ part,
                                                          int64_t nb, double* __restrict__ out) {
  __shared__ double sa[kBlock], sb[kBlock];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < nb; i += kBlock) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sa[0];
    out[1] = sb[0];
  }
}

__global__ void __launch_bounds__(kBlock) k_zero_f64(double* __restrict__ a, int64_t na) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < na) a[i] = 0.0;
}

}  // namespace

void launch_zero_f64(double* a, int64_t na, hipStream_t s) {
  if (na > 0) hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(na)), dim3(kBlock), 0, s, a, na);
}

#define CRK_DISPATCH_KB(kernel, KFN, ...)                                                   \
  do {                                                                                      \
    if ((kernel) == 0)                                                                      \
      hipLaunchKernelGGL((KFN<R, 0>), dim3(grid_for(S.n)), dim3(kBlock), 0, s, __VA_ARGS__); \
    else                                                                                    \
      hipLaunchKernelGGL((KFN<R, 1>), dim3(grid_for(S.n)), dim3(kBlock), 0, s, __VA_ARGS__); \
  } while (0)

template <class R>
void launch_bwd_prep(const State<R>& S, const AdjState<R>& G, hipStream_t s) {
  hipLaunchKernelGGL(k_bwd_prep<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S, G);
}
template <class R>
void launch_bwd_force(const State<R>& S, const AdjState<R>& G, int kernel, hipStream_t s) {
  CRK_DISPATCH_KB(kernel, k_bwd_force, S, G);
}
template <class R>
void launch_bwd_density(const State<R>& S, const AdjState<R>& G, int kernel, hipStream_t s) {
  CRK_DISPATCH_KB(kernel, k_bwd_density, S, G);
}
template <class R>
void launch_bwd_corr(const State<R>& S, const AdjState<R>& G, int kernel, hipStream_t s) {
  CRK_DISPATCH_KB(kernel, k_bwd_corr, S, G);
}
template <class R>
void launch_bwd_moments(const State<R>& S, const AdjState<R>& G, int kernel, int h_mode,
                        hipStream_t s) {
  CRK_DISPATCH_KB(kernel, k_bwd_moments, S, G, h_mode);
}
template <class R>
void launch_bwd_volume(const State<R>& S, const AdjState<R>& G, int kernel, hipStream_t s) {
  CRK_DISPATCH_KB(kernel, k_bwd_volume, S, G);
}
template <class R>
void launch_bwd_finish(const State<R>& S, const AdjState<R>& G, double* g_x, double* g_v,
                       double* g_u, double* g_ab, hipStream_t s) {
  hipLaunchKernelGGL(k_bwd_unpermute<R>, dim3(grid_for(S.n)), dim3(kBlock), 0, s, S, G, g_x, g_v,
                     g_u);
  hipLaunchKernelGGL(k_bwd_reduce_ab, dim3(1), dim3(kBlock), 0, s, (const double*)G.gab,
                     (int64_t)grid_for(S.n), g_ab);
}

#define CRK_INSTANTIATE_BWD(R)                                                                 \
  template void launch_bwd_prep<R>(const State<R>&, const AdjState<R>&, hipStream_t);          \
  template void launch_bwd_force<R>(const State<R>&, const AdjState<R>&, int, hipStream_t);    \
  template void launch_bwd_density<R>(const State<R>&, const AdjState<R>&, int, hipStream_t);  \
  template void launch_bwd_corr<R>(const State<R>&, const AdjState<R>&, int, hipStream_t);     \
  template void launch_bwd_moments<R>(const State<R>&, const AdjState<R>&, int, int,           \
                                      hipStream_t);                                            \
  template void launch_bwd_volume<R>(const State<R>&, const AdjState<R>&, int, hipStream_t);   \
  template void launch_bwd_finish<R>(const State<R>&, const AdjState<R>&, double*, double*,    \
                                     double*, double*, hipStream_t);

CRK_INSTANTIATE_BWD(float)
CRK_INSTANTIATE_BWD(double)

}  // namespace crk
