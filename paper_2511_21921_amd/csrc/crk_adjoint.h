// Reverse-mode (adjoint) building blocks of the CRKSPH passes.
//
// The loss is L = sum_i gA_i . a_i + sum_i gU_i du_i/dt. Every adjoint pass
// is written in gather form: a particle recomputes each pair it belongs to
// and accumulates only the derivatives with respect to its own quantities
// (and, for its reverse role in a neighbour's gather sum, the derivatives
// with respect to the quantities it lends that neighbour). No float atomics
// are used, so the gradients are deterministic.
//
// All functions are __host__ __device__ templates: the pair arithmetic type
// R, the accumulator type A (double).
#pragma once

#include "crk_device.h"

namespace crk {

// --------------------------------------------------------- kernel values ----
// For separation r and 1/h: W, f = (dW/dr)/r (so grad W = f x), fr = df/dr,
// and the h derivatives dW/dh, df/dh. Needs w'' of the shape.

template <int K> struct Shape2;
template <> struct Shape2<0> {
  template <class R> __host__ __device__ static inline void eval(R q, R& w, R& dw, R& d2w) {
    R t = R(1) - q;
    bool in = q <= R(0.5);
    bool sup = q < R(1);
    w = sup ? (in ? R(1) + q * q * (R(6) * q - R(6)) : R(2) * t * t * t) : R(0);
    dw = sup ? (in ? q * (R(18) * q - R(12)) : R(-6) * t * t) : R(0);
    d2w = sup ? (in ? R(36) * q - R(12) : R(12) * t) : R(0);
  }
};
template <> struct Shape2<1> {
  template <class R> __host__ __device__ static inline void eval(R q, R& w, R& dw, R& d2w) {
    R t = R(1) - q;
    t = t > R(0) ? t : R(0);
    R t2 = t * t, t4 = t2 * t2;
    R t5 = t4 * t;
    w = t5 * t * (R(1) + R(6) * q + R(35.0 / 3.0) * q * q);
    dw = R(-56.0 / 3.0) * q * (R(1) + R(5) * q) * t5;
    d2w = R(-56.0 / 3.0) * t4 * (R(1) + R(4) * q - R(35) * q * q);
  }
};

template <class R>
struct KEval {
  R W, f, fr, dWdh, dfdh;
};

template <class R, int K>
__host__ __device__ inline void kernel_eval(R r, R rinv, R hinv, KEval<R>& e) {
  const R q = r * hinv;
  R w, dw, d2w;
  Shape2<K>::eval(q, w, dw, d2w);
  const R C3 = R(Shape<K>::C) * hinv * hinv * hinv;
  const R C4 = C3 * hinv;
  e.W = C3 * w;
  e.f = C4 * dw * rinv;
  e.fr = C4 * (d2w * hinv - dw * rinv) * rinv;
  e.dWdh = -C4 * (R(3) * w + q * dw);
  e.dfdh = -C4 * hinv * rinv * (R(4) * dw + q * d2w);
}

// Self term W(0, h) and its h derivative.
template <class R, int K>
__host__ __device__ inline void kernel_self(R hinv, R& W0, R& dW0dh) {
  const R C3 = R(Shape<K>::C) * hinv * hinv * hinv;
  W0 = C3 * R(Shape<K>::w0);
  dW0dh = R(-3) * W0 * hinv;
}

// ------------------------------------------- corrected kernel and adjoint --
// Forward: s = a + b.x, W^R = s W, g = W (c + M x) + s f x.
template <class R>
__host__ __device__ inline void corr_fwd(const KC<R>& k, const R x[3], const KEval<R>& e, R& WR,
                                         R g[3]) {
  const R s = k.a + k.b[0] * x[0] + k.b[1] * x[1] + k.b[2] * x[2];
  WR = s * e.W;
  for (int gg = 0; gg < 3; ++gg) {
    const R t = k.c[gg] + k.M[gg * 3] * x[0] + k.M[gg * 3 + 1] * x[1] + k.M[gg * 3 + 2] * x[2];
    g[gg] = e.W * t + s * e.f * x[gg];
  }
}

// Adjoint accumulators of the 16 packed coefficients (a, b, c, M).
template <class A>
struct KCBar {
  A a, b[3], c[3], M[9];
  __host__ __device__ void zero() {
    a = 0;
    for (int t = 0; t < 3; ++t) b[t] = c[t] = 0;
    for (int t = 0; t < 9; ++t) M[t] = 0;
  }
};

// Given WRbar and gbar (adjoints of W^R and of the corrected gradient g at
// separation x), accumulate into kcb (if non-null), xb and hb.
template <class R, class A, class AK = A>
__host__ __device__ inline void corr_adj(const KC<R>& k, const R x[3], R r, R rinv,
                                         const KEval<R>& e, R WRbar, const R gbar[3],
                                         KCBar<AK>* kcb, A xb[3], A& hb) {
  const R s = k.a + k.b[0] * x[0] + k.b[1] * x[1] + k.b[2] * x[2];
  R t[3];
  for (int gg = 0; gg < 3; ++gg)
    t[gg] = k.c[gg] + k.M[gg * 3] * x[0] + k.M[gg * 3 + 1] * x[1] + k.M[gg * 3 + 2] * x[2];
  const R gx = gbar[0] * x[0] + gbar[1] * x[1] + gbar[2] * x[2];
  const R Wbar = gbar[0] * t[0] + gbar[1] * t[1] + gbar[2] * t[2] + WRbar * s;
  const R sbar = e.f * gx + WRbar * e.W;
  const R fbar = s * gx;
  // t = c + M x
  R tb[3] = {e.W * gbar[0], e.W * gbar[1], e.W * gbar[2]};
  if (kcb) {
    kcb->a += (AK)sbar;
    for (int a = 0; a < 3; ++a) {
      kcb->b[a] += (AK)(sbar * x[a]);
      kcb->c[a] += (AK)tb[a];
      for (int gg = 0; gg < 3; ++gg) kcb->M[gg * 3 + a] += (AK)(tb[gg] * x[a]);
    }
  }
  // x: from M x, from s = a + b.x, from f x, and from r in W and f
  const R radial = Wbar * e.f + fbar * e.fr * rinv;
  for (int a = 0; a < 3; ++a) {
    R v = k.M[a] * tb[0] + k.M[3 + a] * tb[1] + k.M[6 + a] * tb[2];
    v += sbar * k.b[a] + e.f * s * gbar[a] + radial * x[a];
    xb[a] += (A)v;
  }
  hb += (A)(Wbar * e.dWdh + fbar * e.dfdh);
}

// ------------------------------------------------------ viscosity pieces ----

template <class R>
struct AVFwd {
  R gix[3], gjx[3], nn, dd, s2, phi, vp[3], vpx, Di, Dj, iDi, iDj, mui, muj;
  bool phi_active, mui_on, muj_on;
};

// Velocity jump, limiter and mu_k of the pair (i, j) at x = x_ij.
template <class R>
__host__ __device__ inline void av_fwd(const R gvi[9], const R gvj[9], const R vij[3],
                                       const R x[3], R r2, R hi, R hj, R eps2, AVFwd<R>& o) {
  for (int a = 0; a < 3; ++a) {
    o.gix[a] = gvi[a * 3] * x[0] + gvi[a * 3 + 1] * x[1] + gvi[a * 3 + 2] * x[2];
    o.gjx[a] = gvj[a * 3] * x[0] + gvj[a * 3 + 1] * x[1] + gvj[a * 3 + 2] * x[2];
  }
  o.nn = x[0] * o.gix[0] + x[1] * o.gix[1] + x[2] * o.gix[2];
  o.dd = x[0] * o.gjx[0] + x[1] * o.gjx[1] + x[2] * o.gjx[2];
  const R sum = o.nn + o.dd;
  o.s2 = sum * sum;
  o.phi = R(0);
  o.phi_active = false;
  if (o.s2 > R(0)) {
    const R p = Sc<R>::div(R(4) * o.nn * o.dd, o.s2);
    o.phi = p < R(0) ? R(0) : (p > R(1) ? R(1) : p);
    o.phi_active = p > R(0) && p < R(1);
  }
  const R hp = R(0.5) * o.phi;
  for (int a = 0; a < 3; ++a) o.vp[a] = vij[a] - hp * (o.gix[a] + o.gjx[a]);
  o.vpx = o.vp[0] * x[0] + o.vp[1] * x[1] + o.vp[2] * x[2];
  o.Di = r2 + eps2 * hi * hi;
  o.Dj = r2 + eps2 * hj * hj;
  o.iDi = Sc<R>::rcp(o.Di);
  o.iDj = Sc<R>::rcp(o.Dj);
  const R mi = o.vpx * hi * o.iDi, mj = o.vpx * hj * o.iDj;
  o.mui_on = mi < R(0);
  o.muj_on = mj < R(0);
  o.mui = o.mui_on ? mi : R(0);
  o.muj = o.muj_on ? mj : R(0);
}

// ------------------------------------------------------ force pair, adjoint --
// Everything particle i needs about itself and neighbour j for one pair.
template <class R>
struct PairSide {
  KC<R> kc;      // packed corrections (plain when the pair is relaxed)
  R hinv, h, V, rho, P, c;
  R v[3], gv[9];
  R wam[3], wum;  // loss weights over the mass: w_a / m and w_u / (2 m)
};

template <class A, class AK = A>
struct ForceBar {  // i-side adjoints of one force pass
  A x[3], v[3], h, V, rho, P, c, alpha, beta;
  AK gv[9];      // sums feeding the density adjoint's coefficients
  KCBar<AK> kc;  // sums feeding the correction adjoint
  __host__ __device__ void zero() {
    for (int t = 0; t < 3; ++t) x[t] = v[t] = 0;
    h = V = rho = P = c = alpha = beta = 0;
    for (int t = 0; t < 9; ++t) gv[t] = 0;
    kc.zero();
  }
};

// Adjoint of L_pair = F_ij . w_ij (w_ij = gA_i/m_i - gA_j/m_j - v_ij lambda,
// lambda = gU_i/(2 m_i) + gU_j/(2 m_j)), which is the pair's whole share of
// L. Accumulates the derivatives with respect to i's quantities; the pair
// is seen from j's side by j's own call. corrected = false for a relaxed pair.
// The pair's several terms in x, v and h are summed in the working precision
// and enter the accumulators once per pair.
template <class R, class A, class AK, int K>
__host__ __device__ inline void force_pair_adj(const PairSide<R>& I, const PairSide<R>& J,
                                               const R x[3], R alpha, R beta, R eps2,
                                               bool corrected, ForceBar<A, AK>& ob) {
  const R r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  const R rinv = Sc<R>::rsqrt(r2);
  const R r = r2 * rinv;
  const R xm[3] = {-x[0], -x[1], -x[2]};
  KEval<R> ei, ej;
  kernel_eval<R, K>(r, rinv, I.hinv, ei);
  kernel_eval<R, K>(r, rinv, J.hinv, ej);
  R WRi, Gi[3], WRj, Gj[3];
  corr_fwd(I.kc, x, ei, WRi, Gi);
  corr_fwd(J.kc, xm, ej, WRj, Gj);
  const R G[3] = {Gi[0] - Gj[0], Gi[1] - Gj[1], Gi[2] - Gj[2]};
  const R vij[3] = {I.v[0] - J.v[0], I.v[1] - J.v[1], I.v[2] - J.v[2]};
  AVFwd<R> av;
  av_fwd(I.gv, J.gv, vij, x, r2, I.h, J.h, eps2, av);
  const R Qi = I.rho * (-alpha * I.c * av.mui + beta * av.mui * av.mui);
  const R Qj = J.rho * (-alpha * J.c * av.muj + beta * av.muj * av.muj);
  const R Pi = I.P + J.P + Qi + Qj;
  const R sig = R(-0.5) * I.V * J.V * Pi;
  const R lam = I.wum + J.wum;
  R w[3];
  for (int a = 0; a < 3; ++a) w[a] = I.wam[a] - J.wam[a] - vij[a] * lam;
  // L = sig G.w
  const R gsig = G[0] * w[0] + G[1] * w[1] + G[2] * w[2];
  R vb[3];
  for (int a = 0; a < 3; ++a) vb[a] = -lam * sig * G[a];  // explicit v_ij in w
  ob.V += (A)(gsig * R(-0.5) * J.V * Pi);
  const R Pibar = gsig * R(-0.5) * I.V * J.V;
  ob.P += (A)Pibar;
  // Q_i, Q_j
  R mubar_i = R(0), mubar_j = R(0);
  if (av.mui_on) {
    ob.rho += (A)(Pibar * (-alpha * I.c * av.mui + beta * av.mui * av.mui));
    ob.c += (A)(Pibar * (-alpha * I.rho * av.mui));
    ob.alpha += (A)(Pibar * (-I.rho * I.c * av.mui));
    ob.beta += (A)(Pibar * I.rho * av.mui * av.mui);
    mubar_i = Pibar * I.rho * (-alpha * I.c + R(2) * beta * av.mui);
  }
  if (av.muj_on) mubar_j = Pibar * J.rho * (-alpha * J.c + R(2) * beta * av.muj);
  // mu_k = vpx h_k / D_k, D_k = r^2 + eps2 h_k^2
  const R vpxbar = mubar_i * I.h * av.iDi + mubar_j * J.h * av.iDj;
  const R r2bar = -(mubar_i * av.vpx * I.h * av.iDi * av.iDi +
                    mubar_j * av.vpx * J.h * av.iDj * av.iDj);
  // d mu_i / d h_i, with h = 1/hinv
  R hb = mubar_i * av.vpx * (r2 - eps2 * I.h * I.h) * av.iDi * av.iDi;
  R xb[3];
  for (int a = 0; a < 3; ++a) xb[a] = R(2) * r2bar * x[a] + vpxbar * av.vp[a];
  R vpb[3] = {vpxbar * x[0], vpxbar * x[1], vpxbar * x[2]};
  for (int a = 0; a < 3; ++a) ob.v[a] += (A)(vb[a] + vpb[a]);
  // vp = v_ij - phi/2 (gix + gjx)
  const R phibar = R(-0.5) * (vpb[0] * (av.gix[0] + av.gjx[0]) + vpb[1] * (av.gix[1] + av.gjx[1]) +
                              vpb[2] * (av.gix[2] + av.gjx[2]));
  R gixb[3], gjxb[3];
  for (int a = 0; a < 3; ++a) gixb[a] = gjxb[a] = R(-0.5) * av.phi * vpb[a];
  if (av.phi_active) {
    const R s = av.nn + av.dd;
    const R is3 = Sc<R>::rcp(s * s * s);
    const R nnb = phibar * R(4) * av.dd * (av.dd - av.nn) * is3;
    const R ddb = phibar * R(4) * av.nn * (av.nn - av.dd) * is3;
    for (int a = 0; a < 3; ++a) {
      xb[a] += nnb * av.gix[a] + ddb * av.gjx[a];
      gixb[a] += nnb * x[a];
      gjxb[a] += ddb * x[a];
    }
  }
  // gix = grad v_i x, gjx = grad v_j x
  for (int a = 0; a < 3; ++a)
    for (int g = 0; g < 3; ++g) {
      ob.gv[a * 3 + g] += (AK)(gixb[a] * x[g]);
      xb[g] += gixb[a] * I.gv[a * 3 + g] + gjxb[a] * J.gv[a * 3 + g];
    }
  // G = Gi(x) - Gj(-x); Gbar = sig w
  const R Gb[3] = {sig * w[0], sig * w[1], sig * w[2]};
  corr_adj<R, R, AK>(I.kc, x, r, rinv, ei, R(0), Gb, corrected ? &ob.kc : nullptr, xb, hb);
  // j side: d/dx_i of -Gj(-x) = +dGj/dx_ji . Gbar
  R xj[3] = {0, 0, 0};
  R hj_dummy = 0;
  corr_adj<R, R, AK>(J.kc, xm, r, rinv, ej, R(0), Gb, (KCBar<AK>*)nullptr, xj, hj_dummy);
  for (int a = 0; a < 3; ++a) ob.x[a] += (A)(xb[a] + xj[a]);
  ob.h += (A)hb;
}


// ------------------------------------------------ density / grad v adjoint --
// Particle i's sums: Num_i += m_j V_j W^R_ij, Den_i += V_j^2 W^R_ij,
// gv_i[a][g] -= V_j v_ij[a] g_ij[g], with rho = Num / Den, so
// Numb = rhob / Den and Denb = -rhob rho / Den.

// Own term (i gathers j at x = x_ij with i's corrections and h_i).
template <class R, class A, class AK = A>
__host__ __device__ inline void density_own_adj(const KC<R>& ki, const R x[3], R r, R rinv,
                                                const KEval<R>& e, R mj, R Vj, const R vij[3],
                                                R Numb, R Denb, const R gvb[9], KCBar<AK>* kcb,
                                                A xb[3], A& hb, A vb[3]) {
  R WR, g[3];
  corr_fwd(ki, x, e, WR, g);
  const R WRb = Numb * mj * Vj + Denb * Vj * Vj;
  R gb[3];
  for (int gg = 0; gg < 3; ++gg)
    gb[gg] = -Vj * (gvb[gg] * vij[0] + gvb[3 + gg] * vij[1] + gvb[6 + gg] * vij[2]);
  for (int a = 0; a < 3; ++a)
    vb[a] += (A)(-Vj * (gvb[a * 3] * g[0] + gvb[a * 3 + 1] * g[1] + gvb[a * 3 + 2] * g[2]));
  corr_adj<R, A, AK>(ki, x, r, rinv, e, WRb, gb, kcb, xb, hb);
}

// Reverse term: neighbour j gathers i at x_ji = -x_ij with j's corrections
// and h_j. Accumulates i's volume, velocity and position adjoints.
template <class R, class A>
__host__ __device__ inline void density_rev_adj(const KC<R>& kj, const R x[3], R r, R rinv,
                                                const KEval<R>& ej, R mi, R Vi, const R vij[3],
                                                R Numbj, R Denbj, const R gvbj[9], A xb[3],
                                                A& Vb, A vb[3]) {
  const R xji[3] = {-x[0], -x[1], -x[2]};
  const R vji[3] = {-vij[0], -vij[1], -vij[2]};
  R WR, g[3];
  corr_fwd(kj, xji, ej, WR, g);
  R gvg = R(0);  // sum_ag gvb_j[a][g] v_ji[a] g[g]
  R gb[3];
  for (int gg = 0; gg < 3; ++gg) {
    const R t = gvbj[gg] * vji[0] + gvbj[3 + gg] * vji[1] + gvbj[6 + gg] * vji[2];
    gvg += t * g[gg];
    gb[gg] = -Vi * t;
  }
  Vb += (A)(Numbj * mi * WR + Denbj * R(2) * Vi * WR - gvg);
  for (int a = 0; a < 3; ++a)
    vb[a] += (A)(Vi * (gvbj[a * 3] * g[0] + gvbj[a * 3 + 1] * g[1] + gvbj[a * 3 + 2] * g[2]));
  const R WRb = Numbj * mi * Vi + Denbj * Vi * Vi;
  A xt[3] = {0, 0, 0};
  A hdummy = 0;
  corr_adj<R, A>(kj, xji, r, rinv, ej, WRb, gb, (KCBar<A>*)nullptr, xt, hdummy);
  for (int a = 0; a < 3; ++a) xb[a] -= xt[a];
}

// Self term of i's density sums: m_i V_i A_i W(0), V_i^2 A_i W(0).
template <class R, class A, class AK = A>
__host__ __device__ inline void density_self_adj(R a, R mi, R Vi, R W0, R dW0dh, R Numb, R Denb,
                                                 KCBar<AK>* kcb, A& Vb, A& hb) {
  const R w = Numb * mi * Vi + Denb * Vi * Vi;
  Vb += (A)((Numb * mi + Denb * R(2) * Vi) * a * W0);
  if (kcb) kcb->a += (AK)(w * W0);
  hb += (A)(w * a * dW0dh);
}

// --------------------------------------------------- correction adjoint ----
// Packed-coefficient adjoint (a, b, c, M) -> (A, B, dA, dB) adjoint, then
// through the FP64 moment solve to the 40 stored moment sums
// (m0, m1[3], m2 sym[6], dm0[3], X1[9], X2 sym[18]).

struct MomBar {
  double m0, m1[3], m2[6], dm0[3], X1[9], X2[18];
};

__host__ __device__ inline constexpr int sym6h(int a, int b) {
  return a <= b ? (a == 0 ? b : (a == 1 ? 2 + b : 5)) : (b == 0 ? a : (b == 1 ? 2 + a : 5));
}

// Forward moments in full (expanded) form, FP64.
struct MomFull {
  double m0, m1[3], m2[9], dm0[3], dm1[9], dm2[27];
};

__host__ __device__ inline void mom_expand(const double raw[40], MomFull& D) {
  D.m0 = raw[0];
  for (int a = 0; a < 3; ++a) {
    D.m1[a] = raw[1 + a];
    D.dm0[a] = raw[10 + a];
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) D.m2[a * 3 + b] = raw[4 + sym6h(a, b)];
  for (int g = 0; g < 3; ++g)
    for (int a = 0; a < 3; ++a) {
      D.dm1[g * 3 + a] = raw[13 + g * 3 + a] + (a == g ? D.m0 : 0.0);
      for (int b = 0; b < 3; ++b)
        D.dm2[(g * 3 + a) * 3 + b] =
            raw[22 + g * 6 + sym6h(a, b)] + (a == g ? D.m1[b] : 0.0) + (b == g ? D.m1[a] : 0.0);
    }
}

// Returns false (and zero adjoints) for a singular second moment (tol as the
// forward's, SingularTol of the working precision).
__host__ __device__ inline bool corr_solve_adj(const double raw[40], const double kcbar[16],
                                               double out[40], double tol) {
  for (int t = 0; t < 40; ++t) out[t] = 0.0;
  MomFull D;
  mom_expand(raw, D);
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
  if (!(fabs(det) > tol * tr * tr * tr)) return false;
  double inv[9];
  for (int t = 0; t < 9; ++t) inv[t] = cof[t] / det;
  // forward
  double B[3], dB[9], dA[3], rhs[9], tg[3];
  for (int a = 0; a < 3; ++a)
    B[a] = -(inv[a * 3] * D.m1[0] + inv[a * 3 + 1] * D.m1[1] + inv[a * 3 + 2] * D.m1[2]);
  const double A = 1.0 / (D.m0 + B[0] * D.m1[0] + B[1] * D.m1[1] + B[2] * D.m1[2]);
  for (int g = 0; g < 3; ++g) {
    for (int b = 0; b < 3; ++b) {
      rhs[g * 3 + b] = D.dm1[g * 3 + b];
      for (int e = 0; e < 3; ++e) rhs[g * 3 + b] += D.dm2[(g * 3 + b) * 3 + e] * B[e];
    }
    for (int a = 0; a < 3; ++a)
      dB[g * 3 + a] = -(inv[a * 3] * rhs[g * 3] + inv[a * 3 + 1] * rhs[g * 3 + 1] +
                        inv[a * 3 + 2] * rhs[g * 3 + 2]);
    double t = D.dm0[g];
    for (int a = 0; a < 3; ++a) t += dB[g * 3 + a] * D.m1[a] + B[a] * D.dm1[g * 3 + a];
    tg[g] = t;
    dA[g] = -(A * A) * t;
  }
  // packed adjoint -> (A, B, dA, dB) adjoint.
  // a = A, b = A B, c_g = dA_g + A B_g, M_ga = dA_g B_a + A dB_ga
  const double* ab = kcbar;          // a
  const double* bb = kcbar + 1;      // b[3]
  const double* cb = kcbar + 4;      // c[3]
  const double* Mb = kcbar + 7;      // M[9]
  double Ab = ab[0], Bb[3], dAb[3], dBb[9];
  for (int t = 0; t < 3; ++t) {
    Ab += bb[t] * B[t] + cb[t] * B[t];
    Bb[t] = bb[t] * A + cb[t] * A;
    dAb[t] = cb[t];
  }
  for (int g = 0; g < 3; ++g)
    for (int a = 0; a < 3; ++a) {
      Ab += Mb[g * 3 + a] * dB[g * 3 + a];
      Bb[a] += Mb[g * 3 + a] * dA[g];
      dAb[g] += Mb[g * 3 + a] * B[a];
      dBb[g * 3 + a] = Mb[g * 3 + a] * A;
    }
  // reverse of the solve
  MomFull Db;
  Db.m0 = 0;
  for (int t = 0; t < 3; ++t) Db.m1[t] = Db.dm0[t] = 0;
  for (int t = 0; t < 9; ++t) Db.m2[t] = Db.dm1[t] = 0;
  for (int t = 0; t < 27; ++t) Db.dm2[t] = 0;
  double invb[9];
  for (int t = 0; t < 9; ++t) invb[t] = 0;
  for (int g = 0; g < 3; ++g) {
    // dA_g = -A^2 t_g
    const double tb = -(A * A) * dAb[g];
    Ab += -2.0 * A * tg[g] * dAb[g];
    Db.dm0[g] += tb;
    for (int a = 0; a < 3; ++a) {
      dBb[g * 3 + a] += tb * D.m1[a];
      Db.m1[a] += tb * dB[g * 3 + a];
      Bb[a] += tb * D.dm1[g * 3 + a];
      Db.dm1[g * 3 + a] += tb * B[a];
    }
    // dB_g = -inv rhs_g
    double rb[3];
    for (int b = 0; b < 3; ++b)
      rb[b] = -(inv[b * 3] * dBb[g * 3] + inv[b * 3 + 1] * dBb[g * 3 + 1] +
                inv[b * 3 + 2] * dBb[g * 3 + 2]);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) invb[a * 3 + b] += -dBb[g * 3 + a] * rhs[g * 3 + b];
    // rhs_g = dm1_g + dm2_g B
    for (int b = 0; b < 3; ++b) {
      Db.dm1[g * 3 + b] += rb[b];
      for (int e = 0; e < 3; ++e) {
        Db.dm2[(g * 3 + b) * 3 + e] += rb[b] * B[e];
        Bb[e] += D.dm2[(g * 3 + b) * 3 + e] * rb[b];
      }
    }
  }
  // A = 1 / (m0 + B.m1)
  const double denb = -(A * A) * Ab;
  Db.m0 += denb;
  for (int a = 0; a < 3; ++a) {
    Bb[a] += denb * D.m1[a];
    Db.m1[a] += denb * B[a];
  }
  // B = -inv m1
  for (int a = 0; a < 3; ++a) {
    Db.m1[a] += -(inv[a * 3] * Bb[0] + inv[a * 3 + 1] * Bb[1] + inv[a * 3 + 2] * Bb[2]);
    for (int b = 0; b < 3; ++b) invb[a * 3 + b] += -Bb[a] * D.m1[b];
  }
  // inv = m2^-1: m2bar = -inv^T invb inv^T (inv symmetric)
  double tmp[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      tmp[a * 3 + b] = invb[a * 3] * inv[b] + invb[a * 3 + 1] * inv[3 + b] + invb[a * 3 + 2] * inv[6 + b];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      Db.m2[a * 3 + b] -= inv[a * 3] * tmp[b] + inv[a * 3 + 1] * tmp[3 + b] + inv[a * 3 + 2] * tmp[6 + b];
  // expanded -> raw sums
  out[0] = Db.m0;
  for (int a = 0; a < 3; ++a) {
    out[1 + a] = Db.m1[a];
    out[10 + a] = Db.dm0[a];
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) out[4 + sym6h(a, b)] += Db.m2[a * 3 + b];
  for (int g = 0; g < 3; ++g)
    for (int a = 0; a < 3; ++a) {
      out[13 + g * 3 + a] += Db.dm1[g * 3 + a];
      if (a == g) out[0] += Db.dm1[g * 3 + a];
      for (int b = 0; b < 3; ++b) {
        const double v = Db.dm2[(g * 3 + a) * 3 + b];
        out[22 + g * 6 + sym6h(a, b)] += v;
        if (a == g) out[1 + b] += v;
        if (b == g) out[1 + a] += v;
      }
    }
  return true;
}

// ------------------------------------------------------ moment adjoint ----
// One gather pair of particle i's moments contributes
//   l = V_j [W phi0(x) + f psi(x)],
//   phi0 = m0b + m1b.x + sum_s m2b_s p_s(x),
//   psi  = sum_g x_g (dm0b_g + sum_a X1b_ga x_a + sum_s X2b_gs p_s(x)),
// with p = (xx, xy, xz, yy, yz, zz). Returns l / V_j and writes dl/dx (per
// unit V_j) and dl/dh_i (per unit V_j).
template <class R>
__host__ __device__ inline R mom_pair_adj(const R mb[40], const R x[3], R rinv,
                                          const KEval<R>& e, R gx[3], R& gh) {
  const R p[6] = {x[0] * x[0], x[0] * x[1], x[0] * x[2], x[1] * x[1], x[1] * x[2], x[2] * x[2]};
  R phi0 = mb[0] + mb[1] * x[0] + mb[2] * x[1] + mb[3] * x[2];
  for (int s = 0; s < 6; ++s) phi0 += mb[4 + s] * p[s];
  // grad phi0
  R gphi0[3];
  for (int c = 0; c < 3; ++c) {
    R v = mb[1 + c];
    for (int d = 0; d < 3; ++d) {
      const R coef = (c == d) ? R(2) * mb[4 + sym6h(c, d)] : mb[4 + sym6h(c, d)];
      v += coef * x[d];
    }
    gphi0[c] = v;
  }
  // phi1_g and psi
  R phi1[3], psi = R(0);
  for (int g = 0; g < 3; ++g) {
    R v = mb[10 + g];
    for (int a = 0; a < 3; ++a) v += mb[13 + g * 3 + a] * x[a];
    for (int s = 0; s < 6; ++s) v += mb[22 + g * 6 + s] * p[s];
    phi1[g] = v;
    psi += x[g] * v;
  }
  // grad psi_c = phi1_c + sum_g x_g d phi1_g / dx_c
  R gpsi[3];
  for (int c = 0; c < 3; ++c) {
    R v = phi1[c];
    for (int g = 0; g < 3; ++g) {
      R d = mb[13 + g * 3 + c];
      for (int dd = 0; dd < 3; ++dd) {
        const R coef = (c == dd) ? R(2) * mb[22 + g * 6 + sym6h(c, dd)] : mb[22 + g * 6 + sym6h(c, dd)];
        d += coef * x[dd];
      }
      v += x[g] * d;
    }
    gpsi[c] = v;
  }
  const R radial = phi0 * e.f + psi * e.fr * rinv;
  for (int c = 0; c < 3; ++c) gx[c] = e.W * gphi0[c] + e.f * gpsi[c] + radial * x[c];
  gh = phi0 * e.dWdh + psi * e.dfdh;
  return e.W * phi0 + e.f * psi;
}

}  // namespace crk
