// FP64 CPU oracle for the CRKSPH neighbour-pair passes.
//
// TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the
// GPU library is checked against. Only the tests, the smoke check and the
// benchmark's CPU-baseline leg may load it. It shares no code with the HIP
// library and includes none of its headers.
//
// What it computes, in the order the method defines it (paper citations are
// to arXiv:2511.21921, "Modeling Galaxy Formation in Cosmological Simulations
// with CRK-HACC"):
//   1. smoothing length h_i: the root of the Thacker neighbour condition
//      Delta_N = 1 (App. A.3, eq. thacker, with Delta_N^3 = V n_h^3 / h^3),
//      i.e. h^3 sum_j (m_j/m_i) W(r_ij, h) = n_h^3;
//   2. particle volume, V_i^-1 = m_i^-1 sum_j m_j W(|x_ij|, h_i)
//      (App. A.2, eq. Vg), self term included;
//   3. geometric moments and the reproducing-kernel corrections A_i, B_i and
//      their gradients, from requiring the corrected kernel
//      W^R_ij = A_i (1 + B_i . x_ij) W_ij(h_i) (App. A.1, eq. RK) to
//      reproduce constant and linear fields exactly (Sec. 2.1);
//   4. gas density rho_i = sum m_j V_j W^R_ij / sum V_j^2 W^R_ij (Sec. 2.5.1,
//      eq. rhow, gas-only form) and the velocity gradient
//      grad v_i = -sum_j V_j (v_i - v_j) (x) grad W^R_ij (App. A.1, eq. gradv);
//   5. ideal-gas pressure and sound speed with gamma = 5/3 (Sec. 2.4.1);
//   6. optional RK relaxation: exp(|tr grad v_i| dt) > 8 => A = 1, B = 0 for
//      every pair the particle takes part in (App. A.1);
//   7. pairwise momentum and compatible energy with a limited artificial
//      viscosity (Sec. 2.1; the exact forms are the readings listed in the
//      design notes: antisymmetrised RK gradients, equal work split, a
//      van Leer-limited midpoint-reconstructed Monaghan-Gingold viscosity).
// Kernels have compact support of radius h (App. A.2 and its footnote): the
// cubic spline (M4) and the Wendland C4 kernel.
//
// Parity unpinned: the paper cites, but does not print, the exact form of
// the viscosity limiter and of the compatible-energy work split. The forms
// used here (step 7) are readings; the tests pin their invariants (exact
// momentum and energy conservation, Q = 0 for exactly linear flow, affinity
// in alpha and beta, the textbook SPH limit with A = 1, B = 0), not the forms
// themselves.
//
// Neighbour search is either an O(N^2) minimum-image brute force or a simple
// uniform grid written here and checked against the brute force.
//
// Everything is templated on the scalar so that the same code, run on
// forward-mode dual numbers, returns exact directional derivatives (JVPs).
// Built with -ffp-contract=off and without fast-math.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- scalars --

inline double val(double a) { return a; }

struct Dual {  // one tangent direction
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double a) : v(a), d(0.0) {}  // NOLINT: constants promote
  Dual(double a, double b) : v(a), d(b) {}
};
inline double val(const Dual& a) { return a.v; }
inline Dual operator+(const Dual& a, const Dual& b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(const Dual& a, const Dual& b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(const Dual& a) { return Dual(-a.v, -a.d); }
inline Dual operator*(const Dual& a, const Dual& b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(const Dual& a, const Dual& b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual& operator+=(Dual& a, const Dual& b) { a.v += b.v; a.d += b.d; return a; }
inline Dual& operator-=(Dual& a, const Dual& b) { a.v -= b.v; a.d -= b.d; return a; }
inline Dual sqrt(const Dual& a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
using std::sqrt;

// ---------------------------------------------------------------- params ---

struct Params {
  double box, gamma, alpha, beta, eps2, n_h, dt_relax;
  int kernel;  // 0 cubic spline, 1 Wendland C4
  int h_mode;  // 0 fixed h, 1 solve for h
};

const double PI = 3.14159265358979323846;

// ---------------------------------------------------------------- kernels --
// W(r, h) = C / h^3 * w(q), q = r / h, support q < 1.

double knorm(int kernel) {
  return kernel == 0 ? 8.0 / PI : 495.0 / (32.0 * PI);
}

template <class T>
T kw(int kernel, const T& q) {
  if (kernel == 0) {
    if (val(q) <= 0.5) return 1.0 - 6.0 * q * q + 6.0 * q * q * q;
    if (val(q) < 1.0) {
      T s = 1.0 - q;
      return 2.0 * s * s * s;
    }
    return T(0.0);
  }
  if (val(q) < 1.0) {
    T s = 1.0 - q;
    T s2 = s * s;
    return s2 * s2 * s2 * (1.0 + 6.0 * q + (35.0 / 3.0) * q * q);
  }
  return T(0.0);
}

template <class T>
T kdw(int kernel, const T& q) {  // dw/dq
  if (kernel == 0) {
    if (val(q) <= 0.5) return -12.0 * q + 18.0 * q * q;
    if (val(q) < 1.0) {
      T s = 1.0 - q;
      return -6.0 * s * s;
    }
    return T(0.0);
  }
  if (val(q) < 1.0) {
    T s = 1.0 - q;
    T s2 = s * s;
    return -(56.0 / 3.0) * q * (1.0 + 5.0 * q) * s2 * s2 * s;
  }
  return T(0.0);
}

// W and its gradient with respect to the first particle, for separation x
// (x = x_i - x_j) of length r > 0.
template <class T>
void kernel_and_grad(int kernel, const T x[3], const T& r, const T& h, T& W, T gW[3]) {
  T q = r / h;
  double C = knorm(kernel);
  T h2 = h * h;
  T h3 = h2 * h;
  W = C * kw(kernel, q) / h3;
  T dWdr = C * kdw(kernel, q) / (h3 * h);
  for (int g = 0; g < 3; ++g) gW[g] = dWdr * x[g] / r;
}

// ------------------------------------------------------- periodic geometry --

// Minimum-image separation of double positions: returns r^2 and the image
// shift applied (so that the same shift can be replayed on dual numbers).
inline double min_image(const double* X, int64_t n, int64_t i, int64_t j, double L,
                        double d[3], double shift[3]) {
  double r2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    double t = X[a * n + i] - X[a * n + j];
    double s = -L * std::round(t / L);
    shift[a] = s;
    d[a] = t + s;
    r2 += d[a] * d[a];
  }
  return r2;
}

// ---------------------------------------------------------- neighbour sets --

struct Finder {
  const double* X;  // [3][n], wrapped into [0, L)
  int64_t n;
  double L;
  int mode;  // 0 brute force, 1 grid
  int G = 1;
  double ell = 1.0;
  std::vector<int64_t> start, idx;

  void build(double R) {
    if (mode == 0) return;
    G = (int)std::floor(L / R);
    if (G < 1) G = 1;
    if (G > 512) G = 512;
    while ((double)G * G * G > 8.0 * (double)n + 64 && G > 1) --G;
    ell = L / G;
    std::vector<int64_t> cell(n);
    start.assign((size_t)G * G * G + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
      int c[3];
      for (int a = 0; a < 3; ++a) {
        int k = (int)std::floor(X[a * n + i] / ell);
        c[a] = std::min(std::max(k, 0), G - 1);
      }
      cell[i] = ((int64_t)c[2] * G + c[1]) * G + c[0];
      start[cell[i] + 1]++;
    }
    for (size_t c = 0; c + 1 < start.size(); ++c) start[c + 1] += start[c];
    idx.assign(n, 0);
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < n; ++i) idx[fill[cell[i]]++] = i;  // increasing i within a cell
  }

  // All j (self included) with minimum-image distance r < R, ascending j.
  void within(int64_t i, double R, std::vector<int64_t>& out) const {
    out.clear();
    const double R2 = R * R;
    double d[3], s[3];
    if (mode == 0 || 2 * (int)std::ceil(R / ell) + 1 >= G) {
      for (int64_t j = 0; j < n; ++j)
        if (min_image(X, n, i, j, L, d, s) < R2) out.push_back(j);
      return;
    }
    int k = (int)std::ceil(R / ell);
    int c[3];
    for (int a = 0; a < 3; ++a) {
      int t = (int)std::floor(X[a * n + i] / ell);
      c[a] = std::min(std::max(t, 0), G - 1);
    }
    for (int dz = -k; dz <= k; ++dz)
      for (int dy = -k; dy <= k; ++dy)
        for (int dx = -k; dx <= k; ++dx) {
          int cx = ((c[0] + dx) % G + G) % G;
          int cy = ((c[1] + dy) % G + G) % G;
          int cz = ((c[2] + dz) % G + G) % G;
          int64_t cc = ((int64_t)cz * G + cy) * G + cx;
          for (int64_t p = start[cc]; p < start[cc + 1]; ++p) {
            int64_t j = idx[p];
            if (min_image(X, n, i, j, L, d, s) < R2) out.push_back(j);
          }
        }
    std::sort(out.begin(), out.end());
  }
};

// --------------------------------------------------------------- h solve --
// f_i(h) = C sum_j (m_j/m_i) w(r_ij/h) - n_h^3 (= h^3 sum (m_j/m_i) W - n_h^3).
// Non-decreasing in h. Safeguarded Newton inside a bisection bracket.

struct HResult {
  double h;
  int iters;
  bool ok;
};

double f_of_h(int kernel, double n_h3, const std::vector<double>& r, const std::vector<double>& mr,
              double h, double* dfdh) {
  double C = knorm(kernel), s = 0.0, ds = 0.0;
  for (size_t k = 0; k < r.size(); ++k) {
    double q = r[k] / h;
    if (q < 1.0) {
      s += mr[k] * kw(kernel, q);
      ds += mr[k] * kdw(kernel, q) * (-q / h);
    }
  }
  if (dfdh) *dfdh = C * ds;
  return C * s - n_h3;
}

HResult solve_h(const Finder& F, const double* m, int kernel, double n_h, int64_t i, double guess,
                double rtol) {
  const double n_h3 = n_h * n_h * n_h;
  std::vector<int64_t> nb;
  std::vector<double> r, mr;
  double R = guess * 1.5;
  if (R >= 0.5 * F.L) R = 0.4999 * F.L;
  for (int attempt = 0; attempt < 64; ++attempt) {
    F.within(i, R, nb);
    r.clear();
    mr.clear();
    double d[3], s[3];
    for (int64_t j : nb) {
      r.push_back(std::sqrt(min_image(F.X, F.n, i, j, F.L, d, s)));
      mr.push_back(m[j] / m[i]);
    }
    if (f_of_h(kernel, n_h3, r, mr, R, nullptr) > 0.0) break;
    if (R >= 0.4999 * F.L) return {R, 0, false};
    R = std::min(R * 1.5, 0.4999 * F.L);
  }
  double lo = 0.0, hi = R, h = std::min(guess, R);
  int it = 0;
  bool ok = false;
  for (; it < 300; ++it) {
    double dfdh;
    double f = f_of_h(kernel, n_h3, r, mr, h, &dfdh);
    if (f > 0.0) hi = h; else lo = h;
    double hn = 0.5 * (lo + hi);
    if (dfdh > 0.0) {
      double nt = h - f / dfdh;
      // a Newton step below the tolerance ends the solve (h sits on the root)
      if (std::fabs(nt - h) <= rtol * h) {
        h = std::min(std::max(nt, lo), hi);
        ok = true;
        break;
      }
      if (nt > lo && nt < hi) hn = nt;
    }
    h = hn;
    if ((hi - lo) <= rtol * h) {
      ok = true;
      break;
    }
  }
  return {h, it + 1, ok};
}

// ------------------------------------------------------------- the passes --

struct Lists {
  std::vector<std::vector<int64_t>> gather;  // j with r_ij < h_i, self included
  std::vector<std::vector<int64_t>> sym;     // j != i with r_ij < max(h_i, h_j)
};

// Minimum-image separation x_i - x_j in scalar T, image chosen on values.
template <class T>
void sep(const std::vector<T>& x, int64_t n, int64_t i, int64_t j, double L, T out[3]) {
  for (int a = 0; a < 3; ++a) {
    T t = x[a * n + i] - x[a * n + j];
    out[a] = t - L * std::round(val(t) / L);
  }
}

template <class T>
struct Fields {
  std::vector<T> h, V, A, B, dA, dB, rho, gv, P, c, acc, dudt;
  std::vector<double> sa, su;     // cancellation-aware scales
  std::vector<uint8_t> relaxed, singular;
};

// Corrected-kernel value and gradient for particle i (coefficients of i), at
// separation x = x_i - x_j with uncorrected W and grad W.
template <class T>
void corrected(const T& A, const T B[3], const T dA[3], const T dB[9], const T x[3], const T& W,
               const T gW[3], T& WR, T gWR[3]) {
  T bx = B[0] * x[0] + B[1] * x[1] + B[2] * x[2];
  T lin = 1.0 + bx;
  WR = A * lin * W;
  for (int g = 0; g < 3; ++g) {
    T dbx = dB[g * 3 + 0] * x[0] + dB[g * 3 + 1] * x[1] + dB[g * 3 + 2] * x[2];
    gWR[g] = dA[g] * lin * W + A * (dbx + B[g]) * W + A * lin * gW[g];
  }
}

// Stored state of passive particles in a timestep hierarchy (App. A.3, A.4):
// particles that are not updating forces this substep keep the corrections of
// their last evaluation and carry V and rho from the passive updates; their
// velocity gradient is the one of their last evaluation. Caller layouts.
struct Passive {
  const uint8_t* mask = nullptr;  // [n] 1 = passive
  const double *V = nullptr, *A = nullptr, *B = nullptr, *dA = nullptr, *dB = nullptr,
               *rho = nullptr, *gv = nullptr;
  bool at(int64_t i) const { return mask && mask[i]; }
};

template <class T>
void run_passes(const Params& P, const T& alpha, const T& beta, int64_t n,
                const std::vector<T>& x, const std::vector<T>& v, const std::vector<double>& m,
                const std::vector<T>& u, const std::vector<T>& h, const Lists& Lst,
                Fields<T>& out, const Passive& pas = Passive()) {
  const double L = P.box;
  const int K = P.kernel;
  const double C = knorm(K);
  out.h = h;
  out.V.assign(n, T(0.0));
  out.A.assign(n, T(0.0));
  out.B.assign(3 * n, T(0.0));
  out.dA.assign(3 * n, T(0.0));
  out.dB.assign(9 * n, T(0.0));
  out.rho.assign(n, T(0.0));
  out.gv.assign(9 * n, T(0.0));
  out.P.assign(n, T(0.0));
  out.c.assign(n, T(0.0));
  out.acc.assign(3 * n, T(0.0));
  out.dudt.assign(n, T(0.0));
  out.sa.assign(n, 0.0);
  out.su.assign(n, 0.0);
  out.relaxed.assign(n, 0);
  out.singular.assign(n, 0);

  // Volume (App. A.2, eq. Vg), self term included.
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    T s(0.0);
    for (int64_t j : Lst.gather[i]) {
      if (j == i) {
        s += m[j] * C * kw(K, T(0.0)) / (h[i] * h[i] * h[i]);
        continue;
      }
      T d[3];
      sep(x, n, i, j, L, d);
      T r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      T W, gW[3];
      kernel_and_grad(K, d, r, h[i], W, gW);
      s += m[j] * W;
    }
    out.V[i] = m[i] / s;
  }
  for (int64_t i = 0; i < n; ++i)
    if (pas.at(i)) out.V[i] = T(pas.V[i]);

  // Moments and corrections (App. A.1, eq. RK; reproducing conditions).
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    T m0(0.0), m1[3], m2[9], dm0[3], dm1[9], dm2[27];
    for (auto& t : m1) t = T(0.0);
    for (auto& t : m2) t = T(0.0);
    for (auto& t : dm0) t = T(0.0);
    for (auto& t : dm1) t = T(0.0);
    for (auto& t : dm2) t = T(0.0);
    for (int64_t j : Lst.gather[i]) {
      T d[3] = {T(0.0), T(0.0), T(0.0)}, W, gW[3] = {T(0.0), T(0.0), T(0.0)};
      if (j == i) {
        W = C * kw(K, T(0.0)) / (h[i] * h[i] * h[i]);
      } else {
        sep(x, n, i, j, L, d);
        T r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        kernel_and_grad(K, d, r, h[i], W, gW);
      }
      const T& Vj = out.V[j];
      m0 += Vj * W;
      for (int a = 0; a < 3; ++a) {
        m1[a] += Vj * d[a] * W;
        for (int b = 0; b < 3; ++b) m2[a * 3 + b] += Vj * d[a] * d[b] * W;
      }
      for (int g = 0; g < 3; ++g) {
        dm0[g] += Vj * gW[g];
        for (int a = 0; a < 3; ++a) {
          T t = d[a] * gW[g];
          if (a == g) t += W;
          dm1[g * 3 + a] += Vj * t;
          for (int b = 0; b < 3; ++b) {
            T s = d[a] * d[b] * gW[g];
            if (a == g) s += d[b] * W;
            if (b == g) s += d[a] * W;
            dm2[(g * 3 + a) * 3 + b] += Vj * s;
          }
        }
      }
    }
    // m2^-1 by the adjugate.
    T cof[9];
    cof[0] = m2[4] * m2[8] - m2[5] * m2[7];
    cof[1] = m2[2] * m2[7] - m2[1] * m2[8];
    cof[2] = m2[1] * m2[5] - m2[2] * m2[4];
    cof[3] = m2[5] * m2[6] - m2[3] * m2[8];
    cof[4] = m2[0] * m2[8] - m2[2] * m2[6];
    cof[5] = m2[2] * m2[3] - m2[0] * m2[5];
    cof[6] = m2[3] * m2[7] - m2[4] * m2[6];
    cof[7] = m2[1] * m2[6] - m2[0] * m2[7];
    cof[8] = m2[0] * m2[4] - m2[1] * m2[3];
    T det = m2[0] * cof[0] + m2[1] * cof[3] + m2[2] * cof[6];
    double scale = std::fabs(val(m2[0])) + std::fabs(val(m2[4])) + std::fabs(val(m2[8]));
    if (!(std::fabs(val(det)) > 1e-12 * scale * scale * scale)) {
      // Too few non-coplanar neighbours: uncorrected kernel.
      out.singular[i] = 1;
      out.A[i] = T(1.0);
      continue;
    }
    T inv[9];
    for (int k = 0; k < 9; ++k) inv[k] = cof[k] / det;
    T B[3], dB[9], dA[3];
    for (int a = 0; a < 3; ++a) {
      B[a] = T(0.0);
      for (int b = 0; b < 3; ++b) B[a] -= inv[a * 3 + b] * m1[b];
    }
    T A = 1.0 / (m0 + B[0] * m1[0] + B[1] * m1[1] + B[2] * m1[2]);
    for (int g = 0; g < 3; ++g) {
      T rhs[3];
      for (int b = 0; b < 3; ++b) {
        rhs[b] = dm1[g * 3 + b];
        for (int e = 0; e < 3; ++e) rhs[b] += dm2[(g * 3 + b) * 3 + e] * B[e];
      }
      for (int a = 0; a < 3; ++a) {
        dB[g * 3 + a] = T(0.0);
        for (int b = 0; b < 3; ++b) dB[g * 3 + a] -= inv[a * 3 + b] * rhs[b];
      }
      T t = dm0[g];
      for (int a = 0; a < 3; ++a) t += dB[g * 3 + a] * m1[a] + B[a] * dm1[g * 3 + a];
      dA[g] = -(A * A) * t;
    }
    out.A[i] = A;
    for (int a = 0; a < 3; ++a) {
      out.B[a * n + i] = B[a];
      out.dA[a * n + i] = dA[a];
    }
    for (int k = 0; k < 9; ++k) out.dB[k * n + i] = dB[k];
  }

  for (int64_t i = 0; i < n; ++i)
    if (pas.at(i)) {
      out.singular[i] = 0;
      out.A[i] = T(pas.A[i]);
      for (int a = 0; a < 3; ++a) {
        out.B[a * n + i] = T(pas.B[a * n + i]);
        out.dA[a * n + i] = T(pas.dA[a * n + i]);
      }
      for (int k = 0; k < 9; ++k) out.dB[k * n + i] = T(pas.dB[k * n + i]);
    }

  // Density (Sec. 2.5.1, eq. rhow) and velocity gradient (App. A.1, eq. gradv).
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    if (pas.at(i)) {
      // passive: the carried density and the gradient of the last evaluation
      out.rho[i] = T(pas.rho[i]);
      for (int k = 0; k < 9; ++k) out.gv[k * n + i] = T(pas.gv[k * n + i]);
      out.P[i] = (P.gamma - 1.0) * out.rho[i] * u[i];
      out.c[i] = sqrt(P.gamma * (P.gamma - 1.0) * u[i]);
      if (P.dt_relax > 0.0) {
        double div = pas.gv[i] + pas.gv[4 * n + i] + pas.gv[8 * n + i];
        out.relaxed[i] = std::exp(std::fabs(div) * P.dt_relax) > 8.0 ? 1 : 0;
      }
      continue;
    }
    T Ai = out.A[i], Bi[3], dAi[3], dBi[9];
    for (int a = 0; a < 3; ++a) {
      Bi[a] = out.B[a * n + i];
      dAi[a] = out.dA[a * n + i];
    }
    for (int k = 0; k < 9; ++k) dBi[k] = out.dB[k * n + i];
    T num(0.0), den(0.0), gv[9];
    for (auto& t : gv) t = T(0.0);
    for (int64_t j : Lst.gather[i]) {
      T d[3] = {T(0.0), T(0.0), T(0.0)}, W, gW[3] = {T(0.0), T(0.0), T(0.0)};
      if (j == i) {
        W = C * kw(K, T(0.0)) / (h[i] * h[i] * h[i]);
      } else {
        sep(x, n, i, j, L, d);
        T r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        kernel_and_grad(K, d, r, h[i], W, gW);
      }
      T WR, gWR[3];
      corrected(Ai, Bi, dAi, dBi, d, W, gW, WR, gWR);
      const T& Vj = out.V[j];
      num += m[j] * Vj * WR;
      den += Vj * Vj * WR;
      for (int a = 0; a < 3; ++a) {
        T dv = v[a * n + i] - v[a * n + j];
        for (int g = 0; g < 3; ++g) gv[a * 3 + g] -= Vj * dv * gWR[g];
      }
    }
    out.rho[i] = num / den;
    for (int k = 0; k < 9; ++k) out.gv[k * n + i] = gv[k];
    // Equation of state (gamma-law ideal gas).
    out.P[i] = (P.gamma - 1.0) * out.rho[i] * u[i];
    out.c[i] = sqrt(P.gamma * (P.gamma - 1.0) * u[i]);
    if (P.dt_relax > 0.0) {
      double div = val(gv[0]) + val(gv[4]) + val(gv[8]);
      out.relaxed[i] = std::exp(std::fabs(div) * P.dt_relax) > 8.0 ? 1 : 0;
    }
  }

  // Pairwise momentum and energy with artificial viscosity.
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    T ai[3] = {T(0.0), T(0.0), T(0.0)}, dui(0.0);
    double sa = 0.0, su = 0.0;
    for (int64_t j : Lst.sym[i]) {
      T d[3], dj[3];
      sep(x, n, i, j, L, d);
      for (int a = 0; a < 3; ++a) dj[a] = -d[a];
      T r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      bool plain = out.relaxed[i] || out.relaxed[j];
      // i side: grad_i W^R_ij with h_i and i's corrections (zero outside h_i).
      T Gi[3] = {T(0.0), T(0.0), T(0.0)}, Gj[3] = {T(0.0), T(0.0), T(0.0)};
      if (val(r) < val(h[i])) {
        T W, gW[3], WR;
        kernel_and_grad(K, d, r, h[i], W, gW);
        if (plain) {
          for (int g = 0; g < 3; ++g) Gi[g] = gW[g];
        } else {
          T Bi[3], dAi[3], dBi[9];
          for (int a = 0; a < 3; ++a) {
            Bi[a] = out.B[a * n + i];
            dAi[a] = out.dA[a * n + i];
          }
          for (int k = 0; k < 9; ++k) dBi[k] = out.dB[k * n + i];
          corrected(out.A[i], Bi, dAi, dBi, d, W, gW, WR, Gi);
        }
      }
      // j side: grad_j W^R_ji with h_j, j's corrections and x_ji = -x_ij.
      if (val(r) < val(h[j])) {
        T W, gW[3], WR;
        kernel_and_grad(K, dj, r, h[j], W, gW);
        if (plain) {
          for (int g = 0; g < 3; ++g) Gj[g] = gW[g];
        } else {
          T Bj[3], dAj[3], dBj[9];
          for (int a = 0; a < 3; ++a) {
            Bj[a] = out.B[a * n + j];
            dAj[a] = out.dA[a * n + j];
          }
          for (int k = 0; k < 9; ++k) dBj[k] = out.dB[k * n + j];
          corrected(out.A[j], Bj, dAj, dBj, dj, W, gW, WR, Gj);
        }
      }
      T G[3];
      for (int g = 0; g < 3; ++g) G[g] = Gi[g] - Gj[g];

      // Limited artificial viscosity.
      T gi_x[3], gj_x[3];  // grad v . x for i and j
      for (int a = 0; a < 3; ++a) {
        gi_x[a] = T(0.0);
        gj_x[a] = T(0.0);
        for (int g = 0; g < 3; ++g) {
          gi_x[a] += out.gv[(a * 3 + g) * n + i] * d[g];
          gj_x[a] += out.gv[(a * 3 + g) * n + j] * d[g];
        }
      }
      T num = d[0] * gi_x[0] + d[1] * gi_x[1] + d[2] * gi_x[2];
      T den = d[0] * gj_x[0] + d[1] * gj_x[1] + d[2] * gj_x[2];
      T sum = num + den;
      T phi(0.0);
      if (val(sum * sum) > 0.0) {
        phi = 4.0 * num * den / (sum * sum);
        if (val(phi) < 0.0) phi = T(0.0);
        if (val(phi) > 1.0) phi = T(1.0);
      }
      T vp[3];
      for (int a = 0; a < 3; ++a)
        vp[a] = (v[a * n + i] - 0.5 * phi * gi_x[a]) - (v[a * n + j] + 0.5 * phi * gj_x[a]);
      T Q[2];
      for (int s = 0; s < 2; ++s) {
        int64_t k = s == 0 ? i : j;
        T eta[3];
        for (int a = 0; a < 3; ++a) eta[a] = d[a] / h[k];
        T ee = eta[0] * eta[0] + eta[1] * eta[1] + eta[2] * eta[2];
        T mu = (vp[0] * eta[0] + vp[1] * eta[1] + vp[2] * eta[2]) / (ee + P.eps2);
        if (val(mu) > 0.0) mu = T(0.0);
        Q[s] = out.rho[k] * (-alpha * out.c[k] * mu + beta * mu * mu);
      }
      T Pi = out.P[i] + out.P[j] + Q[0] + Q[1];
      T s = -0.5 * out.V[i] * out.V[j] * Pi;
      T F[3];
      for (int g = 0; g < 3; ++g) F[g] = s * G[g];
      T work(0.0);
      for (int a = 0; a < 3; ++a) {
        ai[a] += F[a];
        work += (v[a * n + i] - v[a * n + j]) * F[a];
      }
      dui -= 0.5 * work;
      sa += std::sqrt(val(F[0]) * val(F[0]) + val(F[1]) * val(F[1]) + val(F[2]) * val(F[2]));
      su += 0.5 * std::fabs(val(work));
    }
    for (int a = 0; a < 3; ++a) out.acc[a * n + i] = ai[a] / m[i];
    out.dudt[i] = dui / m[i];
    out.sa[i] = sa / m[i];
    out.su[i] = su / m[i];
  }
}

// Builds positions wrapped into [0, L), the neighbour finder and the solved
// (or fixed) smoothing lengths; then the gather and symmetric lists.
struct Setup {
  std::vector<double> X, h;
  std::vector<int> iters;
  std::vector<uint8_t> conv;
  Lists lists;
  Finder F;
};

int prepare(const Params& P, int64_t n, const double* x, const double* m, const double* h_in,
            int nbr_mode, double rtol, Setup& S) {
  const double L = P.box;
  S.X.assign(3 * n, 0.0);
  for (int64_t k = 0; k < 3 * n; ++k) S.X[k] = x[k] - L * std::floor(x[k] / L);
  for (int64_t k = 0; k < 3 * n; ++k)
    if (S.X[k] >= L) S.X[k] -= L;
  double hmax0 = 0.0;
  for (int64_t i = 0; i < n; ++i) hmax0 = std::max(hmax0, h_in[i]);
  S.F.X = S.X.data();
  S.F.n = n;
  S.F.L = L;
  S.F.mode = nbr_mode;
  S.F.build(std::max(hmax0, 1e-300));
  S.h.assign(h_in, h_in + n);
  S.iters.assign(n, 0);
  S.conv.assign(n, 1);
  if (P.h_mode == 1) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      HResult r = solve_h(S.F, m, P.kernel, P.n_h, i, h_in[i], rtol);
      S.h[i] = r.h;
      S.iters[i] = r.iters;
      S.conv[i] = r.ok;
    }
  }
  double hmax = 0.0;
  for (int64_t i = 0; i < n; ++i) hmax = std::max(hmax, S.h[i]);
  if (!(hmax < 0.5 * L)) return -4;
  S.F.build(hmax);
  S.lists.gather.assign(n, {});
  S.lists.sym.assign(n, {});
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    std::vector<int64_t> nb;
    S.F.within(i, S.h[i], nb);
    S.lists.gather[i] = nb;
  }
  // Symmetric lists, r_ij < max(h_i, h_j): j is in i's list exactly when
  // j is in i's gather list (r_ij < h_i) or i is in j's (r_ij < h_j). The
  // second part is the transpose of the gather lists; min_image gives the
  // same r_ij^2 from both sides. Ascending j, self excluded.
  std::vector<std::vector<int64_t>> incoming(n);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i : S.lists.gather[j])
      if (i != j) incoming[i].push_back(j);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    std::vector<int64_t> sy;
    for (int64_t j : S.lists.gather[i])
      if (j != i) sy.push_back(j);
    sy.insert(sy.end(), incoming[i].begin(), incoming[i].end());
    std::sort(sy.begin(), sy.end());
    sy.erase(std::unique(sy.begin(), sy.end()), sy.end());
    S.lists.sym[i] = sy;
  }
  return 0;
}

Params make_params(double box, double gamma, double alpha, double beta, double eps2, double n_h,
                   double dt_relax, int kernel, int h_mode) {
  Params P;
  P.box = box;
  P.gamma = gamma;
  P.alpha = alpha;
  P.beta = beta;
  P.eps2 = eps2;
  P.n_h = n_h;
  P.dt_relax = dt_relax;
  P.kernel = kernel;
  P.h_mode = h_mode;
  return P;
}

int forward_impl(int64_t n, const double* x, const double* v, const double* m, const double* u,
                 const double* h_in, double box, double gamma, double alpha, double beta,
                 double eps2, double n_h, double dt_relax, int kernel, int h_mode, int nbr_mode,
                 double* h, double* V, double* rho, double* A, double* B, double* gradA,
                 double* gradB, double* gradv, double* Pr, double* cs, double* accel,
                 double* dudt, double* scale_a, double* scale_u, int64_t* stats,
                 const Passive& pas) {
  Params P = make_params(box, gamma, alpha, beta, eps2, n_h, dt_relax, kernel, h_mode);
  if (n <= 0 || !(box > 0.0)) return -1;
  Setup S;
  int rc = prepare(P, n, x, m, h_in, nbr_mode, 1e-14, S);
  if (rc) return rc;
  std::vector<double> X(S.X), Vv(v, v + 3 * n), U(u, u + n), M(m, m + n);
  Fields<double> f;
  run_passes<double>(P, P.alpha, P.beta, n, X, Vv, M, U, S.h, S.lists, f, pas);
  std::memcpy(h, f.h.data(), n * 8);
  std::memcpy(V, f.V.data(), n * 8);
  std::memcpy(rho, f.rho.data(), n * 8);
  std::memcpy(A, f.A.data(), n * 8);
  std::memcpy(B, f.B.data(), 3 * n * 8);
  std::memcpy(gradA, f.dA.data(), 3 * n * 8);
  std::memcpy(gradB, f.dB.data(), 9 * n * 8);
  std::memcpy(gradv, f.gv.data(), 9 * n * 8);
  std::memcpy(Pr, f.P.data(), n * 8);
  std::memcpy(cs, f.c.data(), n * 8);
  std::memcpy(accel, f.acc.data(), 3 * n * 8);
  std::memcpy(dudt, f.dudt.data(), n * 8);
  std::memcpy(scale_a, f.sa.data(), n * 8);
  std::memcpy(scale_u, f.su.data(), n * 8);
  int64_t ng = 0, ns = 0, itmax = 0, unc = 0, sing = 0, rel = 0;
  for (int64_t i = 0; i < n; ++i) {
    ng += (int64_t)S.lists.gather[i].size() - 1;
    ns += (int64_t)S.lists.sym[i].size();
    itmax = std::max<int64_t>(itmax, S.iters[i]);
    unc += S.conv[i] ? 0 : 1;
    sing += f.singular[i];
    rel += f.relaxed[i];
  }
  stats[0] = ng;
  stats[1] = ns;
  stats[2] = itmax;
  stats[3] = unc;
  stats[4] = sing;
  stats[5] = rel;
  return 0;
}

}  // namespace

extern "C" {

// Threads of the OpenMP loops that follow (n >= 1); the benchmark times the
// oracle on all host cores and on one.
void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

// Threads the OpenMP loops use.
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Shape functions w(q), w'(q) on an array of q (pins of the kernel).
void oracle_kernel_eval(int kernel, int64_t n, const double* q, double* w, double* dw,
                        double* norm) {
  for (int64_t k = 0; k < n; ++k) {
    w[k] = kw(kernel, q[k]);
    dw[k] = kdw(kernel, q[k]);
  }
  *norm = knorm(kernel);
}

// Neighbour counts: kind 0 gather (r < h_i, self included), kind 1 symmetric
// (j != i, r < max(h_i, h_j)). Fills counts[n]; if list is non-null it must
// hold sum(counts) entries and receives the concatenated ascending lists.
int oracle_neighbours(int64_t n, const double* x, const double* h, double box, int mode, int kind,
                      int64_t* counts, int64_t* list) {
  Params P = make_params(box, 5.0 / 3.0, 1, 2, 0.01, 1.0, 0.0, 0, 0);
  Setup S;
  int rc = prepare(P, n, x, h /*unused masses*/, h, mode, 1e-13, S);
  if (rc) return rc;
  int64_t off = 0;
  for (int64_t i = 0; i < n; ++i) {
    const auto& L = kind == 0 ? S.lists.gather[i] : S.lists.sym[i];
    counts[i] = (int64_t)L.size();
    if (list)
      for (int64_t j : L) list[off++] = j;
  }
  return 0;
}

// Full forward evaluation in FP64. Arrays are SoA: vectors [3][n], gradients
// [9][n] with gradB index g*3+a = d_g B^a and gradv index a*3+g = d_g v^a.
// stats[0..5] = gather pairs (j != i), force pairs, max h-iterations,
// unconverged h count, singular m2 count, relaxed count.
int oracle_forward(int64_t n, const double* x, const double* v, const double* m, const double* u,
                   const double* h_in, double box, double gamma, double alpha, double beta,
                   double eps2, double n_h, double dt_relax, int kernel, int h_mode, int nbr_mode,
                   double* h, double* V, double* rho, double* A, double* B, double* gradA,
                   double* gradB, double* gradv, double* Pr, double* cs, double* accel,
                   double* dudt, double* scale_a, double* scale_u, int64_t* stats) {
  return forward_impl(n, x, v, m, u, h_in, box, gamma, alpha, beta, eps2, n_h, dt_relax, kernel,
                      h_mode, nbr_mode, h, V, rho, A, B, gradA, gradB, gradv, Pr, cs, accel, dudt,
                      scale_a, scale_u, stats, Passive());
}

// The forward with passive particles (mask != 0) taking their V, A, B,
// grad A, grad B, rho and grad v from the given arrays (caller layouts);
// their P and c follow from that rho and their u. Outputs of passive
// particles other than those are computed but carry no meaning.
int oracle_forward_passive(int64_t n, const double* x, const double* v, const double* m,
                           const double* u, const double* h_in, double box, double gamma,
                           double alpha, double beta, double eps2, double n_h, double dt_relax,
                           int kernel, int h_mode, int nbr_mode, const uint8_t* mask,
                           const double* pV, const double* pA, const double* pB,
                           const double* pgradA, const double* pgradB, const double* prho,
                           const double* pgradv, double* h, double* V, double* rho, double* A,
                           double* B, double* gradA, double* gradB, double* gradv, double* Pr,
                           double* cs, double* accel, double* dudt, double* scale_a,
                           double* scale_u, int64_t* stats) {
  Passive pas;
  pas.mask = mask;
  pas.V = pV;
  pas.A = pA;
  pas.B = pB;
  pas.dA = pgradA;
  pas.dB = pgradB;
  pas.rho = prho;
  pas.gv = pgradv;
  return forward_impl(n, x, v, m, u, h_in, box, gamma, alpha, beta, eps2, n_h, dt_relax, kernel,
                      h_mode, nbr_mode, h, V, rho, A, B, gradA, gradB, gradv, Pr, cs, accel, dudt,
                      scale_a, scale_u, stats, pas);
}

// Forward-mode derivative (JVP) along one direction (dx, dv, du, dalpha,
// dbeta); masses are held fixed. With h_mode = 1 the smoothing-length
// tangent comes from the implicit-function theorem at the converged root:
// one Newton step taken in dual arithmetic, dh = -(df/dx . dx)/(df/dh).
// Returns the primal accel/dudt and their tangents, plus the tangents of h,
// V and rho.
int oracle_jvp(int64_t n, const double* x, const double* v, const double* m, const double* u,
               const double* h_in, double box, double gamma, double alpha, double beta,
               double eps2, double n_h, double dt_relax, int kernel, int h_mode, int nbr_mode,
               const double* dx, const double* dv, const double* du, double dalpha, double dbeta,
               double* accel, double* dudt, double* d_accel, double* d_dudt, double* d_h,
               double* d_V, double* d_rho) {
  Params P = make_params(box, gamma, alpha, beta, eps2, n_h, dt_relax, kernel, h_mode);
  if (n <= 0 || !(box > 0.0)) return -1;
  Setup S;
  int rc = prepare(P, n, x, m, h_in, nbr_mode, 1e-14, S);
  if (rc) return rc;
  std::vector<Dual> X(3 * n), Vv(3 * n), U(n), H(n);
  std::vector<double> M(m, m + n);
  for (int64_t k = 0; k < 3 * n; ++k) {
    X[k] = Dual(S.X[k], dx[k]);
    Vv[k] = Dual(v[k], dv[k]);
  }
  for (int64_t i = 0; i < n; ++i) U[i] = Dual(u[i], du[i]);
  const double C = knorm(kernel);
  const double n_h3 = n_h * n_h * n_h;
  for (int64_t i = 0; i < n; ++i) H[i] = Dual(S.h[i], 0.0);
  if (h_mode == 1) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      // f(h; x) = C sum_j (m_j/m_i) w(r_ij/h) - n_h^3 at fixed h, dual in x.
      double hi = S.h[i];
      Dual f(-n_h3);
      double dfdh = 0.0;
      for (int64_t j : S.lists.gather[i]) {
        if (j == i) {
          f += C * kw(kernel, 0.0);
          continue;
        }
        Dual d[3];
        sep(X, n, i, j, box, d);
        Dual r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        Dual q = r / hi;
        f += C * (M[j] / M[i]) * kw(kernel, q);
        dfdh += C * (M[j] / M[i]) * kdw(kernel, q.v) * (-q.v / hi);
      }
      H[i] = Dual(hi, -f.d / dfdh);
    }
  }
  Fields<Dual> f;
  run_passes<Dual>(P, Dual(alpha, dalpha), Dual(beta, dbeta), n, X, Vv, M, U, H, S.lists, f);
  for (int64_t k = 0; k < 3 * n; ++k) {
    accel[k] = f.acc[k].v;
    d_accel[k] = f.acc[k].d;
  }
  for (int64_t i = 0; i < n; ++i) {
    dudt[i] = f.dudt[i].v;
    d_dudt[i] = f.dudt[i].d;
    d_h[i] = f.h[i].d;
    d_V[i] = f.V[i].d;
    d_rho[i] = f.rho[i].d;
  }
  return 0;
}

}  // extern "C"
