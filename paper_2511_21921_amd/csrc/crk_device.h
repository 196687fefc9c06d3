// Device-side building blocks shared by the CRKSPH pass kernels: scalar
// helpers, the two smoothing kernels (support radius h, App. A.2), the
// corrected kernel W^R (App. A.1, eq. RK) in its packed per-particle form,
// and the periodic pair separation from cell-relative offsets.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crk {

constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------- scalars ----

template <class R> struct Sc;
template <> struct Sc<float> {
  __device__ static inline float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
  __device__ static inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  __device__ static inline float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
  // a / b through the hardware reciprocal (about 1 ulp): FP32 pair arithmetic
  __device__ static inline float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
};
template <> struct Sc<double> {
  __host__ __device__ static inline double rsqrt(double x) { return 1.0 / __builtin_sqrt(x); }
  __host__ __device__ static inline double rcp(double x) { return 1.0 / x; }
  __host__ __device__ static inline double sqrt(double x) { return __builtin_sqrt(x); }
  __host__ __device__ static inline double div(double a, double b) { return a / b; }
};

template <class R> struct Vec4;
template <> struct Vec4<float> { using T = float4; };
template <> struct Vec4<double> { using T = double4; };
template <class R> using R4 = typename Vec4<R>::T;

// ------------------------------------------------------------ positions ----

// xa wrapped into [0, L). A non-finite xa (which the forward's input check
// rejects) maps to 0, so that every cell index derived from it stays in range
// until that check is read.
__host__ __device__ inline double wrap_pos(double xa, double L) {
  double t = xa - L * __builtin_floor(xa / L);
  if (t >= L) t -= L;
  return t >= 0.0 && t < L ? t : 0.0;
}

// Cell index of a wrapped coordinate t in [0, L), with inv = G / L: in [0, G).
__host__ __device__ inline int cell_coord(double t, double inv, int G) {
  const int k = (int)(t * inv);
  return k < 0 ? 0 : (k < G ? k : G - 1);
}

// ------------------------------------------------------------- kernels ----
// W(r, h) = C / h^3 w(q), q = r / h, compact support q < 1.
// eval() returns w(q) and w'(q) (zero outside the support).

template <int K> struct Shape;

template <> struct Shape<0> {  // cubic spline (M4), radius h
  static constexpr double C = 8.0 / kPi;
  template <class R> __host__ __device__ static inline void eval(R q, R& w, R& dw) {
    R t = R(1) - q;
    R wi = R(1) + q * q * (R(6) * q - R(6));
    R dwi = q * (R(18) * q - R(12));
    R wo = R(2) * t * t * t;
    R dwo = R(-6) * t * t;
    bool in = q <= R(0.5);
    bool sup = q < R(1);
    w = sup ? (in ? wi : wo) : R(0);
    dw = sup ? (in ? dwi : dwo) : R(0);
  }
  static constexpr double w0 = 1.0;
};

template <> struct Shape<1> {  // Wendland C4, radius h
  static constexpr double C = 495.0 / (32.0 * kPi);
  template <class R> __host__ __device__ static inline void eval(R q, R& w, R& dw) {
    R t = R(1) - q;
    t = t > R(0) ? t : R(0);
    R t2 = t * t;
    R t5 = t2 * t2 * t;
    w = t5 * t * (R(1) + R(6) * q + R(35.0 / 3.0) * q * q);
    dw = R(-56.0 / 3.0) * q * (R(1) + R(5) * q) * t5;
  }
  static constexpr double w0 = 1.0;
};

// ----------------------------------------------------- corrected kernel ----
// Per-particle packed coefficients of W^R_ij = A (1 + B.x) W (x = x_ij):
//   s(x)        = a + b.x            with a = A, b = A B
//   W^R         = s W
//   grad_i W^R  = W (c + M x) + s grad W
// where c_g = dA_g + A B_g and M_ga = dA_g B_a + A dB_ga, which is the
// expansion of dA (1 + B.x) W + A (dB^T x + B) W + A (1 + B.x) grad W.
// Layout of the 16 values: [a, b0, b1, b2, c0, c1, c2, M00..M22 (row g)].

template <class R> struct KC {
  R a, b[3], c[3], M[9];
};

template <class R>
__device__ inline void kc_load(const R* __restrict__ kc, int64_t n, int64_t i, KC<R>& k) {
  k.a = kc[i];
#pragma unroll
  for (int t = 0; t < 3; ++t) k.b[t] = kc[(1 + t) * n + i];
#pragma unroll
  for (int t = 0; t < 3; ++t) k.c[t] = kc[(4 + t) * n + i];
#pragma unroll
  for (int t = 0; t < 9; ++t) k.M[t] = kc[(7 + t) * n + i];
}

template <class R>
__host__ __device__ inline void kc_plain(KC<R>& k) {
  k.a = R(1);
#pragma unroll
  for (int t = 0; t < 3; ++t) k.b[t] = k.c[t] = R(0);
#pragma unroll
  for (int t = 0; t < 9; ++t) k.M[t] = R(0);
}

// W^R and grad W^R for separation x, given W and grad W.
template <class R>
__host__ __device__ inline void kc_apply(const KC<R>& k, const R x[3], R W, const R gW[3], R& WR,
                                R gWR[3]) {
  R s = k.a + k.b[0] * x[0] + k.b[1] * x[1] + k.b[2] * x[2];
  WR = s * W;
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    R t = k.c[g] + k.M[g * 3 + 0] * x[0] + k.M[g * 3 + 1] * x[1] + k.M[g * 3 + 2] * x[2];
    gWR[g] = W * t + s * gW[g];
  }
}

// --------------------------------------------------------- cell list ----
// Positions are stored as offsets xi from the centre of their cell (FP64
// difference, rounded once to Real). For a neighbour j found through
// stencil offset d in {-2,...,2}^3 of i's cell (cells are at least half the
// candidate radius wide), the periodic separation is
// x_ij = xi_i - xi_j - d * ell, exact up to one rounding of each term.
// A neighbour-list entry packs the sorted index of j (high 25 bits) with
// the stencil code 25*(dz+2) + 5*(dy+2) + (dx+2) (low 7 bits).

constexpr int kCodeBits = 7;

// A second moment m2 counts as singular (the particle keeps the uncorrected
// kernel: fewer than three non-coplanar neighbours) when |det m2| <= tol tr^3,
// tr = |m2_00| + |m2_11| + |m2_22|. In FP64 tol = 1e-12. FP32 pair arithmetic
// rounds every product x_a x_b to ~6e-8, which alone leaves the sum over a
// rank-deficient neighbourhood with |det| ~ 1e-8 tr^3, so the FP32 passes take
// tol = 1e-6: an inverse that amplifies their rounding by 10^5 or more carries
// no FP32 digit, and would turn a degenerate neighbourhood into arbitrarily
// large corrections.
template <class R> struct SingularTol { static constexpr double v = 1e-12; };
template <> struct SingularTol<float> { static constexpr double v = 1e-6; };
constexpr uint32_t kCodeMask = 127u;
constexpr int kSelfCode = 62;  // d = (0, 0, 0)

__device__ inline uint32_t stencil_code(int dx, int dy, int dz) {
  return (uint32_t)(25 * (dz + 2) + 5 * (dy + 2) + (dx + 2));
}

__device__ inline void code_offset(uint32_t code, int& dx, int& dy, int& dz) {
  dz = int(code / 25u) - 2;
  dy = int((code / 5u) % 5u) - 2;
  dx = int(code % 5u) - 2;
}

template <class R>
__device__ inline void pair_sep(const R4<R>& pi, const R4<R>& pj, uint32_t code, R ell, R x[3]) {
  int dx, dy, dz;
  code_offset(code, dx, dy, dz);
  x[0] = (pi.x - pj.x) - R(dx) * ell;
  x[1] = (pi.y - pj.y) - R(dy) * ell;
  x[2] = (pi.z - pj.z) - R(dz) * ell;
}

// Per-particle lists (candidates, neighbours) use a chunked SELL layout:
// particles in slices of 64 (one wave), entries in chunks of 4. Chunk c of
// particle i starts at word (((i / 64) * cap / 4 + c) * 64 + i % 64) * 4, so
// a wave reading entry k of all its lanes touches one contiguous 1 KiB row,
// and a lane writes its entries four at a time as one 16-byte store.
// cap is a multiple of 4.
__device__ inline int64_t list_index(int64_t i, int cap, int k) {
  return ((((i >> 6) * (int64_t)(cap >> 2) + (k >> 2)) * 64 + (i & 63)) << 2) + (k & 3);
}

// The same layout with a per-wave capacity: the wave of particle i starts at
// chunk row row0 (a row = one 4-entry chunk of all 64 lanes = 256 words).
// slot_base gives the word of entry 0 of particle i, slot_at that of entry k.
__device__ inline int64_t slot_base(int64_t row0, int64_t i) {
  return (row0 * 64 + (i & 63)) << 2;
}
__device__ inline int64_t slot_at(int64_t base, int k) {
  return base + ((int64_t)(k >> 2) << 8) + (k & 3);
}

// Register staging of one lane's appends: four values are collected and
// written with one 16-byte store (the whole chunk, including unused tail
// slots at the final flush; only the counted entries are ever read).
template <class T> struct Vec4T;
template <> struct Vec4T<uint32_t> { using V = uint4; };
template <> struct Vec4T<float> { using V = float4; };
template <> struct Vec4T<double> { using V = double4; };

template <class T>
struct Stage4 {
  T v0 = T(0), v1 = T(0), v2 = T(0), v3 = T(0);
  __device__ inline void put(int slot, T v) {
    v0 = slot == 0 ? v : v0;
    v1 = slot == 1 ? v : v1;
    v2 = slot == 2 ? v : v2;
    v3 = slot == 3 ? v : v3;
  }
  // writes the chunk that holds entry k (k % 4 == 3 for a full chunk)
  __device__ inline void flush(T* base, int64_t i, int cap, int k) const {
    typename Vec4T<T>::V q;
    q.x = v0;
    q.y = v1;
    q.z = v2;
    q.w = v3;
    *reinterpret_cast<typename Vec4T<T>::V*>(base + list_index(i, cap, k & ~3)) = q;
  }
  // the same for a list addressed by its slot_base b
  __device__ inline void flush_at(T* base, int64_t b, int k) const {
    typename Vec4T<T>::V q;
    q.x = v0;
    q.y = v1;
    q.z = v2;
    q.w = v3;
    *reinterpret_cast<typename Vec4T<T>::V*>(base + slot_at(b, k & ~3)) = q;
  }
  // the same for a candidate list addressed by its group_base b
  __device__ inline void flush_group(T* base, int64_t b, int k) const;
};

// Candidate scratch: a lane's entries in groups of 16 held contiguously (64
// bytes of 4-byte entries), the groups of a wave's 64 lanes side by side (a
// row of 1024 entries). A lane fills a group with four 16-byte stores a few
// candidates apart, so each line is complete while it is still in the L2;
// with the 4-entry chunks of all lanes interleaved, lanes that advance at
// different speeds left lines half written and HBM took several partial
// writes per line. Readers take a whole group (four 16-byte loads) at once.
__device__ inline int64_t group_base(int64_t row0, int64_t i) {
  return (row0 * 64 + (i & 63)) << 4;
}
__device__ inline int64_t group_at(int64_t base, int k) {
  return base + ((int64_t)(k >> 4) << 10) + (k & 15);
}

template <class T>
__device__ inline void Stage4<T>::flush_group(T* base, int64_t b, int k) const {
  typename Vec4T<T>::V q;
  q.x = v0;
  q.y = v1;
  q.z = v2;
  q.w = v3;
  *reinterpret_cast<typename Vec4T<T>::V*>(base + group_at(b, k & ~3)) = q;
}

// the 16 entries of the group that starts at p (four vector loads)
template <class T>
__device__ inline void load_group(const T* p, T v[16]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const typename Vec4T<T>::V q = reinterpret_cast<const typename Vec4T<T>::V*>(p)[c];
    v[4 * c] = q.x;
    v[4 * c + 1] = q.y;
    v[4 * c + 2] = q.z;
    v[4 * c + 3] = q.w;
  }
}

}  // namespace crk
