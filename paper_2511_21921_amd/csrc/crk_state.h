// Device state of one evaluation: the cell list and the cell-sorted
// structure-of-arrays intermediates, passed by value to every pass kernel.
#pragma once

#include "crk_device.h"

namespace crk {

// Slots of the device counter array (unsigned long long).
enum Counter {
  CNT_HMAX_BITS = 0,   // max input h as double bits
  CNT_BAD_INPUT,       // h <= 0, m <= 0 or u <= 0
  CNT_PAIRS_GATHER,
  CNT_PAIRS_FORCE,
  CNT_H_ITER_MAX,
  CNT_H_UNCONV,
  CNT_H_CAPPED,
  CNT_SCR_OVERFLOW,    // largest candidate count beyond the candidate capacity
  CNT_LIST_OVERFLOW,   // largest neighbour count beyond the list capacity
  CNT_SINGULAR,
  CNT_RELAXED,
  CNT_NONFINITE,
  CNT_HMAX_OUT_BITS,   // max solved h as double bits
  CNT_COUNT
};

template <class R>
struct State {
  int64_t n;
  int G;              // cells per side
  double box, ell_d;  // box side and cell side (FP64)
  R ell;              // cell side in Real
  // cell list
  const uint32_t* perm;        // sorted -> caller index
  const uint32_t* keys;        // sorted cell keys
  const uint32_t* cell_start;  // [G^3 + 1]
  // sorted particle data
  R4<R>* pos4;  // (xi_x, xi_y, xi_z, 1/h)
  R4<R>* vel4;  // (v_x, v_y, v_z, V)
  R* mass;
  R* uu;
  R* hbuf;      // h (in: input or guess)
  R* Vbuf;
  R4<R>* st4;   // (rho, P, c, den) with den = sum V_j^2 W^R_ij
  R4<R>* gv4;   // 3 per particle: grad v rows, then (gv_22, relaxed, 0, 0)
  R4<R>* kc4;   // 4 per particle: packed corrected-kernel coefficients
  R* mom;       // [40][n] moments kept for the adjoint (may be null)
  // neighbour list (SELL, slices of 64)
  uint32_t* nlist;
  int* ng;      // gather entries (r < h_i), stored from slot 0 upwards
  int* ns;      // scatter-only entries (h_i <= r < h_j), from slot cap-1 down
  int list_cap;
  // candidates within rcap of each particle (SELL, slices of 64):
  // packed entries as in the neighbour list, and (r, m_j/m_i) pairs
  uint32_t* cand;
  R* scr;
  int* ccnt;
  int scr_cap;
  R rcap;
  unsigned long long* cnt;
  // parameters
  double n_h3, gamma, alpha, beta, eps2, dt_relax, rtol;
  int max_iter;
};

// Decoded cell coordinates are packed 10 bits per axis (G <= 1024).
__device__ inline void cell_coords(uint32_t key, int G, int& cx, int& cy, int& cz) {
  cx = (int)(key % (uint32_t)G);
  uint32_t t = key / (uint32_t)G;
  cy = (int)(t % (uint32_t)G);
  cz = (int)(t / (uint32_t)G);
}

__device__ inline int wrap_cell(int c, int G) { return c < 0 ? c + G : (c >= G ? c - G : c); }

// Calls f(j, code) for every particle j of the 27 stencil cells around the
// cell of key, in a fixed order (dz, dy, dx; then sorted order in a cell).
template <class R, class F>
__device__ inline void for_each_candidate(const State<R>& S, uint32_t key, F&& f) {
  int cx, cy, cz;
  cell_coords(key, S.G, cx, cy, cz);
  for (int dz = -1; dz <= 1; ++dz) {
    const int z = wrap_cell(cz + dz, S.G);
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = wrap_cell(cy + dy, S.G);
      for (int dx = -1; dx <= 1; ++dx) {
        const int xx = wrap_cell(cx + dx, S.G);
        const uint32_t c = ((uint32_t)z * S.G + (uint32_t)y) * S.G + (uint32_t)xx;
        const uint32_t code = (uint32_t)(9 * (dz + 1) + 3 * (dy + 1) + (dx + 1));
        const uint32_t b = S.cell_start[c];
        uint32_t e = S.cell_start[c + 1];
        if (e > (uint32_t)S.n) e = (uint32_t)S.n;
        for (uint32_t j = b; j < e; ++j) f(j, code);
      }
    }
  }
}

}  // namespace crk
