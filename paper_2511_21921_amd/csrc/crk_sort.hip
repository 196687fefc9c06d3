// Deterministic device-wide primitives for building the cell list:
// an exclusive prefix sum and a stable LSD radix sort of (key, value) pairs.
// Both are written for 64-wide wavefronts: the sort ranks equal digits
// inside a wave with eight ballots (wave multisplit), so the output order
// never depends on atomic ordering and repeated runs are bitwise equal.
#include "crk_internal.h"

namespace crk {
namespace {

constexpr int kItems = 8;                  // items per thread
constexpr int kTile = kBlock * kItems;     // 2048 items per block
constexpr int kWaves = kBlock / 64;

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t& total) {
  __shared__ uint32_t wsum[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    uint32_t s = wsum[k];
    off += (k < w) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return off + inc - v;
}

__global__ void __launch_bounds__(kBlock) k_chunk_sums(const uint32_t* __restrict__ in, int64_t n,
                                                       uint32_t* __restrict__ part) {
  const int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x * kItems;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k)
    if (base + k < n) s += in[base + k];
  uint32_t tot;
  block_excl_scan(s, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// One block scans the chunk sums in place (exclusive), 2048 at a time.
__global__ void __launch_bounds__(kBlock) k_scan_parts(uint32_t* part, int64_t m) {
  uint32_t carry = 0;
  for (int64_t base = 0; base < m; base += kTile) {
    uint32_t v[kItems], s = 0;
    const int64_t my = base + threadIdx.x * kItems;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      v[k] = (my + k < m) ? part[my + k] : 0u;
      s += v[k];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(s, tot) + carry;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      if (my + k < m) part[my + k] = off;
      off += v[k];
    }
    carry += tot;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBlock) k_scan_apply(const uint32_t* in, uint32_t* out,
                                                       int64_t n,
                                                       const uint32_t* __restrict__ part) {
  const int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x * kItems;
  uint32_t v[kItems], s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t off = block_excl_scan(s, tot) + part[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (base + k < n) out[base + k] = off;
    off += v[k];
  }
}

// ------------------------------------------------------------ radix sort --

__global__ void __launch_bounds__(kBlock) k_radix_hist(const uint32_t* __restrict__ keys,
                                                       int64_t n, int shift, int64_t nblk,
                                                       uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    int64_t i = (int64_t)blockIdx.x * kTile + r * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(kBlock) k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t n, int shift, int64_t nblk,
    const uint32_t* __restrict__ offs) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[kWaves][256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  base[t] = offs[(int64_t)t * nblk + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kItems; ++r) {
#pragma unroll
    for (int k = 0; k < kWaves; ++k) wcnt[k][t] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kTile + r * kBlock + t;
    const bool valid = i < n;
    uint32_t key = valid ? kin[i] : 0u;
    uint32_t val = valid ? vin[i] : 0u;
    uint32_t d = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t rank = __popcll(peers & lt);
    if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    // thread t owns digit t: exclusive prefix over the waves of this round
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      uint32_t c = wcnt[k][t];
      wcnt[k][t] = run;
      run += c;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = base[d] + wcnt[w][d] + rank;
      if ((int64_t)pos < n) {  // always true for a consistent histogram
        kout[pos] = key;
        vout[pos] = val;
      }
    }
    __syncthreads();
    base[t] += run;
  }
}

}  // namespace

int64_t scan_tmp_words(int64_t n) { return (n + kTile - 1) / kTile + 1; }

hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t m = (n + kTile - 1) / kTile;
  hipLaunchKernelGGL(k_chunk_sums, dim3((unsigned)m), dim3(kBlock), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kBlock), 0, s, tmp, m);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)m), dim3(kBlock), 0, s, in, out, n,
                     (const uint32_t*)tmp);
  return hipGetLastError();
}

int64_t radix_tmp_words(int64_t n) {
  const int64_t nblk = (n + kTile - 1) / kTile;
  return 256 * nblk + scan_tmp_words(256 * nblk);
}

hipError_t radix_sort_pairs(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                            uint32_t* vals_b, int64_t n, int key_bits, uint32_t* tmp,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nblk = (n + kTile - 1) / kTile;
  uint32_t* hist = tmp;
  uint32_t* stmp = tmp + 256 * nblk;
  uint32_t *ki = keys_a, *vi = vals_a, *ko = keys_b, *vo = vals_b;
  int passes = 0;
  for (int shift = 0; shift < key_bits; shift += 8, ++passes) {
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nblk), dim3(kBlock), 0, s,
                       (const uint32_t*)ki, n, shift, nblk, hist);
    hipError_t e = exclusive_scan_u32(hist, hist, 256 * nblk, stmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nblk), dim3(kBlock), 0, s,
                       (const uint32_t*)ki, (const uint32_t*)vi, ko, vo, n, shift, nblk,
                       (const uint32_t*)hist);
    uint32_t* t1 = ki; ki = ko; ko = t1;
    uint32_t* t2 = vi; vi = vo; vo = t2;
  }
  if (passes & 1) {
    hipError_t e = hipMemcpyAsync(keys_a, ki, n * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(vals_a, vi, n * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace crk
