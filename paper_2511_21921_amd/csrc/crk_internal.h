// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crk {

constexpr int kBlock = 256;  // threads per block for the particle kernels

inline unsigned grid_for(int64_t n, int block = kBlock) {
  return (unsigned)((n + block - 1) / block);
}

// ---- crk_sort.hip --------------------------------------------------------
// Exclusive prefix sum of n uint32 values (out may alias in). tmp must hold
// scan_tmp_words(n) uint32.
int64_t scan_tmp_words(int64_t n);
hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp,
                              hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by the low key_bits bits of
// key. Ping-pongs between the a and b buffers; the result ends in a (the
// function copies back when the pass count is odd). tmp must hold
// radix_tmp_words(n) uint32.
int64_t radix_tmp_words(int64_t n);
hipError_t radix_sort_pairs(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                            uint32_t* vals_b, int64_t n, int key_bits, uint32_t* tmp,
                            hipStream_t s);

}  // namespace crk
