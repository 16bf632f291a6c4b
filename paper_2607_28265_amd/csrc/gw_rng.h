// Counter-based random numbers shared by the sampler kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gw {

// Philox4x64-10 (Salmon, Moraes, Dror & Shaw 2011): the 4-word counter c is
// replaced by its output under the key (k0, k1).
__device__ inline void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

// A 64-bit output word mapped to (0, 1): ((w >> 11) + 1/2) 2^-53.
__device__ inline double philox_unit(uint64_t w) { return ((double)(w >> 11) + 0.5) * 1.1102230246251565404e-16; }

}  // namespace gw
