// The Gaussian test matrix of the randomised range finder (Algorithm 4):
// Omega[row][col] of sweep step k is one standard normal from the
// counter-based generator Philox-4x32-10 (Salmon, Moraes, Dror and Shaw,
// SC 2011) with counter (row, col, k, 0) and key (seed low, seed high),
// through the Box-Muller transform of its first two output words.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtt {

// ----------------------------------------------------------- Philox 4x32
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ double omega_entry(long long row, int col, int step, uint32_t k0,
                                              uint32_t k1) {
  uint32_t c[4] = {(uint32_t)row, (uint32_t)col, (uint32_t)step, 0u};
  philox4x32_10(c, k0, k1);
  const double u1 = ((double)c[0] + 0.5) * 0x1p-32;
  const double u2 = ((double)c[1] + 0.5) * 0x1p-32;
  return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

}  // namespace qtt
