// Truncation rule of Algorithm 1 (with the max-rank modification (1)) on the
// eigenvalues of the Gram matrix of an unfolding; the eigensolver itself is
// in qtt_syev.hpp.
#pragma once

#include "qtt_internal.hpp"
#include "qtt_syev.hpp"

namespace qtt {

// Algorithm 1's rule on the sorted eigenvalues of the Gram matrix: smallest
// r >= 1 with sum_{i >= r} lam_i <= tau2 (tails summed from the small end),
// then min(r, cap).  *over is set when the eps-rank exceeded cap.
__device__ inline int truncation_rank_dev(const double* lam, int E, double tau2, int cap,
                                          int* over) {
  double tail = 0.0;
  int r = E;
  for (int i = E - 1; i >= 1; --i) {
    const double l = lam[i] > 0.0 ? lam[i] : 0.0;
    const double t2 = tail + l;
    if (t2 <= tau2) {
      tail = t2;
      r = i;
    } else {
      break;
    }
  }
  if (r < 1) r = 1;
  *over = r > cap;
  return r < cap ? r : cap;
}

}  // namespace qtt
