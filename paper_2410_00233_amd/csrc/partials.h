// Device helper for the consumers of the Kronecker apply's partial images.
#pragma once
#include <hip/hip_runtime.h>

namespace kpsb {

// v + P[g0] + P[g0 + 1] + ... + P[ng - 1] (P[g] at p + g NN), added one by one
// in that order, with the loads of up to 8 partials issued before their adds
// (a loop that waits for each load before the next spends one memory latency
// per partial; the adds, and so the bits, are those of the plain loop).
__device__ __forceinline__ double add_partials_in_order(double v, const double* __restrict__ p,
                                                        int g0, int ng, long NN) {
  for (int g = g0; g < ng; g += 8) {
    const int m = ng - g;
    double t[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) t[j] = j < m ? p[(long)(g + j) * NN] : 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < m) v += t[j];
  }
  return v;
}

}  // namespace kpsb
