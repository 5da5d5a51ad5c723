// Small device helpers shared by the kernel translation units.
#pragma once
#include "pitmg_internal.h"

namespace pitmg {

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Value of the interpolated coarse vector (one node-type segment of nc coarse
// steps, width p) at fine step k (1-based), component i.  Variant 0 follows
// the printed transfer: fine step 2m-1 takes coarse step m, fine step 2m the
// mean of coarse steps m and m+1, with the missing step nc+1 replaced by nc.
// Variant 1 aligns coarse step m with fine step 2m and averages m-1, m into
// fine step 2m-1 (coarse step 0 is zero).
__device__ __forceinline__ double interp_node(const double* __restrict__ seg, int nc, int p,
                                              int k, int i, int variant) {
  if (variant == 0) {
    if (k & 1) return seg[(long long)((k + 1) / 2 - 1) * p + i];
    const int m = k / 2, m2 = m < nc ? m + 1 : nc;
    return 0.5 * (seg[(long long)(m - 1) * p + i] + seg[(long long)(m2 - 1) * p + i]);
  }
  if (!(k & 1)) return seg[(long long)(k / 2 - 1) * p + i];
  const int m = (k + 1) / 2;
  const double a = seg[(long long)(m - 1) * p + i];
  const double b = m >= 2 ? seg[(long long)(m - 2) * p + i] : 0.0;
  return 0.5 * (a + b);
}

}  // namespace pitmg
