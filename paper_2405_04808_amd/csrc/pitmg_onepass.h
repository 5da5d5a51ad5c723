// One pass of a 512-thread work-group over a row-major P x P time-step block
// (P = 64 MB): both its row product and its column product from the same
// loads.  Thread (r, c) = (tid / 32, tid % 32) takes row 16 i + r of row
// panel i and the columns 2c + 64m + e (m < MB, e < 2: 16-byte loads, a
// half-wave reading 512 contiguous bytes).  Each entry serves
//   srow[row] = (M x)_row   (summed over the 32 lanes of the row) and
//   red[w][j] += M_row,j y_row  (column partials, summed over the rows of
//                                 the panel's two rows per wave, lane ^ 32),
// so that (M^T y)_j = sum over the 8 waves of red[w][j], which the caller
// forms after a barrier, in a fixed order.  The next panel's loads are
// issued before the current one is used.
#pragma once
#include "pitmg_internal.h"
#include "pitmg_device.h"

namespace pitmg {

constexpr int kOnePassThreads = 512;
constexpr int kOnePassWaves = kOnePassThreads / kWave;

// x: the row product's vector in global memory (16-byte aligned, P values);
// sy: the column product's vector in LDS, ready (after a barrier) before
// the call; srow, red: LDS outputs ([P], [8][P]).  All threads call it.
template <int MB>
__device__ __forceinline__ void onepass_products(const double* __restrict__ M,
                                                 const double* __restrict__ x, const double* sy,
                                                 double* srow, double (*red)[64 * MB]) {
  constexpr int P = 64 * MB, CT = 2 * MB, NP = P / 16;
  static_assert(NP % 2 == 0, "panels in pairs");
  const int tid = threadIdx.x, r = tid / 32, c = tid % 32, w = tid / kWave;
  double xu[CT];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const double2 v = *reinterpret_cast<const double2*>(x + 2 * c + 64 * m);
    xu[2 * m] = v.x;
    xu[2 * m + 1] = v.y;
  }
  double acc[CT];
#pragma unroll
  for (int t = 0; t < CT; ++t) acc[t] = 0.0;
  auto load = [&](int pn, double (&dst)[CT]) {
    const double* row = M + (long long)(16 * pn + r) * P + 2 * c;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const double2 v = *reinterpret_cast<const double2*>(row + 64 * m);
      dst[2 * m] = v.x;
      dst[2 * m + 1] = v.y;
    }
  };
  auto use = [&](int pn, const double (&cur)[CT]) {
    const int row = 16 * pn + r;
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < CT; ++t) s += cur[t] * xu[t];
    s = xor16_sum(row_sum16(s));                 // over the 32 lanes of the row
    if (c == 0) srow[row] = s;
    const double yr = sy[row];
#pragma unroll
    for (int t = 0; t < CT; ++t) acc[t] += cur[t] * yr;
  };
  double A[CT], B[CT];
  load(0, A);
#pragma unroll 1
  for (int pn = 0; pn < NP; pn += 2) {
    load(pn + 1, B);
    use(pn, A);
    if (pn + 2 < NP) load(pn + 2, A);
    use(pn + 1, B);
  }
#pragma unroll
  for (int t = 0; t < CT; ++t) acc[t] = xor32_sum(acc[t]);
  if (r % 2 == 0) {
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      red[w][2 * c + 64 * m] = acc[2 * m];
      red[w][2 * c + 64 * m + 1] = acc[2 * m + 1];
    }
  }
}

}  // namespace pitmg
