// Factorisation of the time-step blocks on the matrix cores, every level in
// one launch: for each block k of each level (p = 16 NT <= 128, FP64)
//
//     S_k = N_k N_k^T + Z~_k Z~_k^T,   S_k = G_k G_k^T (Cholesky),   G_k^{-1},
//
// written row-major into the factor buffer with zeros above the diagonal.
// (Block algebra: pitmg_kernels.hip; S_k is positive definite when N_k is
// invertible, Thm. 1.)  One work-group of 512 threads per block keeps S_k and
// then G_k^{-1} in LDS as 16x16 tiles of the lower triangle and works tile by
// tile with v_mfma_f64_16x16x4f64:
//
//   1. S = X X^T, X = [N_k | Z~_k]: column panels of X staged in LDS through
//      coalesced row loads, each wave accumulating its lower tiles in
//      registers;
//   2. right-looking blocked Cholesky: factor the diagonal tile (one wave),
//      solve the panel below it (one thread per row), update the trailing
//      tiles S_IJ -= G_IK G_JK^T (matrix cores);
//   3. blocked inverse X = G^{-1}: the diagonal tiles' inverses (a lane per
//      column), then the off-diagonal tiles by diagonals,
//      X_IJ = -X_II sum_{K=J}^{I-1} G_IK X_KJ (matrix cores);
//   4. X to global memory, row-major, zero above the diagonal.
//
// Tiles are stored row-major with the column index rotated by the row
// ((c + r) mod 16), so a wave's operand reads (16 rows at one column, or 16
// columns of one row) fall in distinct banks.
#include "pitmg_internal.h"
#include "pitmg_device.h"

namespace pitmg {
namespace {

constexpr int kFacThreads = 512;
constexpr int kFacWaves = kFacThreads / kWave;
constexpr int kPanel = 32;                     // columns of X staged per pass

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mfma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Element (r, c) of a 16x16 tile.
__device__ __forceinline__ int tix(int r, int c) { return r * 16 + ((c + r) & 15); }

template <int NT>
struct Tiles {
  static constexpr int P = 16 * NT;
  static constexpr int kTiles = NT * (NT + 1) / 2;       // lower tiles (I >= J)
  __device__ static int id(int I, int J) { return I * (I + 1) / 2 + J; }
};

}  // namespace

template <int NT>
__global__ __launch_bounds__(kFacThreads, 1) void k_factor_mfma(FactorBatch F, int* fail) {
  using TL = Tiles<NT>;
  constexpr int P = TL::P;
  extern __shared__ double lds[];
  double* St = lds;                                     // S, then G: kTiles tiles
  double* Xt = lds + TL::kTiles * 256;                  // G^{-1} tiles
  double* stage = Xt;                                   // X panel (before step 3)
  __shared__ int sfail;
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const int r = lane & 15, g = lane >> 4;

  // which level and block this work-group factors
  int lev = 0;
  while (lev + 1 < F.nlev && (int)blockIdx.x >= F.start[lev + 1]) ++lev;
  const int k = blockIdx.x - F.start[lev];
  const int q = F.q;
  const double* __restrict__ Nk = F.N[lev] + (long long)k * F.sN;
  const double* __restrict__ Zk = F.Z[lev] + (long long)k * F.sZ;
  double* __restrict__ Gk = F.Gi[lev] + (long long)k * P * P;
  if (tid == 0) sfail = 0;

  // ---- 1. S = X X^T --------------------------------------------------------
  // lower tiles t = w, w + 8, ... of this wave, numbered row by row
  constexpr int kMine = (TL::kTiles + kFacWaves - 1) / kFacWaves;
  f64x4 acc[kMine];
  int tI[kMine], tJ[kMine];
#pragma unroll
  for (int m = 0; m < kMine; ++m) {
    acc[m] = f64x4{0, 0, 0, 0};
    int t = w + m * kFacWaves, I = 0;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    tI[m] = I;
    tJ[m] = t - I * (I + 1) / 2;
  }
  const int K = P + q;
  for (int c0 = 0; c0 < K; c0 += kPanel) {
    __syncthreads();
    // stage X[:, c0 .. c0+31] as [row][32] (zero past the last column)
    for (int e = tid; e < P * kPanel; e += kFacThreads) {
      const int i = e / kPanel, c = c0 + e % kPanel;
      double v = 0.0;
      if (c < P) v = Nk[(long long)i * P + c];
      else if (c < K) v = Zk[(long long)i * q + (c - P)];
      stage[i * (kPanel + 1) + e % kPanel] = v;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kMine; ++m) {
      if (w + m * kFacWaves < TL::kTiles) {
        const double* A = stage + (16 * tI[m] + r) * (kPanel + 1);
        const double* B = stage + (16 * tJ[m] + r) * (kPanel + 1);
#pragma unroll
        for (int s = 0; s < kPanel / 4; ++s) acc[m] = mfma(A[4 * s + g], B[4 * s + g], acc[m]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < kMine; ++m) {
    if (w + m * kFacWaves < TL::kTiles) {
      double* T = St + TL::id(tI[m], tJ[m]) * 256;
#pragma unroll
      for (int i = 0; i < 4; ++i) T[tix(g + 4 * i, r)] = acc[m][i];
    }
  }
  __syncthreads();

  // ---- 2. blocked Cholesky, right-looking ---------------------------------
  for (int Kt = 0; Kt < NT; ++Kt) {
    double* D = St + TL::id(Kt, Kt) * 256;
    if (w == 0) {
      // unblocked Cholesky of the diagonal tile by one wave (lanes in order)
      for (int j = 0; j < 16; ++j) {
        const double d = D[tix(j, j)];
        if (!(d > 0.0) || !isfinite(d)) {
          if (lane == 0) sfail = 1;
          break;                                         // uniform in the wave
        }
        const double s = sqrt(d), inv = 1.0 / s;
        if (lane > j && lane < 16) D[tix(lane, j)] *= inv;
        if (lane == 0) D[tix(j, j)] = s;
        // rank-1 update of the trailing part of the tile (rows, columns > j)
        for (int e = lane; e < 256; e += kWave) {
          const int i = e >> 4, c = e & 15;
          if (i > j && c > j && c <= i) D[tix(i, c)] -= D[tix(i, j)] * D[tix(c, j)];
        }
      }
    }
    __syncthreads();
    if (sfail) {
      if (tid == 0) atomicMin(fail, (F.level0 + lev) << 20 | k);
      return;                                            // uniform: after the barrier
    }
    // panel: G_IK = S_IK G_KK^{-T}, one thread per row of the tiles below
    {
      const int row = tid;                               // row within the panel
      const int I = Kt + 1 + row / 16;
      if (I < NT) {
        double* T = St + TL::id(I, Kt) * 256;
        const int rr = row & 15;
        double x[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          double v = T[tix(rr, c)];
#pragma unroll
          for (int j = 0; j < c; ++j) v -= x[j] * D[tix(c, j)];
          x[c] = v / D[tix(c, c)];
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) T[tix(rr, c)] = x[c];
      }
    }
    __syncthreads();
    // trailing update S_IJ -= G_IK G_JK^T, Kt < J <= I
    const int m = NT - 1 - Kt;
    const int ntr = m * (m + 1) / 2;
    for (int t = w; t < ntr; t += kFacWaves) {
      int ii = 0;
      while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
      const int I = Kt + 1 + ii, J = Kt + 1 + (t - ii * (ii + 1) / 2);
      double* C = St + TL::id(I, J) * 256;
      const double* A = St + TL::id(I, Kt) * 256;
      const double* B = St + TL::id(J, Kt) * 256;
      f64x4 c4;
#pragma unroll
      for (int i = 0; i < 4; ++i) c4[i] = C[tix(g + 4 * i, r)];
#pragma unroll
      for (int s = 0; s < 4; ++s) c4 = mfma(-A[tix(r, 4 * s + g)], B[tix(r, 4 * s + g)], c4);
#pragma unroll
      for (int i = 0; i < 4; ++i) C[tix(g + 4 * i, r)] = c4[i];
    }
    __syncthreads();
  }

  // ---- 3. X = G^{-1}, blocked ---------------------------------------------
  // diagonal tiles: column j of X_KK solves G_KK x = e_j (lane j of a wave)
  for (int Kt = w; Kt < NT; Kt += kFacWaves) {
    if (lane < 16) {
      const double* D = St + TL::id(Kt, Kt) * 256;
      double* X = Xt + TL::id(Kt, Kt) * 256;
      const int j = lane;
      double x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double v = i == j ? 1.0 : 0.0;
#pragma unroll
        for (int c = 0; c < i; ++c) v -= D[tix(i, c)] * x[c];
        x[i] = i < j ? 0.0 : v / D[tix(i, i)];
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) X[tix(i, j)] = x[i];
    }
  }
  __syncthreads();
  // off-diagonal tiles by diagonals d = I - J
  for (int d = 1; d < NT; ++d) {
    for (int J = w; J + d < NT; J += kFacWaves) {
      const int I = J + d;
      f64x4 t4 = f64x4{0, 0, 0, 0};
      for (int Kt = J; Kt < I; ++Kt) {
        const double* A = St + TL::id(I, Kt) * 256;      // G_IK
        const double* B = Xt + TL::id(Kt, J) * 256;      // X_KJ
#pragma unroll
        for (int s = 0; s < 4; ++s) t4 = mfma(A[tix(r, 4 * s + g)], B[tix(4 * s + g, r)], t4);
      }
      // X_IJ = -X_II T: T's accumulator element s is its row 4s + g, column
      // r, which is the B operand of the k-chunk s
      const double* A = Xt + TL::id(I, I) * 256;
      f64x4 x4 = f64x4{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) x4 = mfma(-A[tix(r, 4 * s + g)], t4[s], x4);
      double* X = Xt + TL::id(I, J) * 256;
#pragma unroll
      for (int i = 0; i < 4; ++i) X[tix(g + 4 * i, r)] = x4[i];
    }
    __syncthreads();
  }

  // ---- 4. G^{-1} to global memory, zero above the diagonal ----------------
  for (int e = tid; e < P * P; e += kFacThreads) {
    const int i = e / P, j = e % P;
    const int I = i >> 4, J = j >> 4;
    double v = 0.0;
    if (J < I) v = Xt[TL::id(I, J) * 256 + tix(i & 15, j & 15)];
    else if (J == I && (j & 15) <= (i & 15)) v = Xt[TL::id(I, I) * 256 + tix(i & 15, j & 15)];
    Gk[e] = v;
  }
}

bool factor_mfma_supported(int p) { return p == 64 || p == 128; }

size_t factor_mfma_lds(int p) {
  const int nt = p / 16;
  return (size_t)nt * (nt + 1) * 256 * sizeof(double);   // S tiles + X tiles
}

hipError_t launch_factor_mfma(const FactorBatch& F, int* fail, hipStream_t s) {
  const int total = F.start[F.nlev];
  if (total <= 0) return hipSuccess;
  const size_t lds = factor_mfma_lds(F.p);
  if (F.p == 128) {
    hipError_t e = hipFuncSetAttribute((const void*)k_factor_mfma<8>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return launch_k(k_factor_mfma<8>, dim3(total), dim3(kFacThreads), lds, s, F, fail);
  }
  if (F.p == 64) {
    hipError_t e = hipFuncSetAttribute((const void*)k_factor_mfma<4>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return launch_k(k_factor_mfma<4>, dim3(total), dim3(kFacThreads), lds, s, F, fail);
  }
  return hipErrorInvalidValue;
}

}  // namespace pitmg
