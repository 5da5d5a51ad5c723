// Dense P x P FP64 products for one work-group of 512 threads on the matrix
// cores (v_mfma_f64_16x16x4f64), P = 16 NT <= 128:
//
//     C = alpha op(A) op(B),   op(M) = M or M^T,
//
// with K-panels of 32 columns of op(A) and 32 rows of op(B) staged in LDS
// through coalesced loads (a row segment of 32 or a column segment of P
// values per group of threads, depending on the operand's layout), and each
// wave accumulating its 16x16 tiles of C in registers.  Lane l supplies
// op(A)[I0 + l%16][k0 + l/16] and op(B)[k0 + l/16][J0 + l%16]; element i of
// its result is C[I0 + l/16 + 4i][J0 + l%16].
#pragma once
#include "pitmg_internal.h"

namespace pitmg {

// One step of a 16x16 product with K = 4 on the matrix cores in the element
// type's arithmetic.  Lane l supplies A[l%16][l/16] and B[l/16][l%16];
// element i of its result is C[row(l/16, i)][l%16] (the FP64 and FP32
// instructions lay rows out differently).
template <class T>
struct Mfma4;
template <>
struct Mfma4<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 step(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int group, int i) { return group + 4 * i; }
};
template <>
struct Mfma4<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 step(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int group, int i) { return 4 * group + i; }
};

constexpr int kGemmThreads = 512;
constexpr int kGemmPanel = 32;

// LDS doubles wg_gemm needs for P x P operands.
__host__ __device__ constexpr int wg_gemm_lds_doubles(int P) {
  return P * (kGemmPanel + 1) + kGemmPanel * (P + 1);
}

template <int NT, bool TA, bool TB>
__device__ void wg_gemm(const double* __restrict__ A, long long lda,
                        const double* __restrict__ B, long long ldb, double alpha,
                        double* __restrict__ C, long long ldc, double* lds) {
  typedef double f64x4 __attribute__((ext_vector_type(4)));
  constexpr int P = 16 * NT;
  constexpr int kTiles = NT * NT;
  constexpr int kWaves = kGemmThreads / 64;
  constexpr int kMine = (kTiles + kWaves - 1) / kWaves;
  double* As = lds;                                      // [P][33]
  double* Bs = lds + P * (kGemmPanel + 1);               // [32][P+1]
  const int tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  const int r = lane & 15, g = lane >> 4;
  f64x4 acc[kMine];
#pragma unroll
  for (int m = 0; m < kMine; ++m) acc[m] = f64x4{0, 0, 0, 0};
  for (int k0 = 0; k0 < P; k0 += kGemmPanel) {
    __syncthreads();
    for (int e = tid; e < P * kGemmPanel; e += kGemmThreads) {
      if (!TA) {                                         // A row-major: rows of 32
        const int i = e / kGemmPanel, kk = e % kGemmPanel;
        As[i * (kGemmPanel + 1) + kk] = A[(long long)i * lda + k0 + kk];
      } else {                                           // A^T: columns of P
        const int kk = e / P, i = e % P;
        As[i * (kGemmPanel + 1) + kk] = A[(long long)(k0 + kk) * lda + i];
      }
      if (!TB) {                                         // B row-major: rows of P
        const int kk = e / P, j = e % P;
        Bs[kk * (P + 1) + j] = B[(long long)(k0 + kk) * ldb + j];
      } else {                                           // B^T: rows of 32
        const int j = e / kGemmPanel, kk = e % kGemmPanel;
        Bs[kk * (P + 1) + j] = B[(long long)j * ldb + k0 + kk];
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kMine; ++m) {
      const int t = w + m * kWaves;
      if (t < kTiles) {
        const int I = t / NT, J = t % NT;
        const double* Ar = As + (16 * I + r) * (kGemmPanel + 1);
        const double* Bc = Bs + 16 * J + r;
#pragma unroll
        for (int s = 0; s < kGemmPanel / 4; ++s)
          acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ar[4 * s + g],
                                                        Bc[(4 * s + g) * (P + 1)], acc[m], 0, 0,
                                                        0);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < kMine; ++m) {
    const int t = w + m * kWaves;
    if (t < kTiles) {
      const int I = t / NT, J = t % NT;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        C[(long long)(16 * I + g + 4 * i) * ldc + 16 * J + r] = alpha * acc[m][i];
    }
  }
}

// A 128 x 128 block of a product for one work-group of 512 threads, in the
// element type's arithmetic, accumulated in registers over any number of
// calls (K a multiple of 32 per call):
//
//     acc += op(A) op(B),   op(A): 128 x K,  op(B): K x 128,
//
// with K-panels of op(A) (128 x 32) and op(B) (32 x 128) staged in LDS
// through coalesced loads.  Wave w holds the eight 16x16 tiles of tile
// column w, so each B operand it reads serves eight matrix-core steps.
// Every call starts with a barrier, so consecutive calls may reuse the
// staging area and read what an earlier store() of the work-group wrote;
// a store() may overwrite the operands of the call before it (all of that
// call's global reads precede its last barrier).
template <class T>
struct Gemm128 {
  typedef typename Mfma4<T>::v4 v4;
  static constexpr int kPadA = kGemmPanel + 1, kPadB = 128 + 1;
  static constexpr int kLdsElems = 128 * kPadA + kGemmPanel * kPadB;
  v4 acc[8];

  __device__ void zero() {
#pragma unroll
    for (int m = 0; m < 8; ++m) acc[m] = v4{0, 0, 0, 0};
  }

  template <bool TA, bool TB>
  __device__ void mul(const T* __restrict__ A, long long lda, const T* __restrict__ B,
                      long long ldb, int K, T* lds) {
    T* As = lds;                                  // [128][33]
    T* Bs = lds + 128 * kPadA;                    // [32][129]
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int r = lane & 15, g = lane >> 4;
    for (int k0 = 0; k0 < K; k0 += kGemmPanel) {
      __syncthreads();
      for (int e = tid; e < 128 * kGemmPanel; e += kGemmThreads) {
        if (!TA) {                                // rows of 32
          const int i = e / kGemmPanel, kk = e % kGemmPanel;
          As[i * kPadA + kk] = A[(long long)i * lda + k0 + kk];
        } else {                                  // columns of 128
          const int kk = e / 128, i = e % 128;
          As[i * kPadA + kk] = A[(long long)(k0 + kk) * lda + i];
        }
        if (!TB) {
          const int kk = e / 128, j = e % 128;
          Bs[kk * kPadB + j] = B[(long long)(k0 + kk) * ldb + j];
        } else {
          const int j = e / kGemmPanel, kk = e % kGemmPanel;
          Bs[kk * kPadB + j] = B[(long long)j * ldb + k0 + kk];
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < kGemmPanel / 4; ++s) {
        const T b = Bs[(4 * s + g) * kPadB + 16 * w + r];
#pragma unroll
        for (int m = 0; m < 8; ++m)
          acc[m] = Mfma4<T>::step(As[(16 * m + r) * kPadA + 4 * s + g], b, acc[m]);
      }
    }
  }

  // C = alpha acc + beta C (C is not read when beta is 0)
  __device__ void store(T* C, long long ldc, T alpha, T beta) const {
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        T* c = C + (long long)(16 * m + Mfma4<T>::row(g, i)) * ldc + 16 * w + r;
        const T v = alpha * acc[m][i];
        *c = beta != T(0) ? v + beta * *c : v;
      }
  }
};

}  // namespace pitmg
