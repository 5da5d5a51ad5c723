// Factorisation of the time-step blocks on the matrix cores, every level of
// one element type in one launch: for each block k of each level
//
//     S_k = N_k N_k^T + Z~_k Z~_k^T,   S_k = G_k G_k^T (Cholesky),   G_k^{-1},
//
// written row-major into the factor buffer with zeros above the diagonal.
// (Block algebra: pitmg_kernels.hip; S_k is positive definite when N_k is
// invertible, Thm. 1.)  FP64 blocks use v_mfma_f64_16x16x4f64, FP32 blocks
// (the FP32 smoother's levels) v_mfma_f32_16x16x4f32.  One work-group of 512
// threads per block.
//
// p = 16 NT <= 128 (k_factor_mfma): S_k, then G_k, then G_k^{-1} stay in one
// LDS array of 16x16 tiles of the lower triangle (73.7 KB for p = 128 in
// FP64, so two work-groups share a CU and one's sequential pivot steps
// overlap the other's), worked on tile by tile:
//
//   1. S = X X^T, X = [N_k | Z~_k]: column panels of X staged in the same
//      LDS array through coalesced row loads, each wave accumulating its
//      lower tiles in registers;
//   2. right-looking blocked Cholesky: factor the diagonal tile (one wave),
//      solve the panel below it (one thread per row), update the trailing
//      tiles S_IJ -= G_IK G_JK^T (matrix cores);
//   3. blocked inverse X = G^{-1} in place: the diagonal tiles' inverses (a
//      lane per column), then the off-diagonal tiles by tile columns from
//      the right, X_IJ = -(sum_{K=J+1}^{I} X_IK G_KJ) X_JJ (matrix cores);
//   4. X to global memory, row-major, zero above the diagonal.
//
// p = 128 NB, NB in {2, 4} (k_factor_big): the same algorithm one level up,
// on 128 x 128 super-blocks kept in the factor buffer itself (global
// memory; the block's 0.5-2 MB mostly stays in the caches), each product a
// 128 x 128 matrix-core GEMM of the work-group (Gemm128):
//
//   1. S_IJ = N_I N_J^T + Z~_I Z~_J^T for J <= I (N_I: rows 128I.. of N_k),
//      zeros above;
//   2. for K = 0 .. NB-1: the diagonal super-block through steps 2-3 above
//      in LDS (G_KK and X_KK = G_KK^{-1}), X_KK stored in its place (G_KK is
//      not needed again), the panel G_IK = S_IK X_KK^T, the trailing update
//      S_IJ -= G_IK G_JK^T;
//   3. the inverse in place, super-block column J from right to left and
//      within it I from the bottom up: from X G = I,
//      X_IJ = -(sum_{K=J+1}^{I} X_IK G_KJ) X_JJ, where the sum reads G_KJ
//      only for K <= I, none of which the bottom-up order has overwritten.
//
// Tiles in LDS are stored row-major with the column index rotated by the row
// ((c + r) mod 16), so a wave's operand reads (16 rows at one column, or 16
// columns of one row) fall in distinct banks.
#include "pitmg_internal.h"
#include "pitmg_device.h"
#include "pitmg_mfma.h"

namespace pitmg {
namespace {

constexpr int kFacThreads = 512;
constexpr int kFacWaves = kFacThreads / kWave;
constexpr int kPanel = 32;                     // columns of X staged per pass

// Element (r, c) of a 16x16 tile.
__device__ __forceinline__ int tix(int r, int c) { return r * 16 + ((c + r) & 15); }

template <int NT>
struct Tiles {
  static constexpr int P = 16 * NT;
  static constexpr int kTiles = NT * (NT + 1) / 2;       // lower tiles (I >= J)
  __device__ static int id(int I, int J) { return I * (I + 1) / 2 + J; }
};

// Row of element i of a lane of group g in a matrix-core result tile.
template <class T>
__device__ __forceinline__ int arow(int g, int i) { return Mfma4<T>::row(g, i); }

// Steps 2 and 3 on the lower tiles of a P x P symmetric matrix in St:
// Cholesky in place (St then holds G), then the inverse of G in place (St
// then holds G^{-1}).  Returns false (uniformly, after a barrier) when a
// pivot is not positive.
template <class T, int NT>
__device__ __forceinline__ bool tile_cholesky_inverse(T* St, int* sfail) {
  using TL = Tiles<NT>;
  typedef typename Mfma4<T>::v4 v4;
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const int r = lane & 15, g = lane >> 4;

  // ---- blocked Cholesky, right-looking ------------------------------------
  for (int Kt = 0; Kt < NT; ++Kt) {
    T* D = St + TL::id(Kt, Kt) * 256;
    if (w == 0) {
      // unblocked Cholesky of the diagonal tile by one wave (lanes in order)
      for (int j = 0; j < 16; ++j) {
        const T d = D[tix(j, j)];
        if (!(d > T(0)) || !isfinite(d)) {
          if (lane == 0) *sfail = 1;
          break;                                         // uniform in the wave
        }
        const T s = sqrt(d), inv = T(1) / s;
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
    if (*sfail) return false;                            // uniform: after the barrier
    // panel: G_IK = S_IK G_KK^{-T}, one thread per row of the tiles below
    {
      const int row = tid;                               // row within the panel
      const int I = Kt + 1 + row / 16;
      if (I < NT) {
        T* Tp = St + TL::id(I, Kt) * 256;
        const int rr = row & 15;
        T x[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          T v = Tp[tix(rr, c)];
#pragma unroll
          for (int j = 0; j < c; ++j) v -= x[j] * D[tix(c, j)];
          x[c] = v / D[tix(c, c)];
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) Tp[tix(rr, c)] = x[c];
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
      T* C = St + TL::id(I, J) * 256;
      const T* A = St + TL::id(I, Kt) * 256;
      const T* B = St + TL::id(J, Kt) * 256;
      v4 c4;
#pragma unroll
      for (int i = 0; i < 4; ++i) c4[i] = C[tix(arow<T>(g, i), r)];
#pragma unroll
      for (int s = 0; s < 4; ++s)
        c4 = Mfma4<T>::step(-A[tix(r, 4 * s + g)], B[tix(r, 4 * s + g)], c4);
#pragma unroll
      for (int i = 0; i < 4; ++i) C[tix(arow<T>(g, i), r)] = c4[i];
    }
    __syncthreads();
  }

  // ---- X = G^{-1}, blocked, in place ---------------------------------------
  // diagonal tiles: column j of X_KK solves G_KK x = e_j (lane j of a wave);
  // the wave reads the whole tile before any lane writes its column
  for (int Kt = w; Kt < NT; Kt += kFacWaves) {
    if (lane < 16) {
      T* D = St + TL::id(Kt, Kt) * 256;
      const int j = lane;
      T x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        T v = i == j ? T(1) : T(0);
#pragma unroll
        for (int c = 0; c < i; ++c) v -= D[tix(i, c)] * x[c];
        x[i] = i < j ? T(0) : v / D[tix(i, i)];
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) D[tix(i, j)] = x[i];
    }
  }
  __syncthreads();
  // off-diagonal tiles by tile columns J from the right: from X G = I,
  // X_IJ = -(sum_{K=J+1}^{I} X_IK G_KJ) X_JJ.  The X_IK (K > J) are done, and
  // column J still holds G until all of its tiles have been formed.
  for (int J = NT - 2; J >= 0; --J) {
    const int nI = NT - 1 - J;                           // tiles I = J+1 .. NT-1
    v4 x4 = v4{0, 0, 0, 0};
    const int I = J + 1 + w;
    if (w < nI) {
      // T^T = sum_K G_KJ^T X_IK^T (accumulator: T[r][arow(g, i)])
      v4 t4 = v4{0, 0, 0, 0};
      for (int Kt = J + 1; Kt <= I; ++Kt) {
        const T* A = St + TL::id(Kt, J) * 256;           // G_KJ
        const T* B = St + TL::id(I, Kt) * 256;           // X_IK
#pragma unroll
        for (int s = 0; s < 4; ++s)
          t4 = Mfma4<T>::step(A[tix(4 * s + g, r)], B[tix(r, 4 * s + g)], t4);
      }
      // X_IJ^T = -X_JJ^T T^T with T^T's accumulator as the B operand (element
      // s of the lane is T^T[arow(g, s)][r], so k-chunk s takes the inner
      // indices arow(g, s) of the A operand too)
      const T* X = St + TL::id(J, J) * 256;
#pragma unroll
      for (int s = 0; s < 4; ++s) x4 = Mfma4<T>::step(-X[tix(arow<T>(g, s), r)], t4[s], x4);
    }
    __syncthreads();                                     // column J's G read
    if (w < nI) {
      T* X = St + TL::id(I, J) * 256;
#pragma unroll
      for (int i = 0; i < 4; ++i) X[tix(r, arow<T>(g, i))] = x4[i];
    }
    __syncthreads();
  }
  return true;
}

// The same as a call of its own (k_factor_big keeps its GEMM state in
// registers around it).
template <class T>
__device__ __noinline__ bool tile_cholesky_inverse_call(T* St, int* sfail) {
  return tile_cholesky_inverse<T, 8>(St, sfail);
}

// Which level and block a work-group of a batch launch factors.
template <class T>
__device__ void batch_block(const FactorBatchT<T>& F, int& lev, int& k) {
  lev = 0;
  while (lev + 1 < F.nlev && (int)blockIdx.x >= F.start[lev + 1]) ++lev;
  k = blockIdx.x - F.start[lev];
}

}  // namespace

template <class T, int NT>
__global__ __launch_bounds__(kFacThreads, 4) void k_factor_mfma(FactorBatchT<T> F, int* fail) {
  using TL = Tiles<NT>;
  typedef typename Mfma4<T>::v4 v4;
  constexpr int P = TL::P;
  extern __shared__ double lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  T* St = lds;                                          // S, G, then G^{-1}: kTiles tiles
  T* stage = St;                                        // X panels (step 1, before S)
  __shared__ int sfail;
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const int r = lane & 15, g = lane >> 4;
  int lev, k;
  batch_block(F, lev, k);
  const int q = F.q;
  const T* __restrict__ Nk = F.N[lev] + (long long)k * F.sN;
  const T* __restrict__ Zk = F.Z[lev] + (long long)k * F.sZ;
  T* __restrict__ Gk = F.Gi[lev] + (long long)k * P * P;
  // diagonal Z~: S = N N^T + diag(Zd)^2, the panels of N alone
  const T* __restrict__ zd = (F.zflag && F.zflag[F.level0 + lev]) ? F.Zd[lev] : nullptr;
  if (tid == 0) sfail = 0;

  // ---- 1. S = X X^T --------------------------------------------------------
  // lower tiles t = w, w + 8, ... of this wave, numbered row by row
  constexpr int kMine = (TL::kTiles + kFacWaves - 1) / kFacWaves;
  v4 acc[kMine];
  int tI[kMine], tJ[kMine];
#pragma unroll
  for (int m = 0; m < kMine; ++m) {
    acc[m] = v4{0, 0, 0, 0};
    int t = w + m * kFacWaves, I = 0;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    tI[m] = I;
    tJ[m] = t - I * (I + 1) / 2;
  }
  const int K = zd ? P : P + q;
  for (int c0 = 0; c0 < K; c0 += kPanel) {
    __syncthreads();
    // stage X[:, c0 .. c0+31] as [row][32] (zero past the last column)
    for (int e = tid; e < P * kPanel; e += kFacThreads) {
      const int i = e / kPanel, c = c0 + e % kPanel;
      T v = T(0);
      if (c < P) v = Nk[(long long)i * P + c];
      else if (c < K) v = Zk[(long long)i * q + (c - P)];
      stage[i * (kPanel + 1) + e % kPanel] = v;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kMine; ++m) {
      if (w + m * kFacWaves < TL::kTiles) {
        const T* A = stage + (16 * tI[m] + r) * (kPanel + 1);
        const T* B = stage + (16 * tJ[m] + r) * (kPanel + 1);
#pragma unroll
        for (int s = 0; s < kPanel / 4; ++s)
          acc[m] = Mfma4<T>::step(A[4 * s + g], B[4 * s + g], acc[m]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < kMine; ++m) {
    if (w + m * kFacWaves < TL::kTiles) {
      T* Tp = St + TL::id(tI[m], tJ[m]) * 256;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        T v = acc[m][i];
        if (zd && tI[m] == tJ[m] && arow<T>(g, i) == r) {
          const T z = zd[16 * tI[m] + r];
          v += z * z;
        }
        Tp[tix(arow<T>(g, i), r)] = v;
      }
    }
  }
  __syncthreads();

  // ---- 2-3. Cholesky and inverse ------------------------------------------
  if (!tile_cholesky_inverse<T, NT>(St, &sfail)) {
    if (tid == 0) atomicMin(fail, (F.level0 + lev) << 20 | k);
    return;
  }

  // ---- 4. G^{-1} to global memory, zero above the diagonal ----------------
  for (int e = tid; e < P * P; e += kFacThreads) {
    const int i = e / P, j = e % P;
    const int I = i >> 4, J = j >> 4;
    T v = T(0);
    if (J < I) v = St[TL::id(I, J) * 256 + tix(i & 15, j & 15)];
    else if (J == I && (j & 15) <= (i & 15)) v = St[TL::id(I, I) * 256 + tix(i & 15, j & 15)];
    Gk[e] = v;
  }
}

template <class T>
__global__ __launch_bounds__(kFacThreads, 1) void k_factor_big(FactorBatchT<T> F, int* fail) {
  using TL = Tiles<8>;
  extern __shared__ double lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  T* St = lds;                                          // diagonal super-block, then its inverse
  __shared__ int sfail;
  const int tid = threadIdx.x;
  int lev, k;
  batch_block(F, lev, k);
  const int P = F.p, q = F.q, NB = P / 128;
  const T* __restrict__ Nk = F.N[lev] + (long long)k * F.sN;
  const T* __restrict__ Zk = F.Z[lev] + (long long)k * F.sZ;
  T* __restrict__ Gk = F.Gi[lev] + (long long)k * P * P;
  auto at = [&](int I, int J) { return Gk + (long long)128 * I * P + 128 * J; };
  // diagonal Z~: S = N N^T + diag(Zd)^2, no product with the dense Z~
  const T* __restrict__ zd = (F.zflag && F.zflag[F.level0 + lev]) ? F.Zd[lev] : nullptr;
  if (tid == 0) sfail = 0;
  Gemm128<T> gm;

  // ---- 1. S_IJ = N_I N_J^T + Z~_I Z~_J^T, J <= I; zeros above ---------------
  for (int I = 0; I < NB; ++I) {
    for (int J = 0; J <= I; ++J) {
      gm.zero();
      gm.template mul<false, true>(Nk + (long long)128 * I * P, P, Nk + (long long)128 * J * P, P,
                                   P, lds);
      if (!zd)
        gm.template mul<false, true>(Zk + (long long)128 * I * q, q, Zk + (long long)128 * J * q,
                                     q, q, lds);
      gm.store(at(I, J), P, T(1), T(0));
      if (zd && I == J) {
        __syncthreads();                                // the stored block, then its diagonal
        for (int i = tid; i < 128; i += kFacThreads) {
          const T z = zd[128 * I + i];
          at(I, I)[(long long)i * P + i] += z * z;
        }
        __syncthreads();
      }
    }
    for (int J = I + 1; J < NB; ++J)
      for (int e = tid; e < 128 * 128; e += kFacThreads) at(I, J)[(long long)(e >> 7) * P + (e & 127)] = T(0);
  }

  // ---- 2. blocked Cholesky by super-blocks ---------------------------------
  for (int K = 0; K < NB; ++K) {
    __syncthreads();                                    // S_KK written, LDS free
    const T* Skk = at(K, K);
    for (int e = tid; e < TL::kTiles * 256; e += kFacThreads) {
      const int t = e >> 8, rc = e & 255;
      int I = 0;
      while ((I + 1) * (I + 2) / 2 <= t) ++I;
      const int J = t - I * (I + 1) / 2, rr = rc >> 4, cc = rc & 15;
      St[t * 256 + tix(rr, cc)] = Skk[(long long)(16 * I + rr) * P + 16 * J + cc];
    }
    __syncthreads();
    if (!tile_cholesky_inverse_call<T>(St, &sfail)) {
      if (tid == 0) atomicMin(fail, (F.level0 + lev) << 20 | k);
      return;
    }
    // X_KK in place of S_KK, zero above the diagonal
    T* Xkk = at(K, K);
    for (int e = tid; e < 128 * 128; e += kFacThreads) {
      const int i = e >> 7, j = e & 127, I = i >> 4, J = j >> 4;
      T v = T(0);
      if (J < I) v = St[TL::id(I, J) * 256 + tix(i & 15, j & 15)];
      else if (J == I && (j & 15) <= (i & 15)) v = St[TL::id(I, I) * 256 + tix(i & 15, j & 15)];
      Xkk[(long long)i * P + j] = v;
    }
    // panel: G_IK = S_IK X_KK^T (in place)
    for (int I = K + 1; I < NB; ++I) {
      gm.zero();
      gm.template mul<false, true>(at(I, K), P, Xkk, P, 128, lds);
      gm.store(at(I, K), P, T(1), T(0));
    }
    // trailing: S_IJ -= G_IK G_JK^T, K < J <= I
    for (int I = K + 1; I < NB; ++I)
      for (int J = K + 1; J <= I; ++J) {
        gm.zero();
        gm.template mul<false, true>(at(I, K), P, at(J, K), P, 128, lds);
        gm.store(at(I, J), P, T(-1), T(1));
      }
  }

  // ---- 3. X = G^{-1} in place by super-blocks ------------------------------
  for (int J = NB - 2; J >= 0; --J) {
    for (int I = NB - 1; I > J; --I) {
      gm.zero();
      for (int K = J + 1; K <= I; ++K)
        gm.template mul<false, false>(at(I, K), P, at(K, J), P, 128, lds);
      gm.store(at(I, J), P, T(1), T(0));                // the sum, over G_IJ
      gm.zero();
      gm.template mul<false, false>(at(I, J), P, at(J, J), P, 128, lds);
      gm.store(at(I, J), P, T(-1), T(0));
    }
  }
}

bool factor_mfma_supported(int p, int q) {
  if (p == 64 || p == 128) return true;
  return (p == 256 || p == 512) && q > 0 && q % kPanel == 0;
}

template <class T>
static hipError_t launch_t(const FactorBatchT<T>& F, int* fail, hipStream_t s) {
  const int total = F.start[F.nlev];
  if (total <= 0) return hipSuccess;
  if (!factor_mfma_supported(F.p, F.q)) return hipErrorInvalidValue;
  const int nt = F.p <= 128 ? F.p / 16 : 8;
  const size_t lds = (size_t)nt * (nt + 1) / 2 * 256 * sizeof(T);   // the lower tiles
  auto go = [&](auto kern) -> hipError_t {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return launch_k(kern, dim3(total), dim3(kFacThreads), lds, s, F, fail);
  };
  if (F.p == 64) return go(k_factor_mfma<T, 4>);
  if (F.p == 128) return go(k_factor_mfma<T, 8>);
  return go(k_factor_big<T>);
}

hipError_t launch_factor_mfma(const FactorBatchT<double>& F, int* fail, hipStream_t s) {
  return launch_t(F, fail, s);
}

hipError_t launch_factor_mfma(const FactorBatchT<float>& F, int* fail, hipStream_t s) {
  return launch_t(F, fail, s);
}

}  // namespace pitmg
