// Block Jacobi sweep for large blocks (p = 256 or 512) whose V and Z~ are
// shared by every step (theta = 1).  A block of p = 512 holds 3 MB of N_k and
// G_k^{-1} in FP64, too much for one work-group's registers and LDS, and the
// shared V, Z~ (2 MB each) would be re-read by every block.  The sweep is
// therefore split (Schur form as in pitmg_kernels.hip):
//
//   1. prepare: R_mu[:, k] = r_mu of block k+1 (b_mu minus the u coupling);
//   2. GEMM:    U = Z~ R_z - V R_mu          (all steps at once)
//   3. blocks:  t = N r_u + U_k - r_l, lambda = G^{-T} G^{-1} t,
//               u = r_u - N^T lambda          (N_k, G_k^{-1} streamed twice)
//   4. GEMM:    W_z = Z~^T Lambda,  W_v = V^T Lambda
//   5. finish:  z = r_z - W_z,  mu = W_v - r_mu - r_v,  v = -r_mu
//
// so every block reads only its own N_k and G_k^{-1}, and V, Z~ are read once
// per 64-step tile of the GEMMs, which run on the matrix cores (k_gemm_rows).
// The output is the unweighted sweep; launch_jacobi weights it afterwards.
#include "pitmg_internal.h"
#include "pitmg_device.h"
#include "pitmg_tiled.h"
#include "pitmg_mfma.h"


namespace pitmg {
namespace {

constexpr int kSplitThreads = 512;
constexpr int kSplitWaves = kSplitThreads / kWave;

// coupling values of the previous iterate: yold + P ec (u and mu only)
struct Coupling {
  PrevIterate prev;
  __device__ double cu(int k1, int i) const { return prev.at(0, k1, i); }
  __device__ double cm(int k1, int i) const { return prev.at(4, k1, i); }
};

// R_mu (p x (n+1), column k-1 for block k; column 0 is zero) and, for the
// FP32 smoother, FP32 copies of R_mu and R_z (q x n).
__global__ void k_split_prepare(Coupling C, const double* __restrict__ b, double* __restrict__ Rm,
                                float* __restrict__ Rm32, float* __restrict__ Rz32) {
  const int p = C.prev.p, q = C.prev.q, n = C.prev.n;
  const TypeMajor Tm(p, q, n);
  const long long total = (long long)p * (n + 1);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int col = (int)(e / p), i = (int)(e % p);   // block col+1
    double v = 0.0;
    if (col >= 1) v = b[Tm.m + (long long)(col - 1) * p + i] - C.cu(col, i);
    Rm[e] = v;
    if (Rm32 && col < n) Rm32[e] = (float)v;
  }
  if (Rz32) {
    const long long nz = (long long)q * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nz;
         e += (long long)gridDim.x * blockDim.x)
      Rz32[e] = (float)b[Tm.z + e];
  }
}

// One block per work-group, 512 threads: thread (a, b) = (tid/16, tid%16)
// covers rows RT a .. RT a + RT-1 and the CT columns tile_col(c) of N_k and
// G_k^{-1}, streamed row by row.  Row sums reduce over the 16 lanes sharing
// a; column sums over the 4 row groups of a wave and then over the 8 waves
// through LDS, in a fixed order.
template <int RT, int CT, class T>
__global__ __launch_bounds__(kSplitThreads) void k_split_blocks(LevelView L, Coupling C,
                                                                const double* __restrict__ b,
                                                                const T* __restrict__ U,
                                                                double* __restrict__ ynew,
                                                                T* __restrict__ Lam32) {
  constexpr int P = 32 * RT;
  static_assert(P == 16 * CT, "tile shape");
  extern __shared__ double sm_raw[];
  T* sm = reinterpret_cast<T*>(sm_raw);
  T* sru = sm;
  T* srl = sru + P;
  T* st = srl + P;
  T* ss = st + P;
  T* slam = ss + P;
  T* red = slam + P;                        // [kSplitWaves][P]
  const int n = L.n, q = L.q;
  const TypeMajor Tm(P, q, n);
  const int k = blockIdx.x + 1;
  const long long kk = k - 1;
  const int tid = threadIdx.x, a = tid / 16, bq = tid % 16;
  const int lane = tid % kWave, w = tid / kWave;
  const int r0 = RT * a;
  const T* __restrict__ Nk = Mats<T>::N(L) + kk * L.sN;
  const T* __restrict__ Gk = Mats<T>::Gi(L) + kk * (long long)P * P;
  for (int i = tid; i < P; i += kSplitThreads) {
    sru[i] = (T)(b[Tm.u + kk * P + i] - C.cm(k, i));
    srl[i] = (T)b[Tm.l + kk * P + i];
  }
  __syncthreads();
  // t = N r_u + U_k - r_l
#pragma unroll 2
  for (int r = 0; r < RT; ++r) {
    T row[CT];
    tile_load_row<CT, T>(Nk + (long long)(r0 + r) * P, row);
    T s = 0;
#pragma unroll
    for (int c = 0; c < CT; ++c) s += row[c] * sru[tile_col<T>(c)];
    s = tile_sum16(s);
    if (bq == 0) st[r0 + r] = s + U[kk * P + r0 + r] - srl[r0 + r];
  }
  __syncthreads();
  // s = G^{-1} t
#pragma unroll 2
  for (int r = 0; r < RT; ++r) {
    T row[CT];
    tile_load_row_lower<CT, T>(Gk + (long long)(r0 + r) * P, r0 + r, row);
    T s = 0;
#pragma unroll
    for (int c = 0; c < CT; ++c) s += row[c] * st[tile_col<T>(c)];
    s = tile_sum16(s);
    if (bq == 0) ss[r0 + r] = s;
  }
  __syncthreads();
  // column sums over this thread's rows, then over the 4 row groups of the
  // wave (lanes xor 16, 32), then over the waves through red
  auto columns = [&](const T* __restrict__ M, bool lower, const T* x) {
    T acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c] = 0;
#pragma unroll 2
    for (int r = 0; r < RT; ++r) {
      T row[CT];
      if (lower)
        tile_load_row_lower<CT, T>(M + (long long)(r0 + r) * P, r0 + r, row);
      else
        tile_load_row<CT, T>(M + (long long)(r0 + r) * P, row);
      const T xr = x[r0 + r];
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[c] += row[c] * xr;
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      acc[c] = xor32_sum(xor16_sum(acc[c]));
    }
    if (lane < 16) {
#pragma unroll
      for (int c = 0; c < CT; ++c) red[w * P + tile_col<T>(c)] = acc[c];
    }
    __syncthreads();
  };
  // lambda = G^{-T} s
  columns(Gk, true, ss);
  for (int j = tid; j < P; j += kSplitThreads) {
    T s = 0;
#pragma unroll
    for (int ww = 0; ww < kSplitWaves; ++ww) s += red[ww * P + j];
    slam[j] = s;
    ynew[Tm.l + kk * P + j] = (double)s;
    if (Lam32) Lam32[kk * P + j] = s;
  }
  __syncthreads();
  // u = r_u - N^T lambda
  columns(Nk, false, slam);
  for (int j = tid; j < P; j += kSplitThreads) {
    T s = 0;
#pragma unroll
    for (int ww = 0; ww < kSplitWaves; ++ww) s += red[ww * P + j];
    ynew[Tm.u + kk * P + j] = (double)(sru[j] - s);
  }
}

// z = r_z - W_z, v = -r_mu, mu = W_v - r_mu - r_v (blocks 2..n+1; block n+1
// has no W_v term, V_{n+1} := 0).
template <class T>
__global__ void k_split_finish(int p, int q, int n, const double* __restrict__ b,
                               const double* __restrict__ Rm, const T* __restrict__ Wz,
                               const T* __restrict__ Wv, double* __restrict__ ynew) {
  const TypeMajor Tm(p, q, n);
  const long long nz = (long long)q * n, nm = (long long)p * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nz + nm;
       e += (long long)gridDim.x * blockDim.x) {
    if (e < nz) {
      ynew[Tm.z + e] = b[Tm.z + e] - (double)Wz[e];
      continue;
    }
    const long long f = e - nz;                 // (v_m, mu_m), m = f/p + 1 = 1..n
    const int m = (int)(f / p), i = (int)(f % p);
    const double rmu = Rm[(long long)(m + 1) * p + i];   // block m+2's r_mu
    const double rv = b[Tm.v + (long long)m * p + i];
    ynew[Tm.v + (long long)m * p + i] = -rmu;
    const double wv = m + 1 < n ? (double)Wv[(long long)(m + 1) * p + i] : 0.0;
    ynew[Tm.m + (long long)m * p + i] = wv - rmu - rv;
  }
}

int grid_for_split(long long len) {
  long long g = (len + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

size_t split_lds(int p, size_t elem) { return (size_t)(5 + kSplitWaves) * p * elem; }

// C (m x P, row-major, ld P) = alpha A op(B) + beta C with A (m x K, row-major,
// ld lda) and op(B) = B (K x P, row-major) or B^T (B: P x K, row-major): the
// per-step products of the split sweep, one 64 x 64 tile of C per work-group
// of 256 threads (four waves of 32 x 32), K in panels of 32 staged in LDS.
// Rows of A beyond m and columns beyond K read as zero.  FP64 on
// v_mfma_f64_16x16x4f64, FP32 on v_mfma_f32_16x16x4f32 (Mfma4 layouts).
constexpr int kGemmTile = 64;
constexpr int kGemmK = 32;

template <class T, bool TB>
__global__ __launch_bounds__(256) void k_gemm_rows(int m, int P, int K, double alpha,
                                                   const T* __restrict__ A, long long lda,
                                                   const T* __restrict__ B, double beta,
                                                   T* __restrict__ C) {
  __shared__ T As[kGemmTile][kGemmK + 1];
  __shared__ T Bs[kGemmK][kGemmTile + 1];
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const int r = lane & 15, g = lane >> 4;
  const int row0 = blockIdx.x * kGemmTile, col0 = blockIdx.y * kGemmTile;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;          // the wave's 32 x 32
  typename Mfma4<T>::v4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = {0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += kGemmK) {
    __syncthreads();
    for (int e = tid; e < kGemmTile * kGemmK; e += 256) {
      const int i = e / kGemmK, kk = e % kGemmK;            // A: rows of 32
      const int gi = row0 + i, gk = k0 + kk;
      As[i][kk] = gi < m && gk < K ? A[(long long)gi * lda + gk] : T(0);
      if (!TB) {                                            // B: rows of 64
        const int k2 = e / kGemmTile, j = e % kGemmTile;
        Bs[k2][j] = k0 + k2 < K ? B[(long long)(k0 + k2) * P + col0 + j] : T(0);
      } else {                                              // B^T: rows of 32
        const int j = e / kGemmK, k2 = e % kGemmK;
        Bs[k2][j] = k0 + k2 < K ? B[(long long)(col0 + j) * K + k0 + k2] : T(0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kGemmK / 4; ++s) {
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const T av = As[wr + 16 * a + r][4 * s + g];
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = Mfma4<T>::step(av, Bs[4 * s + g][wc + 16 * b + r], acc[a][b]);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gi = row0 + wr + 16 * a + Mfma4<T>::row(g, i);
        const int gj = col0 + wc + 16 * b + r;
        if (gi < m) {
          T* c = C + (long long)gi * P + gj;
          *c = (T)(alpha * (double)acc[a][b][i] + (beta != 0.0 ? beta * (double)*c : 0.0));
        }
      }
}

template <class T, bool TB>
hipError_t gemm_rows(int m, int P, int K, double alpha, const T* A, long long lda, const T* B,
                     double beta, T* C, hipStream_t s) {
  if (P % kGemmTile) return hipErrorInvalidValue;
  const dim3 grid((m + kGemmTile - 1) / kGemmTile, P / kGemmTile);
  return launch_k(k_gemm_rows<T, TB>, grid, dim3(256), 0, s, m, P, K, alpha, A, lda, B, beta,
                  C);
}

// The same row products when V and Z~ are diagonal: C[r][j] = a A[r][j] d[j]
// (+ a2 A2[r][j] d2[j] when A2 is given), for m rows of P.
template <class T>
__global__ void k_diag_rows(int m, int P, const T* __restrict__ A, long long lda,
                            const T* __restrict__ d, double a, const T* __restrict__ A2,
                            long long lda2, const T* __restrict__ d2, double a2,
                            T* __restrict__ C) {
  const long long total = (long long)m * P;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / P;
    const int j = (int)(e % P);
    double v = a * (double)A[r * lda + j] * (double)d[j];
    if (A2) v += a2 * (double)A2[r * lda2 + j] * (double)d2[j];
    C[r * P + j] = (T)v;
  }
}

template <class T>
hipError_t diag_rows(int m, int P, const T* A, long long lda, const T* d, double a, const T* A2,
                     long long lda2, const T* d2, double a2, T* C, hipStream_t s) {
  return launch_k(k_diag_rows<T>, dim3(grid_for_split((long long)m * P)), dim3(256), 0, s, m,
                  P, A, lda, d, a, A2, lda2, d2, a2, C);
}

template <int RT, int CT, class T>
hipError_t run_split(const LevelView& L, const SplitBuffers& S, const double* b,
                     const double* yold, const double* ecoarse, int variant, double* ynew,
                     hipStream_t s) {
  constexpr int P = 32 * RT;
  const int n = L.n, q = L.q;
  const bool f32 = sizeof(T) == 4;
  const TypeMajor Tm(P, q, n);
  Coupling C{PrevIterate{yold, ecoarse, P, q, n, variant, L.mu_scale}};
  hipError_t e = launch_k(k_split_prepare, dim3(grid_for_split((long long)P * (n + 1))),
                          dim3(256), 0, s, C, b, S.Rm, f32 ? S.Rm32 : (float*)nullptr,
                          f32 ? S.Rz32 : (float*)nullptr);
  if (e != hipSuccess) return e;
  const T* Z = Mats<T>::Z(L);
  const T* V = Mats<T>::V(L);
  T* U = f32 ? (T*)S.U32 : (T*)S.U;
  T* Wz = f32 ? (T*)S.Wz32 : (T*)S.Wz;
  T* Wv = f32 ? (T*)S.Wv32 : (T*)S.Wv;
  const T* Rz = f32 ? (const T*)S.Rz32 : (const T*)(b + Tm.z);
  const T* Rm = f32 ? (const T*)S.Rm32 : (const T*)S.Rm;
  // per step k (rows): U_k = Z~ r_z,k - V r_mu,k, i.e. U = R_z Z~^T - R_mu V^T
  // (elementwise when V and Z~ are diagonal)
  const bool dg = L.vz_diag != 0;
  if (dg) {
    if ((e = diag_rows<T>(n, P, Rz, q, Mats<T>::Zd(L), 1.0, Rm, P, Mats<T>::Vd(L), -1.0, U, s)))
      return e;
  } else {
    if ((e = gemm_rows<T, true>(n, P, q, 1.0, Rz, q, Z, 0.0, U, s))) return e;
    if ((e = gemm_rows<T, true>(n, P, P, -1.0, Rm, P, V, 1.0, U, s))) return e;
  }
  const size_t lds = split_lds(P, sizeof(T));
  e = hipFuncSetAttribute((const void*)k_split_blocks<RT, CT, T>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  e = launch_k(k_split_blocks<RT, CT, T>, dim3(n), dim3(kSplitThreads), lds, s, L, C, b,
               (const T*)U, ynew, f32 ? (T*)S.L32 : (T*)nullptr);
  if (e != hipSuccess) return e;
  // W_z,k = Z~^T lambda_k, W_v,k = V^T lambda_k: W = Lambda Z~, Lambda V
  const T* Lam = f32 ? (const T*)S.L32 : (const T*)(ynew + Tm.l);
  if (dg) {
    if ((e = diag_rows<T>(n, P, Lam, P, Mats<T>::Zd(L), 1.0, nullptr, 0, nullptr, 0.0, Wz, s)))
      return e;
    if ((e = diag_rows<T>(n, P, Lam, P, Mats<T>::Vd(L), 1.0, nullptr, 0, nullptr, 0.0, Wv, s)))
      return e;
  } else {
    if ((e = gemm_rows<T, false>(n, q, P, 1.0, Lam, P, Z, 0.0, Wz, s))) return e;
    if ((e = gemm_rows<T, false>(n, P, P, 1.0, Lam, P, V, 0.0, Wv, s))) return e;
  }
  return launch_k(k_split_finish<T>, dim3(grid_for_split((long long)(P + q) * n)), dim3(256), 0,
                  s, P, q, n, b, (const double*)S.Rm, (const T*)Wz, (const T*)Wv, ynew);
}

}  // namespace

bool split_supported(const LevelView& L) {
  return L.split && L.sV == 0 && L.sZ == 0 && (L.p == 256 || L.p == 512) && L.q % 64 == 0;
}

hipError_t launch_jacobi_split(const LevelView& L, const double* b, const double* yold,
                               const double* ecoarse, int variant, double* ynew, hipStream_t s) {
  const SplitBuffers& S = *L.split;
  if (L.p == 512)
    return L.fp32 ? run_split<16, 32, float>(L, S, b, yold, ecoarse, variant, ynew, s)
                  : run_split<16, 32, double>(L, S, b, yold, ecoarse, variant, ynew, s);
  return L.fp32 ? run_split<8, 16, float>(L, S, b, yold, ecoarse, variant, ynew, s)
                : run_split<8, 16, double>(L, S, b, yold, ecoarse, variant, ynew, s);
}

}  // namespace pitmg
