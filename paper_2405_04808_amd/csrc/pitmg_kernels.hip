// HIP kernels for gfx950: block factorisation, block Jacobi sweep, operator
// apply, transfers in time, the coarse GMRES+SGS solve and Krylov helpers.
//
// Block algebra (time-major block k of Fig. 5, unknowns
// (v_{k-1}, u_k, z_k, lambda_k, mu_{k-1})).  The diagonal block D_k is
//     [ I    .    .    V_k^T  -I ]   v_{k-1}
//     [ .    I    .    N_k^T   . ]   u_k
//     [ .    .    I    Z_k^T   . ]   z_k
//     [ V_k  N_k  Z_k  .       . ]   lambda_k
//     [ -I   .    .    .       . ]   mu_{k-1}
// Eliminating v, u, z gives the Schur complement in lambda,
//     S_k = N_k N_k^T + Z_k Z_k^T       (the V_k V_k^T terms cancel),
// which is positive definite when N_k is invertible (Thm. 1).  With
// S_k = G_k G_k^T and the right-hand side (r_v, r_u, r_z, r_l, r_m):
//     t = N r_u + Z r_z - V r_m - r_l,  lambda = G^{-T} G^{-1} t,
//     u = r_u - N^T lambda,  z = r_z - Z^T lambda,
//     mu = V^T lambda - r_m - r_v,  v = -r_m.
// Block 1 has no v, mu (and V_1 is unused); block n+1 is (v_n, mu_n) with
// v_n = -r_m, mu_n = -r_m - r_v.  Between blocks the only couplings are the
// +I entries u_k <-> mu_k (Sec. 5.3.2), so a Jacobi sweep needs just u_{k-1}
// and mu_k of the previous iterate.
#include "pitmg_internal.h"
#include "pitmg_device.h"
#include "pitmg_onepass.h"
#include "pitmg_blocks.h"
#include "pitmg_mfma.h"
#include <algorithm>
#include <climits>

namespace pitmg {

// ---------------------------------------------------------------------------
// K1/K2: factorisation of S_k = N N^T + Z Z^T, Cholesky, triangular inverse
// ---------------------------------------------------------------------------

constexpr int kFactorThreads = 256;

// S = X X^T with X = [N_k | Z_k] (p x (p+q)) on the matrix cores: one
// work-group per block, each wave accumulating 16x16 tiles of the lower
// triangle with v_mfma_f64_16x16x4f64 (v_mfma_f32_16x16x4f32 for FP32).
// Lane l supplies X[I0 + l%16][k0 + l/16] as the A operand and
// X[J0 + l%16][k0 + l/16] as the B operand (B = X^T).  Element i of lane l's
// result is S[I0 + row(l/16, i)][J0 + l%16], with row = l/16 + 4i for the
// FP64 instruction and 4(l/16) + i for the FP32 one (the layouts of the two
// instructions differ).  Rows beyond p and columns beyond p+q read as zero.
// S goes to the factor buffer (lower triangle; the factorisation kernel
// reads it from there).
template <class T>
__global__ __launch_bounds__(kFactorThreads) void k_syrk_mfma(LevelView L, T* Gi) {
  const int p = L.p, q = L.q, K = p + q;
  const int k = blockIdx.x;
  const T* __restrict__ Nk = Mats<T>::N(L) + (long long)k * L.sN;
  const T* __restrict__ Zk = Mats<T>::Z(L) + (long long)k * L.sZ;
  T* S = Gi + (long long)k * p * p;
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int r = lane & 15, kq = lane >> 4;
  const int nt = (p + 15) / 16;
  auto x = [&](int row, int col) -> T {
    if (row >= p || col >= K) return T(0);
    return col < p ? Nk[(long long)row * p + col] : Zk[(long long)row * q + (col - p)];
  };
  // tiles (I, J) with J <= I, numbered row by row
  const int ntiles = nt * (nt + 1) / 2;
  for (int t = w; t < ntiles; t += kFactorThreads / kWave) {
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = t - I * (I + 1) / 2;
    const int I0 = 16 * I, J0 = 16 * J;
    typename Mfma4<T>::v4 acc = {0, 0, 0, 0};
    for (int k0 = 0; k0 < K; k0 += 4) {
      const T a = x(I0 + r, k0 + kq);
      const T b = x(J0 + r, k0 + kq);
      acc = Mfma4<T>::step(a, b, acc);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = I0 + Mfma4<T>::row(kq, i), col = J0 + r;
      if (row < p && col <= row) S[(long long)row * p + col] = acc[i];
    }
  }
}

template <class T, bool USE_LDS>
__global__ __launch_bounds__(kFactorThreads) void k_factor(LevelView L, T* Gi,
                                                           int level, int* fail) {
  extern __shared__ double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int p = L.p;
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  const T* __restrict__ Nk = Mats<T>::N(L) + (long long)k * L.sN;
  const T* __restrict__ Zk = Mats<T>::Z(L) + (long long)k * L.sZ;
  T* Gk = Gi + (long long)k * p * p;
  const int ld = USE_LDS ? p + 1 : p;
  T* S = USE_LDS ? smem : Gk;
  T* tmp = USE_LDS ? smem + (size_t)p * ld : smem;

  // S = N N^T + Z Z^T (lower triangle) was formed by k_syrk_mfma in Gk
  (void)Nk;
  (void)Zk;
  if (USE_LDS) {
    for (int idx = tid; idx < p * p; idx += kFactorThreads) {
      const int i = idx / p, j = idx % p;
      if (j <= i) S[(long long)i * ld + j] = Gk[idx];
    }
  }
  // Cholesky, right-looking, column by column
  for (int j = 0; j < p; ++j) {
    __syncthreads();
    T d = S[(long long)j * ld + j];
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0) atomicMin(fail, (level << 20) | k);
      return;                                  // uniform: every thread read d
    }
    d = sqrt(d);
    __syncthreads();
    if (tid == 0) S[(long long)j * ld + j] = d;
    const T inv = T(1) / d;
    for (int i = j + 1 + tid; i < p; i += kFactorThreads) S[(long long)i * ld + j] *= inv;
    __syncthreads();
    const int m = p - j - 1;
    for (int idx = tid; idx < m * m; idx += kFactorThreads) {
      const int ii = idx / m, cc = idx % m;
      if (cc > ii) continue;
      const int i = j + 1 + ii, c = j + 1 + cc;
      S[(long long)i * ld + c] -= S[(long long)i * ld + j] * S[(long long)c * ld + j];
    }
  }
  // In-place inverse of the lower-triangular G, columns right to left:
  // X[j][j] = 1/G[j][j], X[i][j] = -X[j][j] sum_{m=j+1..i} X[i][m] G[m][j].
  for (int j = p - 1; j >= 0; --j) {
    __syncthreads();
    const T djj = T(1) / S[(long long)j * ld + j];
    for (int i = j + 1 + tid; i < p; i += kFactorThreads) {
      T acc = 0;
      for (int m = j + 1; m <= i; ++m) acc += S[(long long)i * ld + m] * S[(long long)m * ld + j];
      tmp[i] = -djj * acc;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < p; i += kFactorThreads) S[(long long)i * ld + j] = tmp[i];
    if (tid == 0) S[(long long)j * ld + j] = djj;
  }
  __syncthreads();
  for (int idx = tid; idx < p * p; idx += kFactorThreads) {
    const int i = idx / p, j = idx % p;
    const T v = j <= i ? S[(long long)i * ld + j] : T(0);
    Gk[idx] = v;
  }
}

template <class T>
static size_t factor_lds(int p) {
  if (p <= 128) return ((size_t)p * (p + 1) + p) * sizeof(T);
  return (size_t)p * sizeof(T);
}

template <class T>
static hipError_t launch_factor_t(const LevelView& L, T* Gi, int level, int* fail, hipStream_t s) {
  hipLaunchKernelGGL(k_syrk_mfma<T>, dim3(L.n), dim3(kFactorThreads), 0, s, L, Gi);
  const size_t lds = factor_lds<T>(L.p);
  if (L.p <= 128) {
    hipError_t e = hipFuncSetAttribute((const void*)k_factor<T, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_factor<T, true>), dim3(L.n), dim3(kFactorThreads), lds, s, L, Gi,
                       level, fail);
  } else {
    hipLaunchKernelGGL((k_factor<T, false>), dim3(L.n), dim3(kFactorThreads), lds, s, L, Gi,
                       level, fail);
  }
  return hipGetLastError();
}

hipError_t launch_factor(const LevelView& L, double* Gi, int level, int* fail, hipStream_t s) {
  return launch_factor_t<double>(L, Gi, level, fail, s);
}

hipError_t launch_factor32(const LevelView& L, float* Gi32, int level, int* fail,
                           hipStream_t s) {
  return launch_factor_t<float>(L, Gi32, level, fail, s);
}

__global__ void k_to_f32(float* __restrict__ dst, const double* __restrict__ src,
                         long long count) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

hipError_t launch_to_f32(float* dst, const double* src, long long count, hipStream_t s) {
  long long g = (count + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)g), dim3(256), 0, s, dst, src, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K3: block Jacobi sweep, one work-group per time-major block
// ---------------------------------------------------------------------------

constexpr int kSweepThreads = 256;

template <int NT, class T>
__global__ __launch_bounds__(NT) void k_jacobi(LevelView L, const double* __restrict__ b,
                                               const double* __restrict__ yold,
                                               const double* __restrict__ ec, int variant,
                                               double* __restrict__ ynew) {
  extern __shared__ double sm_raw[];
  T* sm = reinterpret_cast<T*>(sm_raw);
  const int p = L.p, q = L.q, n = L.n;
  const TypeMajor Tm(p, q, n);
  const int kb = blockIdx.x, tid = threadIdx.x;
  const double w = L.omega;
  // the iterate the sweep starts from: yold + P ec; its u and mu slots are
  // the couplings, and every slot enters the weighted update
  const PrevIterate prev{yold, ec, p, q, n, variant, L.mu_scale};

  if (kb == n) {                               // block n+1 = (v_n, mu_n)
    for (int i = tid; i < p; i += NT) {
      const double rvv = b[Tm.v + (long long)(n - 1) * p + i];
      const double rmm = b[Tm.m + (long long)(n - 1) * p + i] - prev.at(0, n, i);
      ynew[Tm.v + (long long)(n - 1) * p + i] = weigh(w, -rmm, prev, 1, n, i);
      ynew[Tm.m + (long long)(n - 1) * p + i] = weigh(w, -rmm - rvv, prev, 4, n, i);
    }
    return;
  }
  const int k = kb + 1;
  const bool hv = k >= 2;
  T* rv = sm;
  T* ru = rv + p;
  T* rz = ru + p;
  T* rl = rz + q;
  T* rm = rl + p;
  T* ov = rm + p;
  T* ou = ov + p;
  T* oz = ou + p;
  T* ol = oz + q;
  T* om = ol + p;
  T* t = om + p;
  T* s = t + p;
  T* part = s + p;
  for (int i = tid; i < p; i += NT) {
    ru[i] = (T)(b[Tm.u + (long long)(k - 1) * p + i] - prev.at(4, k, i));
    rl[i] = (T)b[Tm.l + (long long)(k - 1) * p + i];
    if (hv) {
      rv[i] = (T)b[Tm.v + (long long)(k - 2) * p + i];
      rm[i] = (T)(b[Tm.m + (long long)(k - 2) * p + i] - prev.at(0, k - 1, i));
    } else {
      rv[i] = 0;
      rm[i] = 0;
    }
  }
  for (int i = tid; i < q; i += NT) rz[i] = (T)b[Tm.z + (long long)(k - 1) * q + i];
  __syncthreads();
  const long long kk = k - 1;
  block_solve<NT, T>(p, q, Mats<T>::N(L) + kk * L.sN, Mats<T>::V(L) + kk * L.sV,
                     Mats<T>::Z(L) + kk * L.sZ, Mats<T>::Gi(L) + kk * p * p, hv, rv, ru, rz, rl,
                     rm, ov, ou, oz, ol, om, t, s, part);
  for (int i = tid; i < p; i += NT) {
    ynew[Tm.u + kk * p + i] = weigh(w, (double)ou[i], prev, 0, k, i);
    ynew[Tm.l + kk * p + i] = weigh(w, (double)ol[i], prev, 3, k, i);
    if (hv) {
      ynew[Tm.v + (kk - 1) * p + i] = weigh(w, (double)ov[i], prev, 1, k - 1, i);
      ynew[Tm.m + (kk - 1) * p + i] = weigh(w, (double)om[i], prev, 4, k - 1, i);
    }
  }
  for (int i = tid; i < q; i += NT) ynew[Tm.z + kk * q + i] = weigh(w, (double)oz[i], prev, 2, k, i);
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

template <class T>
static hipError_t launch_jacobi_generic(const LevelView& L, const double* b, const double* yold,
                                        const double* ecoarse, int variant, double* ynew,
                                        hipStream_t s) {
  const size_t lds = solve_lds_doubles(L.p, L.q, kSweepThreads) * sizeof(T);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_jacobi<kSweepThreads, T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return launch_k(k_jacobi<kSweepThreads, T>, dim3(L.n + 1), dim3(kSweepThreads), lds, s, L, b,
                  yold, ecoarse, variant, ynew);
}

hipError_t launch_jacobi(const LevelView& L, const double* b, const double* yold,
                         const double* ecoarse, int variant, double* ynew, hipStream_t s,
                         double* restrict_out, double rbeta, double ra) {
  if (restrict_out && ecoarse) return hipErrorInvalidValue;
  const bool al = L.fp32 ? aligned16(L.N32) && aligned16(L.V32) && aligned16(L.Z32) &&
                               aligned16(L.Gi32)
                         : aligned16(L.N) && aligned16(L.V) && aligned16(L.Z) && aligned16(L.Gi);
  const bool small = small_supported(L.p, L.q);
  if (!small && al && jacobi_shared_supported(L) && L.sweep_cfg >= 0)
    return launch_jacobi_shared(L, b, yold, ecoarse, variant, ynew, restrict_out, rbeta, ra, s);
  if (!small && al && jacobi_tiled_supported(L.p, L.q))
    return launch_jacobi_tiled(L, b, yold, ecoarse, variant, ynew, restrict_out, rbeta, ra, s);
  hipError_t e;
  if (small) {
    e = launch_jacobi_small(L, b, yold, ecoarse, variant, ynew, s);
  } else if (al && split_supported(L)) {
    // the split sweep writes the unweighted block solves; weight afterwards
    e = launch_jacobi_split(L, b, yold, ecoarse, variant, ynew, s);
    if (e == hipSuccess && L.omega != 1.0)
      e = launch_weight(L.p, L.q, L.n, L.omega, yold, ecoarse, variant, L.mu_scale, ynew, s);
  } else {
    e = L.fp32 ? launch_jacobi_generic<float>(L, b, yold, ecoarse, variant, ynew, s)
               : launch_jacobi_generic<double>(L, b, yold, ecoarse, variant, ynew, s);
  }
  if (e != hipSuccess || !restrict_out) return e;
  return launch_restrict_delta(L.p, L.q, L.n, b, rbeta, yold, ra, ynew, variant, L.mu_scale,
                               restrict_out, s);
}

static bool sweeps_tiled(const LevelView& L) {
  const bool al = L.fp32 ? aligned16(L.N32) && aligned16(L.V32) && aligned16(L.Z32) &&
                               aligned16(L.Gi32)
                         : aligned16(L.N) && aligned16(L.V) && aligned16(L.Z) && aligned16(L.Gi);
  if (small_supported(L.p, L.q) || !al) return false;
  if (jacobi_shared_supported(L) && L.sweep_cfg >= 0) return false;
  return jacobi_tiled_supported(L.p, L.q);
}

static bool sweeps_shared_fp64(const LevelView& L) {
  if (L.fp32 || small_supported(L.p, L.q)) return false;
  if (!(aligned16(L.N) && aligned16(L.V) && aligned16(L.Z) && aligned16(L.Gi))) return false;
  return jacobi_shared_supported(L) && L.sweep_cfg >= 0;
}

bool jacobi_pair_supported(const LevelView& L, hipStream_t s) {
  if (!sweeps_tiled(L) && !sweeps_shared_fp64(L)) return false;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st == hipStreamCaptureStatusNone;
}

bool jacobi_chain_supported(const LevelView& L, hipStream_t s) {
  if (!sweeps_tiled(L)) return false;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st == hipStreamCaptureStatusNone;
}

hipError_t launch_jacobi_pair(const LevelView& L, const double* b, const double* yold,
                              const double* ecoarse, int variant, double* y1, double* y2,
                              double* restrict_out, double rbeta, double ra,
                              const PairSync& ps, int* groups, hipStream_t s) {
  *groups = 0;
  if (!ps.ticket || !ps.flag || !ps.timeout) return hipErrorNotSupported;
  if (y1 == y2 || y1 == yold || y1 == b || y2 == b) return hipErrorInvalidValue;
  if (sweeps_shared_fp64(L))
    return launch_jacobi_shared2(L, b, yold, ecoarse, variant, y1, y2, restrict_out, rbeta, ra,
                                 ps, groups, s);
  if (!sweeps_tiled(L)) return hipErrorNotSupported;
  *groups = L.n;                                   // one work-group per block 1..n
  return launch_jacobi_tiled2(L, b, yold, ecoarse, variant, y1, y2, restrict_out, rbeta, ra,
                              ps, s);
}

// ---------------------------------------------------------------------------
// K4: out = beta*b + alpha*(A~ x), one work-group per time step
// ---------------------------------------------------------------------------

constexpr int kApplyThreads = 256;


template <int NT>
__global__ __launch_bounds__(NT) void k_apply(LevelView L, const double* __restrict__ x,
                                              const double* __restrict__ b, double alpha,
                                              double beta, double* __restrict__ out) {
  extern __shared__ double sm[];
  apply_step<NT>(L, blockIdx.x + 1, x, b, alpha, beta, out, sm);
}

// The same product for p = q = 64 MB in {64, 128, 256, 512} with V and Z~ diagonal
// (shared by every step), one work-group of 512 threads per step and one
// pass over N_k (onepass_products, pitmg_onepass.h): the row product
// N u_k and the column product N^T lambda_k from the same loads.  Rows of
// block k as in apply_step; the products with V and Z~ are elementwise with
// their diagonals.
template <int MB>
__global__ __launch_bounds__(kOnePassThreads) void k_apply_big(LevelView L,
                                                               const double* __restrict__ x,
                                                               const double* __restrict__ b,
                                                               double alpha, double beta,
                                                               double* __restrict__ out) {
  constexpr int P = 64 * MB, NTH = kOnePassThreads, NW = kOnePassWaves;
  __shared__ double sxu[P], sxl[P], sxz[P], sxv[P], srow[P];
  __shared__ double red[NW][P];
  const int tid = threadIdx.x;
  const int n = L.n, k = blockIdx.x + 1;
  const long long kk = k - 1;
  const bool hv = k >= 2;
  const TypeMajor T(P, P, n);
  for (int i = tid; i < P; i += NTH) {
    sxu[i] = x[T.u + kk * P + i];
    sxl[i] = x[T.l + kk * P + i];
    sxz[i] = x[T.z + kk * P + i];
    sxv[i] = hv ? x[T.v + (kk - 1) * P + i] : 0.0;
  }
  __syncthreads();
  onepass_products<MB>(L.N + kk * L.sN, x + T.u + kk * P, sxl, srow, red);
  __syncthreads();
  const double* __restrict__ Vd = L.Vd;
  const double* __restrict__ Zd = L.Zd;
  auto put = [&](long long idx, double val) {
    out[idx] = (beta != 0.0 ? beta * b[idx] : 0.0) + alpha * val;
  };
  for (int i = tid; i < P; i += NTH) {
    double nl = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) nl += red[q][i];
    const double lam = sxl[i];
    // lambda_k = N u_k + V v_{k-1} + Z~ z_k
    put(T.l + kk * P + i, srow[i] + (hv ? Vd[i] * sxv[i] : 0.0) + Zd[i] * sxz[i]);
    // u_k = u_k + N^T lambda_k + mu_k;  z_k = z_k + Z~^T lambda_k
    put(T.u + kk * P + i, sxu[i] + nl + x[T.m + kk * P + i]);
    put(T.z + kk * P + i, sxz[i] + Zd[i] * lam);
    if (hv) {
      // v_{k-1} = v_{k-1} + V^T lambda_k - mu_{k-1};  mu_{k-1} = u_{k-1} - v_{k-1}
      put(T.v + (kk - 1) * P + i, sxv[i] + Vd[i] * lam - x[T.m + (kk - 1) * P + i]);
      put(T.m + (kk - 1) * P + i, x[T.u + (kk - 1) * P + i] - sxv[i]);
    }
    if (k == n) {
      const double vn = x[T.v + kk * P + i], mn = x[T.m + kk * P + i];
      put(T.v + kk * P + i, vn - mn);
      put(T.m + kk * P + i, sxu[i] - vn);
    }
  }
}

static bool apply_big_supported(const LevelView& L, const double* x) {
  return L.vz_diag && L.Vd && L.Zd && L.p == L.q &&
         (L.p == 64 || L.p == 128 || L.p == 256 || L.p == 512) && aligned16(L.N) && aligned16(x);
}

hipError_t launch_apply(const LevelView& L, const double* x, const double* b, double alpha,
                        double beta, double* out, hipStream_t s) {
  if (small_supported(L.p, L.q)) return launch_apply_small(L, x, b, alpha, beta, out, s);
  if (apply_big_supported(L, x)) {
    const dim3 g(L.n), t(kOnePassThreads);
    switch (L.p) {
      case 64: hipLaunchKernelGGL(k_apply_big<1>, g, t, 0, s, L, x, b, alpha, beta, out); break;
      case 128: hipLaunchKernelGGL(k_apply_big<2>, g, t, 0, s, L, x, b, alpha, beta, out); break;
      case 256: hipLaunchKernelGGL(k_apply_big<4>, g, t, 0, s, L, x, b, alpha, beta, out); break;
      default: hipLaunchKernelGGL(k_apply_big<8>, g, t, 0, s, L, x, b, alpha, beta, out); break;
    }
    return hipGetLastError();
  }
  if (apply_shared_supported(L)) return launch_apply_shared(L, x, b, alpha, beta, out, s);
  const size_t lds = apply_lds_doubles(L.p, L.q, kApplyThreads) * sizeof(double);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_apply<kApplyThreads>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_apply<kApplyThreads>, dim3(L.n), dim3(kApplyThreads), lds, s, L, x,
                     b, alpha, beta, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K5: transfers in time
// ---------------------------------------------------------------------------

// Locate coarse element idx: type (0 u,1 v,2 z,3 l,4 m), step m (1-based),
// component i.
__device__ __forceinline__ void locate(long long idx, const TypeMajor& T, int p, int q,
                                       int& type, int& m, int& i) {
  long long off;
  if (idx < T.v) { type = 0; off = idx - T.u; }
  else if (idx < T.z) { type = 1; off = idx - T.v; }
  else if (idx < T.l) { type = 2; off = idx - T.z; m = (int)(off / q) + 1; i = (int)(off % q); return; }
  else if (idx < T.m) { type = 3; off = idx - T.l; }
  else { type = 4; off = idx - T.m; }
  m = (int)(off / p) + 1;
  i = (int)(off % p);
}

// Coarse step m of the restriction takes fine step kf = 2m-1 (variant 0) or
// 2m (variant 1) for u, v, lambda, mu and the mean of fine steps 2m-1, 2m
// for the control; the mu rows are weighted by mu_scale.
__device__ __forceinline__ int restrict_fine_step(int m, int variant) {
  return variant == 0 ? 2 * m - 1 : 2 * m;
}

__global__ void k_restrict_delta(int p, int q, int nf, const double* __restrict__ b, double beta,
                                 const double* __restrict__ ya, double a,
                                 const double* __restrict__ y, int variant, double mu_scale,
                                 double* __restrict__ bc) {
  const int nc = nf / 2;
  const TypeMajor Tf(p, q, nf), Tc(p, q, nc);
  const long long segf[5] = {Tf.u, Tf.v, Tf.z, Tf.l, Tf.m};
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < Tc.len;
       idx += (long long)gridDim.x * blockDim.x) {
    int type, m, i;
    locate(idx, Tc, p, q, type, m, i);
    const int kf = restrict_fine_step(m, variant);
    double v = 0.0;
    if (beta != 0.0) {
      if (type == 2)
        v = 0.5 * beta * (b[Tf.z + (long long)(2 * m - 2) * q + i] +
                          b[Tf.z + (long long)(2 * m - 1) * q + i]);
      else
        v = beta * b[segf[type] + (long long)(kf - 1) * p + i];
    }
    // (L+L^T) c: the u_k row couples mu_k, the mu_k row couples u_k
    if (type == 0 || type == 4) {
      const long long f = (type == 0 ? Tf.m : Tf.u) + (long long)(kf - 1) * p + i;
      v += (ya ? a * ya[f] : 0.0) - y[f];
    }
    bc[idx] = type == 4 ? mu_scale * v : v;
  }
}

__global__ void k_restrict(int p, int q, int nf, const double* __restrict__ r, int variant,
                           double mu_scale, double* __restrict__ bc) {
  const int nc = nf / 2;
  const TypeMajor Tf(p, q, nf), Tc(p, q, nc);
  const long long segf[5] = {Tf.u, Tf.v, Tf.z, Tf.l, Tf.m};
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < Tc.len;
       idx += (long long)gridDim.x * blockDim.x) {
    int type, m, i;
    locate(idx, Tc, p, q, type, m, i);
    double v;
    if (type == 2) {
      v = 0.5 * (r[Tf.z + (long long)(2 * m - 2) * q + i] + r[Tf.z + (long long)(2 * m - 1) * q + i]);
    } else {
      const int kf = restrict_fine_step(m, variant);
      v = r[segf[type] + (long long)(kf - 1) * p + i];
    }
    bc[idx] = type == 4 ? mu_scale * v : v;
  }
}

__global__ void k_interp_add(int p, int q, int nf, const double* __restrict__ e, int variant,
                             double mu_scale, double* __restrict__ y) {
  const int nc = nf / 2;
  const TypeMajor Tf(p, q, nf), Tc(p, q, nc);
  const long long segc[5] = {Tc.u, Tc.v, Tc.z, Tc.l, Tc.m};
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < Tf.len;
       idx += (long long)gridDim.x * blockDim.x) {
    int type, k, i;
    locate(idx, Tf, p, q, type, k, i);
    double v;
    if (type == 2) v = e[Tc.z + (long long)((k + 1) / 2 - 1) * q + i];
    else v = interp_node(e + segc[type], nc, p, k, i, variant);
    y[idx] += type == 4 ? mu_scale * v : v;
  }
}

// Transfers for a step ratio c between levels (coarse step k at fine step
// c(k-1)+1): injection for u, v, lambda, mu; the control averaged over the
// c fine steps; interpolation linear over the c fine steps of a coarse step
// (s^c_{nc+1} := s^c_{nc}) and the control copied.  The mu block is scaled
// by mu_fac (mu_scale per halving of the step).
__global__ void k_restrict_c(int p, int q, int nf, int c, const double* __restrict__ r,
                             double mu_fac, double* __restrict__ bc) {
  const int nc = nf / c;
  const TypeMajor Tf(p, q, nf), Tc(p, q, nc);
  const long long segf[5] = {Tf.u, Tf.v, Tf.z, Tf.l, Tf.m};
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < Tc.len;
       idx += (long long)gridDim.x * blockDim.x) {
    int type, m, i;
    locate(idx, Tc, p, q, type, m, i);
    double v;
    if (type == 2) {
      v = 0.0;
      for (int j = 0; j < c; ++j) v += r[Tf.z + (long long)(c * (m - 1) + j) * q + i];
      v /= c;
    } else {
      v = r[segf[type] + (long long)(c * (m - 1)) * p + i];
    }
    bc[idx] = type == 4 ? mu_fac * v : v;
  }
}

__global__ void k_interp_add_c(int p, int q, int nf, int c, const double* __restrict__ e,
                               double mu_fac, double* __restrict__ y) {
  const int nc = nf / c;
  const TypeMajor Tf(p, q, nf), Tc(p, q, nc);
  const long long segc[5] = {Tc.u, Tc.v, Tc.z, Tc.l, Tc.m};
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < Tf.len;
       idx += (long long)gridDim.x * blockDim.x) {
    int type, k, i;
    locate(idx, Tf, p, q, type, k, i);
    const int kc = (k - 1) / c + 1, j = (k - 1) % c;    // coarse step, position in it
    double v;
    if (type == 2) {
      v = e[Tc.z + (long long)(kc - 1) * q + i];
    } else {
      const int kn = kc < nc ? kc + 1 : nc;
      const double* seg = e + segc[type];
      v = ((double)(c - j) * seg[(long long)(kc - 1) * p + i] +
           (double)j * seg[(long long)(kn - 1) * p + i]) / c;
    }
    y[idx] += type == 4 ? mu_fac * v : v;
  }
}

// y = w y + (1 - w)(yold + P ec)
__global__ void k_weight(int p, int q, int n, double w, const double* __restrict__ yold,
                         const double* __restrict__ ec, int variant, double mu_scale,
                         double* __restrict__ y) {
  const TypeMajor Tm(p, q, n);
  const PrevIterate prev{yold, ec, p, q, n, variant, mu_scale};
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < Tm.len;
       idx += (long long)gridDim.x * blockDim.x) {
    int type, k, i;
    locate(idx, Tm, p, q, type, k, i);
    y[idx] = w * y[idx] + (1.0 - w) * prev.at(type, k, i);
  }
}

static inline int grid_for(long long len, int nt) {
  long long g = (len + nt - 1) / nt;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

// ---------------------------------------------------------------------------
// A~ z after a sweep.  When z = D^{-1}(b - (L+L^T) yprev) was the last sweep
// of a cycle, A~ z = D z + (L+L^T) z = b - (L+L^T)(yprev - z).  The only
// couplings are +I between u_k and mu_k, so the result is b except in the u
// and mu slots: w_u = b_u - (yprev_mu - z_mu), w_mu = b_mu - (yprev_u - z_u).
// ---------------------------------------------------------------------------

__global__ void k_apply_identity(int p, int q, int n, const double* __restrict__ b,
                                 const double* __restrict__ yprev,
                                 const double* __restrict__ z, double* __restrict__ w) {
  const TypeMajor T(p, q, n);
  const long long np = (long long)n * p;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < T.len;
       e += (long long)gridDim.x * blockDim.x) {
    double v = b[e];
    if (e < np) {
      v -= yprev[T.m + e] - z[T.m + e];
    } else if (e >= T.m) {
      const long long i = e - T.m;
      v -= yprev[T.u + i] - z[T.u + i];
    }
    w[e] = v;
  }
}

hipError_t launch_apply_identity(int p, int q, int n, const double* b, const double* yprev,
                                 const double* z, double* w, hipStream_t s) {
  const TypeMajor T(p, q, n);
  hipLaunchKernelGGL(k_apply_identity, dim3(grid_for(T.len, 256)), dim3(256), 0, s, p, q, n, b,
                     yprev, z, w);
  return hipGetLastError();
}


hipError_t launch_restrict_delta(int p, int q, int nf, const double* b, double beta,
                                 const double* ya, double a, const double* y, int variant,
                                 double mu_scale, double* bc, hipStream_t s) {
  const TypeMajor Tc(p, q, nf / 2);
  hipLaunchKernelGGL(k_restrict_delta, dim3(grid_for(Tc.len, 256)), dim3(256), 0, s, p, q, nf,
                     b, beta, ya, a, y, variant, mu_scale, bc);
  return hipGetLastError();
}

hipError_t launch_restrict(int p, int q, int nf, const double* r, int variant, double mu_scale,
                           double* bc, hipStream_t s) {
  const TypeMajor Tc(p, q, nf / 2);
  hipLaunchKernelGGL(k_restrict, dim3(grid_for(Tc.len, 256)), dim3(256), 0, s, p, q, nf, r,
                     variant, mu_scale, bc);
  return hipGetLastError();
}

hipError_t launch_interp_add(int p, int q, int nf, const double* e, int variant,
                             double mu_scale, double* y, hipStream_t s) {
  const TypeMajor Tf(p, q, nf);
  hipLaunchKernelGGL(k_interp_add, dim3(grid_for(Tf.len, 256)), dim3(256), 0, s, p, q, nf, e,
                     variant, mu_scale, y);
  return hipGetLastError();
}

hipError_t launch_restrict_c(int p, int q, int nf, int c, const double* r, double mu_fac,
                             double* bc, hipStream_t s) {
  const TypeMajor Tc(p, q, nf / c);
  hipLaunchKernelGGL(k_restrict_c, dim3(grid_for(Tc.len, 256)), dim3(256), 0, s, p, q, nf, c, r,
                     mu_fac, bc);
  return hipGetLastError();
}

hipError_t launch_interp_add_c(int p, int q, int nf, int c, const double* e, double mu_fac,
                               double* y, hipStream_t s) {
  const TypeMajor Tf(p, q, nf);
  hipLaunchKernelGGL(k_interp_add_c, dim3(grid_for(Tf.len, 256)), dim3(256), 0, s, p, q, nf, c,
                     e, mu_fac, y);
  return hipGetLastError();
}

hipError_t launch_weight(int p, int q, int n, double w, const double* yold, const double* ec,
                         int variant, double mu_scale, double* y, hipStream_t s) {
  const TypeMajor Tm(p, q, n);
  hipLaunchKernelGGL(k_weight, dim3(grid_for(Tm.len, 256)), dim3(256), 0, s, p, q, n, w, yold,
                     ec, variant, mu_scale, y);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K7: Krylov helpers.  Vectors are split into krylov_partial_blocks(len)
// contiguous slices, one work-group each; partial results are stored
// value-major ([value][slice]) and reduced by one wave per value, in a fixed
// order (no atomics, bitwise reproducible).
// ---------------------------------------------------------------------------

constexpr int kVecThreads = 256;
constexpr long long kSliceTarget = 1024;

int krylov_partial_blocks(long long len) {
  long long g = (len + kSliceTarget - 1) / kSliceTarget;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (int)g;
}

// slices of exactly kSliceLen elements for the dot / update kernels
int krylov_slices(long long len) { return (int)((len + 1023) / 1024); }

__device__ __forceinline__ void slice_of(long long len, long long& e0, long long& e1) {
  const long long per = (len + gridDim.x - 1) / gridDim.x;
  e0 = (long long)blockIdx.x * per;
  e1 = e0 + per < len ? e0 + per : len;
}

// Dots of a basis against one or two vectors over this work-group's slice,
// value-major partials:
//   value i          = basis_i . x1                 (i < nb)
//   value nb + i     = basis_i . x2                 (i < nb, when x2)
//   then x1.x1, and when x2 also x1.x2 and x2.x2.
// Each wave takes every 4th basis vector and keeps the slices of x1, x2 in
// registers (kSliceLen / 64 elements per lane): one coalesced pass over the
// basis, no barriers.
constexpr int kSliceLen = 1024;
constexpr int kPerLane = kSliceLen / kWave;

// The dot pass runs 4 waves per slice: every wave holds the slice of x1 and
// x2, and the waves share out the basis vectors.
constexpr int kDotThreads = 256;

__global__ __launch_bounds__(kDotThreads) void k_dots(const double* __restrict__ basis, int nb,
                                                      const double* __restrict__ x1,
                                                      const double* __restrict__ x2,
                                                      long long len,
                                                      double* __restrict__ partial) {
  const long long e0 = (long long)blockIdx.x * kSliceLen;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int nblk = gridDim.x;
  const bool two = x2 != nullptr;
  // blockIdx.y: a contiguous group of basis vectors (short-lived work-groups
  // that drain evenly; for short vectors also enough of them to fill the
  // device)
  const int per = (nb + gridDim.y - 1) / gridDim.y;
  const int i0 = blockIdx.y * per, i1 = min(nb, i0 + per);
  double a[kPerLane], c[kPerLane];
#pragma unroll
  for (int t = 0; t < kPerLane; ++t) {
    const long long e = e0 + lane + (long long)kWave * t;
    a[t] = e < len ? x1[e] : 0.0;
    c[t] = (two && e < len) ? x2[e] : 0.0;
  }
  for (int i = i0 + wv; i < i1; i += kDotThreads / kWave) {
    const double* __restrict__ bi = basis + (size_t)i * len;
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int t = 0; t < kPerLane; ++t) {
      const long long e = e0 + lane + (long long)kWave * t;
      const double bv = e < len ? bi[e] : 0.0;
      s1 += bv * a[t];
      s2 += bv * c[t];
    }
    s1 = wave_sum(s1);
    if (two) s2 = wave_sum(s2);
    if (lane == 0) {
      partial[(size_t)i * nblk + blockIdx.x] = s1;
      if (two) partial[(size_t)(nb + i) * nblk + blockIdx.x] = s2;
    }
  }
  if (wv == 0 && blockIdx.y == 0) {
    double s11 = 0.0, s12 = 0.0, s22 = 0.0;
#pragma unroll
    for (int t = 0; t < kPerLane; ++t) {
      s11 += a[t] * a[t];
      s12 += a[t] * c[t];
      s22 += c[t] * c[t];
    }
    s11 = wave_sum(s11);
    if (two) {
      s12 = wave_sum(s12);
      s22 = wave_sum(s22);
    }
    if (lane == 0) {
      const int base = two ? 2 * nb : nb;
      partial[(size_t)base * nblk + blockIdx.x] = s11;
      if (two) {
        partial[(size_t)(base + 1) * nblk + blockIdx.x] = s12;
        partial[(size_t)(base + 2) * nblk + blockIdx.x] = s22;
      }
    }
  }
}

// The two scalars of one delayed re-orthogonalisation step from the dot
// pass's results c (s = c[0..j), h = c[j..2j), v.v = c[2j], v.w = c[2j+1]):
//   alpha = sqrt(v.v - |s|^2)  (1 for j = 0),   cq = (v.w - s.h) / alpha,
// into out[0], out[1]; out[2] = 1 when v.v - |s|^2 is not positive and
// finite (the basis lost orthogonality; alpha is then left at 1).  One
// thread, the sums in index order.
__global__ void k_arnoldi_coeffs(const double* __restrict__ c, int j, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double ss = 0.0, sh = 0.0;
  for (int i = 0; i < j; ++i) {
    ss += c[i] * c[i];
    sh += c[i] * c[j + i];
  }
  double alpha = 1.0, bad = 0.0;
  if (j > 0) {
    const double a2 = c[2 * j] - ss;
    if (a2 > 0.0 && isfinite(a2)) alpha = sqrt(a2);
    else bad = 1.0;
  }
  out[0] = alpha;
  out[1] = (c[2 * j + 1] - sh) / alpha;
  out[2] = bad;
}

// Delayed re-orthogonalisation update over this work-group's slice:
//   q  = (x1 - basis^T s) / alpha     (written back to x1 when reorth)
//   x2 = x2 - basis^T h - c q
// with alpha = acq[0], c = acq[1] (device scalars), and norm_partial[slice]
// = sum of the new x2 squared.
__global__ __launch_bounds__(kVecThreads) void k_update(const double* __restrict__ basis, int nb,
                                                        double* __restrict__ x1,
                                                        double* __restrict__ x2,
                                                        const double* __restrict__ scoef,
                                                        const double* __restrict__ hcoef,
                                                        const double* __restrict__ acq,
                                                        int reorth, long long len,
                                                        double* __restrict__ norm_partial) {
  const double alpha = acq[0], cq = acq[1];
  __shared__ double red[kVecThreads / kWave];
  constexpr int kPer = kSliceLen / kVecThreads;
  const long long e0 = (long long)blockIdx.x * kSliceLen;
  double a1[kPer], a2[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    a1[t] = 0.0;
    a2[t] = 0.0;
  }
  for (int i = 0; i < nb; ++i) {
    const double* __restrict__ bi = basis + (size_t)i * len;
    const double si = scoef[i], hi = hcoef[i];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const long long e = e0 + threadIdx.x + (long long)kVecThreads * t;
      const double bv = e < len ? bi[e] : 0.0;
      a1[t] += si * bv;
      a2[t] += hi * bv;
    }
  }
  double nrm = 0.0;
  const double inv = 1.0 / alpha;
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const long long e = e0 + threadIdx.x + (long long)kVecThreads * t;
    if (e < len) {
      double q = x1[e];
      if (reorth) {
        q = (q - a1[t]) * inv;
        x1[e] = q;
      }
      const double u = x2[e] - a2[t] - cq * q;
      x2[e] = u;
      nrm += u * u;
    }
  }
  nrm = wave_sum(nrm);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kVecThreads / kWave; ++q) t += red[q];
    norm_partial[blockIdx.x] = t;
  }
}

// The update for short vectors, in two passes.  Pass 1, grid (slices,
// groups): part[g][0][e] = sum_{i in group g} s_i basis_i[e] and
// part[g][1][e] = sum h_i basis_i[e].  Pass 2, grid (slices): the group sums
// in order, then the same update and norm partials as k_update.
__global__ __launch_bounds__(kVecThreads) void k_update_part(const double* __restrict__ basis,
                                                             int nb,
                                                             const double* __restrict__ scoef,
                                                             const double* __restrict__ hcoef,
                                                             long long len,
                                                             double* __restrict__ part) {
  constexpr int kPer = kSliceLen / kVecThreads;
  const long long e0 = (long long)blockIdx.x * kSliceLen;
  const int per = (nb + gridDim.y - 1) / gridDim.y;
  const int i0 = blockIdx.y * per, i1 = min(nb, i0 + per);
  double a1[kPer], a2[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    a1[t] = 0.0;
    a2[t] = 0.0;
  }
  for (int i = i0; i < i1; ++i) {
    const double* __restrict__ bi = basis + (size_t)i * len;
    const double si = scoef[i], hi = hcoef[i];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const long long e = e0 + threadIdx.x + (long long)kVecThreads * t;
      const double bv = e < len ? bi[e] : 0.0;
      a1[t] += si * bv;
      a2[t] += hi * bv;
    }
  }
  double* p1 = part + (size_t)blockIdx.y * 2 * len;
  double* p2 = p1 + len;
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const long long e = e0 + threadIdx.x + (long long)kVecThreads * t;
    if (e < len) {
      p1[e] = a1[t];
      p2[e] = a2[t];
    }
  }
}

__global__ __launch_bounds__(kVecThreads) void k_update_apply(double* __restrict__ x1,
                                                              double* __restrict__ x2,
                                                              const double* __restrict__ part,
                                                              int ngroups,
                                                              const double* __restrict__ acq,
                                                              int reorth, long long len,
                                                              double* __restrict__ norm_partial) {
  const double alpha = acq[0], cq = acq[1];
  __shared__ double red[kVecThreads / kWave];
  constexpr int kPer = kSliceLen / kVecThreads;
  const long long e0 = (long long)blockIdx.x * kSliceLen;
  double nrm = 0.0;
  const double inv = 1.0 / alpha;
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const long long e = e0 + threadIdx.x + (long long)kVecThreads * t;
    if (e < len) {
      double a1 = 0.0, a2 = 0.0;
      for (int g = 0; g < ngroups; ++g) {
        a1 += part[(size_t)g * 2 * len + e];
        a2 += part[(size_t)g * 2 * len + len + e];
      }
      double q = x1[e];
      if (reorth) {
        q = (q - a1) * inv;
        x1[e] = q;
      }
      const double u = x2[e] - a2 - cq * q;
      x2[e] = u;
      nrm += u * u;
    }
  }
  nrm = wave_sum(nrm);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kVecThreads / kWave; ++q) t += red[q];
    norm_partial[blockIdx.x] = t;
  }
}

// out[i] = sum over slices of partial[i * nblk + slice]; one wave per value.
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ partial,
                                                         int nblk, int nval,
                                                         double* __restrict__ out) {
  const int i = blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (i >= nval) return;
  double s = 0.0;
  for (int b = lane; b < nblk; b += kWave) s += partial[(size_t)i * nblk + b];
  s = wave_sum(s);
  if (lane == 0) out[i] = s;
}

// w += sign * sum_i coef[i] basis_i; if norm_partial != NULL also
// norm_partial[slice] = sum over the slice of (new w)^2.
__global__ __launch_bounds__(kVecThreads) void k_multi_axpy(double* __restrict__ w,
                                                            const double* __restrict__ basis,
                                                            int nvec,
                                                            const double* __restrict__ coef,
                                                            double sign, long long len,
                                                            double* __restrict__ norm_partial) {
  __shared__ double red[kVecThreads / kWave];
  long long e0, e1;
  slice_of(len, e0, e1);
  double nrm = 0.0;
  for (long long e = e0 + threadIdx.x; e < e1; e += kVecThreads) {
    double acc = 0.0;
    int i = 0;
    for (; i + 4 <= nvec; i += 4) {
      acc += coef[i] * basis[(size_t)i * len + e];
      acc += coef[i + 1] * basis[(size_t)(i + 1) * len + e];
      acc += coef[i + 2] * basis[(size_t)(i + 2) * len + e];
      acc += coef[i + 3] * basis[(size_t)(i + 3) * len + e];
    }
    for (; i < nvec; ++i) acc += coef[i] * basis[(size_t)i * len + e];
    const double nw = w[e] + sign * acc;
    w[e] = nw;
    nrm += nw * nw;
  }
  if (norm_partial) {
    nrm = wave_sum(nrm);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < kVecThreads / kWave; ++q) t += red[q];
      norm_partial[blockIdx.x] = t;
    }
  }
}

__global__ void k_scale(double* __restrict__ dst, const double* __restrict__ src, double alpha,
                        long long len) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < len;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = alpha * src[e];
}

__global__ void k_axpby(double* __restrict__ y, const double* __restrict__ x, double a,
                        double b, long long len) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < len;
       e += (long long)gridDim.x * blockDim.x)
    y[e] = a * x[e] + b * y[e];
}

// Groups of basis vectors per launch of the dot and update passes: one when
// the vector alone gives enough work-groups, else enough groups of at least
// 8 vectors to bring the grid to about 1024 work-groups.
int krylov_groups(long long len, int nb) {
  const int sl = krylov_slices(len);
  if (sl >= 128 || nb < 16) return 1;
  const int by_size = (nb + 7) / 8;
  const int by_grid = (1024 + sl - 1) / sl;
  return std::max(1, std::min(by_size, by_grid));
}

// Basis groups of the dot pass: at most kDotGroup vectors per work-group.
// Each work-group then lives for a short stretch of the pass, so the grid
// drains evenly instead of ending on a partial round of long-lived groups
// (the slices of x1 and x2 are re-read per group, 2 / kDotGroup extra).
constexpr int kDotGroup = 32;

int dot_groups(long long len, int nb) {
  return std::max(krylov_groups(len, nb), (nb + kDotGroup - 1) / kDotGroup);
}

hipError_t launch_dots(const double* basis, int nb, const double* x1, const double* x2,
                       long long len, double* partial, hipStream_t s) {
  const int ng = dot_groups(len, nb);
  hipLaunchKernelGGL(k_dots, dim3(krylov_slices(len), ng), dim3(kDotThreads), 0, s, basis, nb,
                     x1, x2, len, partial);
  return hipGetLastError();
}

// One work-group per level (VZDiagBatch); the off-diagonal test over all
// threads by a barrier reduction.
__global__ __launch_bounds__(1024) void k_vz_diag(VZDiagBatch B, int* __restrict__ flags) {
  const int l = blockIdx.x, p = B.p;
  const double* __restrict__ V = B.V[l];
  const double* __restrict__ Z = B.Z[l];
  const long long pp = (long long)p * p;
  int off = 0;
  for (long long e = threadIdx.x; e < pp; e += blockDim.x) {
    const long long i = e / p, j = e % p;
    if (i != j && (V[e] != 0.0 || Z[e] != 0.0)) off = 1;
  }
  const int any = __syncthreads_or(off);
  for (int i = threadIdx.x; i < p; i += blockDim.x) {
    B.out[l][i] = V[(long long)i * p + i];
    B.out[l][p + i] = Z[(long long)i * p + i];
  }
  if (threadIdx.x == 0) flags[l] = any ? 0 : 1;
}

hipError_t launch_vz_diag(const VZDiagBatch& B, int* flags, hipStream_t s) {
  if (B.nlev < 1 || B.nlev > 20) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_vz_diag, dim3(B.nlev), dim3(1024), 0, s, B, flags);
  return hipGetLastError();
}

hipError_t launch_arnoldi_coeffs(const double* coef, int j, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_arnoldi_coeffs, dim3(1), dim3(kWave), 0, s, coef, j, out);
  return hipGetLastError();
}

hipError_t launch_update(const double* basis, int nb, double* x1, double* x2,
                         const double* scoef, const double* hcoef, const double* acq,
                         int reorth, long long len, double* norm_partial, double* scratch,
                         hipStream_t s) {
  const int ng = krylov_groups(len, nb);
  if (ng == 1 || !scratch) {
    hipLaunchKernelGGL(k_update, dim3(krylov_slices(len)), dim3(kVecThreads), 0, s, basis, nb,
                       x1, x2, scoef, hcoef, acq, reorth, len, norm_partial);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_update_part, dim3(krylov_slices(len), ng), dim3(kVecThreads), 0, s, basis,
                     nb, scoef, hcoef, len, scratch);
  hipLaunchKernelGGL(k_update_apply, dim3(krylov_slices(len)), dim3(kVecThreads), 0, s, x1, x2,
                     scratch, ng, acq, reorth, len, norm_partial);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partial, int nblk, int nval, double* out,
                                  hipStream_t s) {
  const int per = 256 / kWave;
  hipLaunchKernelGGL(k_reduce_partials, dim3((nval + per - 1) / per), dim3(256), 0, s, partial,
                     nblk, nval, out);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(double* w, const double* basis, int nvec, const double* coef,
                             double sign, long long len, double* norm_partial, hipStream_t s) {
  hipLaunchKernelGGL(k_multi_axpy, dim3(krylov_partial_blocks(len)), dim3(kVecThreads), 0, s,
                     w, basis, nvec, coef, sign, len, norm_partial);
  return hipGetLastError();
}

hipError_t launch_scale(double* dst, const double* src, double alpha, long long len,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(len, 256)), dim3(256), 0, s, dst, src, alpha, len);
  return hipGetLastError();
}

__global__ void k_fill(double* __restrict__ dst, double value, long long len) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < len;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = value;
}

hipError_t launch_fill(double* dst, double value, long long len, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(len, 256)), dim3(256), 0, s, dst, value, len);
  return hipGetLastError();
}

hipError_t launch_axpby(double* y, const double* x, double a, double b, long long len,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(len, 256)), dim3(256), 0, s, y, x, a, b, len);
  return hipGetLastError();
}

}  // namespace pitmg
