// Work-group level building blocks shared by the sweep, apply and coarse
// kernels: reductions, the generic block solve, the operator rows of one
// time step, and the two block-solve policies used by the coarse solver.
#pragma once
#include "pitmg_internal.h"
#include "pitmg_device.h"

namespace pitmg {

// Sum over the work-group; every thread returns the same value.  red must
// hold NT/64 doubles.  Fixed summation order (deterministic).
template <int NT>
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < NT / kWave; ++i) r += red[i];
  return r;
}

// out[j] = sum_{i in rows} A[i*lda + j] * x[i] for j < ncols; rows are
// 0..nrows-1, or j..nrows-1 when `lower`.  Consecutive threads take
// consecutive columns (coalesced rows); row slices are summed through part
// (NT doubles).  Ends with a barrier.
template <int NT, class T = double>
__device__ void col_dot(int nrows, int ncols, const T* __restrict__ A,
                        long long lda, const T* x, bool lower,
                        T* part, T* out) {
  const int tid = threadIdx.x;
  for (int j0 = 0; j0 < ncols; j0 += NT) {
    const int nc = min(NT, ncols - j0);
    const int G = NT / nc;
    const int jl = tid % nc, g = tid / nc;
    const int j = j0 + jl;
    T acc = 0;
    if (g < G) {
      int i = g;
      if (lower && j > g) i = g + ((j - g + G - 1) / G) * G;
      for (; i < nrows; i += G) acc += A[(long long)i * lda + j] * x[i];
      part[g * nc + jl] = acc;
    }
    __syncthreads();
    if (tid < nc) {
      T s = 0;
      for (int gg = 0; gg < G; ++gg) s += part[gg * nc + tid];
      out[j0 + tid] = s;
    }
    __syncthreads();
  }
}

// Solve D_k (v,u,z,lambda,mu) = (rv,ru,rz,rl,rm) for one time-step block with
// the whole work-group.  All vector arguments live in LDS; the matrices in
// global memory.  has_vm = false for block 1 (no v, mu; V unused).
template <int NT, class T = double>
__device__ void block_solve(int p, int q, const T* __restrict__ Nk,
                            const T* __restrict__ Vk,
                            const T* __restrict__ Zk,
                            const T* __restrict__ Gk, bool has_vm,
                            const T* rv, const T* ru, const T* rz,
                            const T* rl, const T* rm, T* ov,
                            T* ou, T* oz, T* ol, T* om,
                            T* t, T* s, T* part) {
  constexpr int NW = NT / kWave;
  const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
  // t = N r_u + Z r_z - V r_m - r_l   (row dots, one wave per row)
  for (int i = w; i < p; i += NW) {
    T acc = 0;
    const T* Ni = Nk + (long long)i * p;
    for (int j = lane; j < p; j += kWave) acc += Ni[j] * ru[j];
    if (has_vm) {
      const T* Vi = Vk + (long long)i * p;
      for (int j = lane; j < p; j += kWave) acc -= Vi[j] * rm[j];
    }
    const T* Zi = Zk + (long long)i * q;
    for (int j = lane; j < q; j += kWave) acc += Zi[j] * rz[j];
    acc = wave_sum(acc);
    if (lane == 0) t[i] = acc - rl[i];
  }
  __syncthreads();
  // s = G^{-1} t  (lower triangular)
  for (int i = w; i < p; i += NW) {
    T acc = 0;
    const T* Gr = Gk + (long long)i * p;
    for (int j = lane; j <= i; j += kWave) acc += Gr[j] * t[j];
    acc = wave_sum(acc);
    if (lane == 0) s[i] = acc;
  }
  __syncthreads();
  // lambda = G^{-T} s
  col_dot<NT, T>(p, p, Gk, p, s, true, part, ol);
  // u = r_u - N^T lambda ; z = r_z - Z^T lambda ; mu = V^T lambda - r_m - r_v
  col_dot<NT, T>(p, p, Nk, p, ol, false, part, ou);
  col_dot<NT, T>(p, q, Zk, q, ol, false, part, oz);
  if (has_vm) col_dot<NT, T>(p, p, Vk, p, ol, false, part, om);
  for (int i = tid; i < p; i += NT) {
    ou[i] = ru[i] - ou[i];
    if (has_vm) {
      om[i] = om[i] - rm[i] - rv[i];
      ov[i] = -rm[i];
    }
  }
  for (int i = tid; i < q; i += NT) oz[i] = rz[i] - oz[i];
  __syncthreads();
}

// LDS doubles used by one block solve: 5 inputs, 5 outputs, t, s, part.
__host__ __device__ inline size_t solve_lds_doubles(int p, int q, int nt) {
  return (size_t)8 * p + 2 * q + 2 * p + nt + (size_t)2 * p;
}

// Rows of time-major block k (1-based): v_{k-1}, u_k, z_k, lambda_k,
// mu_{k-1}; block n also writes block n+1's rows v_n, mu_n.
template <int NT>
__device__ void apply_step(const LevelView& L, int k, const double* __restrict__ x,
                           const double* __restrict__ b, double alpha, double beta,
                           double* __restrict__ out, double* sm) {
  const int p = L.p, q = L.q, n = L.n;
  const TypeMajor T(p, q, n);
  const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
  constexpr int NW = NT / kWave;
  const bool hv = k >= 2;
  const long long kk = k - 1;
  const double* Nk = L.N + kk * L.sN;
  const double* Vk = L.V + kk * L.sV;
  const double* Zk = L.Z + kk * L.sZ;
  double* xu = sm;
  double* xv = xu + p;
  double* xz = xv + p;
  double* xl = xz + q;
  double* t = xl + p;
  double* part = t + p;
  for (int i = tid; i < p; i += NT) {
    xu[i] = x[T.u + kk * p + i];
    xl[i] = x[T.l + kk * p + i];
    xv[i] = hv ? x[T.v + (kk - 1) * p + i] : 0.0;
  }
  for (int i = tid; i < q; i += NT) xz[i] = x[T.z + kk * q + i];
  __syncthreads();
  auto put = [&](long long idx, double val) {
    out[idx] = (beta != 0.0 ? beta * b[idx] : 0.0) + alpha * val;
  };
  // row lambda_k = N u_k + V v_{k-1} + Z z_k
  for (int i = w; i < p; i += NW) {
    double acc = 0.0;
    const double* Ni = Nk + (long long)i * p;
    for (int j = lane; j < p; j += kWave) acc += Ni[j] * xu[j];
    if (hv) {
      const double* Vi = Vk + (long long)i * p;
      for (int j = lane; j < p; j += kWave) acc += Vi[j] * xv[j];
    }
    const double* Zi = Zk + (long long)i * q;
    for (int j = lane; j < q; j += kWave) acc += Zi[j] * xz[j];
    acc = wave_sum(acc);
    if (lane == 0) put(T.l + kk * p + i, acc);
  }
  // rows u_k, z_k, v_{k-1}
  col_dot<NT>(p, p, Nk, p, xl, false, part, t);
  for (int i = tid; i < p; i += NT)
    put(T.u + kk * p + i, xu[i] + t[i] + x[T.m + kk * p + i]);
  __syncthreads();
  col_dot<NT>(p, q, Zk, q, xl, false, part, t);
  for (int i = tid; i < q; i += NT) put(T.z + kk * q + i, xz[i] + t[i]);
  __syncthreads();
  if (hv) {
    col_dot<NT>(p, p, Vk, p, xl, false, part, t);
    for (int i = tid; i < p; i += NT) {
      put(T.v + (kk - 1) * p + i, xv[i] + t[i] - x[T.m + (kk - 1) * p + i]);
      put(T.m + (kk - 1) * p + i, x[T.u + (kk - 1) * p + i] - xv[i]);
    }
    __syncthreads();
  }
  if (k == n) {
    for (int i = tid; i < p; i += NT) {
      const double vn = x[T.v + kk * p + i], mn = x[T.m + kk * p + i];
      put(T.v + kk * p + i, vn - mn);
      put(T.m + kk * p + i, xu[i] - vn);
    }
  }
  __syncthreads();
}

__host__ __device__ inline size_t apply_lds_doubles(int p, int q, int nt) {
  return (size_t)4 * p + q + nt + p;
}

}  // namespace pitmg
