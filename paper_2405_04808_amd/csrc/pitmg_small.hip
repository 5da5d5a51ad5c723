// Block Jacobi sweep and operator apply for small blocks (p, q <= 4, e.g.
// van der Pol with p = 2): one thread per time step, the step's blocks and
// vectors in registers.  A work-group per step would spend its time on
// barriers for a 9-unknown block; here a level of n steps is n threads.
//
// Block algebra as in pitmg_kernels.hip (Schur complement in lambda):
//     t = N r_u + Z r_z - V r_m - r_l,  lambda = G^{-T} G^{-1} t,
//     u = r_u - N^T lambda,  z = r_z - Z^T lambda,
//     mu = V^T lambda - r_m - r_v,  v = -r_m,
// and block n+1: v_n = -r_m, mu_n = -r_m - r_v.
#include "pitmg_internal.h"
#include "pitmg_device.h"

#include <type_traits>

namespace pitmg {
namespace {

constexpr int kSmallThreads = 256;

template <int P, int Q, class T>
__global__ __launch_bounds__(kSmallThreads) void k_jacobi_small(LevelView L,
                                                                 const double* __restrict__ b,
                                                                 const double* __restrict__ yold,
                                                                 const double* __restrict__ ec,
                                                                 int variant,
                                                                 double* __restrict__ ynew) {
  const int n = L.n;
  const int kb = blockIdx.x * kSmallThreads + threadIdx.x;
  if (kb > n) return;
  const TypeMajor Tm(P, Q, n);
  const double w = L.omega;
  // the iterate the sweep starts from: yold + P ec (couplings in u and mu)
  const PrevIterate prev{yold, ec, P, Q, n, variant, L.mu_scale};
  auto cu = [&](int k1, int i) -> double { return prev.at(0, k1, i); };
  auto cm = [&](int k1, int i) -> double { return prev.at(4, k1, i); };
  if (kb == n) {                                 // block n+1 = (v_n, mu_n)
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const double rvv = b[Tm.v + (long long)(n - 1) * P + i];
      const double rmm = b[Tm.m + (long long)(n - 1) * P + i] - cu(n, i);
      ynew[Tm.v + (long long)(n - 1) * P + i] = weigh(w, -rmm, prev, 1, n, i);
      ynew[Tm.m + (long long)(n - 1) * P + i] = weigh(w, -rmm - rvv, prev, 4, n, i);
    }
    return;
  }
  const int k = kb + 1;
  const bool hv = k >= 2;
  const long long kk = k - 1;
  T ru[P], rl[P], rv[P], rm[P], rz[Q];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    ru[i] = (T)(b[Tm.u + kk * P + i] - cm(k, i));
    rl[i] = (T)b[Tm.l + kk * P + i];
    rv[i] = hv ? (T)b[Tm.v + (kk - 1) * P + i] : T(0);
    rm[i] = hv ? (T)(b[Tm.m + (kk - 1) * P + i] - cu(k - 1, i)) : T(0);
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) rz[j] = (T)b[Tm.z + kk * Q + j];
  const T* __restrict__ N = Mats<T>::N(L) + kk * L.sN;
  const T* __restrict__ V = Mats<T>::V(L) + kk * L.sV;
  const T* __restrict__ Z = Mats<T>::Z(L) + kk * L.sZ;
  const T* __restrict__ G = Mats<T>::Gi(L) + kk * P * P;
  T t[P], s[P], lam[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    T acc = 0;
#pragma unroll
    for (int j = 0; j < P; ++j) acc += N[i * P + j] * ru[j];
    if (hv) {
#pragma unroll
      for (int j = 0; j < P; ++j) acc -= V[i * P + j] * rm[j];
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) acc += Z[i * Q + j] * rz[j];
    t[i] = acc - rl[i];
  }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    T acc = 0;
#pragma unroll
    for (int j = 0; j <= i; ++j) acc += G[i * P + j] * t[j];
    s[i] = acc;
  }
#pragma unroll
  for (int j = 0; j < P; ++j) {
    T acc = 0;
#pragma unroll
    for (int i = j; i < P; ++i) acc += G[i * P + j] * s[i];
    lam[j] = acc;
  }
#pragma unroll
  for (int j = 0; j < P; ++j) {
    T nu = 0, vu = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      nu += N[i * P + j] * lam[i];
      if (hv) vu += V[i * P + j] * lam[i];
    }
    ynew[Tm.u + kk * P + j] = weigh(w, (double)(ru[j] - nu), prev, 0, k, j);
    ynew[Tm.l + kk * P + j] = weigh(w, (double)lam[j], prev, 3, k, j);
    if (hv) {
      ynew[Tm.v + (kk - 1) * P + j] = weigh(w, (double)(-rm[j]), prev, 1, k - 1, j);
      ynew[Tm.m + (kk - 1) * P + j] = weigh(w, (double)(vu - rm[j] - rv[j]), prev, 4, k - 1, j);
    }
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    T zu = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) zu += Z[i * Q + j] * lam[i];
    ynew[Tm.z + kk * Q + j] = weigh(w, (double)(rz[j] - zu), prev, 2, k, j);
  }
}

// out = beta*b + alpha*(A~ x): thread k-1 writes the rows of time-major
// block k (v_{k-1}, u_k, z_k, lambda_k, mu_{k-1}) and, for k = n, block n+1.
template <int P, int Q>
__global__ __launch_bounds__(kSmallThreads) void k_apply_small(LevelView L,
                                                                const double* __restrict__ x,
                                                                const double* __restrict__ b,
                                                                double alpha, double beta,
                                                                double* __restrict__ out) {
  const int n = L.n;
  const int k = blockIdx.x * kSmallThreads + threadIdx.x + 1;
  if (k > n) return;
  const TypeMajor T(P, Q, n);
  const bool hv = k >= 2;
  const long long kk = k - 1;
  const double* __restrict__ N = L.N + kk * L.sN;
  const double* __restrict__ V = L.V + kk * L.sV;
  const double* __restrict__ Z = L.Z + kk * L.sZ;
  double xu[P], xl[P], xv[P], xz[Q];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    xu[i] = x[T.u + kk * P + i];
    xl[i] = x[T.l + kk * P + i];
    xv[i] = hv ? x[T.v + (kk - 1) * P + i] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) xz[j] = x[T.z + kk * Q + j];
  auto put = [&](long long idx, double val) {
    out[idx] = (beta != 0.0 ? beta * b[idx] : 0.0) + alpha * val;
  };
#pragma unroll
  for (int i = 0; i < P; ++i) {                  // lambda_k = N u_k + V v_{k-1} + Z z_k
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) acc += N[i * P + j] * xu[j];
    if (hv) {
#pragma unroll
      for (int j = 0; j < P; ++j) acc += V[i * P + j] * xv[j];
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) acc += Z[i * Q + j] * xz[j];
    put(T.l + kk * P + i, acc);
  }
#pragma unroll
  for (int j = 0; j < P; ++j) {                  // u_k, v_{k-1}, mu_{k-1}
    double nt = 0.0, vt = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      nt += N[i * P + j] * xl[i];
      if (hv) vt += V[i * P + j] * xl[i];
    }
    put(T.u + kk * P + j, xu[j] + nt + x[T.m + kk * P + j]);
    if (hv) {
      put(T.v + (kk - 1) * P + j, xv[j] + vt - x[T.m + (kk - 1) * P + j]);
      put(T.m + (kk - 1) * P + j, x[T.u + (kk - 1) * P + j] - xv[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {                  // z_k
    double zt = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) zt += Z[i * Q + j] * xl[i];
    put(T.z + kk * Q + j, xz[j] + zt);
  }
  if (k == n) {                                  // block n+1
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const double vn = x[T.v + kk * P + i], mn = x[T.m + kk * P + i];
      put(T.v + kk * P + i, vn - mn);
      put(T.m + kk * P + i, xu[i] - vn);
    }
  }
}

template <class F>
hipError_t dispatch_pq(int p, int q, F&& f) {
#define PITMG_PQ(P_, Q_) \
  if (p == P_ && q == Q_) return f(std::integral_constant<int, P_>{}, std::integral_constant<int, Q_>{});
  PITMG_PQ(1, 1) PITMG_PQ(1, 2) PITMG_PQ(1, 3) PITMG_PQ(1, 4)
  PITMG_PQ(2, 1) PITMG_PQ(2, 2) PITMG_PQ(2, 3) PITMG_PQ(2, 4)
  PITMG_PQ(3, 1) PITMG_PQ(3, 2) PITMG_PQ(3, 3) PITMG_PQ(3, 4)
  PITMG_PQ(4, 1) PITMG_PQ(4, 2) PITMG_PQ(4, 3) PITMG_PQ(4, 4)
#undef PITMG_PQ
  return hipErrorInvalidValue;
}

}  // namespace

bool small_supported(int p, int q) { return p >= 1 && p <= 4 && q >= 1 && q <= 4; }

hipError_t launch_jacobi_small(const LevelView& L, const double* b, const double* yold,
                               const double* ecoarse, int variant, double* ynew, hipStream_t s) {
  const dim3 grid((L.n + 1 + kSmallThreads - 1) / kSmallThreads);
  return dispatch_pq(L.p, L.q, [&](auto P_, auto Q_) {
    constexpr int P = decltype(P_)::value, Q = decltype(Q_)::value;
    if (L.fp32)
      return launch_k(k_jacobi_small<P, Q, float>, grid, dim3(kSmallThreads), 0, s, L, b, yold,
                      ecoarse, variant, ynew);
    return launch_k(k_jacobi_small<P, Q, double>, grid, dim3(kSmallThreads), 0, s, L, b, yold,
                    ecoarse, variant, ynew);
  });
}

hipError_t launch_apply_small(const LevelView& L, const double* x, const double* b, double alpha,
                              double beta, double* out, hipStream_t s) {
  const dim3 grid((L.n + kSmallThreads - 1) / kSmallThreads);
  return dispatch_pq(L.p, L.q, [&](auto P_, auto Q_) {
    constexpr int P = decltype(P_)::value, Q = decltype(Q_)::value;
    hipLaunchKernelGGL((k_apply_small<P, Q>), grid, dim3(kSmallThreads), 0, s, L, x, b, alpha,
                       beta, out);
    return hipGetLastError();
  });
}

}  // namespace pitmg
