// Block Jacobi sweep for p = q = 32*RT = 16*CT with the Jacobian block N_k and
// the inverse Cholesky factor G_k^{-1} held in registers.
//
// One work-group of 512 threads (8 waves) per time-major block.  Thread
// (a, b) = (tid / 16, tid % 16) owns rows [RT a, RT a + RT) and columns
// [CT b, CT b + CT) of both matrices, so every entry of N_k and of the lower
// triangle of G_k^{-1} is read from HBM exactly once per sweep and serves
// both the row products (t = N r_u + ..., s = G^{-1} t) and the column
// products (lambda = G^{-T} s, N^T lambda).  Row sums reduce over the 16
// lanes sharing a; column sums reduce over the 4 row groups in a wave
// (lane xor 16, 32) and then over the 8 waves through LDS, in a fixed
// order.  V_k and Z~_k are read in the same tile shape (from L2 when one
// block is shared by every step).  The block algebra is the Schur form
// documented in pitmg_kernels.hip.
#include "pitmg_internal.h"
#include "pitmg_device.h"

namespace pitmg {

namespace {

constexpr int kTiledThreads = 512;
constexpr int kTiledWaves = kTiledThreads / kWave;

template <int CT>
__device__ __forceinline__ void load_row(const double* __restrict__ src, double (&dst)[CT]) {
#pragma unroll
  for (int c = 0; c < CT; c += 2) {
    const double2 v = *reinterpret_cast<const double2*>(src + c);
    dst[c] = v.x;
    dst[c + 1] = v.y;
  }
}

__device__ __forceinline__ double sum16(double v) {
  v += __shfl_xor(v, 8, kWave);
  v += __shfl_xor(v, 4, kWave);
  v += __shfl_xor(v, 2, kWave);
  v += __shfl_xor(v, 1, kWave);
  return v;
}

// Column partials of one thread -> per-wave slot of red (lanes 0..15 write).
template <int P, int CT>
__device__ __forceinline__ void col_partial(double (&v)[CT], double (*red)[P]) {
  const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave, bq = tid % 16;
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    v[c] += __shfl_xor(v[c], 16, kWave);
    v[c] += __shfl_xor(v[c], 32, kWave);
  }
  if (lane < 16) {
#pragma unroll
    for (int c = 0; c < CT; ++c) red[w][CT * bq + c] = v[c];
  }
}

template <int P>
__device__ __forceinline__ double col_total(const double (*red)[P], int j) {
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kTiledWaves; ++w) s += red[w][j];
  return s;
}

}  // namespace

template <int RT, int CT>
__global__ __launch_bounds__(kTiledThreads, 1) void k_jacobi_tiled(
    LevelView L, const double* __restrict__ b, const double* __restrict__ yold,
    const double* __restrict__ ec, int variant, double* __restrict__ ynew) {
  constexpr int P = 32 * RT;
  static_assert(P == 16 * CT, "tile shape");
  __shared__ double sru[P], srz[P], srm[P], srl[P], srv[P], st[P], ss[P], slam[P];
  __shared__ double red[3][kTiledWaves][P];
  const int tid = threadIdx.x, a = tid / 16, bq = tid % 16;
  const int n = L.n;
  const TypeMajor T(P, P, n);
  const int nc = n / 2;
  const TypeMajor Tc(P, P, nc > 0 ? nc : 1);
  const int kb = blockIdx.x;

  auto cu = [&](int k1, int i) -> double {
    double v = yold ? yold[T.u + (long long)(k1 - 1) * P + i] : 0.0;
    if (ec) v += interp_node(ec + Tc.u, nc, P, k1, i, variant);
    return v;
  };
  auto cm = [&](int k1, int i) -> double {
    double v = yold ? yold[T.m + (long long)(k1 - 1) * P + i] : 0.0;
    if (ec) v += interp_node(ec + Tc.m, nc, P, k1, i, variant);
    return v;
  };

  if (kb == n) {                               // block n+1 = (v_n, mu_n)
    for (int i = tid; i < P; i += kTiledThreads) {
      const double rvv = b[T.v + (long long)(n - 1) * P + i];
      const double rmm = b[T.m + (long long)(n - 1) * P + i] - cu(n, i);
      ynew[T.v + (long long)(n - 1) * P + i] = -rmm;
      ynew[T.m + (long long)(n - 1) * P + i] = -rmm - rvv;
    }
    return;
  }
  const int k = kb + 1;
  const bool hv = k >= 2;
  const long long kk = k - 1;
  const double* __restrict__ Nk = L.N + kk * L.sN;
  const double* __restrict__ Gk = L.Gi + kk * (long long)P * P;
  const double* __restrict__ Vk = L.V + kk * L.sV;
  const double* __restrict__ Zk = L.Z + kk * L.sZ;
  const int r0 = RT * a, c0 = CT * bq;

  // register tiles: every HBM byte of N_k and of G_k^{-1}'s lower part once
  double nt[RT][CT], gt[RT][CT];
#pragma unroll
  for (int r = 0; r < RT; ++r) load_row<CT>(Nk + (long long)(r0 + r) * P + c0, nt[r]);
  const bool gnz = c0 <= r0 + RT - 1;          // tile meets the lower triangle
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    if (gnz) {
      load_row<CT>(Gk + (long long)(r0 + r) * P + c0, gt[r]);
    } else {
#pragma unroll
      for (int c = 0; c < CT; ++c) gt[r][c] = 0.0;
    }
  }
  // right-hand side of this block with the coupling values of the previous
  // iterate: r_u = b_u,k - mu_k, r_mu = b_mu,k-1 - u_{k-1}
  for (int i = tid; i < P; i += kTiledThreads) {
    sru[i] = b[T.u + kk * P + i] - cm(k, i);
    srl[i] = b[T.l + kk * P + i];
    srz[i] = b[T.z + kk * P + i];
    if (hv) {
      srv[i] = b[T.v + (kk - 1) * P + i];
      srm[i] = b[T.m + (kk - 1) * P + i] - cu(k - 1, i);
    } else {
      srv[i] = 0.0;
      srm[i] = 0.0;
    }
  }
  __syncthreads();

  // t = N r_u + Z r_z - V r_m - r_l
  double acc[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < CT; ++c) s += nt[r][c] * sru[c0 + c];
    double zr[CT];
    load_row<CT>(Zk + (long long)(r0 + r) * P + c0, zr);
#pragma unroll
    for (int c = 0; c < CT; ++c) s += zr[c] * srz[c0 + c];
    if (hv) {
      double vr[CT];
      load_row<CT>(Vk + (long long)(r0 + r) * P + c0, vr);
#pragma unroll
      for (int c = 0; c < CT; ++c) s -= vr[c] * srm[c0 + c];
    }
    acc[r] = sum16(s);
  }
  if (bq == 0) {
#pragma unroll
    for (int r = 0; r < RT; ++r) st[r0 + r] = acc[r] - srl[r0 + r];
  }
  __syncthreads();

  // s = G^{-1} t
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < CT; ++c) s += gt[r][c] * st[c0 + c];
    acc[r] = sum16(s);
  }
  if (bq == 0) {
#pragma unroll
    for (int r = 0; r < RT; ++r) ss[r0 + r] = acc[r];
  }
  __syncthreads();

  // lambda = G^{-T} s
  double cacc[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < RT; ++r) s += gt[r][c] * ss[r0 + r];
    cacc[c] = s;
  }
  col_partial<P, CT>(cacc, red[0]);
  __syncthreads();
  for (int j = tid; j < P; j += kTiledThreads) slam[j] = col_total<P>(red[0], j);
  __syncthreads();

  // N^T lambda, Z^T lambda, V^T lambda
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < RT; ++r) s += nt[r][c] * slam[r0 + r];
    cacc[c] = s;
  }
  col_partial<P, CT>(cacc, red[0]);
  {
    double zacc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) zacc[c] = 0.0;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      double zr[CT];
      load_row<CT>(Zk + (long long)(r0 + r) * P + c0, zr);
#pragma unroll
      for (int c = 0; c < CT; ++c) zacc[c] += zr[c] * slam[r0 + r];
    }
    col_partial<P, CT>(zacc, red[1]);
  }
  if (hv) {
    double vacc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) vacc[c] = 0.0;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      double vr[CT];
      load_row<CT>(Vk + (long long)(r0 + r) * P + c0, vr);
#pragma unroll
      for (int c = 0; c < CT; ++c) vacc[c] += vr[c] * slam[r0 + r];
    }
    col_partial<P, CT>(vacc, red[2]);
  }
  __syncthreads();

  // u = r_u - N^T lambda, z = r_z - Z^T lambda, mu = V^T lambda - r_m - r_v,
  // v = -r_m
  for (int i = tid; i < P; i += kTiledThreads) {
    ynew[T.u + kk * P + i] = sru[i] - col_total<P>(red[0], i);
    ynew[T.z + kk * P + i] = srz[i] - col_total<P>(red[1], i);
    ynew[T.l + kk * P + i] = slam[i];
    if (hv) {
      ynew[T.m + (kk - 1) * P + i] = col_total<P>(red[2], i) - srm[i] - srv[i];
      ynew[T.v + (kk - 1) * P + i] = -srm[i];
    }
  }
}

bool jacobi_tiled_supported(int p, int q) { return p == q && (p == 128 || p == 64); }

hipError_t launch_jacobi_tiled(const LevelView& L, const double* b, const double* yold,
                               const double* ecoarse, int variant, double* ynew,
                               hipStream_t s) {
  if (L.p == 128 && L.q == 128) {
    hipLaunchKernelGGL((k_jacobi_tiled<4, 8>), dim3(L.n + 1), dim3(kTiledThreads), 0, s, L, b,
                       yold, ecoarse, variant, ynew);
  } else if (L.p == 64 && L.q == 64) {
    hipLaunchKernelGGL((k_jacobi_tiled<2, 4>), dim3(L.n + 1), dim3(kTiledThreads), 0, s, L, b,
                       yold, ecoarse, variant, ynew);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pitmg
