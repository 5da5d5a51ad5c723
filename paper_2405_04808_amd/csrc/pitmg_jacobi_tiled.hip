// Block Jacobi sweep for p = q in {64, 128}: one work-group of 512 threads
// per time-major block, with N_k and G_k^{-1} in registers (pitmg_tiled.h),
// so each Jacobian / factor entry is read from HBM once per sweep.
#include "pitmg_internal.h"
#include "pitmg_device.h"
#include "pitmg_tiled.h"

namespace pitmg {

template <int RT, int CT>
__global__ __launch_bounds__(kTiledThreads, 1) void k_jacobi_tiled(
    LevelView L, const double* __restrict__ b, const double* __restrict__ yold,
    const double* __restrict__ ec, int variant, double* __restrict__ ynew) {
  using TS = TiledSolve<RT, CT>;
  constexpr int P = TS::P;
  __shared__ double sru[P], srz[P], srm[P], srl[P], srv[P], slam[P];
  __shared__ double scr[TS::kScratch];
  const int tid = threadIdx.x;
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
  typename TS::Regs R;
  TS::load(L, kk, R);                          // HBM loads in flight during the gather
  // right-hand side with the coupling values of the previous iterate:
  // r_u = b_u,k - mu_k, r_mu = b_mu,k-1 - u_{k-1}
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
  TS::solve(L, kk, hv, R, sru, srz, srm, srl, slam, scr);
  for (int i = tid; i < P; i += kTiledThreads) {
    ynew[T.u + kk * P + i] = TS::u_of(scr, sru, i);
    ynew[T.z + kk * P + i] = TS::z_of(scr, srz, i);
    ynew[T.l + kk * P + i] = slam[i];
    if (hv) {
      ynew[T.m + (kk - 1) * P + i] = TS::mu_of(scr, srm, srv, i);
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
