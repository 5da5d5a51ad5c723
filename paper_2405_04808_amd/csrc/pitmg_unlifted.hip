// The augmented system without virtual variables (Fig. 2, B = dF), in the
// type-major order x = [u_1..u_n | z_1..z_n | lambda_1..lambda_n]:
//
//     u_k row:       u_k + K_k^T lambda_k + C_{k+1}^T lambda_{k+1}   (C_{n+1} := 0)
//     z_k row:       z_k + B_k^T lambda_k
//     lambda_k row:  K_k u_k + C_k u_{k-1} + B_k z_k                 (u_0 := 0)
//
// with K_k, C_k, B_k the lifted blocks N_k, V_k, Z~_k at v = u (Sec. 5.1).
// A handle set up for this system holds sqrt2 N_k and sqrt2 V_k (the lifted
// problem whose exact solve, read through the maps below, is the unlifted
// inverse), so the product multiplies its N and V blocks by bscale = 1/sqrt2.
//
// Lift and project: E r = (u/sqrt2, u/sqrt2, z, lambda, 0) in the lifted
// type-major order, E^T y = ((u + v)/sqrt2, z, lambda).  E^T A~' E is the
// unlifted operator and E^T A~'^{-1} E its inverse, so E^T MG(E r) carries
// the lifted cycle to the unlifted system.
#include "pitmg_internal.h"
#include "pitmg_device.h"
#include "pitmg_onepass.h"

namespace pitmg {
namespace {

constexpr int kUnlThreads = 256;
constexpr int kUnlWaves = kUnlThreads / kWave;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
  return v;
}

// One work-group per step k: the step's three rows.  Row products (the
// lambda row) go a wave per row with the lanes across the columns; column
// products (the u and z rows) a thread per column, so both read the
// row-major blocks with consecutive lanes on consecutive addresses.
__global__ __launch_bounds__(kUnlThreads) void k_unlifted_apply(
    int p, int q, int n, const double* __restrict__ N, long long sN,
    const double* __restrict__ V, long long sV, const double* __restrict__ Z, long long sZ,
    double bscale, const double* __restrict__ x, const double* __restrict__ b, double alpha,
    double beta, double* __restrict__ out) {
  extern __shared__ double lds[];
  double* uk = lds;                 // u_k
  double* um = uk + p;              // u_{k-1}
  double* zk = um + p;              // z_k
  double* lk = zk + q;              // lambda_k
  double* ln = lk + p;              // lambda_{k+1}
  const int k = blockIdx.x, tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const long long pn = (long long)p * n, qn = (long long)q * n;
  const double* xu = x;
  const double* xz = x + pn;
  const double* xl = x + pn + qn;
  for (int i = tid; i < p; i += kUnlThreads) {
    uk[i] = xu[(long long)k * p + i];
    um[i] = k > 0 ? xu[(long long)(k - 1) * p + i] : 0.0;
    lk[i] = xl[(long long)k * p + i];
    ln[i] = k + 1 < n ? xl[(long long)(k + 1) * p + i] : 0.0;
  }
  for (int i = tid; i < q; i += kUnlThreads) zk[i] = xz[(long long)k * q + i];
  __syncthreads();
  const double* Nk = N + (long long)k * sN;
  const double* Vk = V + (long long)k * sV;
  const double* Vn = k + 1 < n ? V + (long long)(k + 1) * sV : nullptr;
  const double* Zk = Z + (long long)k * sZ;
  auto put = [&](long long idx, double val) {
    out[idx] = (beta != 0.0 ? beta * b[idx] : 0.0) + alpha * val;
  };
  // lambda row: bscale (N_k u_k + V_k u_{k-1}) + Z~_k z_k
  for (int i = w; i < p; i += kUnlWaves) {
    double a = 0.0, c = 0.0;
    for (int j = lane; j < p; j += kWave) {
      a += Nk[(long long)i * p + j] * uk[j];
      if (k > 0) a += Vk[(long long)i * p + j] * um[j];
    }
    for (int j = lane; j < q; j += kWave) c += Zk[(long long)i * q + j] * zk[j];
    const double s = wave_sum(bscale * a + c);
    if (lane == 0) put(pn + qn + (long long)k * p + i, s);
  }
  // u row: u_k + bscale (N_k^T lambda_k + V_{k+1}^T lambda_{k+1})
  for (int j = tid; j < p; j += kUnlThreads) {
    double a = 0.0;
    for (int i = 0; i < p; ++i) {
      a += Nk[(long long)i * p + j] * lk[i];
      if (Vn) a += Vn[(long long)i * p + j] * ln[i];
    }
    put((long long)k * p + j, uk[j] + bscale * a);
  }
  // z row: z_k + Z~_k^T lambda_k
  for (int j = tid; j < q; j += kUnlThreads) {
    double a = 0.0;
    for (int i = 0; i < p; ++i) a += Zk[(long long)i * q + j] * lk[i];
    put(pn + (long long)k * q + j, zk[j] + a);
  }
}

// The same rows for p = q = 64 MB with V and Z~ diagonal (shared by every
// step): one pass over N_k gives N u_k and N^T lambda_k (onepass_products),
// the V and Z~ terms are elementwise with their diagonals.
template <int MB>
__global__ __launch_bounds__(kOnePassThreads) void k_unlifted_apply_big(
    LevelView L, double bscale, const double* __restrict__ x, const double* __restrict__ b,
    double alpha, double beta, double* __restrict__ out) {
  constexpr int P = 64 * MB, NTH = kOnePassThreads, NW = kOnePassWaves;
  __shared__ double sl[P], srow[P];
  __shared__ double red[NW][P];
  const int tid = threadIdx.x, n = L.n, k = blockIdx.x;      // k 0-based
  const long long pn = (long long)P * n;
  const double* xu = x;
  const double* xz = x + pn;
  const double* xl = x + 2 * pn;
  for (int i = tid; i < P; i += NTH) sl[i] = xl[(long long)k * P + i];
  __syncthreads();
  onepass_products<MB>(L.N + (long long)k * L.sN, xu + (long long)k * P, sl, srow, red);
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
    const long long o = (long long)k * P + i;
    const double uk = xu[o], zk = xz[o], lk = sl[i];
    const double um = k > 0 ? xu[o - P] : 0.0;
    const double ln = k + 1 < n ? xl[o + P] : 0.0;
    // lambda row: bscale (N_k u_k + V u_{k-1}) + Z~ z_k
    put(2 * pn + o, bscale * (srow[i] + Vd[i] * um) + Zd[i] * zk);
    // u row: u_k + bscale (N_k^T lambda_k + V^T lambda_{k+1});  z row: z_k + Z~^T lambda_k
    put(o, uk + bscale * (nl + Vd[i] * ln));
    put(pn + o, zk + Zd[i] * lk);
  }
}

constexpr double kRsqrt2 = 0.70710678118654752440;

__global__ void k_lift(long long pn, long long qn, const double* __restrict__ r,
                       double* __restrict__ y) {
  const long long len = 4 * pn + qn;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < len;
       e += (long long)gridDim.x * blockDim.x) {
    double v;
    if (e < pn) v = kRsqrt2 * r[e];                           // u
    else if (e < 2 * pn) v = kRsqrt2 * r[e - pn];             // v
    else if (e < 3 * pn + qn) v = r[e - pn];                  // z, lambda
    else v = 0.0;                                             // mu
    y[e] = v;
  }
}

__global__ void k_project(long long pn, long long qn, const double* __restrict__ y,
                          double* __restrict__ x) {
  const long long len = 2 * pn + qn;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < len;
       e += (long long)gridDim.x * blockDim.x)
    x[e] = e < pn ? kRsqrt2 * (y[e] + y[e + pn]) : y[e + pn];
}

unsigned grid_for(long long len) {
  long long g = (len + 255) / 256;
  return (unsigned)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

}  // namespace

hipError_t launch_unlifted_apply(const LevelView& L, double bscale, const double* x,
                                 const double* b, double alpha, double beta, double* out,
                                 hipStream_t s) {
  const int MB = L.p / 64;
  const bool big = L.vz_diag && L.Vd && L.Zd && L.p == L.q && L.p % 64 == 0 &&
                   (MB == 1 || MB == 2 || MB == 4 || MB == 8) &&
                   ((reinterpret_cast<uintptr_t>(L.N) | reinterpret_cast<uintptr_t>(x)) & 15u) == 0;
  if (big) {
    const dim3 g(L.n), t(kOnePassThreads);
    switch (MB) {
      case 1: hipLaunchKernelGGL(k_unlifted_apply_big<1>, g, t, 0, s, L, bscale, x, b, alpha, beta, out); break;
      case 2: hipLaunchKernelGGL(k_unlifted_apply_big<2>, g, t, 0, s, L, bscale, x, b, alpha, beta, out); break;
      case 4: hipLaunchKernelGGL(k_unlifted_apply_big<4>, g, t, 0, s, L, bscale, x, b, alpha, beta, out); break;
      default: hipLaunchKernelGGL(k_unlifted_apply_big<8>, g, t, 0, s, L, bscale, x, b, alpha, beta, out); break;
    }
    return hipGetLastError();
  }
  const size_t lds = (size_t)(4 * L.p + L.q) * sizeof(double);
  hipLaunchKernelGGL(k_unlifted_apply, dim3(L.n), dim3(kUnlThreads), lds, s, L.p, L.q, L.n, L.N,
                     L.sN, L.V, L.sV, L.Z, L.sZ, bscale, x, b, alpha, beta, out);
  return hipGetLastError();
}

hipError_t launch_lift(int p, int q, int n, const double* r, double* y, hipStream_t s) {
  const long long pn = (long long)p * n, qn = (long long)q * n;
  hipLaunchKernelGGL(k_lift, dim3(grid_for(4 * pn + qn)), dim3(256), 0, s, pn, qn, r, y);
  return hipGetLastError();
}

hipError_t launch_project(int p, int q, int n, const double* y, double* x, hipStream_t s) {
  const long long pn = (long long)p * n, qn = (long long)q * n;
  hipLaunchKernelGGL(k_project, dim3(grid_for(2 * pn + qn)), dim3(256), 0, s, pn, qn, y, x);
  return hipGetLastError();
}

}  // namespace pitmg
