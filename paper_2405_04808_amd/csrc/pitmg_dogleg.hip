// Burgers' equation by Powell's dogleg with Gauss-Newton steps from
// minimum-norm augmented systems, and viscosity continuation (Sec. 6, the
// nonlinear solver of Sec. 6.2 and Table 6; the minimum-norm problem of
// Sec. 3).
//
// Unknowns x = [u_1..u_n | z~_1..z~_n] (p = q = nx per step), z~ = gamma z.
// State equation (backward Euler, upwind differences on nx interior nodes
// of [0, 1], h = 1/(nx+1), zero Dirichlet values, the convective term in
// flux form (u^2/2)_x by the backward difference):
//
//     F_k = (u_k - u_{k-1}) / dt - nu (u_{i+1} - 2 u_i + u_{i-1}) / h^2
//           + (u_i^2 - u_{i-1}^2) / (2h) - z~_k / gamma,        u_0 = w0.
//
// B = dF has the blocks of the unlifted augmented system (Fig. 2):
// dF_k/du_k = N_k (tridiagonal: 1/dt + 2 nu/h^2 + u_i/h on the diagonal,
// -(nu/h^2 + u_{i-1}/h) below, -nu/h^2 above), dF_k/du_{k-1} = V = -I/dt,
// dF_k/dz~_k = Z~ = -I/gamma.  Coarse levels take the states injected at
// the transfer's fine steps and their own time step c^l dt (Sec. 5.3.1).
//
// One dogleg iteration: the Gauss-Newton step s_N is the (u, z~) part of
// the unlifted solve A (s, y) = (0, -F) (FGMRES with the lifted cycle);
// g = B^T F and B g, B s come from unlifted products A (0, F) and A (v, 0);
// the dogleg point for radius delta, the ratio rho of actual to predicted
// decrease of |F|^2 / 2 and the radius update follow the standard
// trust-region form of Powell's method (constants in the header).
#include "../../include/pitmg.h"
#include "pitmg_internal.h"
#include "pitmg_device.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

namespace pitmg {
namespace {

thread_local std::string g_dogleg_err;

int dl_err(int code, const std::string& msg) {
  g_dogleg_err = msg;
  return code;
}

unsigned grid1(long long len) {
  long long g = (len + 255) / 256;
  return (unsigned)(g > 16384 ? 16384 : (g < 1 ? 1 : g));
}

// F(x) for steps k = 1..n, entry i (thread per entry).
__global__ void k_burgers_residual(int p, int n, double nu, double h, double dt, double gamma,
                                   const double* __restrict__ w0, const double* __restrict__ x,
                                   double* __restrict__ F) {
  const long long len = (long long)p * n;
  const double a = nu / (h * h);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < len;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / p), i = (int)(e % p);
    const double* u = x + (long long)k * p;
    const double ui = u[i];
    const double ul = i > 0 ? u[i - 1] : 0.0;
    const double ur = i + 1 < p ? u[i + 1] : 0.0;
    const double up = k > 0 ? x[(long long)(k - 1) * p + i] : w0[i];
    const double zt = x[len + e];
    const double f = a * (ur - 2.0 * ui + ul) - (ui * ui - ul * ul) / (2.0 * h) + zt / gamma;
    F[e] = (ui - up) / dt - f;
  }
}

// N_k of one level, dense row-major p x p per step, at the states of the
// fine steps f(k) = (first + k * stride) (0-based) of x.
__global__ void k_burgers_blocks(int p, int nl, long long first, long long stride, double nu,
                                 double h, double dt, const double* __restrict__ x,
                                 double* __restrict__ N) {
  const int k = blockIdx.y;
  const double* u = x + (first + (long long)k * stride) * p;
  const double a = nu / (h * h);
  double* Nk = N + (long long)k * p * p;
  const long long pp = (long long)p * p;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < pp;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / p), j = (int)(e % p);
    double v = 0.0;
    if (j == i) v = 1.0 / dt + 2.0 * a + u[i] / h;
    else if (j == i - 1) v = -(a + u[i - 1] / h);
    else if (j == i + 1) v = -a;
    Nk[e] = v;
  }
}

// value * I (p x p, dense)
__global__ void k_scaled_identity(int p, double value, double* __restrict__ M) {
  const long long pp = (long long)p * p;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < pp;
       e += (long long)gridDim.x * blockDim.x)
    M[e] = (e / p == e % p) ? value : 0.0;
}

// y = a x1 + b x2 (x2 may be NULL: b ignored)
__global__ void k_lincomb(long long len, double a, const double* __restrict__ x1, double b,
                          const double* __restrict__ x2, double* __restrict__ y) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < len;
       e += (long long)gridDim.x * blockDim.x)
    y[e] = a * x1[e] + (x2 ? b * x2[e] : 0.0);
}

// Unlifted vector [first (m) | 0 (m) ... ]: dst[0 .. off) = 0, dst[off ..
// off + m) = sign * src, dst[off + m .. len) = 0.
__global__ void k_place(long long len, long long off, long long m, double sign,
                        const double* __restrict__ src, double* __restrict__ dst) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < len;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = (e >= off && e < off + m) ? sign * src[e - off] : 0.0;
}

// Up to 8 dot products, one work-group of 1024 threads each, in a fixed
// order: out[j] = sum_e a_j[e] * b_j[e] (b_j = a_j for a squared norm).
struct DotJobs {
  const double* a[8];
  const double* b[8];
  long long len[8];
};
constexpr int kDotThreads = 1024;
__global__ __launch_bounds__(kDotThreads) void k_dot_jobs(DotJobs J, double* __restrict__ out) {
  __shared__ double red[kDotThreads / kWave];
  const int j = blockIdx.x;
  const double* a = J.a[j];
  const double* b = J.b[j];
  double s = 0.0;
  for (long long e = threadIdx.x; e < J.len[j]; e += kDotThreads) s += a[e] * b[e];
  s = wave_sum(s);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kDotThreads / kWave; ++w) t += red[w];
    out[j] = t;
  }
}

struct Dogleg {
  const pitmg_burgers* bp = nullptr;
  hipStream_t s = nullptr;
  int p = 0, n = 0, L = 0, c = 2, variant = 0;
  long long np = 0;
  double h = 0.0;
  std::vector<double*> N, V, Z;
  std::vector<int> nl;
  double *w0 = nullptr, *F = nullptr, *Fn = nullptr, *sN = nullptr, *g = nullptr, *sv = nullptr,
         *xt = nullptr, *ain = nullptr, *aout = nullptr, *rhs = nullptr, *sol = nullptr,
         *dsc = nullptr, *FBs = nullptr;
  double* hsc = nullptr;                 // pinned mirror of dsc
  pitmg_handle* hd = nullptr;
  std::vector<const double*> pn, pv, pz;
  pitmg_problem pb{};

  ~Dogleg() {
    if (hd) pitmg_destroy(hd);
    for (auto* q : N) (void)hipFree(q);
    for (auto* q : V) (void)hipFree(q);
    for (auto* q : Z) (void)hipFree(q);
    double* bufs[] = {w0, F, Fn, sN, g, sv, xt, ain, aout, rhs, sol, dsc, FBs};
    for (auto* q : bufs)
      if (q) (void)hipFree(q);
    if (hsc) (void)hipHostFree(hsc);
  }

  int alloc(double** q, long long count) {
    if (hipMalloc((void**)q, (size_t)count * sizeof(double)) != hipSuccess)
      return dl_err(PITMG_ERR_OOM, "device allocation failed");
    return PITMG_OK;
  }

  // blocks of every level at x and viscosity nu
  int blocks(const double* x, double nu) {
    long long stride = 1;
    for (int l = 0; l < L; ++l) {
      const double dt = bp->T * (double)stride / n;
      const long long first = variant == 0 ? 0 : stride - 1;
      const dim3 grid((unsigned)std::min<long long>(((long long)p * p + 255) / 256, 1024),
                      (unsigned)nl[l]);
      hipLaunchKernelGGL(k_burgers_blocks, grid, dim3(256), 0, s, p, nl[l], first, stride, nu, h,
                         dt, x, N[l]);
      stride *= c;
    }
    return hipGetLastError() == hipSuccess ? PITMG_OK
                                           : dl_err(PITMG_ERR_HIP, "block kernel launch failed");
  }

  int residual(const double* x, double nu, double* out) {
    hipLaunchKernelGGL(k_burgers_residual, dim3(grid1(np)), dim3(256), 0, s, p, n, nu, h,
                       bp->T / n, bp->gamma, w0, x, out);
    return hipGetLastError() == hipSuccess ? PITMG_OK
                                           : dl_err(PITMG_ERR_HIP, "residual kernel launch failed");
  }

  int lincomb(long long len, double a, const double* x1, double b, const double* x2, double* y) {
    hipLaunchKernelGGL(k_lincomb, dim3(grid1(len)), dim3(256), 0, s, len, a, x1, b, x2, y);
    return hipGetLastError() == hipSuccess ? PITMG_OK : dl_err(PITMG_ERR_HIP, "launch failed");
  }

  int place(long long off, long long m, double sign, const double* src, double* dst) {
    const long long len = 3 * np;
    hipLaunchKernelGGL(k_place, dim3(grid1(len)), dim3(256), 0, s, len, off, m, sign, src, dst);
    return hipGetLastError() == hipSuccess ? PITMG_OK : dl_err(PITMG_ERR_HIP, "launch failed");
  }

  // the dot jobs, read back into hsc[0 .. count)
  int dots(const DotJobs& J, int count) {
    hipLaunchKernelGGL(k_dot_jobs, dim3(count), dim3(kDotThreads), 0, s, J, dsc);
    if (hipGetLastError() != hipSuccess) return dl_err(PITMG_ERR_HIP, "launch failed");
    if (hipMemcpyAsync(hsc, dsc, count * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return dl_err(PITMG_ERR_HIP, "readback failed");
    return PITMG_OK;
  }

  // B v for v of length 2np: the lambda part of A (v, 0), into aout + 2np
  int bprod(const double* v) {
    int rc = place(0, 2 * np, 1.0, v, ain);
    if (rc) return rc;
    rc = pitmg_unlifted_apply(hd, ain, aout);
    return rc ? dl_err(rc, std::string("unlifted product: ") + pitmg_last_error(hd)) : PITMG_OK;
  }
};

}  // namespace
}  // namespace pitmg

using namespace pitmg;

extern "C" const char* pitmg_burgers_last_error(void) { return g_dogleg_err.c_str(); }

static int check_burgers(const pitmg_burgers* bp, int c) {
  if (!bp || !bp->w0) return dl_err(PITMG_ERR_INVALID, "null problem or w0");
  if (bp->nx < 2 || bp->n < 1 || bp->n_levels < 1)
    return dl_err(PITMG_ERR_INVALID, "nx >= 2, n >= 1 and n_levels >= 1 are needed");
  if (!(bp->T > 0.0) || !(bp->gamma > 0.0))
    return dl_err(PITMG_ERR_INVALID, "T and gamma must be positive");
  long long cl = 1;
  for (int l = 1; l < bp->n_levels; ++l) cl *= c;
  if (bp->n % cl != 0 || bp->n / cl < 1)
    return dl_err(PITMG_ERR_INVALID, "n must be divisible by coarsen^(n_levels-1)");
  return PITMG_OK;
}

extern "C" int pitmg_burgers_residual(const pitmg_burgers* bp, double nu, const double* x,
                                      double* F, void* stream) {
  int rc = check_burgers(bp, 2);
  if (rc) return rc;
  if (!x || !F) return dl_err(PITMG_ERR_INVALID, "null vector");
  Dogleg D;
  D.bp = bp;
  D.s = (hipStream_t)stream;
  D.p = bp->nx;
  D.n = bp->n;
  D.np = (long long)bp->nx * bp->n;
  D.h = 1.0 / (bp->nx + 1);
  if ((rc = D.alloc(&D.w0, D.p))) return rc;
  if (hipMemcpyAsync(D.w0, bp->w0, D.p * sizeof(double), hipMemcpyHostToDevice, D.s) != hipSuccess)
    return dl_err(PITMG_ERR_HIP, "copy of w0 failed");
  if ((rc = D.residual(x, nu, F))) return rc;
  if (hipStreamSynchronize(D.s) != hipSuccess) return dl_err(PITMG_ERR_HIP, "residual failed");
  return PITMG_OK;
}

extern "C" void pitmg_default_dogleg_params(pitmg_dogleg_params* dp) {
  if (!dp) return;
  dp->ftol = 1e-8;
  dp->lin_tol = 1e-6;
  dp->maxit = 50;
  dp->eta = 1e-4;
}

extern "C" int pitmg_burgers_dogleg(const pitmg_burgers* bp, const pitmg_options* opt,
                                    const double* nus, int n_nu, double* x,
                                    const pitmg_dogleg_params* dpar, pitmg_dogleg_stats* st,
                                    void* stream) {
  pitmg_options o;
  pitmg_default_options(&o);
  if (opt) o = *opt;
  o.unlifted = 1;
  int rc = check_burgers(bp, o.coarsen);
  if (rc) return rc;
  if (!x || !nus || n_nu < 1 || !st) return dl_err(PITMG_ERR_INVALID, "null argument");
  if (o.transfer_variant == 1 && o.coarsen != 2)
    return dl_err(PITMG_ERR_INVALID, "transfer variant 1 needs coarsen = 2");
  pitmg_dogleg_params dp;
  pitmg_default_dogleg_params(&dp);
  if (dpar) dp = *dpar;
  if (!(dp.ftol > 0.0) || !(dp.lin_tol > 0.0) || dp.maxit < 1)
    return dl_err(PITMG_ERR_INVALID, "ftol, lin_tol > 0 and maxit >= 1 are needed");
  for (int i = 0; i < n_nu; ++i)
    if (!(nus[i] >= 0.0)) return dl_err(PITMG_ERR_INVALID, "viscosities must be >= 0");

  Dogleg D;
  D.bp = bp;
  D.s = (hipStream_t)stream;
  D.p = bp->nx;
  D.n = bp->n;
  D.L = bp->n_levels;
  D.c = o.coarsen;
  D.variant = o.transfer_variant;
  D.np = (long long)bp->nx * bp->n;
  D.h = 1.0 / (bp->nx + 1);
  const int p = D.p;
  const long long np = D.np, pp = (long long)p * p;
  {
    int nlv = D.n;
    for (int l = 0; l < D.L; ++l) {
      D.nl.push_back(nlv);
      nlv /= D.c;
    }
  }
  D.N.assign(D.L, nullptr);
  D.V.assign(D.L, nullptr);
  D.Z.assign(D.L, nullptr);
  for (int l = 0; l < D.L; ++l) {
    if ((rc = D.alloc(&D.N[l], (long long)D.nl[l] * pp))) return rc;
    if ((rc = D.alloc(&D.V[l], pp))) return rc;
    if ((rc = D.alloc(&D.Z[l], pp))) return rc;
  }
  double** vecs2[] = {&D.sN, &D.g, &D.sv, &D.xt};
  for (auto** q : vecs2)
    if ((rc = D.alloc(q, 2 * np))) return rc;
  double** vecs3[] = {&D.ain, &D.aout, &D.rhs, &D.sol};
  for (auto** q : vecs3)
    if ((rc = D.alloc(q, 3 * np))) return rc;
  if ((rc = D.alloc(&D.F, np)) || (rc = D.alloc(&D.Fn, np)) || (rc = D.alloc(&D.FBs, np)) ||
      (rc = D.alloc(&D.w0, p)) || (rc = D.alloc(&D.dsc, 8)))
    return rc;
  if (hipHostMalloc((void**)&D.hsc, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return dl_err(PITMG_ERR_OOM, "pinned allocation failed");
  if (hipMemcpyAsync(D.w0, bp->w0, p * sizeof(double), hipMemcpyHostToDevice, D.s) != hipSuccess)
    return dl_err(PITMG_ERR_HIP, "copy of w0 failed");
  {
    long long stride = 1;
    for (int l = 0; l < D.L; ++l) {
      const double dt = bp->T * (double)stride / D.n;
      hipLaunchKernelGGL(k_scaled_identity, dim3(grid1(pp)), dim3(256), 0, D.s, p, -1.0 / dt,
                         D.V[l]);
      hipLaunchKernelGGL(k_scaled_identity, dim3(grid1(pp)), dim3(256), 0, D.s, p,
                         -1.0 / bp->gamma, D.Z[l]);
      stride *= D.c;
    }
  }
  D.pn.assign(D.N.begin(), D.N.end());
  D.pv.assign(D.V.begin(), D.V.end());
  D.pz.assign(D.Z.begin(), D.Z.end());
  D.pb.p = p;
  D.pb.q = p;
  D.pb.n = D.n;
  D.pb.n_levels = D.L;
  D.pb.N = D.pn.data();
  D.pb.V = D.pv.data();
  D.pb.Z = D.pz.data();
  D.pb.N_stride = pp;
  D.pb.V_stride = 0;
  D.pb.Z_stride = 0;
  D.pb.blocks_on_device = 1;
  if ((rc = D.blocks(x, nus[0]))) return rc;
  if ((rc = pitmg_setup(&D.hd, &D.pb, &o, stream)))
    return dl_err(rc, "setup of the augmented solver failed");

  for (int iv = 0; iv < n_nu; ++iv) {
    const double nu = nus[iv];
    const auto t0 = std::chrono::steady_clock::now();
    pitmg_dogleg_stats S{};
    if ((rc = D.residual(x, nu, D.F))) return rc;
    DotJobs J{};
    J.a[0] = J.b[0] = D.F;
    J.len[0] = np;
    if ((rc = D.dots(J, 1))) return rc;
    double ff = D.hsc[0];
    const double f0 = std::sqrt(ff);
    S.fnorm0 = f0;
    double delta = -1.0;
    // the factored blocks are those of (x, nu) unless x moved or nu changed
    // (setup factored them at the first viscosity and the starting point)
    bool stale = iv > 0;
    for (int it = 0; it < dp.maxit; ++it) {
      if (std::sqrt(ff) <= dp.ftol * f0 || f0 == 0.0) {
        S.converged = 1;
        break;
      }
      if (stale) {
        if ((rc = D.blocks(x, nu))) return rc;
        if ((rc = pitmg_refactor(D.hd, &D.pb)))
          return dl_err(rc, std::string("refactor: ") + pitmg_last_error(D.hd));
        stale = false;
      }
      // Gauss-Newton step: A (s, y) = (0, -F)
      if ((rc = D.place(2 * np, np, -1.0, D.F, D.rhs))) return rc;
      pitmg_stats ls{};
      rc = pitmg_unlifted_fgmres_solve(D.hd, D.rhs, D.sol, dp.lin_tol, 0, &ls);
      if (rc < 0) return dl_err(rc, std::string("Gauss-Newton solve: ") + pitmg_last_error(D.hd));
      S.solves += 1;
      S.fgmres_iters += ls.iters;
      S.coarse_calls += ls.coarse_calls;
      S.coarse_its += ls.coarse_its_total;
      if ((rc = D.lincomb(2 * np, 1.0, D.sol, 0.0, nullptr, D.sN))) return rc;
      // g = B^T F (the (u, z~) part of A (0, F)), then B g
      if ((rc = D.place(2 * np, np, 1.0, D.F, D.ain))) return rc;
      if ((rc = pitmg_unlifted_apply(D.hd, D.ain, D.aout)))
        return dl_err(rc, std::string("unlifted product: ") + pitmg_last_error(D.hd));
      if ((rc = D.lincomb(2 * np, 1.0, D.aout, 0.0, nullptr, D.g))) return rc;
      if ((rc = D.bprod(D.g))) return rc;
      DotJobs K{};
      K.a[0] = K.b[0] = D.sN;
      K.len[0] = 2 * np;
      K.a[1] = K.b[1] = D.g;
      K.len[1] = 2 * np;
      K.a[2] = K.b[2] = D.aout + 2 * np;
      K.len[2] = np;
      K.a[3] = D.g;
      K.b[3] = D.sN;
      K.len[3] = 2 * np;
      if ((rc = D.dots(K, 4))) return rc;
      const double nN2 = D.hsc[0], gg = D.hsc[1], bgbg = D.hsc[2], gsN = D.hsc[3];
      const double nN = std::sqrt(nN2);
      if (delta < 0.0) delta = nN;
      // the dogleg point s = al sN + be g
      double al = 1.0, be = 0.0;
      if (nN > delta) {
        if (gg == 0.0) {
          al = delta / nN;
        } else {
          const double tau = gg / bgbg;
          const double nC = tau * std::sqrt(gg);
          if (nC >= delta) {
            al = 0.0;
            be = -delta / std::sqrt(gg);
          } else {
            // |sC + b (sN - sC)| = delta with sC = -tau g
            const double a2 = nN2 + 2.0 * tau * gsN + tau * tau * gg;
            const double b2 = 2.0 * (-tau * gsN - tau * tau * gg);
            const double c2 = tau * tau * gg - delta * delta;
            const double bt = (-b2 + std::sqrt(b2 * b2 - 4.0 * a2 * c2)) / (2.0 * a2);
            al = bt;
            be = -(1.0 - bt) * tau;
          }
        }
      }
      if ((rc = D.lincomb(2 * np, al, D.sN, be, D.g, D.sv))) return rc;
      if ((rc = D.lincomb(2 * np, 1.0, x, 1.0, D.sv, D.xt))) return rc;
      if ((rc = D.residual(D.xt, nu, D.Fn))) return rc;
      if ((rc = D.bprod(D.sv))) return rc;
      if ((rc = D.lincomb(np, 1.0, D.F, 1.0, D.aout + 2 * np, D.FBs))) return rc;
      DotJobs M{};
      M.a[0] = M.b[0] = D.Fn;
      M.len[0] = np;
      M.a[1] = M.b[1] = D.FBs;
      M.len[1] = np;
      M.a[2] = M.b[2] = D.sv;
      M.len[2] = 2 * np;
      if ((rc = D.dots(M, 3))) return rc;
      const double fn2 = D.hsc[0], model2 = D.hsc[1], ns = std::sqrt(D.hsc[2]);
      const double pred = ff - model2, ared = ff - fn2;
      const double rho = pred > 0.0 ? ared / pred : -1.0;
      if (!std::isfinite(fn2)) return dl_err(PITMG_ERR_NONFINITE, "residual not finite");
      if (rho < 0.25) delta = 0.25 * ns;
      else if (rho > 0.75 && ns >= 0.99 * delta) delta = 2.0 * delta;
      S.iters += 1;
      if (rho > dp.eta) {
        if (hipMemcpyAsync(x, D.xt, 2 * np * sizeof(double), hipMemcpyDeviceToDevice, D.s) !=
                hipSuccess ||
            hipMemcpyAsync(D.F, D.Fn, np * sizeof(double), hipMemcpyDeviceToDevice, D.s) !=
                hipSuccess)
          return dl_err(PITMG_ERR_HIP, "copy failed");
        ff = fn2;
        S.accepted += 1;
        stale = true;
      }
    }
    if (!S.converged && std::sqrt(ff) <= dp.ftol * f0) S.converged = 1;
    if (hipStreamSynchronize(D.s) != hipSuccess) return dl_err(PITMG_ERR_HIP, "sync failed");
    S.fnorm = std::sqrt(ff);
    S.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st[iv] = S;
  }
  for (int iv = 0; iv < n_nu; ++iv)
    if (!st[iv].converged) return PITMG_NOT_CONVERGED;
  return PITMG_OK;
}
