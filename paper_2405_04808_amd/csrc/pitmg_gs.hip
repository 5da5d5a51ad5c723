// Forward and backward block Gauss-Seidel in time (Sec. 5.3.4: the FGS and
// BGS iterations, the symmetric one as their product), used as multigrid
// smoothers on the levels above the coarsest.
//
// In the time-major order of Fig. 5 the strictly lower block part L of A~
// has one nonzero block, +I from column u_{k-1} (block k-1) to row mu_{k-1}
// (block k).  Forward substitution (D + L) d = r therefore couples block k
// to the block before it only through u_{k-1}, and the block solve of the
// Schur form (pitmg_kernels.hip) gives, for a right-hand side x in the mu
// slot alone, u_k = N_k^T S_k^{-1} V_k x = Phi_k x.  Hence
//
//     u_1 = c_1,   u_k = c_k - Phi_k u_{k-1}   (k = 2 .. n),   c = u-part of D^{-1} r,
//
// after which d = D^{-1}(r - L u_hat) with u_hat the vector holding those u
// values (a block Jacobi solve with u_hat as its coupling iterate).  Backward
// substitution (D + L^T) d = r couples block k-1's u row to mu_{k-1} of
// block k, and a right-hand side x in the u slot alone gives
// mu_{k-1} = V_k^T S_k^{-1} N_k x = Phi_k^T x, so with e the mu-part of
// D^{-1} r:
//
//     mu_n = e_n,   mu_{k-1} = e_{k-1} - Phi_k^T mu_k   (k = n .. 2),
//
// then d = D^{-1}(r - L^T mu_hat).  Both recurrences are a chain of n - 1
// dependent p x p products: k_gs_chain runs one chain in one work-group of
// 1024 threads, each step a coalesced pass over the step's matrix (thread
// (row r, chunk c) reads the 16 entries M_s[16c .. 16c+15][r] with
// M_s = Phi_s^T for the forward and Phi_s for the backward chain, so
// consecutive threads read consecutive addresses, all 16 loads in flight at
// once), a sum over the chunks in LDS, and two barriers per step.  For
// p <= 128 each thread holds one (row, chunk) pair and loads the next step's
// entries while the current step's sums and barriers run.  This is the
// serial part the paper attributes to Gauss-Seidel smoothing: it does not
// parallelise in time.
#include "pitmg_internal.h"
#include "pitmg_device.h"

namespace pitmg {
namespace {

constexpr int kChainThreads = 1024;
constexpr int kCW = 16;                                 // columns per (row, chunk)

// PRE: every thread holds at most one (row, chunk) pair (p * ceil(p/16) <=
// 1024, i.e. p <= 128), so it can load the next step's 16 matrix values
// into registers while the current step's sums and barriers run.
template <bool PRE>
__global__ __launch_bounds__(kChainThreads) void k_gs_chain(int p, int q, int n,
                                                            const double* __restrict__ M,
                                                            const double* __restrict__ t,
                                                            double* __restrict__ hat,
                                                            int backward) {
  extern __shared__ double lds[];
  const int nch = (p + kCW - 1) / kCW;
  const int pairs = p * nch;
  double* part = lds;                                   // [nch][p]
  double* xs = lds + pairs;                             // [2][p]
  const int tid = threadIdx.x;
  const TypeMajor T(p, q, n);
  const long long slot = backward ? T.m : T.u;          // mu or u slots
  const long long pp = (long long)p * p;
  // step i of the chain: forward x_s = t_s - Phi_s x_{s-1} (M_s = Phi_s^T,
  // s = i); backward x_s = t_s - Phi_{s+1}^T x_{s+1} (M = Phi, s = n-1-i)
  auto step_of = [&](int i) { return backward ? n - 1 - i : i; };
  auto mat_of = [&](int i) {
    return M + (long long)(backward ? step_of(i) + 1 : step_of(i)) * pp;
  };
  const int c0 = tid / (p > 0 ? p : 1), r0 = tid % (p > 0 ? p : 1);
  double cur[kCW];
  if (PRE && tid < pairs && n > 1) {
    const double* Ms = mat_of(1);
#pragma unroll
    for (int jj = 0; jj < kCW; ++jj) {
      const int j = c0 * kCW + jj;
      cur[jj] = j < p ? Ms[(long long)j * p + r0] : 0.0;
    }
  }
  // first link: u_1 = c_1 (forward) or mu_n = e_n (backward)
  const int s0 = step_of(0);
  for (int r = tid; r < p; r += kChainThreads) {
    const double x = t[slot + (long long)s0 * p + r];
    xs[r] = x;
    hat[slot + (long long)s0 * p + r] = x;
  }
  __syncthreads();
  int pc = 0;
  for (int i = 1; i < n; ++i) {
    const int s = step_of(i);
    const double* xp = xs + pc * p;
    if (PRE) {
      if (tid < pairs) {
        double acc = 0.0;
#pragma unroll
        for (int jj = 0; jj < kCW; ++jj) {
          const int j = c0 * kCW + jj;
          acc += cur[jj] * (j < p ? xp[j] : 0.0);
        }
        part[tid] = acc;
        if (i + 1 < n) {                                // the next step's values
          const double* Mn = mat_of(i + 1);
#pragma unroll
          for (int jj = 0; jj < kCW; ++jj) {
            const int j = c0 * kCW + jj;
            cur[jj] = j < p ? Mn[(long long)j * p + r0] : 0.0;
          }
        }
      }
    } else {
      const double* Ms = mat_of(i);
      for (int idx = tid; idx < pairs; idx += kChainThreads) {
        const int c = idx / p, r = idx % p;
        double v[kCW];
#pragma unroll
        for (int jj = 0; jj < kCW; ++jj) {
          const int j = c * kCW + jj;
          v[jj] = j < p ? Ms[(long long)j * p + r] : 0.0;
        }
        double acc = 0.0;
#pragma unroll
        for (int jj = 0; jj < kCW; ++jj) {
          const int j = c * kCW + jj;
          acc += v[jj] * (j < p ? xp[j] : 0.0);
        }
        part[idx] = acc;
      }
    }
    __syncthreads();
    double* xn = xs + (pc ^ 1) * p;
    for (int r = tid; r < p; r += kChainThreads) {
      double sum = 0.0;
      for (int c = 0; c < nch; ++c) sum += part[c * p + r];
      const double x = t[slot + (long long)s * p + r] - sum;
      xn[r] = x;
      hat[slot + (long long)s * p + r] = x;
    }
    __syncthreads();
    pc ^= 1;
  }
}

}  // namespace

hipError_t launch_gs_chain(int p, int q, int n, const double* M, const double* t, double* hat,
                           int backward, hipStream_t s) {
  const int pairs = p * ((p + kCW - 1) / kCW);
  const size_t lds = (size_t)(pairs + 2 * p) * sizeof(double);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const bool pre = pairs <= kChainThreads;
  const void* fn = pre ? (const void*)k_gs_chain<true> : (const void*)k_gs_chain<false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (pre)
    return launch_k(k_gs_chain<true>, dim3(1), dim3(kChainThreads), lds, s, p, q, n, M, t, hat,
                    backward);
  return launch_k(k_gs_chain<false>, dim3(1), dim3(kChainThreads), lds, s, p, q, n, M, t, hat,
                  backward);
}

}  // namespace pitmg
