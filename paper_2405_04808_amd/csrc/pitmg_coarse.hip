// Coarsest-grid solve: GMRES right-preconditioned by symmetric block
// Gauss-Seidel (Sec. 5.3.4), from x0 = 0 to a relative residual tolerance
// (or a fixed number of steps), entirely inside one work-group.
//
// SGS couples the time blocks only through p-vectors: the forward sweep
// (D + L) a = r needs u_{k-1} in row mu_{k-1}, the backward sweep
// (D + L^T) y = D a needs mu_k in row u_k.  With the block propagator
//     Phi_k = N_k^T S_k^{-1} V_k     (S_k = N_k N_k^T + Z~_k Z~_k^T),
// the u-part of the forward result obeys a_u[k] = c_u[k] - Phi_k a_u[k-1]
// with c = D^{-1} r, and the mu-part of the backward result obeys
// y_mu[k-1] = a_mu[k-1] - Phi_k^T y_mu[k].  Both recurrences are linear, so
// their solutions are products with precomputed block-triangular matrices
// P (forward) and Q (backward) built from the Phi_k at setup.  One SGS
// application is then three block-parallel sweeps (c = D^{-1} r;
// a = D^{-1}(r - L a) with a_u known; d = -D^{-1} L^T y with y_mu known;
// result a + d) and two parallel triangular products -- no walk over the
// blocks.  The GMRES control (Arnoldi with modified Gram-Schmidt, Givens
// rotations, the stopping test) runs in a one-work-group kernel per step
// with its state in device memory, so the host never waits.  The host
// enqueues as many steps as the previous coarse solve needed; if a solve
// needs more, a one-work-group kernel finishes it with the sequential
// block sweep (same SGS, walked block by block).
#include "pitmg_internal.h"
#include "pitmg_device.h"
#include "pitmg_blocks.h"
#include "pitmg_mfma.h"
#include "pitmg_tiled.h"

namespace pitmg {

namespace {

// Block solve with every output left in LDS (ov, ou, oz, ol, om).
template <int NT>
struct GenericPolicy {
  static constexpr int kThreads = NT;
  struct Regs {};
  __host__ __device__ static size_t scratch(int p, int /*q*/) { return (size_t)2 * p + NT; }
  __device__ static void load(const LevelView&, long long, Regs&) {}
  __device__ static void solve(const LevelView& L, long long kk, bool hv, Regs&,
                               const double* rv, const double* ru, const double* rz,
                               const double* rl, const double* rm, double* ov, double* ou,
                               double* oz, double* ol, double* om, double* scr) {
    const int p = L.p, q = L.q;
    block_solve<NT>(p, q, L.N + kk * L.sN, L.V + kk * L.sV, L.Z + kk * L.sZ,
                    L.Gi + kk * p * p, hv, rv, ru, rz, rl, rm, ov, ou, oz, ol, om, scr,
                    scr + p, scr + 2 * p);
  }
};

struct CoarseLds {
  double *rv, *ru, *rz, *rl, *rm, *ov, *ou, *oz, *ol, *om, *scr, *app;
};

template <int NT>
__device__ double wg_dot(const double* a, const double* b, long long len, double* red) {
  double acc = 0.0;
  for (long long i = threadIdx.x; i < len; i += NT) acc += a[i] * b[i];
  return block_sum<NT>(acc, red);
}

// dst = M^{-1} src for M = (D+L) D^{-1} (D+L^T): forward block sweep into a,
// then the backward sweep dst_k = a_k - D_k^{-1} (L^T dst)_k.  The only
// coupling is mu_{k-1} <- u_{k-1} (forward) and u_k <- mu_k (backward).
template <class Pol>
__device__ void sgs_apply(const LevelView& L, const double* src, double* a, double* dst,
                          const CoarseLds& S) {
  constexpr int NT = Pol::kThreads;
  const int p = L.p, q = L.q, n = L.n;
  const TypeMajor T(p, q, n);
  const int tid = threadIdx.x;
  typename Pol::Regs R;
  for (int kb = 0; kb <= n; ++kb) {
    if (kb == n) {                             // block n+1 = (v_n, mu_n)
      for (int i = tid; i < p; i += NT) {
        const long long o = (long long)(n - 1) * p + i;
        const double rmm = src[T.m + o] - a[T.u + o];
        a[T.v + o] = -rmm;
        a[T.m + o] = -rmm - src[T.v + o];
      }
      __syncthreads();
      break;
    }
    const int k = kb + 1;
    const bool hv = k >= 2;
    const long long kk = k - 1;
    Pol::load(L, kk, R);
    for (int i = tid; i < p; i += NT) {
      S.ru[i] = src[T.u + kk * p + i];
      S.rl[i] = src[T.l + kk * p + i];
      S.rv[i] = hv ? src[T.v + (kk - 1) * p + i] : 0.0;
      S.rm[i] = hv ? src[T.m + (kk - 1) * p + i] - a[T.u + (kk - 1) * p + i] : 0.0;
    }
    for (int i = tid; i < q; i += NT) S.rz[i] = src[T.z + kk * q + i];
    __syncthreads();
    Pol::solve(L, kk, hv, R, S.rv, S.ru, S.rz, S.rl, S.rm, S.ov, S.ou, S.oz, S.ol, S.om, S.scr);
    for (int i = tid; i < p; i += NT) {
      a[T.u + kk * p + i] = S.ou[i];
      a[T.l + kk * p + i] = S.ol[i];
      if (hv) {
        a[T.v + (kk - 1) * p + i] = S.ov[i];
        a[T.m + (kk - 1) * p + i] = S.om[i];
      }
    }
    for (int i = tid; i < q; i += NT) a[T.z + kk * q + i] = S.oz[i];
    __syncthreads();
  }
  for (int i = tid; i < p; i += NT) {          // block n+1 has no upper coupling
    const long long o = (long long)(n - 1) * p + i;
    dst[T.v + o] = a[T.v + o];
    dst[T.m + o] = a[T.m + o];
  }
  __syncthreads();
  for (int k = n; k >= 1; --k) {
    const bool hv = k >= 2;
    const long long kk = k - 1;
    Pol::load(L, kk, R);
    for (int i = tid; i < p; i += NT) {
      S.rv[i] = 0.0;
      S.rm[i] = 0.0;
      S.rl[i] = 0.0;
      S.ru[i] = dst[T.m + kk * p + i];          // (L^T dst) in row u_k is mu_k
    }
    for (int i = tid; i < q; i += NT) S.rz[i] = 0.0;
    __syncthreads();
    Pol::solve(L, kk, hv, R, S.rv, S.ru, S.rz, S.rl, S.rm, S.ov, S.ou, S.oz, S.ol, S.om, S.scr);
    for (int i = tid; i < p; i += NT) {
      dst[T.u + kk * p + i] = a[T.u + kk * p + i] - S.ou[i];
      dst[T.l + kk * p + i] = a[T.l + kk * p + i] - S.ol[i];
      if (hv) {
        dst[T.v + (kk - 1) * p + i] = a[T.v + (kk - 1) * p + i] - S.ov[i];
        dst[T.m + (kk - 1) * p + i] = a[T.m + (kk - 1) * p + i] - S.om[i];
      }
    }
    for (int i = tid; i < q; i += NT) dst[T.z + kk * q + i] = a[T.z + kk * q + i] - S.oz[i];
    __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// GMRES state in device memory (capacity cap steps)
// ---------------------------------------------------------------------------

struct CState {
  int cap;
  __host__ __device__ static size_t doubles(int cap) {
    return 1 + (size_t)(cap + 1) * cap + 2 * (size_t)cap + (cap + 1) + cap;
  }
  __device__ double& beta(double* c) const { return c[0]; }
  __device__ double* H(double* c) const { return c + 1; }
  __device__ double* cs(double* c) const { return c + 1 + (size_t)(cap + 1) * cap; }
  __device__ double* sn(double* c) const { return cs(c) + cap; }
  __device__ double* g(double* c) const { return sn(c) + cap; }
  __device__ double* y(double* c) const { return g(c) + cap + 1; }
};

// One Arnoldi step on the coarse Krylov basis: w = A z_j is orthogonalised
// against v_0..v_j (modified Gram-Schmidt), column j of H is rotated, and
// the stopping test is taken.  ist = {steps done, stop}.  Returns stop.
template <int NT>
__device__ bool arnoldi_step(int j, double* __restrict__ wv, double* __restrict__ Vb,
                             long long len, double* cst,
                             int* ist, CState S, double tol, int fixed_its, int nsteps,
                             double* red, int* sflag) {
  const int tid = threadIdx.x;
  const double w0 = sqrt(wg_dot<NT>(wv, wv, len, red));
  double* H = S.H(cst);
  for (int i = 0; i <= j; ++i) {
    const double* vi = Vb + (size_t)i * len;
    const double h = wg_dot<NT>(wv, vi, len, red);
    for (long long e = tid; e < len; e += NT) wv[e] -= h * vi[e];
    if (tid == 0) H[(size_t)i * S.cap + j] = h;
    __syncthreads();
  }
  const double hn = sqrt(wg_dot<NT>(wv, wv, len, red));
  if (tid == 0) {
    double* cs = S.cs(cst);
    double* sn = S.sn(cst);
    double* g = S.g(cst);
    const int cap = S.cap;
    H[(size_t)(j + 1) * cap + j] = hn;
    for (int i = 0; i < j; ++i) {
      const double a0 = H[(size_t)i * cap + j], a1 = H[(size_t)(i + 1) * cap + j];
      H[(size_t)i * cap + j] = cs[i] * a0 + sn[i] * a1;
      H[(size_t)(i + 1) * cap + j] = -sn[i] * a0 + cs[i] * a1;
    }
    const double a0 = H[(size_t)j * cap + j], a1 = hn;
    const double r = hypot(a0, a1);
    cs[j] = r > 0.0 ? a0 / r : 1.0;
    sn[j] = r > 0.0 ? a1 / r : 0.0;
    H[(size_t)j * cap + j] = r;
    H[(size_t)(j + 1) * cap + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    const double res = fabs(g[j + 1]);
    int st = fixed_its > 0 ? (j + 1 == fixed_its) : (res <= tol * S.beta(cst));
    if (!st && hn <= 1e-14 * w0) st = 1;
    if (j + 1 >= nsteps) st = 1;
    ist[0] = j + 1;
    ist[1] = st;
    *sflag = st;
  }
  __syncthreads();
  const bool stop = *sflag != 0;
  if (!stop) {
    double* vn = Vb + (size_t)(j + 1) * len;
    for (long long e = tid; e < len; e += NT) vn[e] = wv[e] / hn;
  }
  __syncthreads();
  return stop;
}

constexpr int kCtrlThreads = 512;

__global__ __launch_bounds__(kCtrlThreads) void k_coarse_init(const double* __restrict__ b,
                                                              long long len, double* Vb,
                                                              double* cst, int* ist, int cap) {
  __shared__ double red[kCtrlThreads / kWave];
  const CState S{cap};
  const double beta = sqrt(wg_dot<kCtrlThreads>(b, b, len, red));
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (long long e = threadIdx.x; e < len; e += kCtrlThreads) Vb[e] = b[e] * inv;
  if (threadIdx.x == 0) {
    S.beta(cst) = beta;
    double* g = S.g(cst);
    g[0] = beta;
    for (int i = 1; i <= cap; ++i) g[i] = 0.0;
    ist[0] = 0;
    ist[1] = beta > 0.0 ? 0 : 1;
  }
}

__global__ __launch_bounds__(kCtrlThreads) void k_coarse_arnoldi(int j, double* wv, double* Vb,
                                                                 long long len, double* cst,
                                                                 int* ist, int cap, double tol,
                                                                 int fixed_its, int nsteps) {
  __shared__ double red[kCtrlThreads / kWave];
  __shared__ int sflag;
  if (ist[1]) return;                          // solved at an earlier step
  arnoldi_step<kCtrlThreads>(j, wv, Vb, len, cst, ist, CState{cap}, tol, fixed_its, nsteps,
                             red, &sflag);
}

// The same step, with the SGS result and its product formed first from the
// two sweeps: z_j = a + d and A~ z_j without reading the blocks.  With
// (D + L) a = v (forward sweep) and (D + L^T) z = D a (backward sweep,
// d = z - a), D z = v - L a - L^T z, so A~ z = (D + L + L^T) z = v + L d;
// L is the identity from u_k into row mu_k (k = 1..n), hence w = v except
// w_mu = v_mu + d_u (mu0 = offset of the mu segment).
__global__ __launch_bounds__(kCtrlThreads) void k_coarse_arnoldi_sgs(
    int j, double* __restrict__ wv, double* __restrict__ Vb, double* __restrict__ zj,
    const double* __restrict__ a, const double* __restrict__ d, long long mu0, long long len,
    double* cst, int* ist, int cap, double tol, int fixed_its, int nsteps) {
  __shared__ double red[kCtrlThreads / kWave];
  __shared__ int sflag;
  if (ist[1]) return;                          // solved at an earlier step
  const double* __restrict__ v = Vb + (size_t)j * len;
  for (long long e = threadIdx.x; e < len; e += kCtrlThreads) {
    zj[e] = a[e] + d[e];
    wv[e] = e >= mu0 ? v[e] + d[e - mu0] : v[e];
  }
  __syncthreads();
  arnoldi_step<kCtrlThreads>(j, wv, Vb, len, cst, ist, CState{cap}, tol, fixed_its, nsteps,
                             red, &sflag);
}

// The same step with w held in registers: thread t keeps entries t, t + NT,
// ... (at most MAXE) of w, so the orthogonalisation makes no round trip
// through memory.  The sums and updates are those of arnoldi_step in the
// same order (per-thread partials in index order, then block_sum), so the
// results are the same doubles; w is stored back at the end.
template <int NT, int MAXE>
__global__ __launch_bounds__(NT) void k_coarse_arnoldi_sgs_reg(
    int j, double* __restrict__ wv, double* __restrict__ Vb, double* __restrict__ zj,
    const double* __restrict__ a, const double* __restrict__ d, long long mu0, long long len,
    double* cst, int* ist, int cap, double tol, int fixed_its, int nsteps) {
  __shared__ double red[NT / kWave];
  __shared__ int sflag;
  if (ist[1]) return;                          // solved at an earlier step
  const int tid = threadIdx.x;
  const CState S{cap};
  const double* __restrict__ v = Vb + (size_t)j * len;
  double w[MAXE];
#pragma unroll
  for (int k = 0; k < MAXE; ++k) {
    const long long e = tid + (long long)k * NT;
    w[k] = 0.0;
    if (e < len) {
      zj[e] = a[e] + d[e];
      w[k] = e >= mu0 ? v[e] + d[e - mu0] : v[e];
    }
  }
  auto dot_w = [&](const double* __restrict__ x) -> double {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < MAXE; ++k) {
      const long long e = tid + (long long)k * NT;
      if (e < len) acc += w[k] * (x ? x[e] : w[k]);
    }
    return block_sum<NT>(acc, red);
  };
  const double w0 = sqrt(dot_w(nullptr));
  double* H = S.H(cst);
  for (int i = 0; i <= j; ++i) {
    const double* __restrict__ vi = Vb + (size_t)i * len;
    const double h = dot_w(vi);
#pragma unroll
    for (int k = 0; k < MAXE; ++k) {
      const long long e = tid + (long long)k * NT;
      if (e < len) w[k] -= h * vi[e];
    }
    if (tid == 0) H[(size_t)i * S.cap + j] = h;
  }
  const double hn = sqrt(dot_w(nullptr));
  if (tid == 0) {
    double* cs = S.cs(cst);
    double* sn = S.sn(cst);
    double* g = S.g(cst);
    H[(size_t)(j + 1) * cap + j] = hn;
    for (int i = 0; i < j; ++i) {
      const double a0 = H[(size_t)i * cap + j], a1 = H[(size_t)(i + 1) * cap + j];
      H[(size_t)i * cap + j] = cs[i] * a0 + sn[i] * a1;
      H[(size_t)(i + 1) * cap + j] = -sn[i] * a0 + cs[i] * a1;
    }
    const double a0 = H[(size_t)j * cap + j], a1 = hn;
    const double r = hypot(a0, a1);
    cs[j] = r > 0.0 ? a0 / r : 1.0;
    sn[j] = r > 0.0 ? a1 / r : 0.0;
    H[(size_t)j * cap + j] = r;
    H[(size_t)(j + 1) * cap + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    const double res = fabs(g[j + 1]);
    int st = fixed_its > 0 ? (j + 1 == fixed_its) : (res <= tol * S.beta(cst));
    if (!st && hn <= 1e-14 * w0) st = 1;
    if (j + 1 >= nsteps) st = 1;
    ist[0] = j + 1;
    ist[1] = st;
    sflag = st;
  }
  __syncthreads();
  const bool stop = sflag != 0;
  double* vn = Vb + (size_t)(j + 1) * len;
#pragma unroll
  for (int k = 0; k < MAXE; ++k) {
    const long long e = tid + (long long)k * NT;
    if (e < len) {
      wv[e] = w[k];
      if (!stop) vn[e] = w[k] / hn;
    }
  }
}

// Finish the coarse solve: continue block by block if the enqueued steps did
// not meet the test, then x = Z y with H y = g.
template <class Pol>
__global__ __launch_bounds__(Pol::kThreads) void k_coarse_finish(
    LevelView L, double* __restrict__ x, double tol, int fixed_its, int nsteps,
    double* __restrict__ work, double* cst, int* ist, int cap, int* its_out) {
  constexpr int NT = Pol::kThreads;
  extern __shared__ double sm[];
  const int p = L.p, q = L.q, n = L.n;
  const TypeMajor T(p, q, n);
  const long long len = T.len;
  const int tid = threadIdx.x;
  const CState S{cap};
  double* Vb = work;
  double* Zb = Vb + (size_t)(cap + 1) * len;
  double* wv = Zb + (size_t)cap * len;
  double* av = wv + len;
  const int pm = p > q ? p : q;
  CoarseLds C;
  C.rv = sm;
  C.ru = C.rv + pm;
  C.rz = C.ru + pm;
  C.rl = C.rz + pm;
  C.rm = C.rl + pm;
  C.ov = C.rm + pm;
  C.ou = C.ov + pm;
  C.oz = C.ou + pm;
  C.ol = C.oz + pm;
  C.om = C.ol + pm;
  C.scr = C.om + pm;
  C.app = C.scr + Pol::scratch(p, q);
  double* red = C.app + apply_lds_doubles(p, q, NT);
  __shared__ int sflag;
  if (S.beta(cst) == 0.0) {
    for (long long e = tid; e < len; e += NT) x[e] = 0.0;
    if (tid == 0) *its_out = 0;
    return;
  }
  int j = ist[0];
  bool stop = ist[1] != 0;
  __syncthreads();
  while (!stop && j < nsteps) {
    double* vj = Vb + (size_t)j * len;
    double* zj = Zb + (size_t)j * len;
    sgs_apply<Pol>(L, vj, av, zj, C);
    for (int k = 1; k <= n; ++k) apply_step<NT>(L, k, zj, nullptr, 1.0, 0.0, wv, C.app);
    __syncthreads();
    stop = arnoldi_step<NT>(j, wv, Vb, len, cst, ist, S, tol, fixed_its, nsteps, red, &sflag);
    ++j;
  }
  const int its = ist[0];
  double* H = S.H(cst);
  double* g = S.g(cst);
  double* yv = S.y(cst);
  if (tid == 0) {
    for (int i = its - 1; i >= 0; --i) {
      double acc = g[i];
      for (int c = i + 1; c < its; ++c) acc -= H[(size_t)i * cap + c] * yv[c];
      yv[i] = acc / H[(size_t)i * cap + i];
    }
    *its_out = its;
  }
  __syncthreads();
  for (long long e = tid; e < len; e += NT) {
    double acc = 0.0;
    for (int i = 0; i < its; ++i) acc += yv[i] * Zb[(size_t)i * len + e];
    x[e] = acc;
  }
}

// ---------------------------------------------------------------------------
// propagators for the block-parallel SGS
// ---------------------------------------------------------------------------

// out_s = G_s^{-1} M_s for every step s of the level (M = N or V).
__global__ __launch_bounds__(512) void k_gi_times(LevelView L, int which,
                                                  double* __restrict__ out) {
  const int p = L.p;
  const long long s = blockIdx.x;
  const double* __restrict__ Gk = L.Gi + s * p * p;
  const double* __restrict__ Mk = which == 0 ? L.N + s * L.sN : L.V + s * L.sV;
  double* o = out + s * p * p;
  for (int idx = threadIdx.x; idx < p * p; idx += 512) {
    const int i = idx / p, j = idx % p;
    double acc = 0.0;
    for (int m = 0; m <= i; ++m) acc += Gk[(long long)i * p + m] * Mk[(long long)m * p + j];
    o[idx] = acc;
  }
}

// Phi_s = W_s^T X_s  (= N^T S^{-1} V with W = G^{-1} N, X = G^{-1} V).
__global__ __launch_bounds__(512) void k_phi(int p, const double* __restrict__ W,
                                             const double* __restrict__ X,
                                             double* __restrict__ Phi) {
  const long long s = blockIdx.x;
  const double* Ws = W + s * p * p;
  const double* Xs = X + s * p * p;
  double* o = Phi + s * p * p;
  for (int idx = threadIdx.x; idx < p * p; idx += 512) {
    const int i = idx / p, j = idx % p;
    double acc = 0.0;
    for (int l = 0; l < p; ++l) acc += Ws[(long long)l * p + i] * Xs[(long long)l * p + j];
    o[idx] = acc;
  }
}

// Column i of the propagators (steps 0-based, nc steps, p x p blocks, row
// length nc*p):  P[i][i] = I, P[s][i] = -Phi_s P[s-1][i] (s > i);
//                Q[i][i] = I, Q[m][i] = -Phi_{m+1}^T Q[m+1][i] (m < i).
__global__ __launch_bounds__(512) void k_propagators(int p, int nc, const double* __restrict__ Phi,
                                                     double* __restrict__ P, double* __restrict__ Q) {
  const int i = blockIdx.x;
  const long long ld = (long long)nc * p;
  auto blk = [&](double* M, int r, int c) { return M + (long long)r * p * ld + (long long)c * p; };
  for (int idx = threadIdx.x; idx < p * p; idx += 512) {
    const int a = idx / p, b = idx % p;
    blk(P, i, i)[(long long)a * ld + b] = a == b ? 1.0 : 0.0;
    blk(Q, i, i)[(long long)a * ld + b] = a == b ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int s = i + 1; s < nc; ++s) {
    const double* F = Phi + (long long)s * p * p;
    const double* prev = blk(P, s - 1, i);
    double* cur = blk(P, s, i);
    for (int idx = threadIdx.x; idx < p * p; idx += 512) {
      const int a = idx / p, b = idx % p;
      double acc = 0.0;
      for (int l = 0; l < p; ++l) acc += F[(long long)a * p + l] * prev[(long long)l * ld + b];
      cur[(long long)a * ld + b] = -acc;
    }
    __syncthreads();
  }
  for (int m = i - 1; m >= 0; --m) {
    const double* F = Phi + (long long)(m + 1) * p * p;
    const double* prev = blk(Q, m + 1, i);
    double* cur = blk(Q, m, i);
    for (int idx = threadIdx.x; idx < p * p; idx += 512) {
      const int a = idx / p, b = idx % p;
      double acc = 0.0;
      for (int l = 0; l < p; ++l) acc += F[(long long)l * p + a] * prev[(long long)l * ld + b];
      cur[(long long)a * ld + b] = -acc;
    }
    __syncthreads();
  }
}

// y = M x for a block-lower (upper = 0) or block-upper (upper = 1) matrix of
// nc x nc blocks of p x p whose diagonal blocks are the identity (the
// propagators): y_r = x_r + the off-diagonal blocks of row r times x.  One
// wave per row, eight independent loads in flight per lane.
__global__ __launch_bounds__(256) void k_gemv_tri(const double* __restrict__ M, int nc, int p,
                                                  int upper, const double* __restrict__ x,
                                                  double* __restrict__ y) {
  const long long ld = (long long)nc * p;
  const long long r = (long long)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (r >= ld) return;
  const int s = (int)(r / p);
  const long long c0 = upper ? (long long)(s + 1) * p : 0;
  const long long c1 = upper ? ld : (long long)s * p;
  const double* __restrict__ Mr = M + r * ld;
  double a[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) a[t] = 0.0;
  long long c = c0 + lane;
  for (; c + 7 * kWave < c1; c += 8 * kWave) {
#pragma unroll
    for (int t = 0; t < 8; ++t) a[t] += Mr[c + t * kWave] * x[c + t * kWave];
  }
  for (; c < c1; c += kWave) a[0] += Mr[c] * x[c];
  double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  acc = wave_sum(acc);
  if (lane == 0) y[r] = x[r] + acc;
}

__global__ void k_add(double* __restrict__ z, const double* __restrict__ a,
                      const double* __restrict__ d, long long len) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < len;
       e += (long long)gridDim.x * blockDim.x)
    z[e] = a[e] + d[e];
}

using FinishPol = GenericPolicy<512>;

size_t finish_lds_doubles(int p, int q) {
  const size_t pm = p > q ? p : q;
  return 10 * pm + FinishPol::scratch(p, q) + apply_lds_doubles(p, q, FinishPol::kThreads) +
         FinishPol::kThreads / kWave;
}

}  // namespace

// ---------------------------------------------------------------------------
// host-side pieces
// ---------------------------------------------------------------------------

size_t coarse_work_doubles(int p, int q, int n, int cap) {
  const TypeMajor T(p, q, n);
  return (size_t)T.len * (2 * (size_t)cap + 3);
}

size_t coarse_state_doubles(int cap) { return CState::doubles(cap); }

hipError_t launch_coarse_init(const double* b, long long len, double* Vb, double* cst, int* ist,
                              int cap, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_init, dim3(1), dim3(kCtrlThreads), 0, s, b, len, Vb, cst, ist, cap);
  return hipGetLastError();
}

hipError_t launch_coarse_arnoldi(int j, double* w, double* Vb, long long len, double* cst,
                                 int* ist, int cap, double tol, int fixed_its, int nsteps,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_arnoldi, dim3(1), dim3(kCtrlThreads), 0, s, j, w, Vb, len, cst,
                     ist, cap, tol, fixed_its, nsteps);
  return hipGetLastError();
}

hipError_t launch_coarse_arnoldi_sgs(int j, double* w, double* Vb, double* zj, const double* a,
                                     const double* d, int p, int q, int n, double* cst, int* ist,
                                     int cap, double tol, int fixed_its, int nsteps,
                                     hipStream_t s) {
  const TypeMajor T(p, q, n);
  if (T.len <= 16LL * kCtrlThreads)
    hipLaunchKernelGGL((k_coarse_arnoldi_sgs_reg<kCtrlThreads, 16>), dim3(1), dim3(kCtrlThreads),
                       0, s, j, w, Vb, zj, a, d, T.m, T.len, cst, ist, cap, tol, fixed_its, nsteps);
  else if (T.len <= 48LL * kCtrlThreads)
    hipLaunchKernelGGL((k_coarse_arnoldi_sgs_reg<kCtrlThreads, 48>), dim3(1), dim3(kCtrlThreads),
                       0, s, j, w, Vb, zj, a, d, T.m, T.len, cst, ist, cap, tol, fixed_its, nsteps);
  else
    hipLaunchKernelGGL(k_coarse_arnoldi_sgs, dim3(1), dim3(kCtrlThreads), 0, s, j, w, Vb, zj, a,
                       d, T.m, T.len, cst, ist, cap, tol, fixed_its, nsteps);
  return hipGetLastError();
}

hipError_t launch_coarse_finish(const LevelView& L, double* x, double tol, int fixed_its,
                                int nsteps, double* work, double* cst, int* ist, int cap,
                                int* its_out, hipStream_t s) {
  const size_t lds = finish_lds_doubles(L.p, L.q) * sizeof(double);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void*)k_coarse_finish<FinishPol>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_coarse_finish<FinishPol>, dim3(1), dim3(FinishPol::kThreads), lds, s, L,
                     x, tol, fixed_its, nsteps, work, cst, ist, cap, its_out);
  return hipGetLastError();
}

// The same products on the matrix cores for p in {64, 128} (pitmg_mfma.h):
// W_s = G_s^{-1} N_s and X_s = G_s^{-1} V_s (which = 0, 1), Phi_s = W_s^T X_s,
// and the propagators (below).
template <int NT>
__global__ __launch_bounds__(kGemmThreads) void k_gi_times_mfma(LevelView L, int which,
                                                                double* __restrict__ out) {
  extern __shared__ double lds[];
  constexpr int P = 16 * NT;
  const long long s = blockIdx.x;
  const double* Gk = L.Gi + s * P * P;
  const double* Mk = which == 0 ? L.N + s * L.sN : L.V + s * L.sV;
  wg_gemm<NT, false, false>(Gk, P, Mk, P, 1.0, out + s * P * P, P, lds);
}

template <int NT>
__global__ __launch_bounds__(kGemmThreads) void k_phi_mfma(const double* __restrict__ W,
                                                           const double* __restrict__ X,
                                                           double* __restrict__ Phi) {
  extern __shared__ double lds[];
  constexpr int P = 16 * NT;
  const long long s = blockIdx.x;
  wg_gemm<NT, true, false>(W + s * P * P, P, X + s * P * P, P, 1.0, Phi + s * P * P, P, lds);
}

// The propagators by doubling spans: P[s][i] = (-1)^(s-i) Phi_s ... Phi_{i+1}
// composes, P[s][i] = P[s][m] P[m][i] for i < m < s, and Q[m][i] =
// P[i][m]^T likewise, Q[m][i] = Q[m][k] Q[k][i].  k_prop_init writes the
// identity blocks and the span-1 blocks (-Phi_{i+1}, -Phi_{i+1}^T); round r
// forms every block of span d in (2^(r-1), 2^r] from a span-2^(r-1) block
// and a shorter one, one work-group per block (P blocks in the first half of
// the grid, Q in the second): ceil(log2(nc - 1)) rounds of independent
// products instead of a chain of nc - 1.
template <int NT>
__global__ __launch_bounds__(kGemmThreads) void k_prop_init(int nc, const double* __restrict__ Phi,
                                                            double* P_, double* Q_) {
  constexpr int P = 16 * NT;
  const long long ld = (long long)nc * P;
  const int i = blockIdx.x;                     // block column of P (row of Q)
  for (int idx = threadIdx.x; idx < P * P; idx += kGemmThreads) {
    const int a = idx / P, b = idx % P;
    const double id = a == b ? 1.0 : 0.0;
    P_[(long long)i * P * ld + (long long)i * P + (long long)a * ld + b] = id;
    Q_[(long long)i * P * ld + (long long)i * P + (long long)a * ld + b] = id;
    if (i + 1 < nc) {
      const double* F = Phi + (long long)(i + 1) * P * P;
      P_[(long long)(i + 1) * P * ld + (long long)i * P + (long long)a * ld + b] = -F[a * P + b];
      Q_[(long long)i * P * ld + (long long)(i + 1) * P + (long long)a * ld + b] = -F[b * P + a];
    }
  }
}

// Blocks of round r: span d = h + e, h = 2^(r-1), e in [1, h], d <= nc - 1,
// row s = i + d for i = 0 .. nc-1-d, enumerated by e, then i.
__host__ __device__ inline int prop_round_count(int nc, int h) {
  int c = 0;
  for (int e = 1; e <= h && h + e <= nc - 1; ++e) c += nc - (h + e);
  return c;
}

template <int NT>
__global__ __launch_bounds__(kGemmThreads) void k_prop_round(int nc, int h, double* P_,
                                                             double* Q_) {
  extern __shared__ double lds[];
  constexpr int P = 16 * NT;
  const long long ld = (long long)nc * P;
  const int per = prop_round_count(nc, h);
  const bool lower = (int)blockIdx.x < per;
  int t = lower ? blockIdx.x : blockIdx.x - per;
  int e = 1;
  while (t >= nc - (h + e)) {
    t -= nc - (h + e);
    ++e;
  }
  const int i = t, d = h + e;
  double* M = lower ? P_ : Q_;
  auto blk = [&](int rr, int cc) { return M + (long long)rr * P * ld + (long long)cc * P; };
  if (lower) {                                  // P[i+d][i] = P[i+d][i+e] P[i+e][i]
    wg_gemm<NT, false, false>(blk(i + d, i + e), ld, blk(i + e, i), ld, 1.0, blk(i + d, i), ld,
                              lds);
  } else {                                      // Q[i][i+d] = Q[i][i+h] Q[i+h][i+d]
    wg_gemm<NT, false, false>(blk(i, i + h), ld, blk(i + h, i + d), ld, 1.0, blk(i, i + d), ld,
                              lds);
  }
}

template <int NT>
static hipError_t launch_propagators_mfma(const LevelView& L, double* W, double* X, double* Phi,
                                          double* P, double* Q, hipStream_t s) {
  const int nc = L.n;
  const size_t lds = wg_gemm_lds_doubles(16 * NT) * sizeof(double);
  const void* fns[4] = {(const void*)k_gi_times_mfma<NT>, (const void*)k_phi_mfma<NT>,
                        (const void*)k_prop_round<NT>, nullptr};
  for (int f = 0; f < 3; ++f) {
    hipError_t e = hipFuncSetAttribute(fns[f], hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_gi_times_mfma<NT>, dim3(nc), dim3(kGemmThreads), lds, s, L, 0, W);
  hipLaunchKernelGGL(k_gi_times_mfma<NT>, dim3(nc), dim3(kGemmThreads), lds, s, L, 1, X);
  hipLaunchKernelGGL(k_phi_mfma<NT>, dim3(nc), dim3(kGemmThreads), lds, s, W, X, Phi);
  hipLaunchKernelGGL(k_prop_init<NT>, dim3(nc), dim3(kGemmThreads), 0, s, nc, Phi, P, Q);
  for (int h = 1; h < nc - 1; h *= 2) {
    const int per = prop_round_count(nc, h);
    hipLaunchKernelGGL(k_prop_round<NT>, dim3(2 * per), dim3(kGemmThreads), lds, s, nc, h, P, Q);
  }
  return hipGetLastError();
}

// p = 128 NB (NB >= 2): every P x P product split into NB^2 super-blocks of
// 128 x 128, one work-group each (Gemm128, K = P).
//   k_batched_gemm128: C_s = op(A_s) B_s for every step s (W, X, Phi);
//   k_propagator_step: chain step j of both propagators, P[j][i] for i < j
//   (from P[j-1][i]) and Q[nc-1-j][i] for i > nc-1-j (from Q[nc-j][i]), each
//   column's super-blocks in parallel; the host launches j = 1 .. nc-1 in
//   order, so every launch reads blocks the previous one wrote.
template <bool TA>
__global__ __launch_bounds__(kGemmThreads) void k_batched_gemm128(
    int P, const double* __restrict__ A, long long sA, const double* __restrict__ B,
    long long sB, double* __restrict__ C) {
  extern __shared__ double lds[];
  const int NB = P / 128, per = NB * NB;
  const long long s = blockIdx.x / per;
  const int t = blockIdx.x % per, R = t / NB, Cc = t % NB;
  const double* a = A + s * sA + (TA ? 128LL * R : 128LL * R * P);
  Gemm128<double> gm;
  gm.zero();
  gm.template mul<TA, false>(a, P, B + s * sB + 128 * Cc, P, P, lds);
  gm.store(C + s * (long long)P * P + 128LL * R * P + 128 * Cc, P, 1.0, 0.0);
}

__global__ __launch_bounds__(kGemmThreads) void k_propagator_step(
    int P, int nc, int j, const double* __restrict__ Phi, double* P_, double* Q_) {
  extern __shared__ double lds[];
  const int NB = P / 128, per = NB * NB;
  const int c = blockIdx.x / per, t = blockIdx.x % per, R = t / NB, Cc = t % NB;
  const bool lower = c < j;
  const long long ld = (long long)nc * P;
  auto blk = [&](double* M, int rr, int cc) {
    return M + (long long)rr * P * ld + (long long)cc * P;
  };
  Gemm128<double> gm;
  gm.zero();
  double* out;
  if (lower) {                                 // P[j][i] = -Phi_j P[j-1][i], i = c
    const double* a = Phi + (long long)j * P * P + 128LL * R * P;
    gm.template mul<false, false>(a, P, blk(P_, j - 1, c) + 128 * Cc, ld, P, lds);
    out = blk(P_, j, c);
  } else {                                     // Q[m][i] = -Phi_{m+1}^T Q[m+1][i]
    const int m = nc - 1 - j, i = m + 1 + (c - j);
    const double* a = Phi + (long long)(m + 1) * P * P + 128 * R;
    gm.template mul<true, false>(a, P, blk(Q_, m + 1, i) + 128 * Cc, ld, P, lds);
    out = blk(Q_, m, i);
  }
  gm.store(out + 128LL * R * ld + 128 * Cc, ld, -1.0, 0.0);
}

__global__ void k_propagator_identity(int P, int nc, double* P_, double* Q_) {
  const long long ld = (long long)nc * P;
  const long long total = (long long)nc * P * P;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / ((long long)P * P)), a = (int)(e / P % P), b = (int)(e % P);
    const long long off = (long long)i * P * ld + (long long)i * P + (long long)a * ld + b;
    const double v = a == b ? 1.0 : 0.0;
    P_[off] = v;
    Q_[off] = v;
  }
}

static hipError_t launch_propagators_big(const LevelView& L, double* W, double* X, double* Phi,
                                         double* P, double* Q, hipStream_t s) {
  const int p = L.p, nc = L.n, per = (p / 128) * (p / 128);
  const size_t lds = Gemm128<double>::kLdsElems * sizeof(double);
  const void* fns[3] = {(const void*)k_batched_gemm128<false>,
                        (const void*)k_batched_gemm128<true>, (const void*)k_propagator_step};
  for (int f = 0; f < 3; ++f) {
    hipError_t e = hipFuncSetAttribute(fns[f], hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  const dim3 g(nc * per), b(kGemmThreads);
  const long long pp = (long long)p * p;
  hipLaunchKernelGGL(k_batched_gemm128<false>, g, b, lds, s, p, L.Gi, pp, L.N, L.sN, W);
  hipLaunchKernelGGL(k_batched_gemm128<false>, g, b, lds, s, p, L.Gi, pp, L.V, L.sV, X);
  hipLaunchKernelGGL(k_batched_gemm128<true>, g, b, lds, s, p, W, pp, X, pp, Phi);
  hipLaunchKernelGGL(k_propagator_identity, dim3(nc * 8), dim3(256), 0, s, p, nc, P, Q);
  for (int j = 1; j < nc; ++j)
    hipLaunchKernelGGL(k_propagator_step, dim3(2 * j * per), b, lds, s, p, nc, j, Phi, P, Q);
  return hipGetLastError();
}

hipError_t launch_propagators(const LevelView& L, double* scratch, double* Phi, double* P,
                              double* Q, hipStream_t s) {
  const int p = L.p, nc = L.n;
  double* W = scratch;
  double* X = scratch + (size_t)nc * p * p;
  if (p == 128) return launch_propagators_mfma<8>(L, W, X, Phi, P, Q, s);
  if (p == 64) return launch_propagators_mfma<4>(L, W, X, Phi, P, Q, s);
  if (p >= 256 && p % 128 == 0) return launch_propagators_big(L, W, X, Phi, P, Q, s);
  hipLaunchKernelGGL(k_gi_times, dim3(nc), dim3(512), 0, s, L, 0, W);
  hipLaunchKernelGGL(k_gi_times, dim3(nc), dim3(512), 0, s, L, 1, X);
  hipLaunchKernelGGL(k_phi, dim3(nc), dim3(512), 0, s, p, W, X, Phi);
  hipLaunchKernelGGL(k_propagators, dim3(nc), dim3(512), 0, s, p, nc, Phi, P, Q);
  return hipGetLastError();
}

template <int NT>
__global__ __launch_bounds__(kGemmThreads) void k_gi_times_batch(GiNBatch B) {
  extern __shared__ double lds[];
  constexpr int P = 16 * NT;
  const int b = blockIdx.x;
  int l = 0;
  while (l + 1 < B.nlev && b >= B.start[l + 1]) ++l;
  const long long s = b - B.start[l];
  wg_gemm<NT, false, false>(B.Gi[l] + s * P * P, P, B.N[l] + s * B.sN, P, 1.0,
                            B.out[l] + s * P * P, P, lds);
}

hipError_t launch_gi_times_batch(const GiNBatch& B, hipStream_t s) {
  if (B.nlev < 1 || B.nlev > 20 || (B.p != 64 && B.p != 128)) return hipErrorInvalidValue;
  const size_t lds = wg_gemm_lds_doubles(B.p) * sizeof(double);
  const void* fn = B.p == 128 ? (const void*)k_gi_times_batch<8> : (const void*)k_gi_times_batch<4>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 g(B.start[B.nlev]);
  if (B.p == 128)
    hipLaunchKernelGGL(k_gi_times_batch<8>, g, dim3(kGemmThreads), lds, s, B);
  else
    hipLaunchKernelGGL(k_gi_times_batch<4>, g, dim3(kGemmThreads), lds, s, B);
  return hipGetLastError();
}

// Phi_k = N_k^T S_k^{-1} V_k and its transpose for every step of a level
// (the block Gauss-Seidel smoothers' coupling, see pitmg_gs.hip):
// W = G^{-1} N, X = G^{-1} V, Phi = W^T X, Phi^T = X^T W.
hipError_t launch_phi_pair(const LevelView& L, double* W, double* X, double* Phi, double* PhiT,
                           hipStream_t s) {
  const int p = L.p, n = L.n;
  const long long pp = (long long)p * p;
  if (p == 64 || p == 128) {
    const size_t lds = wg_gemm_lds_doubles(p) * sizeof(double);
    const void* fns[2] = {p == 128 ? (const void*)k_gi_times_mfma<8> : (const void*)k_gi_times_mfma<4>,
                          p == 128 ? (const void*)k_phi_mfma<8> : (const void*)k_phi_mfma<4>};
    for (int f = 0; f < 2; ++f) {
      hipError_t e = hipFuncSetAttribute(fns[f], hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds);
      if (e != hipSuccess) return e;
    }
    if (p == 128) {
      hipLaunchKernelGGL(k_gi_times_mfma<8>, dim3(n), dim3(kGemmThreads), lds, s, L, 0, W);
      hipLaunchKernelGGL(k_gi_times_mfma<8>, dim3(n), dim3(kGemmThreads), lds, s, L, 1, X);
      hipLaunchKernelGGL(k_phi_mfma<8>, dim3(n), dim3(kGemmThreads), lds, s, W, X, Phi);
      hipLaunchKernelGGL(k_phi_mfma<8>, dim3(n), dim3(kGemmThreads), lds, s, X, W, PhiT);
    } else {
      hipLaunchKernelGGL(k_gi_times_mfma<4>, dim3(n), dim3(kGemmThreads), lds, s, L, 0, W);
      hipLaunchKernelGGL(k_gi_times_mfma<4>, dim3(n), dim3(kGemmThreads), lds, s, L, 1, X);
      hipLaunchKernelGGL(k_phi_mfma<4>, dim3(n), dim3(kGemmThreads), lds, s, W, X, Phi);
      hipLaunchKernelGGL(k_phi_mfma<4>, dim3(n), dim3(kGemmThreads), lds, s, X, W, PhiT);
    }
    return hipGetLastError();
  }
  if (p >= 256 && p % 128 == 0) {
    const int per = (p / 128) * (p / 128);
    const size_t lds = Gemm128<double>::kLdsElems * sizeof(double);
    const void* fns[2] = {(const void*)k_batched_gemm128<false>,
                          (const void*)k_batched_gemm128<true>};
    for (int f = 0; f < 2; ++f) {
      hipError_t e = hipFuncSetAttribute(fns[f], hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds);
      if (e != hipSuccess) return e;
    }
    const dim3 g(n * per), b(kGemmThreads);
    hipLaunchKernelGGL(k_batched_gemm128<false>, g, b, lds, s, p, L.Gi, pp, L.N, L.sN, W);
    hipLaunchKernelGGL(k_batched_gemm128<false>, g, b, lds, s, p, L.Gi, pp, L.V, L.sV, X);
    hipLaunchKernelGGL(k_batched_gemm128<true>, g, b, lds, s, p, W, pp, X, pp, Phi);
    hipLaunchKernelGGL(k_batched_gemm128<true>, g, b, lds, s, p, X, pp, W, pp, PhiT);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_gi_times, dim3(n), dim3(512), 0, s, L, 0, W);
  hipLaunchKernelGGL(k_gi_times, dim3(n), dim3(512), 0, s, L, 1, X);
  hipLaunchKernelGGL(k_phi, dim3(n), dim3(512), 0, s, p, W, X, Phi);
  hipLaunchKernelGGL(k_phi, dim3(n), dim3(512), 0, s, p, X, W, PhiT);
  return hipGetLastError();
}

hipError_t launch_gemv_tri(const double* M, int nc, int p, int upper, const double* x, double* y,
                           hipStream_t s) {
  const long long rows = (long long)nc * p;
  hipLaunchKernelGGL(k_gemv_tri, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, M, nc, p,
                     upper, x, y);
  return hipGetLastError();
}

hipError_t launch_add(double* z, const double* a, const double* d, long long len, hipStream_t s) {
  long long g = (len + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_add, dim3((unsigned)g), dim3(256), 0, s, z, a, d, len);
  return hipGetLastError();
}

}  // namespace pitmg
