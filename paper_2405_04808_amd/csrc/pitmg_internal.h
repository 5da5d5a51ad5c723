// Internal declarations shared by the kernel and host translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstdint>

struct pitmg_net;   // learned coarse correction (pitmg_net.hip)

namespace pitmg {

constexpr int kWave = 64;

// Work buffers of the split sweep for large blocks (pitmg_split.hip): the
// coupled right-hand sides R_mu [n+1][p], U = Z~ R_z - V R_mu [n][p],
// W_z = Z~^T Lambda [n][q], W_v = V^T Lambda [n][p] (one row per step, FP64)
// and their FP32 counterparts for an FP32 level.
struct SplitBuffers {
  double *Rm = nullptr, *U = nullptr, *Wz = nullptr, *Wv = nullptr;
  float *Rm32 = nullptr, *Rz32 = nullptr, *U32 = nullptr, *L32 = nullptr, *Wz32 = nullptr,
        *Wv32 = nullptr;
};

// One level of the hierarchy as the kernels see it.
struct LevelView {
  int n;                       // steps on this level
  int p, q;
  const double* N;  long long sN;   // N_k = N + k*sN (k 0-based)
  const double* V;  long long sV;
  const double* Z;  long long sZ;
  const double* Gi;            // [n][p][p] row-major, lower triangle of G_k^{-1}
  // FP32 smoother (levels above the coarsest when enabled): single-precision
  // copies of the blocks and the factor, same layout and strides.
  const float* N32 = nullptr;
  const float* V32 = nullptr;
  const float* Z32 = nullptr;
  const float* Gi32 = nullptr;
  int fp32 = 0;
  // sweep launch shape: 0 built-in rule, k >= 1 steps per work-group of the
  // shared-block kernel, -1 the one-step kernel
  int sweep_cfg = 0;
  // host-side: split-sweep buffers of this level, or NULL (never read on the
  // device)
  const SplitBuffers* split = nullptr;
  // weight of the block Jacobi correction, y <- (1-omega) y + omega D^{-1}(b -
  // (L+L^T) y); 1 on the coarsest level, whose sweeps are the exact block
  // solves of the coarse SGS
  double omega = 1.0;
  // scale of the mu block in the transfers between this level and the next
  // coarser one (interpolation multiplies coarse mu by it, restriction
  // weights the mu residual rows by it)
  double mu_scale = 1.0;
  // V and Z~ shared by every step and diagonal (p == q; theta = 1 with an
  // identity mass matrix and distributed control): the sweeps and the apply
  // use their diagonals Vd, Zd (p values each) instead of the dense blocks
  int vz_diag = 0;
  const double* Vd = nullptr;
  const double* Zd = nullptr;
  const float* Vd32 = nullptr;
  const float* Zd32 = nullptr;
  // W_k = G_k^{-1} N_k ([n][p][p] row-major) on FP64 levels with diagonal
  // shared V, Z~ and p = q in {64, 128}, else NULL: the one-step sweeps then
  // take s = W r_u + G^{-1} d and N^T lambda = W^T s (pitmg_tiled.h)
  const double* GiN = nullptr;
  // 16 zero bytes in device memory (the one-step kernels read the factor's
  // vectors above the diagonal from here)
  const void* zeros = nullptr;
};

// Block pointers of a level in the arithmetic of the smoother.
template <class T>
struct Mats;
template <>
struct Mats<double> {
  __host__ __device__ static const double* N(const LevelView& L) { return L.N; }
  __host__ __device__ static const double* V(const LevelView& L) { return L.V; }
  __host__ __device__ static const double* Z(const LevelView& L) { return L.Z; }
  __host__ __device__ static const double* Gi(const LevelView& L) { return L.Gi; }
  __host__ __device__ static const double* Vd(const LevelView& L) { return L.Vd; }
  __host__ __device__ static const double* Zd(const LevelView& L) { return L.Zd; }
  __host__ __device__ static const double* GiN(const LevelView& L) { return L.GiN; }
};
template <>
struct Mats<float> {
  __host__ __device__ static const float* N(const LevelView& L) { return L.N32; }
  __host__ __device__ static const float* V(const LevelView& L) { return L.V32; }
  __host__ __device__ static const float* Z(const LevelView& L) { return L.Z32; }
  __host__ __device__ static const float* Gi(const LevelView& L) { return L.Gi32; }
  __host__ __device__ static const float* Vd(const LevelView& L) { return L.Vd32; }
  __host__ __device__ static const float* Zd(const LevelView& L) { return L.Zd32; }
  __host__ __device__ static const float* GiN(const LevelView&) { return nullptr; }
};

// Offsets of the five variable types in a type-major vector of n steps.
struct TypeMajor {
  long long u, v, z, l, m, len;
  __host__ __device__ TypeMajor(int p, int q, int n) {
    u = 0; v = (long long)p * n; z = 2LL * p * n; l = z + (long long)q * n;
    m = l + (long long)p * n; len = m + (long long)p * n;
  }
};

// Events armed by the host's kernel timer.  A launcher that issues its kernel
// through launch_k lets the kernel's own dispatch record the start (first
// kernel only) and the end (every kernel, so the last one counts), with no
// marker packets around it; the start slot is cleared once taken.
struct KernelEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
  int taken = 0;
};
KernelEvents& kernel_events();   // per host thread (pitmg_host.hip)

template <class F, class... Args>
hipError_t launch_k(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                    Args... args) {
  KernelEvents& ev = kernel_events();
  hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)lds, s, ev.start, ev.stop, 0u,
                        args...);
  if (ev.stop) {
    ev.start = nullptr;
    ev.taken += 1;
  }
  return hipGetLastError();
}

// ---- launchers (pitmg_kernels.hip) ---------------------------------------
// Factor every block of one level: S_k = N_k N_k^T + Z_k Z_k^T, Cholesky
// S_k = G_k G_k^T, and G_k^{-1} stored in Gi.  fail: device int, atomicMin'd
// with (level << 20 | k) on a non-positive pivot.
hipError_t launch_factor(const LevelView& L, double* Gi, int level, int* fail,
                         hipStream_t s);
// Every level of one element type in one launch on the matrix cores
// (pitmg_factor.hip) for p in {64, 128}, and for p in {256, 512} with q a
// multiple of 32: block b of the launch is block b - start[l] of level l for
// start[l] <= b < start[l+1].  FP64 from N / Z~ into Gi, FP32 from the FP32
// copies into Gi32.
template <class T>
struct FactorBatchT {
  int nlev = 0;
  int level0 = 0;              // hierarchy level of entry 0 (failure codes)
  int p = 0, q = 0;
  long long sN = 0, sZ = 0;
  int start[21] = {0};
  const T* N[20] = {};
  const T* Z[20] = {};
  T* Gi[20] = {};
  // device flags by hierarchy level (launch_vz_diag) and the diagonals of
  // Z~ (p = q): where a flag is set, S = N N^T + diag(Zd)^2 (no product
  // with the dense Z~); NULL flags: always the dense product
  const int* zflag = nullptr;
  const T* Zd[20] = {};
};
// The shared V and Z~ (p x p each) of up to 20 levels: flags[l] = 1 when
// both have only zeros off the diagonal (exact comparison), and then
// out[l] = [diag V | diag Z~] (2p values); flags[l] = 0 otherwise.
struct VZDiagBatch {
  int nlev = 0, p = 0;
  const double* V[20] = {};
  const double* Z[20] = {};
  double* out[20] = {};
};
hipError_t launch_vz_diag(const VZDiagBatch& B, int* flags, hipStream_t s);
bool factor_mfma_supported(int p, int q);
hipError_t launch_factor_mfma(const FactorBatchT<double>& F, int* fail, hipStream_t s);
hipError_t launch_factor_mfma(const FactorBatchT<float>& F, int* fail, hipStream_t s);
// Same in FP32 from L.N32 / L.Z32 into Gi32.
hipError_t launch_factor32(const LevelView& L, float* Gi32, int level, int* fail,
                           hipStream_t s);
// dst = (float) src
hipError_t launch_to_f32(float* dst, const double* src, long long count, hipStream_t s);

// One weighted block Jacobi sweep from yc = yold (NULL = 0) plus, if
// ecoarse != NULL, the interpolation of the coarse vector ecoarse (variant as
// in the options, mu scaled by L.mu_scale):
//     ynew = (1 - w) yc + w D^{-1}(b - (L+L^T) yc),   w = L.omega.
// If restrict_out != NULL (only with ecoarse == NULL), also the restricted
// residual R (rbeta b + (L+L^T)(ra yold - ynew)) of the next coarser level,
// as launch_restrict_delta computes it: inside the sweep where the kernel
// supports it, else by that kernel after the sweep.  The caller picks
// (rbeta, ra) so that this is the residual b - A~ ynew (see vcycle_level).
hipError_t launch_jacobi(const LevelView& L, const double* b, const double* yold,
                         const double* ecoarse, int variant, double* ynew,
                         hipStream_t s, double* restrict_out = nullptr, double rbeta = 0.0,
                         double ra = 1.0);

// Register-tiled sweep for p == q in {64, 128} (16-byte aligned blocks); the
// launchers follow L.fp32 for the arithmetic.  restrict_out as in
// launch_jacobi (the restriction fused into the sweep).
bool jacobi_tiled_supported(int p, int q);
// Hand-off state of the two-sweep kernel (device words owned by the handle).
struct PairSync {
  unsigned long long* ticket;  // ticket counter; only grows
  unsigned long long base;     // its value when this launch starts
  unsigned long long* flag;    // [n+1]: epoch of each block's published first sweep
  unsigned long long epoch;    // this launch's epoch, above every earlier one
  int* timeout;                // bit 0: a wait ran out; bit 1: a ticket out of range
  unsigned long long spin;     // bound of each wait, ticks of the device wall clock
};
// Two consecutive sweeps in one launch (y1 = first, y2 = second sweep; the
// coarse correction, if any, folds into the first, the restriction, if any,
// comes from the second and is R (rbeta b + (L+L^T)(ra y1 - y2))) for levels
// that sweep with the one-step tiled kernel or, in FP64, the shared-block
// kernel.  Only the u and mu entries of y1 are guaranteed (the one-step
// kernel stores no others).  jacobi_pair_supported says whether launch_jacobi_pair applies
// (never while the stream is being captured: the tickets and epochs are
// launch arguments).
bool jacobi_pair_supported(const LevelView& L, hipStream_t s);
// *groups: work-groups (tickets) of the launch, set whenever it is issued.
hipError_t launch_jacobi_pair(const LevelView& L, const double* b, const double* yold,
                              const double* ecoarse, int variant, double* y1, double* y2,
                              double* restrict_out, double rbeta, double ra,
                              const PairSync& ps, int* groups, hipStream_t s);
// Two-sweep smoothing of several levels in one launch (pitmg_jacobi_tiled.hip):
// sw[0..nlev) in ticket order, levels 0, 1, ... (up = 0: pre-smoothing, each
// level restricting into the next one's b) or ..., 1, 0 (up = 1:
// post-smoothing, each level's ec the previous one's y2).  Every level sweeps
// with the one-step tiled kernel (same p, q and precision); flag_off gives
// each level its own range of hand-off flags.  The launch uses the epochs
// ps.epoch (first sweeps) and ps.epoch + 1 (finished blocks).
struct ChainSweep {
  LevelView L;
  const double* b;
  const double* yold;
  const double* ec;
  double* y1;
  double* y2;
  double* restrict_out;
  double rbeta, ra;
  int flag_off;
};
int jacobi_chain_max();
// The coarse solve's block-parallel SGS application (three block sweeps and
// the two propagator products of pitmg_coarse.hip) as one launch with
// dataflow flags between its phases (pitmg_jacobi_tiled.hip).  FP64, p = q in
// {64, 128}, n + 1 <= 64 blocks; ps.flag needs sgs_fused_flags(n, p) words.
int sgs_fused_flags(int n, int p);
hipError_t launch_sgs_fused(const LevelView& L, const double* v, const double* zero, double* c,
                            double* a, double* d, double* yf, double* yb, const double* Pf,
                            const double* Qb, int variant, const PairSync& ps, int* groups,
                            hipStream_t s);
bool jacobi_chain_supported(const LevelView& L, hipStream_t s);
hipError_t launch_jacobi_chain(const ChainSweep* sw, int nlev, int up, int variant,
                               const PairSync& ps, int* groups, hipStream_t s);
hipError_t launch_jacobi_shared2(const LevelView& L, const double* b, const double* yold,
                                 const double* ecoarse, int variant, double* y1, double* y2,
                                 double* restrict_out, double rbeta, double ra,
                                 const PairSync& ps, int* groups, hipStream_t s);
hipError_t launch_jacobi_tiled2(const LevelView& L, const double* b, const double* yold,
                                const double* ecoarse, int variant, double* y1, double* y2,
                                double* restrict_out, double rbeta, double ra,
                                const PairSync& ps, hipStream_t s);
hipError_t launch_jacobi_tiled(const LevelView& L, const double* b, const double* yold,
                               const double* ecoarse, int variant, double* ynew,
                               double* restrict_out, double rbeta, double ra, hipStream_t s);

// Sweep for V and Z~ shared by every step (stride 0), p == q in {64, 128}.
bool jacobi_shared_supported(const LevelView& L);
hipError_t launch_jacobi_shared(const LevelView& L, const double* b, const double* yold,
                                const double* ecoarse, int variant, double* ynew,
                                double* restrict_out, double rbeta, double ra, hipStream_t s);

// out = beta*b + alpha*(A~ x) on one level (b may be NULL when beta == 0).
hipError_t launch_apply(const LevelView& L, const double* x, const double* b,
                        double alpha, double beta, double* out, hipStream_t s);
// The same for p = q in {64, 128} with V and Z~ shared by every step
// (register tiles of N_k, pitmg_jacobi_tiled.hip); apply_shared_supported
// says whether it applies.
bool apply_shared_supported(const LevelView& L);
hipError_t launch_apply_shared(const LevelView& L, const double* x, const double* b,
                               double alpha, double beta, double* out, hipStream_t s);

// Coarse right-hand side from the last pre-smoothing sweep:
// bc = R (beta b + (L+L^T)(a ya - y))  (ya NULL = 0; b unread if beta == 0),
// the mu rows of R scaled by mu_scale.
hipError_t launch_restrict_delta(int p, int q, int nf, const double* b, double beta,
                                 const double* ya, double a, const double* y, int variant,
                                 double mu_scale, double* bc, hipStream_t s);
// bc = R r (general restriction of a full fine vector).
hipError_t launch_restrict(int p, int q, int nf, const double* r, int variant,
                           double mu_scale, double* bc, hipStream_t s);
// y += P e  (interpolate and add).
// Transfers for a step ratio c (variant 0 alignment), mu block times mu_fac.
hipError_t launch_restrict_c(int p, int q, int nf, int c, const double* r, double mu_fac,
                             double* bc, hipStream_t s);
hipError_t launch_interp_add_c(int p, int q, int nf, int c, const double* e, double mu_fac,
                               double* y, hipStream_t s);
hipError_t launch_interp_add(int p, int q, int nf, const double* e, int variant,
                             double mu_scale, double* y, hipStream_t s);
// y = w y + (1 - w)(yold + P ec)  (yold, ec NULL = 0): the weighting of a
// sweep written unweighted by a kernel that does not weight itself.
hipError_t launch_weight(int p, int q, int n, double w, const double* yold, const double* ec,
                         int variant, double mu_scale, double* y, hipStream_t s);

// Coarse GMRES + SGS (pitmg_coarse.hip).  work: coarse_work_doubles(...)
// doubles holding the coarse Krylov bases; cst: coarse_state_doubles(cap)
// doubles of GMRES state; ist: 2 device ints {steps done, stop}.
size_t coarse_work_doubles(int p, int q, int n, int cap);
size_t coarse_state_doubles(int cap);
hipError_t launch_coarse_init(const double* b, long long len, double* Vb, double* cst, int* ist,
                              int cap, hipStream_t s);
hipError_t launch_coarse_arnoldi(int j, double* w, double* Vb, long long len, double* cst,
                                 int* ist, int cap, double tol, int fixed_its, int nsteps,
                                 hipStream_t s);
// The Arnoldi step of an SGS application z_j = a + d (forward sweep a,
// backward correction d): forms z_j and w = A~ z_j = v_j + L d, then the step.
hipError_t launch_coarse_arnoldi_sgs(int j, double* w, double* Vb, double* zj, const double* a,
                                     const double* d, int p, int q, int n, double* cst, int* ist,
                                     int cap, double tol, int fixed_its, int nsteps,
                                     hipStream_t s);
hipError_t launch_coarse_finish(const LevelView& L, double* x, double tol, int fixed_its,
                                int nsteps, double* work, double* cst, int* ist, int cap,
                                int* its_out, hipStream_t s);
// Block propagators Phi_s = N_s^T S_s^{-1} V_s and the block-triangular
// products P (forward SGS chain) and Q (backward chain), each (n p)^2.
// scratch: 2 n p^2 doubles; P and Q must be zero-filled beforehand.
hipError_t launch_propagators(const LevelView& L, double* scratch, double* Phi, double* P,
                              double* Q, hipStream_t s);
// Phi_k = N_k^T S_k^{-1} V_k and Phi_k^T for every step of level L (W, X:
// scratch of n p^2 doubles each).
hipError_t launch_phi_pair(const LevelView& L, double* W, double* X, double* Phi, double* PhiT,
                           hipStream_t s);
// W_k = G_k^{-1} N_k (p in {64, 128}, FP64, out [n][p][p] row-major) on the
// matrix cores for every step of up to 20 levels in one launch (block b of
// the launch is step b - start[l] of entry l).
struct GiNBatch {
  int nlev = 0, p = 0;
  long long sN = 0;
  int start[21] = {0};
  const double* Gi[20] = {};
  const double* N[20] = {};
  double* out[20] = {};
};
hipError_t launch_gi_times_batch(const GiNBatch& B, hipStream_t s);
// The chain of a block Gauss-Seidel substitution (pitmg_gs.hip): from
// t = D^{-1} r (type-major), hat's u slots (forward, M = Phi^T) or mu slots
// (backward, M = Phi) receive the substituted values; its other slots are
// not written.
hipError_t launch_gs_chain(int p, int q, int n, const double* M, const double* t, double* hat,
                           int backward, hipStream_t s);
// The system without virtual variables (pitmg_unlifted.hip): out = beta b +
// alpha A x on unlifted type-major vectors [u | z | lambda] of L's size, the
// N and V blocks of L multiplied by bscale; y = E r and x = E^T y.
hipError_t launch_unlifted_apply(const LevelView& L, double bscale, const double* x,
                                 const double* b, double alpha, double beta, double* out,
                                 hipStream_t s);
hipError_t launch_lift(int p, int q, int n, const double* r, double* y, hipStream_t s);
hipError_t launch_project(int p, int q, int n, const double* y, double* x, hipStream_t s);
hipError_t launch_gemv_tri(const double* M, int nc, int p, int upper, const double* x, double* y,
                           hipStream_t s);
hipError_t launch_add(double* z, const double* a, const double* d, long long len, hipStream_t s);

// Krylov helpers.  Basis vectors are rows of a [k][len] array.  Dot and
// update kernels work on krylov_slices(len) slices of 1024 elements and store
// value-major partials [value][slice]; launch_reduce_partials sums them.
int krylov_slices(long long len);
int krylov_partial_blocks(long long len);
// values: basis_i.x1 (nb), basis_i.x2 (nb, if x2), x1.x1, [x1.x2, x2.x2]
hipError_t launch_dots(const double* basis, int nb, const double* x1, const double* x2,
                       long long len, double* partial, hipStream_t s);
// The Arnoldi step's alpha, cq and a lost-orthogonality flag (out[0..2])
// from the dot values coef of step j (layout of launch_dots).
hipError_t launch_arnoldi_coeffs(const double* coef, int j, double* out, hipStream_t s);
// x1 <- (x1 - basis^T s)/alpha if reorth;  x2 <- x2 - basis^T h - cq*x1
// with (alpha, cq) = acq[0..1] in device memory; norm_partial[slice] =
// |x2|^2 over the slice.  scratch: 2*len doubles per basis group
// (krylov_groups) when there is more than one; NULL forces the single-pass
// kernel.
hipError_t launch_update(const double* basis, int nb, double* x1, double* x2,
                         const double* scoef, const double* hcoef, const double* acq,
                         int reorth, long long len, double* norm_partial, double* scratch,
                         hipStream_t s);
// Basis groups the dot and update passes split nb vectors of length len into.
int krylov_groups(long long len, int nb);
hipError_t launch_reduce_partials(const double* partial, int nblk, int nval,
                                  double* out, hipStream_t s);
// w += sign * basis^T coef; optional per-slice sums of the new w squared.
hipError_t launch_multi_axpy(double* w, const double* basis, int nvec,
                             const double* coef, double sign, long long len,
                             double* norm_partial, hipStream_t s);
hipError_t launch_scale(double* dst, const double* src, double alpha,
                        long long len, hipStream_t s);
// dst[0 .. len) = value (a kernel, so that it may be captured in a graph)
hipError_t launch_fill(double* dst, double value, long long len, hipStream_t s);
hipError_t launch_axpby(double* y, const double* x, double a, double b,
                        long long len, hipStream_t s);   // y = a*x + b*y

// w = A~ z from the last sweep z = D^{-1}(b - (L+L^T) yprev) of a cycle:
// w = b - (L+L^T)(yprev - z) (nonzero corrections in the u and mu slots only).
hipError_t launch_apply_identity(int p, int q, int n, const double* b, const double* yprev,
                                 const double* z, double* w, hipStream_t s);

// ---- large blocks with shared V, Z~ (pitmg_split.hip) ----------------------
bool split_supported(const LevelView& L);
hipError_t launch_jacobi_split(const LevelView& L, const double* b, const double* yold,
                               const double* ecoarse, int variant, double* ynew, hipStream_t s);

// ---- small blocks (pitmg_small.hip): one thread per time step -------------
bool small_supported(int p, int q);
hipError_t launch_jacobi_small(const LevelView& L, const double* b, const double* yold,
                               const double* ecoarse, int variant, double* ynew, hipStream_t s);
hipError_t launch_apply_small(const LevelView& L, const double* x, const double* b, double alpha,
                              double beta, double* out, hipStream_t s);

// ---- learned coarse correction (pitmg_net.hip) ----------------------------
// True if the network takes C channels over T steps.
bool net_matches(const pitmg_net* n, int C, int T);
// e = s * net(r / s) for one type-major coarse vector of the network's shape
// (s = rms(r)), enqueued on stream s; uses the network's work buffers.
hipError_t net_coarse_correction(pitmg_net* n, const double* r, double* e, int p, int q,
                                 hipStream_t s);

}  // namespace pitmg
