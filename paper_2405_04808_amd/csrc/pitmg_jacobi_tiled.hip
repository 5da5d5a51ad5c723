// Block Jacobi sweep for p = q in {64, 128}: one work-group of 512 threads
// per time-major block (or per group of 1-4 blocks when V and Z~ are shared
// by every step), with N_k and G_k^{-1} in registers (pitmg_tiled.h), so
// each Jacobian / factor entry is read from HBM once per sweep.  Each kernel
// also has a form that runs two consecutive sweeps in one launch, handing
// the two coupling values a neighbour needs across work-groups.
#include "pitmg_internal.h"
#include "pitmg_device.h"
#include "pitmg_tiled.h"

#include <type_traits>

namespace pitmg {

// Restriction of the residual after the last pre-smoothing sweep, fused
// into that sweep.  With y_A the iterate before the sweep (single sweep) or
// the first sweep's result (two-sweep launch) and y its output, the caller
// chooses (beta, a) so that the residual is r = beta b + (L+L^T)(a y_A - y):
// beta = 0, a = 1 for undamped sweeps; for weighted sweeps from a zero
// iterate beta = (1-w)^s, a = w (s = 1, 2 sweeps).  (L+L^T) c is nonzero
// only in the u and mu rows (r_u,k = c_mu,k, r_mu,k = c_u,k), and the coarse
// vector takes fine step kf = 2m-1 (variant 0) or 2m (variant 1) for coarse
// step m, the mean of fine steps 2m-1, 2m for the control, and mu_scale on
// the mu rows.  The work-group that produces u_kf writes the coarse mu, v,
// z, lambda entries of m; the one that produces mu_kf (block kf+1) writes
// the coarse u entry.  Same doubles as k_restrict_delta.  p = q here.
struct FusedRestrict {
  double* rc;                  // coarse vector, or NULL (no restriction)
  int variant;
  double beta, a, mu_scale;
  // b written by other work-groups of the same launch (read it with coherent
  // loads); rc read by other work-groups of the same launch (coherent stores)
  int coh_b = 0, coh_rc = 0;
  __device__ __forceinline__ double ldb(const double* __restrict__ b, long long idx) const {
    return coh_b ? coherent_load(b + idx) : b[idx];
  }
  __device__ __forceinline__ void put(long long idx, double v) const {
    if (coh_rc) coherent_store(rc + idx, v);
    else rc[idx] = v;
  }
  // coarse step m (1-based) whose mu, v, z, lambda block k writes, else 0
  __device__ int mu_writer(int k) const {
    if (!rc) return 0;
    if (variant == 0) return (k & 1) ? (k + 1) / 2 : 0;
    return (k & 1) ? 0 : k / 2;
  }
  // coarse step m whose u entry block k (producing mu_{k-1}) writes, else 0
  __device__ int u_writer(int k) const {
    if (!rc || k < 2) return 0;
    const int kf = k - 1;
    if (variant == 0) return (kf & 1) ? (kf + 1) / 2 : 0;
    return (kf & 1) ? 0 : kf / 2;
  }
  __device__ int fine(int m) const { return variant == 0 ? 2 * m - 1 : 2 * m; }
  // coarse mu, v, z, lambda of step m from c_u = a y_A,u - y_u at fine step kf
  __device__ void put_mu(int m, int i, double cu, const double* __restrict__ b,
                         const TypeMajor& Tm, const TypeMajor& Tc, int P) const {
    const long long o = (long long)(m - 1) * P + i;
    const long long f = (long long)(fine(m) - 1) * P + i;
    if (beta != 0.0) {
      put(Tc.m + o, mu_scale * (beta * ldb(b, Tm.m + f) + cu));
      put(Tc.v + o, beta * ldb(b, Tm.v + f));
      put(Tc.l + o, beta * ldb(b, Tm.l + f));
      put(Tc.z + o, 0.5 * beta * (ldb(b, Tm.z + (long long)(2 * m - 2) * P + i) +
                                  ldb(b, Tm.z + (long long)(2 * m - 1) * P + i)));
    } else {
      put(Tc.m + o, mu_scale * cu);
      put(Tc.v + o, 0.0);
      put(Tc.z + o, 0.0);
      put(Tc.l + o, 0.0);
    }
  }
  // coarse u of step m from c_mu = a y_A,mu - y_mu at fine step kf
  __device__ void put_u(int m, int i, double cmu, const double* __restrict__ b,
                        const TypeMajor& Tm, const TypeMajor& Tc, int P) const {
    const long long f = (long long)(fine(m) - 1) * P + i;
    put(Tc.u + (long long)(m - 1) * P + i, (beta != 0.0 ? beta * ldb(b, Tm.u + f) : 0.0) + cmu);
  }
};

// One block of a single sweep (block kb + 1, or block n+1 when kb = n), the
// body of k_jacobi_tiled.  coh_y: yold is written by other work-groups of the
// same launch (coherent loads); coh_out: ynew is read by other work-groups
// of the same launch (coherent stores).
template <int RT, int CT, class T>
__device__ __forceinline__ void one_block(const LevelView& L, const double* __restrict__ b,
                                          const double* yold, const double* __restrict__ ec,
                                          int variant, double* ynew, const FusedRestrict& fr,
                                          int kb, bool coh_y, bool coh_out) {
  using TS = TiledSolve<RT, CT, T>;
  constexpr int P = TS::P;
  __shared__ T sru[P], srz[P], srm[P], srl[P], srv[P], slam[P], srd[P];
  __shared__ T scr[TS::kScratch];
  const int tid = threadIdx.x;
  const int n = L.n;
  const bool gn = Mats<T>::GiN(L) != nullptr;   // W = G^{-1} N form (diagonal V, Z~)
  const TypeMajor Tm(P, P, n);
  const int nc = n / 2;
  const TypeMajor Tc(P, P, nc > 0 ? nc : 1);
  const double w = L.omega;
  const PrevIterate prev{yold, ec, P, P, n, variant, L.mu_scale, false, coh_y};
  auto cu = [&](int k1, int i) -> double { return prev.at(0, k1, i); };
  auto cm = [&](int k1, int i) -> double { return prev.at(4, k1, i); };
  auto ya = [&](long long idx) -> double { return yold ? fr.a * prev.yold_at(idx) : 0.0; };
  auto out = [&](long long idx, double v) {
    if (coh_out) coherent_store(ynew + idx, v);
    else ynew[idx] = v;
  };

  if (kb == n) {                               // block n+1 = (v_n, mu_n)
    const int mu_m = fr.u_writer(n + 1);
    for (int i = tid; i < P; i += kTiledThreads) {
      const double rvv = b[Tm.v + (long long)(n - 1) * P + i];
      const double rmm = b[Tm.m + (long long)(n - 1) * P + i] - cu(n, i);
      const double mo = weigh(w, -rmm - rvv, prev, 4, n, i);
      out(Tm.v + (long long)(n - 1) * P + i, weigh(w, -rmm, prev, 1, n, i));
      out(Tm.m + (long long)(n - 1) * P + i, mo);
      if (mu_m) fr.put_u(mu_m, i, ya(Tm.m + (long long)(n - 1) * P + i) - mo, b, Tm, Tc, P);
    }
    return;
  }
  const int k = kb + 1;
  const bool hv = k >= 2;
  const long long kk = k - 1;
  static_assert(P <= kTiledThreads, "one entry per thread");
  const bool on = tid < P;
  const int i = tid;
  const int rm_m = fr.mu_writer(k), ru_m = fr.u_writer(k);
  // right-hand side with the coupling values of the previous iterate,
  // r_u = b_u,k - mu_k, r_mu = b_mu,k-1 - u_{k-1}, and the previous values
  // that weigh the output, requested before the tiles (loads complete in
  // order, so the gather waits for these alone)
  double bu = 0.0, bm = 0.0, rl = 0.0, rz = 0.0, rv = 0.0, cmk = 0.0, cuk = 0.0;
  double pu = 0.0, pz = 0.0, pl = 0.0, pm = 0.0, pv = 0.0;
  typename TS::Diag dg;
  PrevFetch fcm, fcu, fu, fz, fl, fm, fv;
  if (on) {
    bu = b[Tm.u + kk * P + i];
    rl = b[Tm.l + kk * P + i];
    rz = b[Tm.z + kk * P + i];
    fcm = prev.fetch(4, k, i);
    if (hv) {
      rv = b[Tm.v + (kk - 1) * P + i];
      bm = b[Tm.m + (kk - 1) * P + i];
      fcu = prev.fetch(0, k - 1, i);
    }
    if (w != 1.0) {
      fu = prev.fetch(0, k, i);
      fz = prev.fetch(2, k, i);
      fl = prev.fetch(3, k, i);
      if (hv) {
        fm = prev.fetch(4, k - 1, i);
        fv = prev.fetch(1, k - 1, i);
      }
    }
    dg = TS::diag_at(L, i);
  }
  // a y_A of the fused restriction (restricting launches only)
  const double yau = on && rm_m ? ya(Tm.u + kk * P + i) : 0.0;
  const double yam = on && ru_m && hv ? ya(Tm.m + (kk - 1) * P + i) : 0.0;
  // (1 - omega) y_prev + omega y_hat, as weigh() forms it
  auto weigh0 = [&](double yhat, double yp) -> double {
    return w == 1.0 ? yhat : w * yhat + (1.0 - w) * yp;
  };
  typename TS::Regs R;
  __builtin_amdgcn_sched_barrier(0);           // keep the loads above ahead of the tile's
  TS::load_straight(L, kk, gn, R);
  __builtin_amdgcn_sched_barrier(0);
  if (on) {
    cmk = prev.value(fcm, 4, k);
    if (hv) cuk = prev.value(fcu, 0, k - 1);
    if (w != 1.0) {
      pu = prev.value(fu, 0, k);
      pz = prev.value(fz, 2, k);
      pl = prev.value(fl, 3, k);
      if (hv) {
        pm = prev.value(fm, 4, k - 1);
        pv = prev.value(fv, 1, k - 1);
      }
    }
    sru[i] = (T)(bu - cmk);
    srl[i] = (T)rl;
    srz[i] = (T)rz;
    srv[i] = (T)rv;
    srm[i] = (T)(bm - cuk);                    // 0 for the first block (no mu row)
    if (gn) srd[i] = TS::d_of(dg, srz, srm, srl, i);
  }
  __syncthreads();
  if (gn) TS::solve_gn(R, sru, srd, slam, scr);
  else TS::solve(L, kk, hv, R, sru, srz, srm, srl, slam, scr);
  if (on) {
    const double uo = weigh0((double)TS::u_of(scr, sru, i), pu);
    out(Tm.u + kk * P + i, uo);
    out(Tm.z + kk * P + i, weigh0((double)TS::z_of(L, dg, scr, srz, slam, i), pz));
    out(Tm.l + kk * P + i, weigh0((double)slam[i], pl));
    if (hv) {
      const double mo = weigh0((double)TS::mu_of(L, dg, scr, srm, srv, slam, i), pm);
      out(Tm.m + (kk - 1) * P + i, mo);
      out(Tm.v + (kk - 1) * P + i, weigh0(-(double)srm[i], pv));
      if (ru_m) fr.put_u(ru_m, i, yam - mo, b, Tm, Tc, P);
    }
    if (rm_m) fr.put_mu(rm_m, i, yau - uo, b, Tm, Tc, P);
  }
}

template <int RT, int CT, class T>
__global__ __launch_bounds__(kTiledThreads, 1) void k_jacobi_tiled(
    LevelView L, const double* __restrict__ b, const double* __restrict__ yold,
    const double* __restrict__ ec, int variant, double* __restrict__ ynew, FusedRestrict fr) {
  one_block<RT, CT, T>(L, b, yold, ec, variant, ynew, fr, blockIdx.x, false, false);
}

bool jacobi_tiled_supported(int p, int q) { return p == q && (p == 128 || p == 64); }

template <class T>
static hipError_t launch_tiled_t(const LevelView& L, const double* b, const double* yold,
                                 const double* ecoarse, int variant, double* ynew,
                                 FusedRestrict fr, hipStream_t s) {
  if (L.p == 128 && L.q == 128) {
    return launch_k(k_jacobi_tiled<4, 8, T>, dim3(L.n + 1), dim3(kTiledThreads), 0, s, L, b, yold,
                    ecoarse, variant, ynew, fr);
  } else if (L.p == 64 && L.q == 64) {
    return launch_k(k_jacobi_tiled<2, 4, T>, dim3(L.n + 1), dim3(kTiledThreads), 0, s, L, b, yold,
                    ecoarse, variant, ynew, fr);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_jacobi_tiled(const LevelView& L, const double* b, const double* yold,
                               const double* ecoarse, int variant, double* ynew,
                               double* restrict_out, double rbeta, double ra, hipStream_t s) {
  const FusedRestrict fr{restrict_out, variant, rbeta, ra, L.mu_scale};
  return L.fp32 ? launch_tiled_t<float>(L, b, yold, ecoarse, variant, ynew, fr, s)
                : launch_tiled_t<double>(L, b, yold, ecoarse, variant, ynew, fr, s);
}

// ---------------------------------------------------------------------------
// Two consecutive sweeps in one launch, one step per work-group.  The second
// sweep of block k needs only two values of the first: mu_k (block k+1) and
// u_{k-1} (block k-1), so the work-group keeps N_k and G_k^{-1} in registers,
// publishes its first-sweep block, waits for its two neighbours' and solves
// again.  Same arithmetic in the same order as two k_jacobi_tiled launches.
//
// The two coupling values a neighbour reads (u_k, mu_{k-1}) are stored and
// loaded as agent-scope atomics, which gfx950 performs at the device's
// coherence point with the sc1 bit (neither the store nor the load is held
// in the non-coherent L2 of an XCD).  The hand-off orders them at the ISA
// level: after its coupling stores every wave of the publishing work-group
// passes a compiler fence and then waits for their acknowledgement
// (s_waitcnt vmcnt(0): the stores are performed device-wide); one thread
// stores the flag only after the work-group barrier that follows; the
// waiting thread's flag loads come before the barrier and the compiler
// fence that precede the coupling loads, which the hardware issues in
// program order.  The first sweep's other values stay in the work-group's
// registers; of them only mu_n (block n+1) is stored, as a plain store.  The
// first-sweep vector y1 therefore holds valid u and mu entries only, which
// is all any later step reads of it.  (The same order under the
// HIP memory model's own rules, an agent-scope release fence in every
// thread before the barrier and acquire flag loads, also writes back the
// XCD's L2 at every hand-off: measured at 133 us against 86 us per
// two-sweep launch of the shared-block kernel on Burgers nx=128, n=1024.)
//
// y2 may be the buffer of yold: a work-group writes its second-sweep block
// only after both readers of that block's first-sweep couplings (the
// neighbours) have published, i.e. finished reading yold.
//
// Work-groups take their block from a ticket counter that only grows (the
// handle's launches are stream-ordered, so this launch owns tickets base ..
// base+n-1; the work-group of block n also takes block n+1).  A work-group
// waits only for first sweeps, which never wait, of blocks whose tickets are
// drawn (t-1) or will be drawn once a lower ticket's work-group has finished
// (t+1); the grid therefore drains whatever number of work-groups is
// resident.  Each wait also ends after ps.spin ticks of the wall clock
// (2 s unless a test of the error path shortens it) and raises *timeout, so
// every wave exits.
// ---------------------------------------------------------------------------

namespace {


// Wave 0 of the work-group (all 64 lanes) waits until each lane's flag (NULL:
// none) reads at least epoch, polling all of them at once; after ps.spin
// ticks it gives up and raises bit 0 of *timeout.
__device__ void await_wave(const unsigned long long* mine, unsigned long long epoch,
                           const PairSync& ps) {
  bool ok = !mine || __hip_atomic_load(mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
  if (__all(ok)) return;
  const unsigned long long t0 = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(2);
    if (!ok) ok = __hip_atomic_load(mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
    if (__all(ok)) return;
    if (wall_clock64() - t0 > ps.spin) {
      if (threadIdx.x == 0) atomicOr(ps.timeout, 1);
      return;
    }
  }
}

// Publish this work-group's first sweep (flag = epoch) and wait for the
// flags lo and hi of its neighbours (NULL: none); see above for the order.
__device__ void pair_handoff(unsigned long long* self, const unsigned long long* lo,
                             const unsigned long long* hi, const PairSync& ps) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");   // no store sinks below
  __builtin_amdgcn_s_waitcnt(0x0F70);                      // vmcnt(0): stores performed
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(self, ps.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x < kWave)
    await_wave(threadIdx.x == 0 ? lo : threadIdx.x == 1 ? hi : nullptr, ps.epoch, ps);
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");   // no load rises above
}

// Wait until blocks lo..hi (at most 64) of an earlier level of the launch
// have finished (flag = epoch + 1), same order as the hand-off.
__device__ void await_done(const unsigned long long* f, int lo, int hi, const PairSync& ps) {
  if (threadIdx.x < kWave) {
    const int j = lo + (int)threadIdx.x;
    await_wave(j <= hi ? f + j : nullptr, ps.epoch + 1, ps);
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// This block has finished: its outputs that a later level of the launch
// reads were stored coherently; once they are performed, flag = epoch + 1.
__device__ void publish_done(unsigned long long* self, const PairSync& ps) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(self, ps.epoch + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
}  // namespace

// ---------------------------------------------------------------------------
// Chained levels.  One launch can also run the two-sweep smoothing of
// several levels (k_jacobi_chain): the pre-smoothing of levels 0, 1, ..., L-2
// of a V-cycle, each level's last sweep restricting into the next level's
// right-hand side, or the post-smoothing of levels L-2, ..., 0, each level's
// first sweep interpolating the result of the coarser level of the same
// launch.  Tickets run through the levels in that order.  A block of a
// chained level first requests its tiles (written by an earlier launch), then
// waits for the blocks of the previous level of the chain that write what it
// reads, and only then loads them, with coherent loads; those blocks store
// these values coherently and raise their flag to epoch + 1 once the stores
// are performed.
//   * Restriction: coarse step m is written by the fine blocks that produce
//     fine steps 2m-1 and 2m (0-based blocks 2m-2, 2m-1; 2m-1, 2m in the
//     time-aligned variant), and coarse block k (1-based) reads coarse steps
//     k-1, k and, for the control mean, the fine right-hand side of the step
//     after its own, so it waits for fine blocks 2k-4 .. 2k+2 (0-based).
//   * Interpolation: fine step j takes coarse steps j/2 - 1 .. j/2 + 1 at
//     most, and coarse step m is written by coarse blocks m-1 and m (the
//     work-group of the last block also writes the last step's v and mu), so
//     fine block kb (0-based) waits for coarse blocks kb/2 - 2 .. kb/2 + 2.
// Every wait is for a lower ticket (the previous level) or for a neighbour's
// first sweep, which waits only for lower tickets, so the lowest unfinished
// ticket always progresses and the grid drains as above.
// ---------------------------------------------------------------------------

// One level's share of a two-sweep launch.
struct PairLevel {
  LevelView L;
  const double* b;
  const double* yold;
  const double* ec;
  double* y1;
  double* y2;
  FusedRestrict fr;
  int variant;
  int flag_off;   // flags of this level's blocks: ps.flag + flag_off + kb
  int dep;        // 0: inputs from earlier launches; 1: b is written by the
                  // previous (finer) level of the chain; 2: ec is the result
                  // of the previous (coarser) level of the chain
  int dep_off;    // flags of that level
  int dep_n;      // its block count
  int coh_y2;     // y2 is read by the next level of the chain
  int publish;    // the next level of the chain waits for this level's blocks
};

template <int RT, int CT, class T>
__device__ __forceinline__ void pair_block(const PairLevel& lv, const PairSync& ps, int kb) {
  using TS = TiledSolve<RT, CT, T>;
  constexpr int P = TS::P;
  static_assert(P <= kTiledThreads, "one entry per thread");
  __shared__ T sru[P], srz[P], srm[P], srl[P], srv[P], slam[P], srd[P];
  __shared__ T scr[TS::kScratch];
  const LevelView& L = lv.L;
  const double* __restrict__ b = lv.b;
  double* y1 = lv.y1;
  double* y2 = lv.y2;
  const FusedRestrict& fr = lv.fr;
  const bool gn = Mats<T>::GiN(L) != nullptr;   // W = G^{-1} N form (diagonal V, Z~)
  const int tid = threadIdx.x;
  const int n = L.n;
  const TypeMajor Tm(P, P, n);
  const int nc = n / 2;
  const TypeMajor Tc(P, P, nc > 0 ? nc : 1);
  const double w = L.omega;
  const bool on = tid < P;
  const int i = tid;
  unsigned long long* fl = ps.flag + lv.flag_off;
  const bool cb = lv.dep == 1;                 // b written in this launch
  auto ldb = [&](long long idx) -> double { return cb ? coherent_load(b + idx) : b[idx]; };
  auto put2 = [&](long long idx, double v) {
    if (lv.coh_y2) coherent_store(y2 + idx, v);
    else y2[idx] = v;
  };

  // first sweep: from the previous iterate plus the interpolated coarse
  // correction (first post-smoothing sweep)
  const PrevIterate prev{lv.yold, lv.ec, P, P, n, lv.variant, L.mu_scale, lv.dep == 2};
  // second sweep: weighted against this block's own first-sweep values
  auto weigh1 = [&](double yhat, double y1v) -> double {
    return w == 1.0 ? yhat : w * yhat + (1.0 - w) * y1v;
  };
  // publish this block's first sweep, then wait for the neighbours' (lo, hi:
  // block indices kb-1 and kb+1, or -1)
  auto hand_off = [&](int lo, int hi) {
    pair_handoff(fl + kb, lo >= 0 ? fl + lo : nullptr, hi >= 0 ? fl + hi : nullptr, ps);
  };

  const int k = kb + 1;
  const bool hv = k >= 2;
  const long long kk = k - 1;
  // the block's right-hand side, its couplings and the previous values that
  // weigh the first sweep
  double bu = 0.0, bm = 0.0, rl = 0.0, rz = 0.0, rv = 0.0, cmk = 0.0, cuk = 0.0;
  double pu = 0.0, pz = 0.0, pl = 0.0, pm = 0.0, pv = 0.0;
  typename TS::Diag dg;
  PrevFetch fcm, fcu, fu, fz, fl0, fm, fv;
  auto gather = [&]() {
    if (on) {
      bu = ldb(Tm.u + kk * P + i);
      rl = ldb(Tm.l + kk * P + i);
      rz = ldb(Tm.z + kk * P + i);
      fcm = prev.fetch(4, k, i);
      if (hv) {
        rv = ldb(Tm.v + (kk - 1) * P + i);
        bm = ldb(Tm.m + (kk - 1) * P + i);
        fcu = prev.fetch(0, k - 1, i);
      }
      if (w != 1.0) {
        fu = prev.fetch(0, k, i);
        fz = prev.fetch(2, k, i);
        fl0 = prev.fetch(3, k, i);
        if (hv) {
          fm = prev.fetch(4, k - 1, i);
          fv = prev.fetch(1, k - 1, i);
        }
      }
      dg = TS::diag_at(L, i);
    }
  };
  typename TS::Regs R;
  if (lv.dep == 0) {
    // requested before the tiles: loads complete in order, so the gather
    // waits for these alone and the tiles arrive during it
    gather();
    __builtin_amdgcn_sched_barrier(0);         // keep the loads above ahead of the tile's
    TS::load_straight(L, kk, gn, R);
    __builtin_amdgcn_sched_barrier(0);
  } else {
    // the tiles come from an earlier launch: in flight while this block
    // waits for the previous level of the chain
    TS::load_straight(L, kk, gn, R);
    __builtin_amdgcn_sched_barrier(0);
    const int lo = lv.dep == 1 ? 2 * kb - 2 : kb / 2 - 2;
    const int hi = lv.dep == 1 ? 2 * kb + 4 : kb / 2 + 2;
    await_done(ps.flag + lv.dep_off, lo > 0 ? lo : 0, hi < lv.dep_n - 1 ? hi : lv.dep_n - 1,
               ps);
    gather();
  }
  // first-sweep output (1 - omega) y_prev + omega y_hat, as weigh() forms it
  auto weigh0 = [&](double yhat, double yp) -> double {
    return w == 1.0 ? yhat : w * yhat + (1.0 - w) * yp;
  };
  if (on) {
    cmk = prev.value(fcm, 4, k);
    if (hv) cuk = prev.value(fcu, 0, k - 1);
    if (w != 1.0) {
      pu = prev.value(fu, 0, k);
      pz = prev.value(fz, 2, k);
      pl = prev.value(fl0, 3, k);
      if (hv) {
        pm = prev.value(fm, 4, k - 1);
        pv = prev.value(fv, 1, k - 1);
      }
    }
    sru[i] = (T)(bu - cmk);
    srl[i] = (T)rl;
    srz[i] = (T)rz;
    srv[i] = (T)rv;
    srm[i] = (T)(bm - cuk);                    // 0 for the first block (no mu row)
    if (gn) srd[i] = TS::d_of(dg, srz, srm, srl, i);
  }
  __syncthreads();
  if (gn) TS::solve_gn(R, sru, srd, slam, scr);
  else TS::solve(L, kk, hv, R, sru, srz, srm, srl, slam, scr);
  // the work-group of block n also takes block n+1 = (v_n, mu_n), whose
  // only coupling is u_n of block n: no other work-group reads it, and
  // block n's second sweep takes mu_n from this thread's register
  const bool tail = kb == n - 1;
  double rvn = 0.0, mon1 = 0.0, von1 = 0.0;
  if (tail && on) {
    rvn = ldb(Tm.v + (long long)(n - 1) * P + i);
    const double rmm = ldb(Tm.m + (long long)(n - 1) * P + i) - prev.at(0, n, i);
    mon1 = weigh(w, -rmm - rvn, prev, 4, n, i);
    von1 = weigh(w, -rmm, prev, 1, n, i);
    y1[Tm.m + (long long)(n - 1) * P + i] = mon1;
  }
  // this block's first-sweep values stay in registers for the second sweep;
  // y1 receives only its u and mu entries (the couplings the neighbours read
  // and what the product from the last sweep reads)
  double uo1 = 0.0, mo1 = 0.0, zo1 = 0.0, lo1 = 0.0, vo1 = 0.0;
  if (on) {
    uo1 = weigh0((double)TS::u_of(scr, sru, i), pu);
    zo1 = weigh0((double)TS::z_of(L, dg, scr, srz, slam, i), pz);
    lo1 = weigh0((double)slam[i], pl);
    coherent_store(y1 + Tm.u + kk * P + i, uo1);                    // read by block k+1
    if (hv) {
      mo1 = weigh0((double)TS::mu_of(L, dg, scr, srm, srv, slam, i), pm);
      vo1 = weigh0(-(double)srm[i], pv);
      coherent_store(y1 + Tm.m + (kk - 1) * P + i, mo1);            // read by block k-1
    }
  }
  hand_off(hv ? kb - 1 : -1, tail ? -1 : kb + 1);
  // second sweep: r_u = b_u,k - mu_k, r_mu = b_mu,k-1 - u_{k-1} of the first
  if (on) {
    sru[i] = (T)(bu - (tail ? mon1 : coherent_load(y1 + Tm.m + kk * P + i)));
    if (hv) srm[i] = (T)(bm - coherent_load(y1 + Tm.u + (kk - 1) * P + i));
    if (gn) srd[i] = TS::d_of(dg, srz, srm, srl, i);
  }
  __syncthreads();
  if (gn) TS::solve_gn(R, sru, srd, slam, scr);
  else TS::solve(L, kk, hv, R, sru, srz, srm, srl, slam, scr);
  const int rm_m = fr.mu_writer(k), ru_m = fr.u_writer(k);
  if (on) {
    const double uo = weigh1((double)TS::u_of(scr, sru, i), uo1);
    put2(Tm.u + kk * P + i, uo);
    put2(Tm.z + kk * P + i, weigh1((double)TS::z_of(L, dg, scr, srz, slam, i), zo1));
    put2(Tm.l + kk * P + i, weigh1((double)slam[i], lo1));
    if (hv) {
      const double mo = weigh1((double)TS::mu_of(L, dg, scr, srm, srv, slam, i), mo1);
      put2(Tm.m + (kk - 1) * P + i, mo);
      put2(Tm.v + (kk - 1) * P + i, weigh1(-(double)srm[i], vo1));
      if (ru_m) fr.put_u(ru_m, i, fr.a * mo1 - mo, b, Tm, Tc, P);
    }
    if (rm_m) fr.put_mu(rm_m, i, fr.a * uo1 - uo, b, Tm, Tc, P);
  }
  if (tail && on) {                            // block n+1, second sweep
    const int mu_m = fr.u_writer(n + 1);
    const double rmm = ldb(Tm.m + (long long)(n - 1) * P + i) - uo1;
    const double mo = weigh1(-rmm - rvn, mon1);
    put2(Tm.v + (long long)(n - 1) * P + i, weigh1(-rmm, von1));
    put2(Tm.m + (long long)(n - 1) * P + i, mo);
    if (mu_m) fr.put_u(mu_m, i, fr.a * mon1 - mo, b, Tm, Tc, P);
  }
  if (lv.publish) publish_done(fl + kb, ps);
}

template <int RT, int CT, class T>
__global__ __launch_bounds__(kTiledThreads, 1) void k_jacobi_tiled2(PairLevel lv, PairSync ps) {
  __shared__ int skb;
  if (threadIdx.x == 0) {
    const unsigned long long t = atomicAdd(ps.ticket, 1ull) - ps.base;
    skb = t < (unsigned long long)lv.L.n ? (int)t : -1;
  }
  __syncthreads();
  const int kb = skb;
  if (kb < 0) {                                // more tickets than blocks: a fault
    if (threadIdx.x == 0) atomicOr(ps.timeout, 2);
    return;
  }
  pair_block<RT, CT, T>(lv, ps, kb);
}

constexpr int kChainMax = 8;
struct PairChain {
  PairLevel lv[kChainMax];
  int start[kChainMax + 1];   // first ticket of each level; start[nlev] = all
  int nlev;
};
static_assert(sizeof(PairChain) <= 4096, "kernel argument size");

template <int RT, int CT, class T>
__global__ __launch_bounds__(kTiledThreads, 1) void k_jacobi_chain(PairChain ch, PairSync ps) {
  __shared__ int st;
  if (threadIdx.x == 0) {
    const unsigned long long t = atomicAdd(ps.ticket, 1ull) - ps.base;
    st = t < (unsigned long long)ch.start[ch.nlev] ? (int)t : -1;
  }
  __syncthreads();
  const int t = __builtin_amdgcn_readfirstlane(st);
  if (t < 0) {
    if (threadIdx.x == 0) atomicOr(ps.timeout, 2);
    return;
  }
  int c = 0;
  while (c + 1 < ch.nlev && t >= ch.start[c + 1]) ++c;
  pair_block<RT, CT, T>(ch.lv[c], ps, t - ch.start[c]);
}

static PairLevel pair_level(const LevelView& L, const double* b, const double* yold,
                            const double* ecoarse, int variant, double* y1, double* y2,
                            double* restrict_out, double rbeta, double ra) {
  PairLevel lv{};
  lv.L = L;
  lv.b = b;
  lv.yold = yold;
  lv.ec = ecoarse;
  lv.y1 = y1;
  lv.y2 = y2;
  lv.fr = FusedRestrict{restrict_out, variant, rbeta, ra, L.mu_scale};
  lv.variant = variant;
  return lv;
}

template <class T>
static hipError_t launch_tiled2_t(const PairLevel& lv, const PairSync& ps, hipStream_t s) {
  if (lv.L.p == 128 && lv.L.q == 128)
    return launch_k(k_jacobi_tiled2<4, 8, T>, dim3(lv.L.n), dim3(kTiledThreads), 0, s, lv, ps);
  if (lv.L.p == 64 && lv.L.q == 64)
    return launch_k(k_jacobi_tiled2<2, 4, T>, dim3(lv.L.n), dim3(kTiledThreads), 0, s, lv, ps);
  return hipErrorInvalidValue;
}

hipError_t launch_jacobi_tiled2(const LevelView& L, const double* b, const double* yold,
                                const double* ecoarse, int variant, double* y1, double* y2,
                                double* restrict_out, double rbeta, double ra,
                                const PairSync& ps, hipStream_t s) {
  const PairLevel lv = pair_level(L, b, yold, ecoarse, variant, y1, y2, restrict_out, rbeta, ra);
  return L.fp32 ? launch_tiled2_t<float>(lv, ps, s) : launch_tiled2_t<double>(lv, ps, s);
}

template <class T>
static hipError_t launch_chain_t(const PairChain& ch, const PairSync& ps, hipStream_t s) {
  const LevelView& L = ch.lv[0].L;
  const dim3 grid(ch.start[ch.nlev]);
  if (L.p == 128 && L.q == 128)
    return launch_k(k_jacobi_chain<4, 8, T>, grid, dim3(kTiledThreads), 0, s, ch, ps);
  if (L.p == 64 && L.q == 64)
    return launch_k(k_jacobi_chain<2, 4, T>, grid, dim3(kTiledThreads), 0, s, ch, ps);
  return hipErrorInvalidValue;
}

int jacobi_chain_max() { return kChainMax; }

// ---------------------------------------------------------------------------
// The block-parallel SGS application of the coarse solve (pitmg_coarse.hip)
// in one launch: its three block sweeps and two propagator products as five
// phases of one grid, tickets in phase order,
//   0  c = D^{-1} v                                   (blocks 1 .. n+1)
//   1  y_f,u = P c_u          (rows of the lower block-triangular propagator)
//   2  a = D^{-1} (v - L a), the coupling u_{k-1} from y_f
//   3  y_b,mu = Q a_mu        (rows of the upper block-triangular propagator)
//   4  d = -D^{-1} L^T y, the coupling mu_k from y_b (right-hand side zero).
// Each work-group waits only for the work-groups of the previous phase that
// write what it reads (so only for lower tickets: the grid drains with any
// number of resident work-groups), reads those values with coherent loads,
// and raises its flag to epoch + 1 once its coherent stores are performed.
// Sweeps are one_block (k_jacobi_tiled's body) and the rows k_gemv_tri's
// sums, so the results are those of the five separate launches.
// ---------------------------------------------------------------------------

struct SgsPhases {
  LevelView L;
  const double* v;       // right-hand side of sweeps 1 and 2
  const double* zero;    // zero vector, the right-hand side of sweep 3
  double* c;             // sweep outputs
  double* a;
  double* d;
  double* yf;            // propagated couplings (zero outside the u / mu rows)
  double* yb;
  const double* Pf;      // propagators, [n p][n p]
  const double* Qb;
  int variant;
};

constexpr int kSgsRows = kTiledThreads / kWave;   // propagator rows per work-group

// y[r] = x[r] + (off-diagonal blocks of row r) x, one wave, the sums of
// k_gemv_tri in its order; x read and y written coherently.
__device__ void sgs_row(const double* __restrict__ M, int nc, int p, int upper,
                        const double* x, double* y, long long r) {
  const long long ld = (long long)nc * p;
  const int lane = threadIdx.x % kWave;
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
    for (int t = 0; t < 8; ++t) a[t] += Mr[c + t * kWave] * coherent_load(x + c + t * kWave);
  }
  for (; c < c1; c += kWave) a[0] += Mr[c] * coherent_load(x + c);
  double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  acc = wave_sum(acc);
  if (lane == 0) coherent_store(y + r, coherent_load(x + r) + acc);
}

template <int RT, int CT, class T>
__global__ __launch_bounds__(kTiledThreads, 1) void k_sgs_fused(SgsPhases F, PairSync ps) {
  __shared__ int st;
  const int n = F.L.n, p = F.L.p, nb = n + 1;
  const long long ld = (long long)n * p;
  const int ng = (int)((ld + kSgsRows - 1) / kSgsRows);
  const int b1 = nb, b2 = nb + ng, b3 = 2 * nb + ng, b4 = 2 * nb + 2 * ng, b5 = 3 * nb + 2 * ng;
  if (threadIdx.x == 0) {
    const unsigned long long t = atomicAdd(ps.ticket, 1ull) - ps.base;
    st = t < (unsigned long long)b5 ? (int)t : -1;
  }
  __syncthreads();
  const int t = __builtin_amdgcn_readfirstlane(st);
  if (t < 0) {
    if (threadIdx.x == 0) atomicOr(ps.timeout, 2);
    return;
  }
  const TypeMajor Tm(p, p, n);
  const FusedRestrict none{nullptr, F.variant, 0.0, 1.0, F.L.mu_scale};
  unsigned long long* fl = ps.flag;
  const long long r = (long long)(t - (t < b2 ? b1 : b3)) * kSgsRows + threadIdx.x / kWave;
  // propagator work-groups holding block rows s0 .. s1 of the u / mu rows
  auto wgs = [&](int s0, int s1, int& lo, int& hi) {
    lo = (int)((long long)s0 * p / kSgsRows);
    hi = (int)(((long long)(s1 + 1) * p - 1) / kSgsRows);
  };
  if (t < b1) {                                    // 0: c = D^{-1} v
    one_block<RT, CT, T>(F.L, F.v, nullptr, nullptr, F.variant, F.c, none, t, false, true);
    publish_done(fl + t, ps);
  } else if (t < b2) {                             // 1: forward propagation
    const long long r0 = (long long)(t - b1) * kSgsRows;
    const long long s1 = (r0 + kSgsRows - 1) / p;
    await_done(fl, 0, (int)(s1 < n - 1 ? s1 : n - 1), ps);
    if (r < ld) sgs_row(F.Pf, n, p, 0, F.c + Tm.u, F.yf + Tm.u, r);
    publish_done(fl + t, ps);
  } else if (t < b3) {                             // 2: a = D^{-1}(v - L a)
    const int kb = t - b2;
    int lo, hi;
    wgs(kb < n ? (kb > 0 ? kb - 1 : 0) : n - 1, kb < n ? kb : n - 1, lo, hi);
    await_done(fl + b1, lo, hi < ng - 1 ? hi : ng - 1, ps);
    one_block<RT, CT, T>(F.L, F.v, F.yf, nullptr, F.variant, F.a, none, kb, true, true);
    publish_done(fl + t, ps);
  } else if (t < b4) {                             // 3: backward propagation
    const long long r0 = (long long)(t - b3) * kSgsRows;
    await_done(fl + b2, (int)(r0 / p) + 1, n, ps);
    if (r < ld) sgs_row(F.Qb, n, p, 1, F.a + Tm.m, F.yb + Tm.m, r);
    publish_done(fl + t, ps);
  } else {                                         // 4: d = -D^{-1} L^T y
    const int kb = t - b4;
    int lo, hi;
    wgs(kb < n ? (kb > 0 ? kb - 1 : 0) : n - 1, kb < n ? kb : n - 1, lo, hi);
    await_done(fl + b3, lo, hi < ng - 1 ? hi : ng - 1, ps);
    one_block<RT, CT, T>(F.L, F.zero, F.yb, nullptr, F.variant, F.d, none, kb, true, false);
  }
}

int sgs_fused_flags(int n, int p) {
  const long long ld = (long long)n * p;
  return 2 * (n + 1) + 2 * (int)((ld + kSgsRows - 1) / kSgsRows);
}

hipError_t launch_sgs_fused(const LevelView& L, const double* v, const double* zero, double* c,
                            double* a, double* d, double* yf, double* yb, const double* Pf,
                            const double* Qb, int variant, const PairSync& ps, int* groups,
                            hipStream_t s) {
  *groups = 0;
  if (L.fp32 || L.p != L.q || (L.p != 64 && L.p != 128) || L.n + 1 > 64 || !ps.ticket ||
      !ps.flag || !ps.timeout)
    return hipErrorInvalidValue;
  SgsPhases F{L, v, zero, c, a, d, yf, yb, Pf, Qb, variant};
  const long long ld = (long long)L.n * L.p;
  const int ng = (int)((ld + kSgsRows - 1) / kSgsRows);
  const int total = 3 * (L.n + 1) + 2 * ng;
  *groups = total;
  if (L.p == 128)
    return launch_k(k_sgs_fused<4, 8, double>, dim3(total), dim3(kTiledThreads), 0, s, F, ps);
  return launch_k(k_sgs_fused<2, 4, double>, dim3(total), dim3(kTiledThreads), 0, s, F, ps);
}

hipError_t launch_jacobi_chain(const ChainSweep* sw, int nlev, int up, int variant,
                               const PairSync& ps, int* groups, hipStream_t s) {
  *groups = 0;
  if (nlev < 1 || nlev > kChainMax || !ps.ticket || !ps.flag || !ps.timeout)
    return hipErrorInvalidValue;
  PairChain ch{};
  ch.nlev = nlev;
  int t = 0;
  for (int c = 0; c < nlev; ++c) {
    const ChainSweep& x = sw[c];
    if (x.L.p != sw[0].L.p || x.L.q != sw[0].L.q || x.L.fp32 != sw[0].L.fp32)
      return hipErrorInvalidValue;
    if (x.y1 == x.y2 || x.y1 == x.yold || x.y1 == x.b || x.y2 == x.b) return hipErrorInvalidValue;
    if (c > 0) {
      // the chain's own data flow: the restriction of the previous level is
      // this level's right-hand side (down), or the previous level's result
      // is this level's coarse correction (up)
      const ChainSweep& pr = sw[c - 1];
      const bool ok = up ? (pr.y2 == x.ec && pr.L.n * 2 == x.L.n && !x.restrict_out)
                         : (pr.restrict_out == x.b && x.L.n * 2 == pr.L.n && !x.ec);
      if (!ok) return hipErrorInvalidValue;
    }
    PairLevel lv = pair_level(x.L, x.b, x.yold, x.ec, variant, x.y1, x.y2, x.restrict_out,
                              x.rbeta, x.ra);
    lv.flag_off = x.flag_off;
    lv.dep = c == 0 ? 0 : (up ? 2 : 1);
    lv.dep_off = c == 0 ? 0 : sw[c - 1].flag_off;
    lv.dep_n = c == 0 ? 0 : sw[c - 1].L.n;
    lv.publish = c + 1 < nlev;
    lv.coh_y2 = up && c + 1 < nlev;
    lv.fr.coh_b = !up && c > 0;
    lv.fr.coh_rc = !up && c + 1 < nlev;
    ch.lv[c] = lv;
    ch.start[c] = t;
    t += x.L.n;
  }
  ch.start[nlev] = t;
  *groups = t;
  return sw[0].L.fp32 ? launch_chain_t<float>(ch, ps, s) : launch_chain_t<double>(ch, ps, s);
}

// ---------------------------------------------------------------------------
// Sweep for V_k and Z~_k shared by every step (stride 0, the theta = 1 case).
//
// A work-group takes up to kMaxSteps consecutive steps.  The products with
// the shared blocks are formed for all of its steps in one pass over each
// shared block (Z~ r_z - V r_mu before, Z~^T lambda and V^T lambda after the
// per-step solves), so each shared block crosses the CU's load path once per
// work-group instead of twice per step.  Per step only N_k and G_k^{-1} are
// read (register tiles, as in k_jacobi_tiled); the tiles of the next step are
// requested as soon as the current step has finished with them (G^{-1}
// after lambda, N after N^T lambda), so the HBM stream continues through the
// reductions.
// ---------------------------------------------------------------------------

namespace {
constexpr int kMaxSteps = 4;
}

template <int RT, int CT, class T>
__global__ __launch_bounds__(kTiledThreads, 1) void k_jacobi_shared(
    LevelView L, const double* __restrict__ b, const double* __restrict__ yold,
    const double* __restrict__ ec, int variant, double* __restrict__ ynew, int per_wg,
    FusedRestrict fr) {
  using TS = TiledSolve<RT, CT, T>;
  constexpr int P = TS::P;
  constexpr int G = kTiledThreads / P;                   // row groups of the post pass
  __shared__ T sru[kMaxSteps][P], srz[kMaxSteps][P], srm[kMaxSteps][P],
      srl[kMaxSteps][P], srv[kMaxSteps][P], sT[kMaxSteps][P], slam[kMaxSteps][P];
  __shared__ T st[P], ss[P], red[kTiledWaves * P];
  __shared__ T pz[G][kMaxSteps][P], pv[G][kMaxSteps][P];
  const int tid = threadIdx.x, a = tid / 16, bq = tid % 16;
  const int r0 = RT * a;
  const int n = L.n;
  const TypeMajor Tm(P, P, n);
  const int nc = n / 2;
  const TypeMajor Tc(P, P, nc > 0 ? nc : 1);
  const int k0 = blockIdx.x * per_wg + 1;                // first step (1-based)
  const int nb = min(per_wg, n - k0 + 1);                // steps of this work-group
  const T* __restrict__ Vs = Mats<T>::V(L);             // shared blocks
  const T* __restrict__ Zs = Mats<T>::Z(L);

  const double w = L.omega;
  const PrevIterate prev{yold, ec, P, P, n, variant, L.mu_scale};
  auto cu = [&](int k1, int i) -> double { return prev.at(0, k1, i); };
  auto cm = [&](int k1, int i) -> double { return prev.at(4, k1, i); };
  auto ya = [&](long long idx) -> double { return yold ? fr.a * yold[idx] : 0.0; };

  // tiles of the first step in flight while the right-hand sides are gathered
  typename TS::Regs R;
  TS::load(L, k0 - 1, R);
  for (int bi = 0; bi < nb; ++bi) {
    const int k = k0 + bi;
    const long long kk = k - 1;
    for (int i = tid; i < P; i += kTiledThreads) {
      sru[bi][i] = (T)(b[Tm.u + kk * P + i] - cm(k, i));
      srl[bi][i] = (T)b[Tm.l + kk * P + i];
      srz[bi][i] = (T)b[Tm.z + kk * P + i];
      if (k >= 2) {
        srv[bi][i] = (T)b[Tm.v + (kk - 1) * P + i];
        srm[bi][i] = (T)(b[Tm.m + (kk - 1) * P + i] - cu(k - 1, i));
      } else {
        srv[bi][i] = 0;
        srm[bi][i] = 0;
      }
    }
  }
  if (k0 + nb - 1 == n) {                                // block n+1 = (v_n, mu_n)
    const int mu_m = fr.u_writer(n + 1);
    for (int i = tid; i < P; i += kTiledThreads) {
      const double rvv = b[Tm.v + (long long)(n - 1) * P + i];
      const double rmm = b[Tm.m + (long long)(n - 1) * P + i] - cu(n, i);
      const double mo = weigh(w, -rmm - rvv, prev, 4, n, i);
      ynew[Tm.v + (long long)(n - 1) * P + i] = weigh(w, -rmm, prev, 1, n, i);
      ynew[Tm.m + (long long)(n - 1) * P + i] = mo;
      if (mu_m) fr.put_u(mu_m, i, ya(Tm.m + (long long)(n - 1) * P + i) - mo, b, Tm, Tc, P);
    }
  }
  __syncthreads();

  // sT[s] = Z~ r_z[s] - V r_mu[s] for every step: one pass over Z~ and V
  // (elementwise when they are diagonal)
  const bool dg = L.vz_diag != 0;
  if (dg) {
    const T* __restrict__ Vd = Mats<T>::Vd(L);
    const T* __restrict__ Zd = Mats<T>::Zd(L);
    for (int idx = tid; idx < nb * P; idx += kTiledThreads) {
      const int s = idx / P, i = idx % P;
      sT[s][i] = Zd[i] * srz[s][i] - Vd[i] * srm[s][i];
    }
  } else {
    T acc[kMaxSteps][RT];
#pragma unroll
    for (int s = 0; s < kMaxSteps; ++s)
#pragma unroll
      for (int r = 0; r < RT; ++r) acc[s][r] = 0;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      T zr[CT], vr[CT];
      tile_load_row<CT, T>(Zs + (long long)(r0 + r) * P, zr);
      tile_load_row<CT, T>(Vs + (long long)(r0 + r) * P, vr);
#pragma unroll
      for (int s = 0; s < kMaxSteps; ++s) {
        if (s < nb) {
#pragma unroll
          for (int c = 0; c < CT; ++c)
            acc[s][r] += zr[c] * srz[s][tile_col<T>(c)] - vr[c] * srm[s][tile_col<T>(c)];
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kMaxSteps; ++s) {
      if (s < nb) {
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          const T v = tile_sum16(acc[s][r]);
          if (bq == 0) sT[s][r0 + r] = v;
        }
      }
    }
  }
  __syncthreads();

  for (int bi = 0; bi < nb; ++bi) {
    const long long kk = k0 + bi - 1;
    // t = N r_u + (Z~ r_z - V r_mu) - r_l
    T acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < CT; ++c) s += R.nt[r][c] * sru[bi][tile_col<T>(c)];
      acc[r] = tile_sum16(s);
    }
    if (bq == 0) {
#pragma unroll
      for (int r = 0; r < RT; ++r) st[r0 + r] = acc[r] + sT[bi][r0 + r] - srl[bi][r0 + r];
    }
    __syncthreads();
    // s = G^{-1} t
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < CT; ++c) s += R.gt[r][c] * st[tile_col<T>(c)];
      acc[r] = tile_sum16(s);
    }
    if (bq == 0) {
#pragma unroll
      for (int r = 0; r < RT; ++r) ss[r0 + r] = acc[r];
    }
    __syncthreads();
    // lambda = G^{-T} s
    T cacc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      T s = 0;
#pragma unroll
      for (int r = 0; r < RT; ++r) s += R.gt[r][c] * ss[r0 + r];
      cacc[c] = s;
    }
    TS::col_partial(cacc, red);
    __syncthreads();
    for (int j = tid; j < P; j += kTiledThreads) slam[bi][j] = TS::col_total(red, j);
    __syncthreads();
    if (bi + 1 < nb) TS::load_g(L, kk + 1, R);             // G^{-1} of the next step
    // u = r_u - N^T lambda
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      T s = 0;
#pragma unroll
      for (int r = 0; r < RT; ++r) s += R.nt[r][c] * slam[bi][r0 + r];
      cacc[c] = s;
    }
    TS::col_partial(cacc, red);
    __syncthreads();
    if (bi + 1 < nb) TS::load_n(L, kk + 1, R);             // N of the next step
    const int rm_m = fr.mu_writer((int)kk + 1);
    for (int i = tid; i < P; i += kTiledThreads) {
      const double uo =
          weigh(w, (double)(sru[bi][i] - TS::col_total(red, i)), prev, 0, (int)kk + 1, i);
      ynew[Tm.u + kk * P + i] = uo;
      ynew[Tm.l + kk * P + i] = weigh(w, (double)slam[bi][i], prev, 3, (int)kk + 1, i);
      if (rm_m) fr.put_mu(rm_m, i, ya(Tm.u + kk * P + i) - uo, b, Tm, Tc, P);
    }
    __syncthreads();
  }

  // Z~^T lambda and V^T lambda for every step: one pass over Z~ and V.
  // Thread (j, g) = (tid % P, tid / P) sums rows i = g, g+G, ...
  if (!dg) {
    const int j = tid % P, g = tid / P;
    T za[kMaxSteps], va[kMaxSteps];
#pragma unroll
    for (int s = 0; s < kMaxSteps; ++s) {
      za[s] = 0;
      va[s] = 0;
    }
    for (int i = g; i < P; i += G) {
      const T zi = Zs[(long long)i * P + j], vi = Vs[(long long)i * P + j];
#pragma unroll
      for (int s = 0; s < kMaxSteps; ++s) {
        if (s < nb) {
          za[s] += zi * slam[s][i];
          va[s] += vi * slam[s][i];
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kMaxSteps; ++s) {
      pz[g][s][j] = za[s];
      pv[g][s][j] = va[s];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < nb * P; idx += kTiledThreads) {
    const int s = idx / P, i = idx % P;
    const long long kk = k0 + s - 1;
    T zt = 0, vt = 0;
    if (dg) {
      zt = Mats<T>::Zd(L)[i] * slam[s][i];
      vt = Mats<T>::Vd(L)[i] * slam[s][i];
    } else {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        zt += pz[g][s][i];
        vt += pv[g][s][i];
      }
    }
    const int k = (int)kk + 1;
    ynew[Tm.z + kk * P + i] = weigh(w, (double)(srz[s][i] - zt), prev, 2, k, i);
    if (kk >= 1) {
      const double mo = weigh(w, (double)(vt - srm[s][i] - srv[s][i]), prev, 4, k - 1, i);
      ynew[Tm.m + (kk - 1) * P + i] = mo;
      ynew[Tm.v + (kk - 1) * P + i] = weigh(w, -(double)srm[s][i], prev, 1, k - 1, i);
      const int ru_m = fr.u_writer(k);
      if (ru_m) fr.put_u(ru_m, i, ya(Tm.m + (kk - 1) * P + i) - mo, b, Tm, Tc, P);
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 shared-block sweep with the next step's N_k in flight.
//
// As k_jacobi_shared (register tiles of N_k and G_k^{-1}, products with the
// shared V and Z~ for all steps of the group in one pass each), except that
// N of the next step is requested at the start of the current one: it is
// moved by direct global-to-LDS loads into a staging buffer (128 KB at
// p = 128) and copied into the register tile when its step begins, so the
// HBM stream of N runs under the current step's arithmetic.  G^{-1} of the
// next step is loaded into its register tile once lambda is formed.
// Results stay in LDS and are written after the last step: stores count in
// the same vector-memory counter as the loads the step start waits for.
// ---------------------------------------------------------------------------

// One sweep of steps k0 .. k0+nb-1 (and block n+1 when the group ends at
// step n).  In a two-sweep launch, pub makes the two first-sweep values that
// neighbouring groups read (u of the last step, mu_{k0-1} of the first)
// device-coherent stores, and xin makes the second sweep read those two
// couplings of the neighbours with device-coherent loads; every other
// coupling comes from this work-group's own first sweep.
template <int RT, int CT>
__device__ __forceinline__ void shared_nl_sweep(
    const LevelView& L, const double* __restrict__ b, const double* yold, const double* ec,
    int variant, double* ynew, int k0, int nb, FusedRestrict fr, bool pub, bool xin) {
  using TS = TiledSolve<RT, CT, double>;
  constexpr int P = TS::P;
  constexpr int G = kTiledThreads / P;                   // row groups of the post pass
  constexpr int kUnits = P * P / 2;                      // 16-byte units of N_k
  constexpr int kChunks = kUnits / kWave;                // one wave load (1 KB) each
  static_assert(kChunks % kTiledWaves == 0, "whole chunks per wave");
  static_assert(2 * G * kMaxSteps * P <= P * P, "post-pass slabs fit");
  static_assert(3 * kMaxSteps * P <= P * P, "gathered right-hand sides fit");
  static_assert(RT % 2 == 0, "row pairs of st");
  __shared__ double nbuf[P * P];                         // staged N of the next step
  __shared__ double sru[kMaxSteps][P], sT[kMaxSteps][P], slam[kMaxSteps][P], sou[kMaxSteps][P];
  __shared__ double st[P], ss[P], red[kTiledWaves * P];
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  const int a = tid / 16, bq = tid % 16, r0 = RT * a;
  const int n = L.n;
  const TypeMajor Tm(P, P, n);
  const int nc = n / 2;
  const TypeMajor Tc(P, P, nc > 0 ? nc : 1);
  const int klast = k0 + nb - 1;                         // last step of the group
  const double* __restrict__ Vs = L.V;                   // shared blocks
  const double* __restrict__ Zs = L.Z;

  // couplings of the previous iterate; u_{k0-1} and mu_klast (klast < n)
  // belong to the neighbouring groups
  auto cu = [&](int k1, int i) -> double {
    double v = 0.0;
    if (yold) {
      const double* p = yold + Tm.u + (long long)(k1 - 1) * P + i;
      v = xin && k1 == k0 - 1 ? coherent_load(p) : *p;
    }
    if (ec) v += interp_node(ec + Tc.u, nc, P, k1, i, variant);
    return v;
  };
  auto cm = [&](int k1, int i) -> double {
    double v = 0.0;
    if (yold) {
      const double* p = yold + Tm.m + (long long)(k1 - 1) * P + i;
      v = xin && k1 == klast && klast < n ? coherent_load(p) : *p;
    }
    if (ec) v += L.mu_scale * interp_node(ec + Tc.m, nc, P, k1, i, variant);
    return v;
  };
  // the previous iterate at this group's own slots, for the weighted update
  // and the fused restriction; the two slots the first sweep published with
  // device-coherent stores are read back the same way
  const double w = L.omega;
  const PrevIterate prev{yold, ec, P, P, n, variant, L.mu_scale};
  auto own = [&](int type, int k1, int i) -> double {
    if (xin && yold && ((type == 0 && k1 == klast) || (type == 4 && k1 == k0 - 1)))
      return coherent_load(yold + (type == 0 ? Tm.u : Tm.m) + (long long)(k1 - 1) * P + i);
    return prev.at(type, k1, i);
  };
  auto wt = [&](double yhat, int type, int k1, int i) -> double {
    return w == 1.0 ? yhat : w * yhat + (1.0 - w) * own(type, k1, i);
  };
  auto ya = [&](int type, int k1, int i) -> double {
    return yold ? fr.a * own(type, k1, i) : 0.0;
  };
  // N_k (row-major, contiguous) into nbuf: wave w moves chunks w, w + 8, ...
  auto stage_n = [&](long long kk) {
    const double* Nk = L.N + kk * L.sN;
#pragma unroll
    for (int t = 0; t < kChunks / kTiledWaves; ++t) {
      const int c = wv + kTiledWaves * t;
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)(Nk + 2 * (kWave * c + lane)),
          (__attribute__((address_space(3))) void*)(nbuf + 2 * kWave * c), 16, 0, 0);
    }
  };
  // the thread's register tile of N from the staged copy
  auto unstage_n = [&](typename TS::Regs& R) {
#pragma unroll
    for (int r = 0; r < RT; ++r) tile_load_row<CT, double>(nbuf + (r0 + r) * P, R.nt[r]);
  };
  // barrier inside a step: LDS accesses complete (lgkmcnt(0)); no wait on
  // the vector-memory counter, which holds the staged N in flight
  auto lds_barrier = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);                  // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };

  // tiles of the first step in flight while the right-hand sides are gathered
  typename TS::Regs R;
  TS::load(L, k0 - 1, R);
  double* srz = nbuf;                                    // pre-pass only
  double* srm = nbuf + kMaxSteps * P;
  double* srl = nbuf + 2 * kMaxSteps * P;
  for (int bi = 0; bi < nb; ++bi) {
    const int k = k0 + bi;
    const long long kk = k - 1;
    for (int i = tid; i < P; i += kTiledThreads) {
      sru[bi][i] = b[Tm.u + kk * P + i] - cm(k, i);
      srl[bi * P + i] = b[Tm.l + kk * P + i];
      srz[bi * P + i] = b[Tm.z + kk * P + i];
      srm[bi * P + i] = k >= 2 ? b[Tm.m + (kk - 1) * P + i] - cu(k - 1, i) : 0.0;
    }
  }
  if (k0 + nb - 1 == n) {                                // block n+1 = (v_n, mu_n)
    const int mu_m = fr.u_writer(n + 1);
    for (int i = tid; i < P; i += kTiledThreads) {
      const double rvv = b[Tm.v + (long long)(n - 1) * P + i];
      const double rmm = b[Tm.m + (long long)(n - 1) * P + i] - cu(n, i);
      const double mo = wt(-rmm - rvv, 4, n, i);
      const double vo = wt(-rmm, 1, n, i);
      // the old values are read before this thread's stores replace them
      const double ca = mu_m ? ya(4, n, i) : 0.0;
      ynew[Tm.v + (long long)(n - 1) * P + i] = vo;
      ynew[Tm.m + (long long)(n - 1) * P + i] = mo;
      if (mu_m) fr.put_u(mu_m, i, ca - mo, b, Tm, Tc, P);
    }
  }
  __syncthreads();

  // sT[s] = Z~ r_z[s] - V r_mu[s] - r_lambda[s] for every step (elementwise
  // when V and Z~ are diagonal)
  const bool dg = L.vz_diag != 0;
  if (dg) {
    for (int idx = tid; idx < nb * P; idx += kTiledThreads) {
      const int s2 = idx / P, i = idx % P;
      sT[s2][i] = L.Zd[i] * srz[s2 * P + i] - L.Vd[i] * srm[s2 * P + i] - srl[s2 * P + i];
    }
  } else {
    double acc[kMaxSteps][RT];
#pragma unroll
    for (int s2 = 0; s2 < kMaxSteps; ++s2)
#pragma unroll
      for (int r = 0; r < RT; ++r) acc[s2][r] = 0;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      double zr[CT], vr[CT];
      tile_load_row<CT, double>(Zs + (long long)(r0 + r) * P, zr);
      tile_load_row<CT, double>(Vs + (long long)(r0 + r) * P, vr);
#pragma unroll
      for (int s2 = 0; s2 < kMaxSteps; ++s2) {
        if (s2 < nb) {
#pragma unroll
          for (int c = 0; c < CT; ++c)
            acc[s2][r] += zr[c] * srz[s2 * P + tile_col<double>(c)] -
                          vr[c] * srm[s2 * P + tile_col<double>(c)];
        }
      }
    }
#pragma unroll
    for (int s2 = 0; s2 < kMaxSteps; ++s2) {
      if (s2 < nb) {
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          const double v = tile_sum16(acc[s2][r]);
          if (bq == 0) sT[s2][r0 + r] = v - srl[s2 * P + r0 + r];
        }
      }
    }
  }
  __syncthreads();                                       // staging buffer free

  for (int bi = 0; bi < nb; ++bi) {
    // N (staged, or loaded directly for the first step) and G^{-1} of this
    // step have arrived; waiting on every path leaves no load of this step
    // pending once the next step's loads are issued
    __builtin_amdgcn_s_waitcnt(0x0F70);                  // vmcnt(0)
    __syncthreads();
    if (bi > 0) {
      unstage_n(R);
      lds_barrier();                                     // every wave has its tile
    }
    if (bi + 1 < nb) stage_n(k0 + bi);                   // N of the next step
    // t = N r_u + (Z~ r_z - V r_mu - r_lambda)
    double acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      double sum = 0;
#pragma unroll
      for (int c = 0; c < CT; ++c) sum += R.nt[r][c] * sru[bi][tile_col<double>(c)];
      acc[r] = tile_sum16(sum);
    }
    if (bq == 0) {
#pragma unroll
      for (int r = 0; r < RT; r += 2)
        *reinterpret_cast<double2*>(st + r0 + r) =
            make_double2(acc[r] + sT[bi][r0 + r], acc[r + 1] + sT[bi][r0 + r + 1]);
    }
    lds_barrier();
    // s = G^{-1} t
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      double sum = 0;
#pragma unroll
      for (int c = 0; c < CT; ++c) sum += R.gt[r][c] * st[tile_col<double>(c)];
      acc[r] = tile_sum16(sum);
    }
    if (bq == 0) {
#pragma unroll
      for (int r = 0; r < RT; r += 2)
        *reinterpret_cast<double2*>(ss + r0 + r) = make_double2(acc[r], acc[r + 1]);
    }
    lds_barrier();
    // lambda = G^{-T} s
    double cacc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      double sum = 0;
#pragma unroll
      for (int r = 0; r < RT; ++r) sum += R.gt[r][c] * ss[r0 + r];
      cacc[c] = sum;
    }
    TS::col_partial(cacc, red);
    lds_barrier();
    for (int j = tid; j < P; j += kTiledThreads) slam[bi][j] = TS::col_total(red, j);
    lds_barrier();
    if (bi + 1 < nb) TS::load_g(L, k0 + bi, R);          // G^{-1} of the next step
    // u = r_u - N^T lambda
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      double sum = 0;
#pragma unroll
      for (int r = 0; r < RT; ++r) sum += R.nt[r][c] * slam[bi][r0 + r];
      cacc[c] = sum;
    }
    TS::col_partial(cacc, red);
    lds_barrier();
    for (int i = tid; i < P; i += kTiledThreads) sou[bi][i] = sru[bi][i] - TS::col_total(red, i);
  }
  __syncthreads();

  // Z~^T lambda and V^T lambda for every step (slabs in the idle staging
  // buffer), then every output of the work-group
  double* pz = nbuf;                                     // [G][kMaxSteps][P]
  double* pv = nbuf + G * kMaxSteps * P;
  if (!dg) {
    const int j = tid % P, g = tid / P;
    double za[kMaxSteps], va[kMaxSteps];
#pragma unroll
    for (int s2 = 0; s2 < kMaxSteps; ++s2) {
      za[s2] = 0;
      va[s2] = 0;
    }
    // rows g, g + G, ... in batches of 8: every load of a batch is issued
    // before any of its products, so the L2 latency is paid once per batch;
    // every step slot is formed (slots past nb are never written out)
    constexpr int kRowBatch = 8;
    static_assert((P / G) % kRowBatch == 0, "whole row batches");
#pragma unroll 1
    for (int i0 = g; i0 < P; i0 += G * kRowBatch) {
      double zr[kRowBatch], vr[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        zr[u] = Zs[(long long)(i0 + u * G) * P + j];
        vr[u] = Vs[(long long)(i0 + u * G) * P + j];
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
#pragma unroll
        for (int s2 = 0; s2 < kMaxSteps; ++s2) {
          za[s2] += zr[u] * slam[s2][i0 + u * G];
          va[s2] += vr[u] * slam[s2][i0 + u * G];
        }
      }
    }
#pragma unroll
    for (int s2 = 0; s2 < kMaxSteps; ++s2) {
      pz[(g * kMaxSteps + s2) * P + j] = za[s2];
      pv[(g * kMaxSteps + s2) * P + j] = va[s2];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < nb * P; idx += kTiledThreads) {
    const int s2 = idx / P, i = idx % P;
    const int k = k0 + s2;
    const long long kk = k - 1;
    double zt = 0, vt = 0;
    if (dg) {
      zt = L.Zd[i] * slam[s2][i];
      vt = L.Vd[i] * slam[s2][i];
    } else {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        zt += pz[(g * kMaxSteps + s2) * P + i];
        vt += pv[(g * kMaxSteps + s2) * P + i];
      }
    }
    const int rm_m = fr.mu_writer(k);
    const int ru_m = k >= 2 ? fr.u_writer(k) : 0;
    // every old value of the block is read before any store of this thread
    // replaces it (ynew may be the buffer of yold only in the second sweep of
    // a two-sweep launch, where yold is this group's own first sweep)
    const double uo = wt(sou[s2][i], 0, k, i);
    const double lo = wt(slam[s2][i], 3, k, i);
    const double zo = wt(b[Tm.z + kk * P + i] - zt, 2, k, i);
    const double cua = rm_m ? ya(0, k, i) : 0.0;
    double mo = 0.0, vo = 0.0, cma = 0.0;
    if (k >= 2) {
      const double rm = b[Tm.m + (kk - 1) * P + i] - cu(k - 1, i);
      mo = wt(vt - rm - b[Tm.v + (kk - 1) * P + i], 4, k - 1, i);
      vo = wt(-rm, 1, k - 1, i);
      cma = ru_m ? ya(4, k - 1, i) : 0.0;
    }
    if (pub && k == klast)
      coherent_store(ynew + Tm.u + kk * P + i, uo);      // read by the next group
    else
      ynew[Tm.u + kk * P + i] = uo;
    ynew[Tm.l + kk * P + i] = lo;
    ynew[Tm.z + kk * P + i] = zo;
    if (rm_m) fr.put_mu(rm_m, i, cua - uo, b, Tm, Tc, P);
    if (k >= 2) {
      if (pub && k == k0)
        coherent_store(ynew + Tm.m + (kk - 1) * P + i, mo);   // read by the previous group
      else
        ynew[Tm.m + (kk - 1) * P + i] = mo;
      ynew[Tm.v + (kk - 1) * P + i] = vo;
      if (ru_m) fr.put_u(ru_m, i, cma - mo, b, Tm, Tc, P);
    }
  }
}

template <int RT, int CT>
__global__ __launch_bounds__(kTiledThreads, 1) void k_jacobi_shared_nl(
    LevelView L, const double* __restrict__ b, const double* __restrict__ yold,
    const double* __restrict__ ec, int variant, double* __restrict__ ynew, int per_wg,
    FusedRestrict fr) {
  const int k0 = blockIdx.x * per_wg + 1;                // first step (1-based)
  shared_nl_sweep<RT, CT>(L, b, yold, ec, variant, ynew, k0, min(per_wg, L.n - k0 + 1), fr,
                          false, false);
}

// Two consecutive sweeps of the shared-block kernel in one launch: the
// group's second sweep needs, besides its own first sweep, only u at the
// previous group's last step and mu at the next group's first block.
// Groups draw their index from the ticket counter and hand off as in
// k_jacobi_tiled2 (same deadlock-freedom argument, bounded waits); the
// group's tiles are loaded again for the second sweep.
template <int RT, int CT>
__global__ __launch_bounds__(kTiledThreads, 1) void k_jacobi_shared_nl2(
    LevelView L, const double* __restrict__ b, const double* yold,
    const double* __restrict__ ec, int variant, double* y1, double* y2, int per_wg,
    FusedRestrict fr, PairSync ps) {
  __shared__ int sg;
  const int tid = threadIdx.x;
  const int ng = (L.n + per_wg - 1) / per_wg;
  if (tid == 0) {
    const unsigned long long t = atomicAdd(ps.ticket, 1ull) - ps.base;
    sg = t < (unsigned long long)ng ? (int)t : -1;
  }
  __syncthreads();
  const int g = sg;
  if (g < 0) {                                 // more tickets than groups: a fault
    if (tid == 0) atomicOr(ps.timeout, 2);
    return;
  }
  const int k0 = g * per_wg + 1;
  const int nb = min(per_wg, L.n - k0 + 1);
  shared_nl_sweep<RT, CT>(L, b, yold, ec, variant, y1, k0, nb,
                          FusedRestrict{nullptr, variant, 0.0, 1.0, L.mu_scale}, true, false);
  pair_handoff(ps.flag + g, g > 0 ? ps.flag + g - 1 : nullptr,
               g + 1 < ng ? ps.flag + g + 1 : nullptr, ps);
  shared_nl_sweep<RT, CT>(L, b, y1, nullptr, variant, y2, k0, nb, fr, false, true);
}

bool jacobi_shared_supported(const LevelView& L) {
  return L.sV == 0 && L.sZ == 0 && L.p == L.q && (L.p == 128 || L.p == 64);
}

template <class T>
static hipError_t launch_shared_t(const LevelView& L, const double* b, const double* yold,
                                  const double* ecoarse, int variant, double* ynew, int per,
                                  FusedRestrict fr, hipStream_t s) {
  const int nwg = (L.n + per - 1) / per;
  if constexpr (std::is_same<T, double>::value) {
    if (L.p == 128)
      return launch_k(k_jacobi_shared_nl<4, 8>, dim3(nwg), dim3(kTiledThreads), 0, s, L, b, yold,
                      ecoarse, variant, ynew, per, fr);
    if (L.p == 64)
      return launch_k(k_jacobi_shared_nl<2, 4>, dim3(nwg), dim3(kTiledThreads), 0, s, L, b, yold,
                      ecoarse, variant, ynew, per, fr);
    return hipErrorInvalidValue;
  } else if (L.p == 128) {
    return launch_k(k_jacobi_shared<4, 8, T>, dim3(nwg), dim3(kTiledThreads), 0, s, L, b, yold,
                    ecoarse, variant, ynew, per, fr);
  } else if (L.p == 64) {
    return launch_k(k_jacobi_shared<2, 4, T>, dim3(nwg), dim3(kTiledThreads), 0, s, L, b, yold,
                    ecoarse, variant, ynew, per, fr);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// steps per work-group of the shared-block sweep: the tuned choice, else
// enough to keep the grid near one work-group per CU
int shared_steps_per_group(const LevelView& L) {
  int per = L.sweep_cfg > 0 ? L.sweep_cfg : (L.n + 255) / 256;
  if (per > kMaxSteps) per = kMaxSteps;
  if (per < 1) per = 1;
  return per;
}

hipError_t launch_jacobi_shared2(const LevelView& L, const double* b, const double* yold,
                                 const double* ecoarse, int variant, double* y1, double* y2,
                                 double* restrict_out, double rbeta, double ra,
                                 const PairSync& ps, int* groups, hipStream_t s) {
  const FusedRestrict fr{restrict_out, variant, rbeta, ra, L.mu_scale};
  const int per = shared_steps_per_group(L);
  const int nwg = (L.n + per - 1) / per;
  *groups = nwg;
  if (L.fp32) return hipErrorNotSupported;
  if (L.p == 128)
    return launch_k(k_jacobi_shared_nl2<4, 8>, dim3(nwg), dim3(kTiledThreads), 0, s, L, b, yold,
                    ecoarse, variant, y1, y2, per, fr, ps);
  if (L.p == 64)
    return launch_k(k_jacobi_shared_nl2<2, 4>, dim3(nwg), dim3(kTiledThreads), 0, s, L, b, yold,
                    ecoarse, variant, y1, y2, per, fr, ps);
  return hipErrorInvalidValue;
}

hipError_t launch_jacobi_shared(const LevelView& L, const double* b, const double* yold,
                                const double* ecoarse, int variant, double* ynew,
                                double* restrict_out, double rbeta, double ra, hipStream_t s) {
  const FusedRestrict fr{restrict_out, variant, rbeta, ra, L.mu_scale};
  const int per = shared_steps_per_group(L);
  return L.fp32 ? launch_shared_t<float>(L, b, yold, ecoarse, variant, ynew, per, fr, s)
                : launch_shared_t<double>(L, b, yold, ecoarse, variant, ynew, per, fr, s);
}


// ---------------------------------------------------------------------------
// out = beta b + alpha A~ x for p = q in {64, 128} with V and Z~ shared by
// every step: a work-group takes up to kMaxSteps consecutive steps, N_k in
// the register tile of the sweep (pitmg_tiled.h) serving both its row
// product N u_k and its column product N^T lambda_k, so each N_k is read
// from HBM once; the products with the shared V and Z~ are formed for all
// steps of the group in one pass over each (rows before, columns after).
// Rows of time-major block k: lambda_k = N u_k + V v_{k-1} + Z z_k,
// u_k + N^T lambda_k + mu_k, z_k + Z^T lambda_k, v_{k-1} + V^T lambda_k -
// mu_{k-1}, u_{k-1} - v_{k-1}; block n+1 (with step n): v_n - mu_n, u_n - v_n.
// ---------------------------------------------------------------------------

template <int RT, int CT>
__global__ __launch_bounds__(kTiledThreads, 1) void k_apply_shared(
    LevelView L, const double* __restrict__ x, const double* __restrict__ b, double alpha,
    double beta, double* __restrict__ out, int per_wg) {
  using TS = TiledSolve<RT, CT, double>;
  constexpr int P = TS::P;
  constexpr int G = kTiledThreads / P;
  __shared__ double su[kMaxSteps][P], sl[kMaxSteps][P], svz[kMaxSteps][P];
  __shared__ double sxv[kMaxSteps][P], sxz[kMaxSteps][P];
  __shared__ double red[kTiledWaves * P];
  __shared__ double pz[G][kMaxSteps][P], pv[G][kMaxSteps][P];
  const int tid = threadIdx.x, a = tid / 16, bq = tid % 16;
  const int r0 = RT * a;
  const int n = L.n;
  const TypeMajor Tm(P, P, n);
  const int k0 = blockIdx.x * per_wg + 1;
  const int nb = min(per_wg, n - k0 + 1);
  const double* __restrict__ Vs = L.V;
  const double* __restrict__ Zs = L.Z;
  auto put = [&](long long idx, double val) {
    out[idx] = (beta != 0.0 ? beta * b[idx] : 0.0) + alpha * val;
  };

  typename TS::Regs R;
  TS::load_n(L, k0 - 1, R);
  for (int s = 0; s < nb; ++s) {
    const long long kk = k0 + s - 1;
    for (int i = tid; i < P; i += kTiledThreads) {
      su[s][i] = x[Tm.u + kk * P + i];
      sl[s][i] = x[Tm.l + kk * P + i];
      sxz[s][i] = x[Tm.z + kk * P + i];
      sxv[s][i] = kk >= 1 ? x[Tm.v + (kk - 1) * P + i] : 0.0;
    }
  }
  __syncthreads();
  // svz[s] = V v_{k-1} + Z z_k for every step: one pass over V and Z~
  // (elementwise when they are diagonal)
  const bool dg = L.vz_diag != 0;
  if (dg) {
    for (int idx = tid; idx < nb * P; idx += kTiledThreads) {
      const int s = idx / P, i = idx % P;
      svz[s][i] = L.Vd[i] * sxv[s][i] + L.Zd[i] * sxz[s][i];
    }
  } else {
    double acc[kMaxSteps][RT];
#pragma unroll
    for (int s = 0; s < kMaxSteps; ++s)
#pragma unroll
      for (int r = 0; r < RT; ++r) acc[s][r] = 0;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      double zr[CT], vr[CT];
      tile_load_row<CT, double>(Zs + (long long)(r0 + r) * P, zr);
      tile_load_row<CT, double>(Vs + (long long)(r0 + r) * P, vr);
#pragma unroll
      for (int s = 0; s < kMaxSteps; ++s) {
        if (s < nb) {
#pragma unroll
          for (int c = 0; c < CT; ++c)
            acc[s][r] += zr[c] * sxz[s][tile_col<double>(c)] + vr[c] * sxv[s][tile_col<double>(c)];
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kMaxSteps; ++s) {
      if (s < nb) {
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          const double v = tile_sum16(acc[s][r]);
          if (bq == 0) svz[s][r0 + r] = v;
        }
      }
    }
  }
  __syncthreads();
  for (int s = 0; s < nb; ++s) {
    const long long kk = k0 + s - 1;
    // lambda row: N u_k + (V v_{k-1} + Z z_k)
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      double sum = 0;
#pragma unroll
      for (int c = 0; c < CT; ++c) sum += R.nt[r][c] * su[s][tile_col<double>(c)];
      sum = tile_sum16(sum);
      if (bq == 0) put(Tm.l + kk * P + r0 + r, sum + svz[s][r0 + r]);
    }
    // u row: u_k + N^T lambda_k + mu_k
    double cacc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      double sum = 0;
#pragma unroll
      for (int r = 0; r < RT; ++r) sum += R.nt[r][c] * sl[s][r0 + r];
      cacc[c] = sum;
    }
    TS::col_partial(cacc, red);
    __syncthreads();
    if (s + 1 < nb) TS::load_n(L, kk + 1, R);           // N of the next step
    for (int i = tid; i < P; i += kTiledThreads)
      put(Tm.u + kk * P + i, su[s][i] + TS::col_total(red, i) + x[Tm.m + kk * P + i]);
    __syncthreads();
  }
  // Z^T lambda and V^T lambda for every step: one pass over Z~ and V
  if (!dg) {
    const int j = tid % P, g = tid / P;
    double za[kMaxSteps], va[kMaxSteps];
#pragma unroll
    for (int s = 0; s < kMaxSteps; ++s) {
      za[s] = 0;
      va[s] = 0;
    }
    for (int i = g; i < P; i += G) {
      const double zi = Zs[(long long)i * P + j], vi = Vs[(long long)i * P + j];
#pragma unroll
      for (int s = 0; s < kMaxSteps; ++s) {
        if (s < nb) {
          za[s] += zi * sl[s][i];
          va[s] += vi * sl[s][i];
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kMaxSteps; ++s) {
      pz[g][s][j] = za[s];
      pv[g][s][j] = va[s];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < nb * P; idx += kTiledThreads) {
    const int s = idx / P, i = idx % P;
    const long long kk = k0 + s - 1;
    double zt = 0, vt = 0;
    if (dg) {
      zt = L.Zd[i] * sl[s][i];
      vt = L.Vd[i] * sl[s][i];
    } else {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        zt += pz[g][s][i];
        vt += pv[g][s][i];
      }
    }
    put(Tm.z + kk * P + i, sxz[s][i] + zt);
    if (kk >= 1) {
      put(Tm.v + (kk - 1) * P + i, sxv[s][i] + vt - x[Tm.m + (kk - 1) * P + i]);
      put(Tm.m + (kk - 1) * P + i, x[Tm.u + (kk - 1) * P + i] - sxv[s][i]);
    }
    if (kk == n - 1) {                                    // block n+1
      const double vn = x[Tm.v + kk * P + i], mn = x[Tm.m + kk * P + i];
      put(Tm.v + kk * P + i, vn - mn);
      put(Tm.m + kk * P + i, su[s][i] - vn);
    }
  }
}

bool apply_shared_supported(const LevelView& L) {
  return !L.fp32 && jacobi_shared_supported(L) && (reinterpret_cast<uintptr_t>(L.N) & 15u) == 0 &&
         (reinterpret_cast<uintptr_t>(L.V) & 15u) == 0 &&
         (reinterpret_cast<uintptr_t>(L.Z) & 15u) == 0;
}

hipError_t launch_apply_shared(const LevelView& L, const double* x, const double* b, double alpha,
                               double beta, double* out, hipStream_t s) {
  const int per = L.n >= 1024 ? kMaxSteps : (L.n + 255) / 256 > 0 ? (L.n + 255) / 256 : 1;
  const int nwg = (L.n + per - 1) / per;
  if (L.p == 128)
    return launch_k(k_apply_shared<4, 8>, dim3(nwg), dim3(kTiledThreads), 0, s, L, x, b, alpha,
                    beta, out, per);
  if (L.p == 64)
    return launch_k(k_apply_shared<2, 4>, dim3(nwg), dim3(kTiledThreads), 0, s, L, x, b, alpha,
                    beta, out, per);
  return hipErrorInvalidValue;
}

}  // namespace pitmg
