// C ABI of the solver: setup / refactor, operator apply, Jacobi sweep,
// coarse solve, V-cycle (Alg. 1 recursed) and flexible GMRES, orchestrated
// on one HIP stream.  Declarations and argument contracts: include/pitmg.h.
#include "pitmg_internal.h"
#include "../../include/pitmg.h"

#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

using namespace pitmg;

// Scratch of pitmg_coarse_solve_noalloc: one array per GPU the library runs
// on, held until the process ends.  In host code `scratch` only names the
// array; its device address on each GPU comes from hipGetSymbolAddress with
// that GPU current, and only that address is ever passed to a kernel.
constexpr size_t kNoallocScratchDoubles = (size_t)4 << 20;      // 32 MiB
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch array, resolved once per GPU.
hipError_t noalloc_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

namespace {

struct LevelBuf {
  int n = 0;
  long long len = 0;
  const double* N = nullptr;
  const double* V = nullptr;
  const double* Z = nullptr;
  long long sN = 0, sV = 0, sZ = 0;
  double* N_own = nullptr;           // device copies when blocks came from the host
  double* V_own = nullptr;
  double* Z_own = nullptr;
  double* Gi = nullptr;              // [n][p][p]
  double* b = nullptr;               // right-hand side of this level (l >= 1)
  double* y0 = nullptr;              // smoothing ping-pong buffers
  double* y1 = nullptr;
  double* out = nullptr;             // result of this level's cycle (l >= 1)
  double* res = nullptr;             // explicit FP64 residual (finest level, FP32 smoother)
  bool vz_diag = false;              // shared V, Z~ diagonal: their diagonals in vzd
  double* vzd = nullptr;             // [Vd (p) | Zd (p)]
  float* vzd32 = nullptr;            // FP32 copy (FP32 levels)
  double* gin = nullptr;             // W_k = G_k^{-1} N_k (one-step sweeps), or NULL
  bool gn = false;                   // gin holds W for the current blocks
  double* b2 = nullptr;              // W / F cycles: second coarse right-hand side (l >= 1)
  double* e2 = nullptr;              //   and its correction
  // block Gauss-Seidel smoothers (levels above the coarsest)
  double* Phi = nullptr;             // [n][p][p] N_k^T S_k^{-1} V_k
  double* PhiT = nullptr;            // [n][p][p] its transpose
  double *gs_r = nullptr, *gs_t = nullptr, *gs_d = nullptr, *gs_h = nullptr;
  double *hat_u = nullptr, *hat_m = nullptr;   // chain results (zero elsewhere)
  bool fp32 = false;                 // this level smooths in FP32
  float* N32 = nullptr;
  float* V32 = nullptr;
  float* Z32 = nullptr;
  float* Gi32 = nullptr;
  int sweep_cfg = 0;                 // tuned sweep launch shape (LevelView)
  bool split = false;                // split sweep buffers allocated
  SplitBuffers sp;
};

struct ProfRec {
  int cls;
  hipEvent_t a, b;
};

constexpr int kNumClasses = 6;

}  // namespace

KernelEvents& pitmg::kernel_events() {
  static thread_local KernelEvents ev;
  return ev;
}

struct pitmg_handle {
  hipStream_t stream = nullptr;
  int p = 0, q = 0, n = 0, L = 0;
  pitmg_options opt{};
  int restart_cap = 0, maxit_cap = 0, coarse_cap = 0;
  int blocks_on_device = 0;
  std::vector<LevelBuf> lv;
  double* Vk = nullptr;              // FGMRES basis [restart+1][len]
  double* Zk = nullptr;              // preconditioned vectors [restart][len]
  double* w = nullptr;
  double* r = nullptr;
  double* partial = nullptr;         // [blocks][restart+2]
  double* upd = nullptr;             // [groups][2][len] for the grouped update, or NULL
  double* coef = nullptr;            // device scalars, 2*(restart+2)+8
  double* hbuf = nullptr;            // pinned host mirror of coef
  double* coarse_work = nullptr;     // coarse Krylov bases
  double* cst = nullptr;             // coarse GMRES state
  int* ist = nullptr;                // {steps done, stop}
  bool coarse_fast = false;          // block-parallel SGS available
  int coarse_k = 1;                  // coarse steps enqueued per solve
  int* its_pinned = nullptr;         // host copy of the last coarse step count
  double *cC = nullptr, *cA = nullptr, *cD = nullptr, *cY = nullptr, *cY2 = nullptr,
         *czero = nullptr;           // coarse work vectors
  double *Phi = nullptr, *Pf = nullptr, *Qb = nullptr, *pscr = nullptr;
  double* gs_scr = nullptr;          // W, X of the smoothers' Phi products (finest size)
  double *ul_in = nullptr, *ul_out = nullptr;   // lifted images in the unlifted solve
  int* coarse_its = nullptr;         // device log of coarse step counts
  int coarse_log_cap = 0;
  int coarse_calls = 0;
  int* fail = nullptr;
  int* vz_flags = nullptr;           // [20]: levels whose shared V, Z~ are diagonal
  double* zeros = nullptr;           // 64 zero bytes (LevelView::zeros)
  int fail_code = INT_MAX;
  long long dev_bytes = 0;
  std::string err;
  int prof = 0;                      // 0 off, 1 every launch, 2 the sweep only
  int prof_every = 1;                // time the sweeps of every n-th V-cycle
  long long vcycles = 0;             // finest-level V-cycles run
  std::vector<ProfRec> pending;
  std::vector<hipEvent_t> pool;
  int prof_launches[kNumClasses] = {0};
  double prof_ms[kNumClasses] = {0};
  // learned coarse correction
  pitmg_net* net = nullptr;          // borrowed
  bool fell_back = false;            // stall rule fired in this solve
  bool last_plain = false;           // last coarse correction was GMRES + SGS
  int net_calls = 0;
  double* pair_r = nullptr;          // caller-owned pair buffers
  double* pair_e = nullptr;
  int pair_cap = 0, pair_count = 0;
  int* last_its_slot = nullptr;      // device slot of the last coarse step count
  // captured V-cycle
  hipGraph_t g_graph = nullptr;
  hipGraphExec_t g_exec = nullptr;
  double* g_in = nullptr;            // fixed input / output of the captured cycle
  double* g_out = nullptr;
  int g_K = 0;                       // coarse steps enqueued in the capture
  int* g_its_slot = nullptr;
  long long graph_replays = 0;
  // previous iterate of the finest level's last sweep, when that sweep was
  // FP64 without a folded coarse correction (A~ z from the sweep identity)
  const double* top_prev = nullptr;
  // two-sweep launches: ticket counter, per-block epochs, timeout word
  unsigned long long* hand_ticket = nullptr;
  unsigned long long* hand_flag = nullptr;
  int* hand_timeout = nullptr;
  unsigned long long* sgs_flag = nullptr;   // phase flags of the fused coarse SGS
  unsigned long long hand_tickets = 0;   // tickets issued so far (host mirror)
  unsigned long long hand_epoch = 0;     // last epoch issued
  double wall_hz = 1e8;                  // the device's constant wall clock
  unsigned long long hand_spin = 200000000ull;   // wait bound (ticks): 2 s
};

namespace {

int set_err(pitmg_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

#define HIPCHK(h, call)                                                          \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      return set_err(h, PITMG_ERR_HIP, std::string(#call) + ": " +               \
                                           hipGetErrorString(e_));               \
  } while (0)

int dalloc(pitmg_handle* h, void** ptr, size_t bytes) {
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return set_err(h, e == hipErrorOutOfMemory ? PITMG_ERR_OOM : PITMG_ERR_HIP,
                   std::string("hipMalloc(") + std::to_string(bytes) + "): " +
                       hipGetErrorString(e));
  }
  h->dev_bytes += (long long)bytes;
  return PITMG_OK;
}

hipEvent_t take_event(pitmg_handle* h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Add one finished launch's time to its class (a failed query leaves the
// totals as they are) and return its events to the pool.
void account(pitmg_handle* h, const ProfRec& r) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
    h->prof_ms[r.cls] += ms;
    h->prof_launches[r.cls] += 1;
  }
  h->pool.push_back(r.a);
  h->pool.push_back(r.b);
}

// Events for one timed launch, or an error if the runtime cannot make them.
int take_pair(pitmg_handle* h, int cls, ProfRec& r) {
  r = ProfRec{cls, take_event(h), take_event(h)};
  if (r.a && r.b) return PITMG_OK;
  if (r.a) h->pool.push_back(r.a);
  if (r.b) h->pool.push_back(r.b);
  return set_err(h, PITMG_ERR_HIP, "profiling: hipEventCreate failed");
}

// Accumulate the elapsed time of the recorded launches that have already
// finished (in order), without waiting: called while the device is busy.
void drain_ready(pitmg_handle* h) {
  size_t done = 0;
  for (; done < h->pending.size(); ++done) {
    const ProfRec& r = h->pending[done];
    if (hipEventQuery(r.b) != hipSuccess) break;
    account(h, r);
  }
  h->pending.erase(h->pending.begin(), h->pending.begin() + done);
}

// Accumulate the elapsed time of every recorded launch (waits for them).
void drain(pitmg_handle* h) {
  for (auto& r : h->pending) {
    (void)hipEventSynchronize(r.b);     // a failed wait fails the query below
    account(h, r);
  }
  h->pending.clear();
}

template <class F>
int timed(pitmg_handle* h, int cls, F&& launch) {
  if (h->prof != 1) {            // level 2 times the sweep only
    HIPCHK(h, launch());
    return PITMG_OK;
  }
  ProfRec r;
  if (int rc = take_pair(h, cls, r)) return rc;
  HIPCHK(h, hipEventRecord(r.a, h->stream));
  HIPCHK(h, launch());
  HIPCHK(h, hipEventRecord(r.b, h->stream));
  h->pending.push_back(r);
  if (h->pending.size() > 4096) {
    drain_ready(h);
    if (h->pending.size() > 16384) drain(h);   // bound the records in flight
  }
  return PITMG_OK;
}

// Time a launcher whose kernels go through launch_k: the kernels' own
// dispatches record the start and end times.
template <class F>
int timed_kernel(pitmg_handle* h, int cls, F&& launch) {
  if (!h->prof || (h->prof_every > 1 && (h->vcycles - 1) % h->prof_every != 0)) {
    HIPCHK(h, launch());
    return PITMG_OK;
  }
  ProfRec r;
  if (int rc = take_pair(h, cls, r)) return rc;
  KernelEvents& ev = kernel_events();
  ev.start = r.a;
  ev.stop = r.b;
  ev.taken = 0;
  const hipError_t e = launch();
  const int taken = ev.taken;
  ev = KernelEvents{};
  if (e != hipSuccess)
    return set_err(h, PITMG_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  if (taken == 0) {
    h->pool.push_back(r.a);
    h->pool.push_back(r.b);
    return set_err(h, PITMG_ERR_HIP, "profiling: the launcher issued no timed kernel");
  }
  h->pending.push_back(r);
  if (h->pending.size() > 4096) {
    drain_ready(h);
    if (h->pending.size() > 16384) drain(h);   // bound the records in flight
  }
  return PITMG_OK;
}

LevelView view(const pitmg_handle* h, int l) {
  const LevelBuf& b = h->lv[l];
  LevelView v;
  v.n = b.n;
  v.p = h->p;
  v.q = h->q;
  v.N = b.N;
  v.sN = b.sN;
  v.V = b.V;
  v.sV = b.sV;
  v.Z = b.Z;
  v.sZ = b.sZ;
  v.Gi = b.Gi;
  if (b.fp32) {
    v.fp32 = 1;
    v.N32 = b.N32;
    v.V32 = b.V32;
    v.Z32 = b.Z32;
    v.Gi32 = b.Gi32;
  }
  v.sweep_cfg = b.sweep_cfg;
  if (b.split) v.split = &b.sp;
  // the smoother weight applies above the coarsest level; the coarsest
  // level's sweeps are the exact block solves of its SGS
  v.omega = l < h->L - 1 ? h->opt.omega : 1.0;
  v.mu_scale = h->opt.mu_scale;
  v.vz_diag = b.vz_diag ? 1 : 0;
  v.Vd = b.vzd;
  v.Zd = b.vzd ? b.vzd + h->p : nullptr;
  v.Vd32 = b.vzd32;
  v.Zd32 = b.vzd32 ? b.vzd32 + h->p : nullptr;
  v.GiN = b.gn ? b.gin : nullptr;
  v.zeros = h->zeros;
  // the coarsest level's block solves (inside the coarse SGS) take one step
  // per work-group: at 8 steps the one-step kernel has the shorter latency
  if (l == h->L - 1 && v.sweep_cfg == 0 && jacobi_tiled_supported(h->p, h->q))
    v.sweep_cfg = -1;
  return v;
}

int check_options(pitmg_handle* h, const pitmg_options& o) {
  if (o.nu_pre < 0 || o.nu_post < 0 || o.nu_pre > 64 || o.nu_post > 64)
    return set_err(h, PITMG_ERR_INVALID, "nu_pre/nu_post must be in [0, 64]");
  if (!(o.coarse_tol >= 0.0) || o.coarse_maxit < 1 || o.coarse_fixed_its < 0)
    return set_err(h, PITMG_ERR_INVALID, "bad coarse solver options");
  if (o.restart < 1 || o.maxit < 1)
    return set_err(h, PITMG_ERR_INVALID, "restart and maxit must be >= 1");
  if (o.transfer_variant != 0 && o.transfer_variant != 1)
    return set_err(h, PITMG_ERR_INVALID, "transfer_variant must be 0 or 1");
  if (o.smoother_fp32 < 0) return set_err(h, PITMG_ERR_INVALID, "smoother_fp32 must be >= 0");
  if (o.coarse_mode != 0 && o.coarse_mode != 1)
    return set_err(h, PITMG_ERR_INVALID, "coarse_mode must be 0 or 1");
  if (!(o.stall_ratio > 0.0) || o.stall_steps < 1)
    return set_err(h, PITMG_ERR_INVALID, "stall_ratio must be > 0 and stall_steps >= 1");
  if (o.apply_from_sweep != 0 && o.apply_from_sweep != 1)
    return set_err(h, PITMG_ERR_INVALID, "apply_from_sweep must be 0 or 1");
  if (o.pair_sweeps < 0 || o.pair_sweeps > 2)
    return set_err(h, PITMG_ERR_INVALID, "pair_sweeps must be 0, 1 or 2");
  if (o.vcycle_graph != 0 && o.vcycle_graph != 1)
    return set_err(h, PITMG_ERR_INVALID, "vcycle_graph must be 0 or 1");
  if (o.vcycle_graph && h && h->stream == nullptr)
    return set_err(h, PITMG_ERR_INVALID, "vcycle_graph needs a stream other than the null stream");
  if (!(o.omega > 0.0 && o.omega <= 1.0))
    return set_err(h, PITMG_ERR_INVALID, "omega must be in (0, 1]");
  if (!(o.mu_scale > 0.0) || !std::isfinite(o.mu_scale))
    return set_err(h, PITMG_ERR_INVALID, "mu_scale must be > 0");
  if (o.cycle < 0 || o.cycle > 2)
    return set_err(h, PITMG_ERR_INVALID, "cycle must be 0 (V), 1 (W) or 2 (F)");
  if (o.smoother < 0 || o.smoother > 3)
    return set_err(h, PITMG_ERR_INVALID, "smoother must be 0 (Jacobi), 1 (FGS), 2 (BGS) or 3 (SGS)");
  if (o.smoother != 0 && o.smoother_fp32 != 0)
    return set_err(h, PITMG_ERR_INVALID, "the Gauss-Seidel smoothers run in FP64 only");
  if (o.unlifted != 0 && o.unlifted != 1)
    return set_err(h, PITMG_ERR_INVALID, "unlifted must be 0 or 1");
  if (o.coarsen != 2 && o.coarsen != 4 && o.coarsen != 8 && o.coarsen != 16)
    return set_err(h, PITMG_ERR_INVALID, "coarsen must be 2, 4, 8 or 16");
  if (o.coarsen != 2 && o.transfer_variant != 0)
    return set_err(h, PITMG_ERR_INVALID, "transfer_variant 1 is defined for coarsen = 2 only");
  return PITMG_OK;
}

int check_problem(pitmg_handle* h, const pitmg_problem* pb, int coarsen) {
  if (!pb) return set_err(h, PITMG_ERR_INVALID, "problem is NULL");
  if (pb->p < 1 || pb->q < 1 || pb->n < 1 || pb->n_levels < 1)
    return set_err(h, PITMG_ERR_INVALID, "p, q, n and n_levels must be >= 1");
  if (pb->n_levels > 20) return set_err(h, PITMG_ERR_INVALID, "n_levels must be <= 20");
  if (pb->n >= (1 << 20)) return set_err(h, PITMG_ERR_UNSUPPORTED, "n must be < 2^20");
  long long div = 1;
  for (int l = 1; l < pb->n_levels && div <= pb->n; ++l) div *= coarsen;
  if (div > pb->n || pb->n % div != 0)
    return set_err(h, PITMG_ERR_INVALID, "n must be divisible by coarsen^(n_levels-1)");
  if (pb->p > 512 || pb->q > 512)
    return set_err(h, PITMG_ERR_UNSUPPORTED, "this build supports p, q <= 512");
  if (!pb->N || !pb->V || !pb->Z) return set_err(h, PITMG_ERR_INVALID, "block arrays are NULL");
  const long long pp = (long long)pb->p * pb->p, pq = (long long)pb->p * pb->q;
  if (pb->N_stride != pp && pb->N_stride != 0)
    return set_err(h, PITMG_ERR_INVALID, "N_stride must be p*p or 0");
  if (pb->V_stride != pp && pb->V_stride != 0)
    return set_err(h, PITMG_ERR_INVALID, "V_stride must be p*p or 0");
  if (pb->Z_stride != pq && pb->Z_stride != 0)
    return set_err(h, PITMG_ERR_INVALID, "Z_stride must be p*q or 0");
  if (pb->blocks_on_device != 0 && pb->blocks_on_device != 1)
    return set_err(h, PITMG_ERR_INVALID, "blocks_on_device must be 0 or 1");
  for (int l = 0; l < pb->n_levels; ++l)
    if (!pb->N[l] || !pb->V[l] || !pb->Z[l])
      return set_err(h, PITMG_ERR_INVALID, "NULL block pointer at level " + std::to_string(l));
  return PITMG_OK;
}

// Take the blocks (copy from host or borrow device pointers) and factor.
int load_and_factor(pitmg_handle* h, const pitmg_problem* pb) {
  const long long pp = (long long)h->p * h->p, pq = (long long)h->p * h->q;
  for (int l = 0; l < h->L; ++l) {
    LevelBuf& b = h->lv[l];
    b.sN = pb->N_stride;
    b.sV = pb->V_stride;
    b.sZ = pb->Z_stride;
    const long long cN = (b.sN ? b.n : 1) * pp, cV = (b.sV ? b.n : 1) * pp,
                    cZ = (b.sZ ? b.n : 1) * pq;
    if (pb->blocks_on_device) {
      b.N = pb->N[l];
      b.V = pb->V[l];
      b.Z = pb->Z[l];
    } else {
      HIPCHK(h, hipMemcpyAsync(b.N_own, pb->N[l], cN * 8, hipMemcpyHostToDevice, h->stream));
      HIPCHK(h, hipMemcpyAsync(b.V_own, pb->V[l], cV * 8, hipMemcpyHostToDevice, h->stream));
      HIPCHK(h, hipMemcpyAsync(b.Z_own, pb->Z[l], cZ * 8, hipMemcpyHostToDevice, h->stream));
      b.N = b.N_own;
      b.V = b.V_own;
      b.Z = b.Z_own;
    }
    if (h->opt.unlifted) {
      // the unlifted system's lifted hierarchy holds sqrt2 N_k and sqrt2 V_k
      // (pitmg_unlifted.hip): scaled into the handle's own copies
      const double r2 = std::sqrt(2.0);
      if (launch_scale(b.N_own, b.N, r2, cN, h->stream) != hipSuccess ||
          launch_scale(b.V_own, b.V, r2, cV, h->stream) != hipSuccess)
        return set_err(h, PITMG_ERR_HIP, "scaling of the state blocks failed");
      b.N = b.N_own;
      b.V = b.V_own;
    }
  }
  const int big = INT_MAX;
  HIPCHK(h, hipMemcpyAsync(h->fail, &big, sizeof(int), hipMemcpyHostToDevice, h->stream));
  // FP32 copies of the blocks of the FP32 levels
  for (int l = 0; l < h->L; ++l) {
    LevelBuf& b = h->lv[l];
    if (!b.fp32) continue;
    const long long cN = (b.sN ? b.n : 1) * pp, cV = (b.sV ? b.n : 1) * pp,
                    cZ = (b.sZ ? b.n : 1) * pq;
    int rc = timed(h, 0, [&] { return launch_to_f32(b.N32, b.N, cN, h->stream); });
    if (!rc) rc = timed(h, 0, [&] { return launch_to_f32(b.V32, b.V, cV, h->stream); });
    if (!rc) rc = timed(h, 0, [&] { return launch_to_f32(b.Z32, b.Z, cZ, h->stream); });
    if (rc) return rc;
  }
  // shared V and Z~ that are diagonal (theta = 1 with an identity mass matrix
  // and distributed control) are used through their diagonals: tested on
  // the device for every level at once; the flags come back with the
  // factorisation's status below
  const bool vz_cand = h->p == h->q && pb->V_stride == 0 && pb->Z_stride == 0;
  int vz_flags[20] = {0};
  for (int l = 0; l < h->L; ++l) h->lv[l].vz_diag = false;
  if (vz_cand) {
    VZDiagBatch B;
    B.nlev = h->L;
    B.p = h->p;
    for (int l = 0; l < h->L; ++l) {
      B.V[l] = h->lv[l].V;
      B.Z[l] = h->lv[l].Z;
      B.out[l] = h->lv[l].vzd;
    }
    int rc = timed(h, 0, [&] { return launch_vz_diag(B, h->vz_flags, h->stream); });
    for (int l = 0; l < h->L && !rc; ++l)
      if (h->lv[l].fp32)
        rc = timed(h, 0, [&] {
          return launch_to_f32(h->lv[l].vzd32, h->lv[l].vzd, 2LL * h->p, h->stream);
        });
    if (rc) return rc;
    HIPCHK(h, hipMemcpyAsync(vz_flags, h->vz_flags, h->L * sizeof(int), hipMemcpyDeviceToHost,
                             h->stream));
  }
  if (factor_mfma_supported(h->p, h->q)) {
    // the levels of each element type in one launch on the matrix cores; the
    // FP32 levels are the finest ones, so the FP64 levels are level0 .. L-1
    FactorBatchT<double> F;
    FactorBatchT<float> F32;
    F.p = F32.p = h->p;
    F.q = F32.q = h->q;
    F.sN = F32.sN = pb->N_stride;
    F.sZ = F32.sZ = pb->Z_stride;
    // the diagonal test above runs first on the stream: where it flags a
    // level, the factor forms S from N and the diagonal of Z~ alone
    F.zflag = F32.zflag = vz_cand ? h->vz_flags : nullptr;
    for (int l = 0; l < h->L; ++l) {
      const LevelBuf& b = h->lv[l];
      if (b.fp32) {
        F32.N[F32.nlev] = b.N32;
        F32.Z[F32.nlev] = b.Z32;
        F32.Gi[F32.nlev] = b.Gi32;
        F32.Zd[F32.nlev] = b.vzd32 ? b.vzd32 + h->p : nullptr;
        F32.start[F32.nlev + 1] = F32.start[F32.nlev] + b.n;
        F32.nlev++;
      } else {
        F.N[F.nlev] = b.N;
        F.Z[F.nlev] = b.Z;
        F.Gi[F.nlev] = b.Gi;
        F.Zd[F.nlev] = b.vzd + h->p;
        F.start[F.nlev + 1] = F.start[F.nlev] + b.n;
        F.nlev++;
      }
    }
    F32.level0 = 0;
    F.level0 = h->L - F.nlev;
    int rc = F32.nlev ? timed(h, 0, [&] { return launch_factor_mfma(F32, h->fail, h->stream); })
                      : 0;
    if (!rc) rc = timed(h, 0, [&] { return launch_factor_mfma(F, h->fail, h->stream); });
    if (rc) return rc;
  } else {
    for (int l = 0; l < h->L; ++l) {
      LevelBuf& b = h->lv[l];
      LevelView v = view(h, l);
      int rc = b.fp32 ? timed(h, 0, [&] { return launch_factor32(v, b.Gi32, l, h->fail, h->stream); })
                      : timed(h, 0, [&] { return launch_factor(v, b.Gi, l, h->fail, h->stream); });
      if (rc) return rc;
    }
  }
  int code = INT_MAX;
  HIPCHK(h, hipMemcpyAsync(&code, h->fail, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->fail_code = code;
  for (int l = 0; l < h->L; ++l) h->lv[l].vz_diag = vz_cand && vz_flags[l] == 1;
  if (code != INT_MAX)
    return set_err(h, PITMG_ERR_SINGULAR,
                   "S_k not positive definite at level " + std::to_string(code >> 20) +
                       ", step " + std::to_string((code & 0xFFFFF) + 1));
  // W_k = G_k^{-1} N_k where the one-step sweeps take it (diagonal V, Z~):
  // every such level in one launch
  {
    GiNBatch W;
    W.p = h->p;
    W.sN = h->lv[0].sN;
    for (int l = 0; l < h->L; ++l) {
      LevelBuf& b = h->lv[l];
      b.gn = false;
      if (!b.gin || !b.vz_diag) continue;
      W.Gi[W.nlev] = b.Gi;
      W.N[W.nlev] = b.N;
      W.out[W.nlev] = b.gin;
      W.start[W.nlev + 1] = W.start[W.nlev] + b.n;
      W.nlev++;
      b.gn = true;
    }
    if (W.nlev) {
      const int rc = timed(h, 0, [&] { return launch_gi_times_batch(W, h->stream); });
      if (rc) return rc;
    }
  }
  if (h->coarse_fast) {
    LevelView vc = view(h, h->L - 1);
    int rc = timed(h, 0, [&] {
      return launch_propagators(vc, h->pscr, h->Phi, h->Pf, h->Qb, h->stream);
    });
    if (rc) return rc;
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  if (h->opt.smoother != 0) {
    // Phi_k = N_k^T S_k^{-1} V_k and its transpose on every smoothed level
    for (int l = 0; l + 1 < h->L; ++l) {
      LevelBuf& b = h->lv[l];
      LevelView v = view(h, l);
      double* W = h->gs_scr;
      double* X = h->gs_scr + (size_t)b.n * h->p * h->p;
      int rc = timed(h, 0, [&] { return launch_phi_pair(v, W, X, b.Phi, b.PhiT, h->stream); });
      if (rc) return rc;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  return PITMG_OK;
}

// Device buffers of one coarse solve: the Krylov bases and GMRES state, the
// block-parallel SGS work vectors (cY, cY2 and czero zero outside the slots
// the sweeps write), and the slot that receives the step count.
struct CoarseWork {
  double* work;
  double* cst;
  int* ist;
  double *cC, *cA, *cD, *cY, *cY2, *czero;
  int* its;
};

// Coarsest level: GMRES + SGS.  Enqueue coarse_k steps with the
// block-parallel SGS (no host wait), then a finish kernel that continues
// block by block if the test was not met and forms x = Z y.
int coarse_solve_with(pitmg_handle* h, const double* b, double* out, const CoarseWork& cw) {
  const pitmg_options& o = h->opt;
  const int l = h->L - 1;
  LevelView v = view(h, l);
  const TypeMajor T(h->p, h->q, v.n);
  const long long len = T.len;
  const int cap = h->coarse_cap;
  const int nsteps = o.coarse_fixed_its > 0 ? o.coarse_fixed_its : o.coarse_maxit;
  int K = o.coarse_fixed_its > 0 ? o.coarse_fixed_its : std::min(h->coarse_k, nsteps);
  if (!h->coarse_fast) K = 0;
  double* Vb = cw.work;
  double* Zb = Vb + (size_t)(cap + 1) * len;
  double* W = Zb + (size_t)cap * len;
  const int var = o.transfer_variant;
  int rc = timed(h, 4, [&] {
    return launch_coarse_init(b, len, Vb, cw.cst, cw.ist, cap, h->stream);
  });
  if (rc) return rc;
  // the SGS application as one launch (phases with dataflow flags) where the
  // level sweeps with the one-step kernel
  const bool fused = h->sgs_flag && !v.fp32 && jacobi_chain_supported(v, h->stream);
  for (int j = 0; j < K; ++j) {
    double* vj = Vb + (size_t)j * len;
    double* zj = Zb + (size_t)j * len;
    if (fused) {
      if ((rc = timed(h, 4, [&] {
             const PairSync ps{h->hand_ticket, h->hand_tickets, h->sgs_flag, h->hand_epoch + 1,
                               h->hand_timeout, h->hand_spin};
             int groups = 0;
             const hipError_t e = launch_sgs_fused(v, vj, cw.czero, cw.cC, cw.cA, cw.cD, cw.cY,
                                                   cw.cY2, h->Pf, h->Qb, var, ps, &groups,
                                                   h->stream);
             if (e == hipSuccess) {
               h->hand_tickets += (unsigned long long)groups;
               h->hand_epoch += 2;
             }
             return e;
           })))
        return rc;
    }
    // forward sweep: c = D^{-1} v, a_u = P c_u, a = D^{-1}(v - L a)
    if (!fused && (rc = timed(h, 4, [&] {
           return launch_jacobi(v, vj, nullptr, nullptr, var, cw.cC, h->stream);
         })))
      return rc;
    if (!fused && (rc = timed(h, 4, [&] {
           return launch_gemv_tri(h->Pf, v.n, h->p, 0, cw.cC + T.u, cw.cY + T.u, h->stream);
         })))
      return rc;
    if (!fused && (rc = timed(h, 4, [&] {
           return launch_jacobi(v, vj, cw.cY, nullptr, var, cw.cA, h->stream);
         })))
      return rc;
    // backward sweep: y_mu = Q a_mu, z = a - D^{-1} L^T y
    if (!fused && (rc = timed(h, 4, [&] {
           return launch_gemv_tri(h->Qb, v.n, h->p, 1, cw.cA + T.m, cw.cY2 + T.m, h->stream);
         })))
      return rc;
    if (!fused && (rc = timed(h, 4, [&] {
           return launch_jacobi(v, cw.czero, cw.cY2, nullptr, var, cw.cD, h->stream);
         })))
      return rc;
    if (o.apply_from_sweep) {
      // z = a + d and w = A~ z from the two sweeps' identities (no pass over
      // the blocks), inside the Arnoldi step's own launch
      if ((rc = timed(h, 4, [&] {
             return launch_coarse_arnoldi_sgs(j, W, Vb, zj, cw.cA, cw.cD, h->p, h->q, v.n,
                                              cw.cst, cw.ist, cap, o.coarse_tol,
                                              o.coarse_fixed_its, nsteps, h->stream);
           })))
        return rc;
      continue;
    }
    if ((rc = timed(h, 4, [&] { return launch_add(zj, cw.cA, cw.cD, len, h->stream); })))
      return rc;
    if ((rc = timed(h, 4, [&] { return launch_apply(v, zj, nullptr, 1.0, 0.0, W, h->stream); })))
      return rc;
    if ((rc = timed(h, 4, [&] {
           return launch_coarse_arnoldi(j, W, Vb, len, cw.cst, cw.ist, cap, o.coarse_tol,
                                        o.coarse_fixed_its, nsteps, h->stream);
         })))
      return rc;
  }
  return timed(h, 4, [&] {
    return launch_coarse_finish(v, out, o.coarse_tol, o.coarse_fixed_its, nsteps, cw.work,
                                cw.cst, cw.ist, cap, cw.its, h->stream);
  });
}

// The coarse solve on the handle's own buffers, logging its step count.
int coarse_solve(pitmg_handle* h, const double* b, double* out) {
  int* its = h->coarse_its + (h->coarse_calls % h->coarse_log_cap);
  h->coarse_calls++;
  h->last_its_slot = its;
  const CoarseWork cw{h->coarse_work, h->cst, h->ist, h->cC, h->cA, h->cD,
                      h->cY, h->cY2, h->czero, its};
  return coarse_solve_with(h, b, out, cw);
}

// Coarsest level inside a V-cycle: the attached network while coarse_mode
// is 1 and the stall rule has not fired, else GMRES + SGS (recording the
// pair when armed).
int coarse_dispatch(pitmg_handle* h, const double* b, double* out) {
  if (h->opt.coarse_mode == 1 && !h->fell_back) {
    if (!h->net) return set_err(h, PITMG_ERR_INVALID, "coarse_mode 1 needs an attached network");
    h->last_plain = false;
    h->net_calls++;
    return timed(h, 4, [&] {
      return net_coarse_correction(h->net, b, out, h->p, h->q, h->stream);
    });
  }
  h->last_plain = true;
  int rc = coarse_solve(h, b, out);
  if (rc) return rc;
  if (h->pair_count < h->pair_cap) {
    const long long len = h->lv[h->L - 1].len;
    HIPCHK(h, hipMemcpyAsync(h->pair_r + (size_t)h->pair_count * len, b, len * 8,
                             hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->pair_e + (size_t)h->pair_count * len, out, len * 8,
                             hipMemcpyDeviceToDevice, h->stream));
    h->pair_count++;
  }
  return PITMG_OK;
}

int vcycle_level(pitmg_handle* h, int l, const double* b, double* out, int cyc);

// A two-sweep launch whose neighbour wait ran out leaves a nonzero word in
// the handle: report it (and clear it) as the error of the call it ends.
int handoff_check(pitmg_handle* h) {
  int to = 0;
  HIPCHK(h, hipMemcpyAsync(&to, h->hand_timeout, sizeof(int), hipMemcpyDeviceToHost,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (!to) return PITMG_OK;
  HIPCHK(h, hipMemsetAsync(h->hand_timeout, 0, sizeof(int), h->stream));
  return set_err(h, PITMG_ERR_HIP, to & 2 ? "two-sweep launch: ticket out of range"
                                          : "two-sweep launch: a hand-off wait timed out");
}

void drop_graph(pitmg_handle* h) {
  if (h->g_exec) (void)hipGraphExecDestroy(h->g_exec);
  if (h->g_graph) (void)hipGraphDestroy(h->g_graph);
  h->g_exec = nullptr;
  h->g_graph = nullptr;
  h->g_K = 0;
}

// Capture MG_0(g_in) -> g_out on the handle's stream into a HIP graph.
int capture_vcycle(pitmg_handle* h) {
  drop_graph(h);
  HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
  const int K = h->opt.coarse_fixed_its > 0 ? h->opt.coarse_fixed_its : h->coarse_k;
  const int rc = vcycle_level(h, 0, h->g_in, h->g_out, h->opt.cycle);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess)
    return set_err(h, PITMG_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  h->g_graph = g;
  HIPCHK(h, hipGraphInstantiate(&h->g_exec, g, nullptr, nullptr, 0));
  h->g_K = K;
  h->g_its_slot = h->last_its_slot;
  return PITMG_OK;
}

// MG_0(r) -> e, eagerly or by replaying the captured cycle.
int vcycle_top(pitmg_handle* h, const double* r, double* e) {
  const pitmg_options& o = h->opt;
  h->vcycles++;
  const bool graph = o.vcycle_graph && h->stream != nullptr && !h->prof && o.nu_post > 0 &&
                     o.coarse_mode == 0 && h->pair_count >= h->pair_cap;
  if (!graph) return vcycle_level(h, 0, r, e, h->opt.cycle);
  const long long len = h->lv[0].len;
  int rc;
  if (!h->g_in) {
    if ((rc = dalloc(h, (void**)&h->g_in, len * 8))) return rc;
    if ((rc = dalloc(h, (void**)&h->g_out, len * 8))) return rc;
  }
  const int need = !h->coarse_fast ? 0
                   : o.coarse_fixed_its > 0 ? o.coarse_fixed_its : h->coarse_k;
  if (!h->g_exec || need > h->g_K)
    if ((rc = capture_vcycle(h))) return rc;
  HIPCHK(h, hipMemcpyAsync(h->g_in, r, len * 8, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(h, hipGraphLaunch(h->g_exec, h->stream));
  HIPCHK(h, hipMemcpyAsync(e, h->g_out, len * 8, hipMemcpyDeviceToDevice, h->stream));
  h->last_plain = true;
  h->last_its_slot = h->g_its_slot;
  h->graph_replays++;
  return PITMG_OK;
}

// MG_l(b) -> out (Alg. 1 recursed; zero initial guess on every level).
// Two consecutive sweeps of a level in one launch (y1 then y2), taking the
// next tickets and epoch of the handle's hand-off state.
hipError_t sweep_pair(pitmg_handle* h, const LevelView& v, const double* b, const double* yo,
                      const double* ec, double* y1, double* y2, double* rc_out, double rbeta,
                      double ra) {
  const PairSync ps{h->hand_ticket, h->hand_tickets, h->hand_flag, h->hand_epoch + 1,
                    h->hand_timeout, h->hand_spin};
  int groups = 0;
  const hipError_t e = launch_jacobi_pair(v, b, yo, ec, h->opt.transfer_variant, y1, y2,
                                          rc_out, rbeta, ra, ps, &groups, h->stream);
  if (e == hipSuccess) {
    h->hand_tickets += (unsigned long long)groups;
    h->hand_epoch += 1;
  }
  return e;
}

// MG_l0(b) -> out with the pre-smoothing of levels l0 .. L-2 in one launch
// and their post-smoothing in another (pair_sweeps = 2): the same sweeps,
// fused restrictions and interpolations, into the same buffers, as the level
// by level recursion of vcycle_level with two sweeps per launch.
// chained_cycle says whether the handle's cycle has that form from level l0
// on (an FP32 finest level, whose residual is an explicit FP64 product, is
// swept on its own and the levels below it chain).
int coarse_correction(pitmg_handle* h, int l, int cyc);

bool chain_form(const pitmg_options& o, int n_levels, int l0) {
  const int nc = n_levels - 1 - l0;            // levels that smooth from l0 on
  return o.pair_sweeps == 2 && o.smoother == 0 && o.cycle == 0 && o.coarsen == 2 &&
         o.nu_pre == 2 && o.nu_post == 2 && nc >= 2 && nc <= jacobi_chain_max();
}

bool chained_cycle(pitmg_handle* h, int l0) {
  if (!chain_form(h->opt, h->L, l0)) return false;
  const int fp = view(h, l0).fp32;             // one precision along the chain
  for (int l = l0; l < h->L - 1; ++l) {
    const LevelView v = view(h, l);
    if (h->lv[l].res || v.fp32 != fp || !jacobi_chain_supported(v, h->stream)) return false;
  }
  return true;
}

int vcycle_chained(pitmg_handle* h, int l0, const double* b, double* out) {
  const int ns = h->L - 1 - l0;                // levels in the chain
  ChainSweep dn[16], up[16];
  int off = 0;
  for (int c = 0; c < ns; ++c) {
    const int l = l0 + c;
    const LevelView v = view(h, l);
    LevelBuf& B = h->lv[l];
    LevelBuf& C = h->lv[l + 1];
    const double w = v.omega;
    const double rbeta = w != 1.0 ? (1.0 - w) * (1.0 - w) : 0.0;
    const double ra = w != 1.0 ? w : 1.0;
    const double* bl = c == 0 ? b : B.b;
    dn[c] = ChainSweep{v, bl, nullptr, nullptr, B.y0, B.y1, C.b, rbeta, ra, off};
    up[ns - 1 - c] = ChainSweep{v, bl, B.y1, C.out, B.y0, c == 0 ? out : B.out, nullptr,
                                0.0, 1.0, off};
    off += v.n;
  }
  auto chain = [&](const ChainSweep* sw, int dir) {
    const PairSync ps{h->hand_ticket, h->hand_tickets, h->hand_flag, h->hand_epoch + 1,
                      h->hand_timeout, h->hand_spin};
    int groups = 0;
    const hipError_t e = launch_jacobi_chain(sw, ns, dir, h->opt.transfer_variant, ps, &groups,
                                             h->stream);
    if (e == hipSuccess) {
      h->hand_tickets += (unsigned long long)groups;
      h->hand_epoch += 2;
    }
    return e;
  };
  int rc = timed_kernel(h, 1, [&] { return chain(dn, 0); });
  if (rc) return rc;
  if ((rc = coarse_correction(h, h->L - 2, 0))) return rc;
  rc = timed_kernel(h, 1, [&] { return chain(up, 1); });
  if (rc) return rc;
  // A~ z from the last sweep's identity needs an undamped FP64 sweep
  const LevelView v0 = view(h, 0);
  if (l0 == 0 && v0.omega == 1.0 && !v0.fp32) h->top_prev = h->lv[0].y0;
  return PITMG_OK;
}

// The transfers between level l and l + 1 for the handle's step ratio:
// R r into C.b-shaped bc, and y += P e.
int restrict_level(pitmg_handle* h, int l, const double* r, double* bc) {
  const LevelView v = view(h, l);
  const int c = h->opt.coarsen;
  if (c == 2)
    return timed(h, 3, [&] {
      return launch_restrict(h->p, h->q, v.n, r, h->opt.transfer_variant, v.mu_scale, bc,
                             h->stream);
    });
  const double fac = std::pow(v.mu_scale, std::log2((double)c));
  return timed(h, 3, [&] {
    return launch_restrict_c(h->p, h->q, v.n, c, r, fac, bc, h->stream);
  });
}

int interp_level(pitmg_handle* h, int l, const double* e, double* y) {
  const LevelView v = view(h, l);
  const int c = h->opt.coarsen;
  if (c == 2)
    return timed(h, 3, [&] {
      return launch_interp_add(h->p, h->q, v.n, e, h->opt.transfer_variant, v.mu_scale, y,
                               h->stream);
    });
  const double fac = std::pow(v.mu_scale, std::log2((double)c));
  return timed(h, 3, [&] {
    return launch_interp_add_c(h->p, h->q, v.n, c, e, fac, y, h->stream);
  });
}

// d = (D + L)^{-1} r (forward) or (D + L^T)^{-1} r (backward) on level l:
// the block solves of D^{-1} r, the chain of the coupled slot through Phi_k,
// then the block solves with the chain as the coupling iterate
// (pitmg_gs.hip).
int gs_solve(pitmg_handle* h, int l, bool forward, const double* r, double* d) {
  LevelBuf& B = h->lv[l];
  LevelView v1 = view(h, l);
  v1.omega = 1.0;
  const int var = h->opt.transfer_variant;
  double* hat = forward ? B.hat_u : B.hat_m;
  int rc = timed_kernel(h, 1, [&] {
    return launch_jacobi(v1, r, nullptr, nullptr, var, B.gs_t, h->stream);
  });
  if (!rc)
    rc = timed_kernel(h, 1, [&] {
      return launch_gs_chain(h->p, h->q, B.n, forward ? B.PhiT : B.Phi, B.gs_t, hat, !forward,
                             h->stream);
    });
  if (!rc)
    rc = timed_kernel(h, 1, [&] {
      return launch_jacobi(v1, r, hat, nullptr, var, d, h->stream);
    });
  return rc;
}

// One Gauss-Seidel smoothing sweep on level l (options.smoother 1-3):
// y_out = y_in + w M^{-1}(b - A~ y_in), M = D + L (FGS), D + L^T (BGS), or
// the symmetric sweep (forward, then backward from the forward result,
// equal to M = (D + L) D^{-1} (D + L^T)); y_in NULL = 0; y_out != y_in.
int gs_sweep(pitmg_handle* h, int l, const double* b, const double* y_in, double* y_out) {
  LevelBuf& B = h->lv[l];
  LevelView v = view(h, l);
  const double w = v.omega;
  const long long len = B.len;
  const int kind = h->opt.smoother;
  int rc = 0;
  const double* r = b;
  if (y_in) {
    rc = timed(h, 2, [&] { return launch_apply(v, y_in, b, -1.0, 1.0, B.gs_r, h->stream); });
    if (rc) return rc;
    r = B.gs_r;
  }
  // ys = y_in + M^{-1} r into gs_h (the symmetric sweep's second half from
  // the first half's result), or the correction alone into gs_d
  double* corr = B.gs_d;
  if (kind == 3) {
    if ((rc = gs_solve(h, l, true, r, B.gs_d))) return rc;
    if (y_in) {
      HIPCHK(h, hipMemcpyAsync(B.gs_h, y_in, len * 8, hipMemcpyDeviceToDevice, h->stream));
      rc = timed(h, 3, [&] { return launch_axpby(B.gs_h, B.gs_d, 1.0, 1.0, len, h->stream); });
    } else {
      HIPCHK(h, hipMemcpyAsync(B.gs_h, B.gs_d, len * 8, hipMemcpyDeviceToDevice, h->stream));
    }
    if (!rc) rc = timed(h, 2, [&] {
      return launch_apply(v, B.gs_h, b, -1.0, 1.0, B.gs_r, h->stream);
    });
    if (!rc) rc = gs_solve(h, l, false, B.gs_r, B.gs_d);
    if (!rc) rc = timed(h, 3, [&] {
      return launch_axpby(B.gs_h, B.gs_d, 1.0, 1.0, len, h->stream);
    });
    if (rc) return rc;
    // y_out = (1 - w) y_in + w ys
    if (!y_in) return timed(h, 3, [&] { return launch_scale(y_out, B.gs_h, w, len, h->stream); });
    HIPCHK(h, hipMemcpyAsync(y_out, y_in, len * 8, hipMemcpyDeviceToDevice, h->stream));
    return timed(h, 3, [&] { return launch_axpby(y_out, B.gs_h, w, 1.0 - w, len, h->stream); });
  }
  if ((rc = gs_solve(h, l, kind == 1, r, corr))) return rc;
  if (!y_in) return timed(h, 3, [&] { return launch_scale(y_out, corr, w, len, h->stream); });
  HIPCHK(h, hipMemcpyAsync(y_out, y_in, len * 8, hipMemcpyDeviceToDevice, h->stream));
  return timed(h, 3, [&] { return launch_axpby(y_out, corr, w, 1.0, len, h->stream); });
}

// The coarse correction of level l into C.out: one cycle of level l + 1
// (V), or two, the second from the residual the first leaves (W: both W;
// F: F, then V).
int coarse_correction(pitmg_handle* h, int l, int cyc) {
  LevelBuf& C = h->lv[l + 1];
  int rc = vcycle_level(h, l + 1, C.b, C.out, cyc);
  if (rc || cyc == 0) return rc;
  LevelView vc = view(h, l + 1);
  vc.fp32 = 0;
  rc = timed(h, 2, [&] { return launch_apply(vc, C.out, C.b, -1.0, 1.0, C.b2, h->stream); });
  if (!rc) rc = vcycle_level(h, l + 1, C.b2, C.e2, cyc == 1 ? 1 : 0);
  if (!rc)
    rc = timed(h, 3, [&] { return launch_axpby(C.out, C.e2, 1.0, 1.0, C.len, h->stream); });
  return rc;
}

// MG_l(b) with Gauss-Seidel smoothing: explicit residual, restriction,
// coarse correction, interpolation, explicit sweeps.
int vcycle_level_gs(pitmg_handle* h, int l, const double* b, double* out, int cyc) {
  const pitmg_options& o = h->opt;
  const int var = o.transfer_variant;
  LevelView v = view(h, l);
  LevelBuf& B = h->lv[l];
  LevelBuf& C = h->lv[l + 1];
  double* bufs[2] = {B.y0, B.y1};
  double* y = nullptr;
  int rc = 0;
  for (int s = 0; s < o.nu_pre; ++s) {
    double* dst = bufs[s & 1];
    if ((rc = gs_sweep(h, l, b, y, dst))) return rc;
    y = dst;
  }
  if (!y) {
    rc = restrict_level(h, l, b, C.b);
  } else {
    double* res = y == bufs[0] ? bufs[1] : bufs[0];
    rc = timed(h, 2, [&] { return launch_apply(v, y, b, -1.0, 1.0, res, h->stream); });
    if (!rc) rc = restrict_level(h, l, res, C.b);
  }
  if (rc) return rc;
  if ((rc = coarse_correction(h, l, cyc))) return rc;
  if (!y) {
    y = bufs[0];
    if ((rc = timed(h, 3, [&] { return launch_fill(y, 0.0, B.len, h->stream); }))) return rc;
  }
  if ((rc = interp_level(h, l, C.out, y))) return rc;
  for (int s = 0; s < o.nu_post; ++s) {
    double* dst = s == o.nu_post - 1 ? out : (y == bufs[0] ? bufs[1] : bufs[0]);
    if ((rc = gs_sweep(h, l, b, y, dst))) return rc;
    y = dst;
  }
  if (o.nu_post == 0)
    HIPCHK(h, hipMemcpyAsync(out, y, B.len * 8, hipMemcpyDeviceToDevice, h->stream));
  return PITMG_OK;
}

int vcycle_level(pitmg_handle* h, int l, const double* b, double* out, int cyc) {
  const pitmg_options& o = h->opt;
  const int var = o.transfer_variant;
  LevelView v = view(h, l);
  if (l == 0) h->top_prev = nullptr;
  if (l == h->L - 1) return coarse_dispatch(h, b, out);
  if (o.smoother != 0) return vcycle_level_gs(h, l, b, out, cyc);
  if (cyc == 0 && chained_cycle(h, l)) return vcycle_chained(h, l, b, out);
  LevelBuf& B = h->lv[l];
  LevelBuf& C = h->lv[l + 1];
  double* bufs[2] = {B.y0, B.y1};
  double* ycur = nullptr;
  int rc;
  const bool pairs = o.pair_sweeps && jacobi_pair_supported(v, h->stream);
  // Residual after the pre-smoothing sweeps from y = 0.  A weighted sweep
  // y' = (1-w) y + w D^{-1}(b - (L+L^T) y) leaves r' = (1-w) r + (L+L^T)(y - y'),
  // so one sweep leaves (1-w) b + (L+L^T)(0 - y1) and two leave
  // (1-w)^2 b + (L+L^T)(w y1 - y2); undamped sweeps (w = 1) leave
  // (L+L^T)(y_prev - y) after any number.  Those forms are restricted
  // inside the last sweep as R (rbeta b + (L+L^T)(ra y_prev - y)); more
  // weighted sweeps, and an FP32 finest level, form the residual explicitly.
  const double w = v.omega;
  // step ratios other than 2 use the stand-alone transfers: explicit
  // residual and restriction, interpolation added before the post-sweeps
  const bool c2 = o.coarsen == 2;
  const bool explicit_res = B.res != nullptr || (w != 1.0 && o.nu_pre > 2) || !c2;
  double rbeta = 0.0, ra = 1.0;
  if (w != 1.0 && o.nu_pre == 1) rbeta = 1.0 - w;
  if (w != 1.0 && o.nu_pre == 2) {
    rbeta = (1.0 - w) * (1.0 - w);
    ra = w;
  }
  for (int s = 0; s < o.nu_pre;) {
    const int last = pairs && s + 1 < o.nu_pre ? s + 1 : s;
    double* rc_out = (last == o.nu_pre - 1 && !explicit_res) ? C.b : nullptr;
    const double* yo = ycur;
    if (last > s) {
      double* d1 = bufs[s & 1];
      double* d2 = bufs[last & 1];
      rc = timed_kernel(h, 1, [&] {
        return sweep_pair(h, v, b, yo, nullptr, d1, d2, rc_out, rbeta, ra);
      });
      if (rc) return rc;
      ycur = d2;
      s += 2;
      continue;
    }
    double* dst = bufs[s & 1];
    rc = timed_kernel(h, 1, [&] {
      return launch_jacobi(v, b, yo, nullptr, var, dst, h->stream, rc_out, rbeta, ra);
    });
    if (rc) return rc;
    ycur = dst;
    ++s;
  }
  if (ycur == nullptr) {
    rc = restrict_level(h, l, b, C.b);
  } else if (explicit_res) {
    // r = b - A~ y in FP64 (into the spare smoothing buffer unless the FP32
    // finest level keeps its own), then restricted
    double* res = B.res ? B.res : (ycur == bufs[0] ? bufs[1] : bufs[0]);
    LevelView v64 = v;
    v64.fp32 = 0;
    rc = timed(h, 2, [&] { return launch_apply(v64, ycur, b, -1.0, 1.0, res, h->stream); });
    if (!rc) rc = restrict_level(h, l, res, C.b);
  }
  if (rc) return rc;
  rc = coarse_correction(h, l, cyc);
  if (rc) return rc;
  if (o.nu_post == 0) {
    if (ycur)
      HIPCHK(h, hipMemcpyAsync(out, ycur, B.len * 8, hipMemcpyDeviceToDevice, h->stream));
    else
      HIPCHK(h, hipMemsetAsync(out, 0, B.len * 8, h->stream));
    return interp_level(h, l, C.out, out);
  }
  if (!c2) {
    // y + P e into the iterate the post-sweeps start from
    if (!ycur) {
      ycur = bufs[0];
      if ((rc = timed(h, 3, [&] { return launch_fill(ycur, 0.0, B.len, h->stream); })))
        return rc;
    }
    if ((rc = interp_level(h, l, C.out, ycur))) return rc;
  }
  // A~ z from the last sweep's identity needs an undamped FP64 sweep
  const bool identity = l == 0 && w == 1.0 && !v.fp32;
  for (int s = 0; s < o.nu_post;) {
    double* dst = (s == o.nu_post - 1) ? out : (ycur == bufs[0] ? bufs[1] : bufs[0]);
    const double* yo = ycur;
    const double* ec = s == 0 && c2 ? C.out : nullptr;
    if (pairs && s + 1 < o.nu_post) {
      // second sweep: into out if it is the last, else the other buffer
      double* d2 = (s + 1 == o.nu_post - 1) ? out : (dst == bufs[0] ? bufs[1] : bufs[0]);
      rc = timed_kernel(h, 1, [&] {
        return sweep_pair(h, v, b, yo, ec, dst, d2, nullptr, 0.0, 1.0);
      });
      if (rc) return rc;
      if (identity && s + 1 == o.nu_post - 1) h->top_prev = dst;
      ycur = d2;
      s += 2;
      continue;
    }
    rc = timed_kernel(h, 1, [&] { return launch_jacobi(v, b, yo, ec, var, dst, h->stream); });
    if (rc) return rc;
    if (identity && s == o.nu_post - 1 && ec == nullptr && yo != nullptr) h->top_prev = yo;
    ycur = dst;
    ++s;
  }
  return PITMG_OK;
}

// dots of the first nb basis vectors with x1 (and x2) plus the self dots,
// reduced into device coef[0 ..) in the value order of launch_dots
int dots(pitmg_handle* h, const double* basis, int nb, const double* x1, const double* x2,
         long long len) {
  const int ns = krylov_slices(len);
  const int nval = x2 ? 2 * nb + 3 : nb + 1;
  int rc = timed(h, 5, [&] { return launch_dots(basis, nb, x1, x2, len, h->partial, h->stream); });
  if (rc) return rc;
  return timed(h, 5, [&] {
    return launch_reduce_partials(h->partial, ns, nval, h->coef, h->stream);
  });
}

// Apply the stored rotations 0..j-1 to column j of H (leading dim m), make
// rotation j and update g.  Returns |g[j+1]|.
double givens_column(std::vector<double>& H, int m, int j, std::vector<double>& cs,
                     std::vector<double>& sn, std::vector<double>& g) {
  for (int i = 0; i < j; ++i) {
    const double a0 = H[(size_t)i * m + j], a1 = H[(size_t)(i + 1) * m + j];
    H[(size_t)i * m + j] = cs[i] * a0 + sn[i] * a1;
    H[(size_t)(i + 1) * m + j] = -sn[i] * a0 + cs[i] * a1;
  }
  const double a0 = H[(size_t)j * m + j], a1 = H[(size_t)(j + 1) * m + j];
  const double rr = std::hypot(a0, a1);
  cs[j] = rr > 0.0 ? a0 / rr : 1.0;
  sn[j] = rr > 0.0 ? a1 / rr : 0.0;
  H[(size_t)j * m + j] = rr;
  H[(size_t)(j + 1) * m + j] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  return std::fabs(g[j + 1]);
}

// One FGMRES solve (Saad 1993) as a resumable sequence of phases.  The
// Arnoldi basis is built by classical Gram-Schmidt with delayed
// re-orthogonalisation: step j takes the dots of the finished basis
// q_0..q_{j-1} with both the lagged vector v_j (the preconditioner input)
// and w = A M(v_j) in one pass, then in one update pass re-orthogonalises
// v_j into q_j and orthogonalises w against q_0..q_j.  The correction of v_j
// is folded into Hessenberg column j-1, so A Z = Q H holds with the
// preconditioned vectors actually used.
//
// advance() enqueues device work up to the next point where the host needs
// device results (a coefficient copy into hbuf) and returns kWait; the
// caller synchronises the handle's stream and calls advance() again.  A
// single solve alternates the two; a batch interleaves the phases of many
// solves, each on its own stream, so their kernels overlap on the device
// while the host waits once per round for all of them.
struct FgmresRun {
  enum Phase { kStart, kAfterBnorm, kCycle, kAfterResid, kStepA, kStepB, kStepEnd,
               kCycleEnd, kFinal, kAfterFinal, kFinish, kDone };
  static constexpr int kWait = 1;
  static constexpr int kFinished = 0;

  pitmg_handle* h = nullptr;
  const double* rhs = nullptr;
  double* x = nullptr;
  double tol = 0.0;
  int use_x0 = 0;
  Phase ph = kStart;
  long long len = 0;
  int m = 0, maxit = 0, net0 = 0, ns = 0;
  LevelView v0{};
  std::chrono::steady_clock::time_point t0;
  std::vector<double> H, cs, sn, g, y, hv, sv;
  double bnorm = 0.0, beta = 0.0, est = 1.0, est_prev = 1.0, rho_prev = 0.0, rho = 0.0;
  double ww = 0.0, alpha = 1.0, cq = 0.0, rn = 0.0;
  bool converged = false, first = true, stop = false, plain = false, zero_rhs = false;
  int total = 0, j = 0, k = 0, stalled = 0, fallback_at = -1;
  int coarse_calls = 0;
  long long coarse_its = 0;
  int status = PITMG_OK;
  pitmg_stats S{};

  bool unl = false;                 // the system without virtual variables

  double* Vp(int i) const { return h->Vk + (size_t)i * len; }
  double* Zp(int i) const { return h->Zk + (size_t)i * len; }

  // out = bb * b + a * (system) xin  (b may be NULL when bb = 0)
  int apply_sys(const double* xin, const double* b, double a, double bb, double* out) {
    if (unl)
      return timed(h, 2, [&] {
        return launch_unlifted_apply(v0, 1.0 / std::sqrt(2.0), xin, b, a, bb, out, h->stream);
      });
    return timed(h, 2, [&] { return launch_apply(v0, xin, b, a, bb, out, h->stream); });
  }

  // out = the preconditioner applied to in: one cycle, carried to the
  // unlifted system by the lift / project maps
  int precondition(const double* in, double* out) {
    if (!unl) return vcycle_top(h, in, out);
    int rc = timed(h, 3, [&] { return launch_lift(h->p, h->q, h->n, in, h->ul_in, h->stream); });
    if (!rc) rc = vcycle_top(h, h->ul_in, h->ul_out);
    if (!rc)
      rc = timed(h, 3, [&] {
        return launch_project(h->p, h->q, h->n, h->ul_out, out, h->stream);
      });
    return rc;
  }

  int start(pitmg_handle* hh, const double* b, double* xx, double tl, int x0) {
    h = hh;
    if (!h || !b || !xx) return PITMG_ERR_INVALID;
    if (!(tl >= 0.0)) return set_err(h, PITMG_ERR_INVALID, "tol must be >= 0");
    if (h->opt.coarse_mode == 1 && !h->net)
      return set_err(h, PITMG_ERR_INVALID, "coarse_mode 1 needs an attached network");
    rhs = b;
    x = xx;
    tol = tl;
    use_x0 = x0;
    t0 = std::chrono::steady_clock::now();
    len = unl ? (2LL * h->p + h->q) * h->n : h->lv[0].len;
    m = h->opt.restart;
    maxit = h->opt.maxit;
    net0 = h->net_calls;
    ns = krylov_slices(len);
    v0 = view(h, 0);
    h->fell_back = false;
    ph = kStart;
    return PITMG_OK;
  }

  // enqueue the copy of count coefficients into hbuf, then wait
  int wait_coef(int count) {
    HIPCHK(h, hipMemcpyAsync(h->hbuf, h->coef, count * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
    return kWait;
  }

  void begin_cycle() {
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    k = 0;
    j = 0;
    stop = false;
    rho_prev = 0.0;
  }

  int advance() {
    int rc;
    for (;;) {
      switch (ph) {
        case kStart:
          if ((rc = dots(h, nullptr, 0, rhs, nullptr, len))) return rc;
          ph = kAfterBnorm;
          return wait_coef(1);
        case kAfterBnorm:
          bnorm = std::sqrt(h->hbuf[0]);
          if (!std::isfinite(bnorm))
            return set_err(h, PITMG_ERR_NONFINITE, "right-hand side not finite");
          if (bnorm == 0.0) {
            HIPCHK(h, hipMemsetAsync(x, 0, len * 8, h->stream));
            zero_rhs = converged = true;
            ph = kFinish;
            break;
          }
          if (!use_x0) HIPCHK(h, hipMemsetAsync(x, 0, len * 8, h->stream));
          H.assign((size_t)(m + 1) * m, 0.0);
          cs.assign(m, 0.0);
          sn.assign(m, 0.0);
          g.assign(m + 1, 0.0);
          y.assign(m, 0.0);
          hv.assign(m + 1, 0.0);
          sv.assign(m + 1, 0.0);
          first = !use_x0;
          ph = kCycle;
          break;
        case kCycle:
          if (first) {
            beta = bnorm;
            if ((rc = timed(h, 5, [&] {
                   return launch_scale(Vp(0), rhs, 1.0 / beta, len, h->stream);
                 })))
              return rc;
            first = false;
            begin_cycle();
            ph = kStepA;
            break;
          }
          if ((rc = apply_sys(x, rhs, -1.0, 1.0, h->r))) return rc;
          if ((rc = dots(h, nullptr, 0, h->r, nullptr, len))) return rc;
          ph = kAfterResid;
          return wait_coef(1);
        case kAfterResid:
          beta = std::sqrt(h->hbuf[0]);
          if (!std::isfinite(beta)) return set_err(h, PITMG_ERR_NONFINITE, "residual not finite");
          est = beta / bnorm;
          if (beta <= tol * bnorm) {
            converged = true;
            ph = kFinal;
            break;
          }
          if (total >= maxit) {
            ph = kFinal;
            break;
          }
          if ((rc = timed(h, 5, [&] {
                 return launch_scale(Vp(0), h->r, 1.0 / beta, len, h->stream);
               })))
            return rc;
          begin_cycle();
          ph = kStepA;
          break;
        case kStepA:
          if ((rc = precondition(Vp(j), Zp(j)))) return rc;
          if (unl) {
            if ((rc = apply_sys(Zp(j), nullptr, 1.0, 0.0, h->w))) return rc;
          } else if (h->opt.apply_from_sweep && h->top_prev) {
            if ((rc = timed(h, 2, [&] {
                   return launch_apply_identity(h->p, h->q, h->n, Vp(j), h->top_prev, Zp(j),
                                                h->w, h->stream);
                 })))
              return rc;
          } else if ((rc = timed(h, 2, [&] {
                        return launch_apply(v0, Zp(j), nullptr, 1.0, 0.0, h->w, h->stream);
                      }))) {
            return rc;
          }
          plain = h->last_plain;
          if (plain)
            HIPCHK(h, hipMemcpyAsync(h->its_pinned, h->last_its_slot, sizeof(int),
                                     hipMemcpyDeviceToHost, h->stream));
          // one pass: s = Q^T v_j, hh = Q^T w, v_j.v_j, v_j.w, w.w (coef[0 .. 2j+2])
          if ((rc = dots(h, h->Vk, j, Vp(j), h->w, len))) return rc;
          {
            // alpha, cq and the orthogonality flag from those values on the
            // device (coef[2j+3 .. 2j+5]), then one pass q_j = (v_j - Q s) /
            // alpha, w -= Q hh + cq q_j, |w|^2 (coef[2j+6]): the host reads
            // the step's scalars back in one copy
            const int oa = 2 * j + 3;
            if ((rc = timed(h, 5, [&] {
                   return launch_arnoldi_coeffs(h->coef, j, h->coef + oa, h->stream);
                 })))
              return rc;
            if ((rc = timed(h, 5, [&] {
                   return launch_update(h->Vk, j, Vp(j), h->w, h->coef, h->coef + j,
                                        h->coef + oa, j > 0 ? 1 : 0, len, h->partial, h->upd,
                                        h->stream);
                 })))
              return rc;
            if ((rc = timed(h, 5, [&] {
                   return launch_reduce_partials(h->partial, ns, 1, h->coef + oa + 3, h->stream);
                 })))
              return rc;
            ph = kStepB;
            return wait_coef(oa + 4);
          }
        case kStepB: {
          if (plain) {
            h->coarse_k = std::max(1, h->its_pinned[0]);   // coarse steps next time
            coarse_calls += 1;
            coarse_its += h->its_pinned[0];
          }
          const double* cb = h->hbuf;
          const int oa = 2 * j + 3;
          ww = cb[2 * j + 2];
          for (int i = 0; i < j; ++i) {
            sv[i] = cb[i];
            hv[i] = cb[j + i];
          }
          if (cb[oa + 2] != 0.0)
            return set_err(h, PITMG_ERR_NONFINITE, "lost orthogonality in the Arnoldi basis");
          alpha = cb[oa];
          cq = cb[oa + 1];
          rho = std::sqrt(cb[oa + 3]);
          if (!std::isfinite(rho) || !std::isfinite(ww))
            return set_err(h, PITMG_ERR_NONFINITE, "Krylov vector not finite");
          // finish column j-1: v_j = Q s + alpha q_j, scaled by rho_{j-1}
          if (j > 0) {
            for (int i = 0; i < j; ++i) H[(size_t)i * m + (j - 1)] += rho_prev * sv[i];
            H[(size_t)j * m + (j - 1)] = rho_prev * alpha;
            est = givens_column(H, m, j - 1, cs, sn, g) / bnorm;
            // stall rule of the learned coarse correction
            if (h->opt.coarse_mode == 1 && !h->fell_back) {
              stalled = est > h->opt.stall_ratio * est_prev ? stalled + 1 : 0;
              if (stalled >= h->opt.stall_steps) {
                h->fell_back = true;
                fallback_at = total + 1;      // first step to use GMRES + SGS
              }
            }
            est_prev = est;
          }
          // column j as far as known: w = Q hh + cq q_j + rho v_{j+1}
          for (int i = 0; i < j; ++i) H[(size_t)i * m + j] = hv[i];
          H[(size_t)j * m + j] = cq;
          H[(size_t)(j + 1) * m + j] = rho;
          total++;
          k = j + 1;
          // estimate with the column as it stands (v_{j+1} not yet re-orthogonalised)
          double prov;
          {
            std::vector<double> col(j + 2);
            for (int i = 0; i <= j; ++i) col[i] = H[(size_t)i * m + j];
            for (int i = 0; i < j; ++i) {
              const double c0 = col[i], c1 = col[i + 1];
              col[i] = cs[i] * c0 + sn[i] * c1;
              col[i + 1] = -sn[i] * c0 + cs[i] * c1;
            }
            const double a0 = col[j], a1 = rho;
            const double rr = std::hypot(a0, a1);
            prov = rr > 0.0 ? std::fabs(a1 / rr * g[j]) : 0.0;
          }
          const bool breakdown = rho <= 1e-14 * std::sqrt(ww);
          const bool end = prov <= tol * bnorm || breakdown || total >= maxit || j == m - 1;
          if (!breakdown) {
            if ((rc = timed(h, 5, [&] {
                   return launch_scale(Vp(j + 1), h->w, 1.0 / rho, len, h->stream);
                 })))
              return rc;
          }
          if (end) {
            if (!breakdown) {
              // finish column j: re-orthogonalisation coefficients of v_{j+1}
              if ((rc = dots(h, h->Vk, j + 1, Vp(j + 1), nullptr, len))) return rc;
              ph = kStepEnd;
              return wait_coef(j + 2);
            }
            est = givens_column(H, m, j, cs, sn, g) / bnorm;
            if (total >= maxit) stop = true;
            ph = kCycleEnd;
            break;
          }
          rho_prev = rho;
          ++j;
          ph = kStepA;
          break;
        }
        case kStepEnd: {
          double s2 = 0.0;
          for (int i = 0; i <= j; ++i) {
            H[(size_t)i * m + j] += rho * h->hbuf[i];
            s2 += h->hbuf[i] * h->hbuf[i];
          }
          const double a2 = h->hbuf[j + 1] - s2;
          H[(size_t)(j + 1) * m + j] = rho * std::sqrt(a2 > 0.0 ? a2 : 0.0);
          est = givens_column(H, m, j, cs, sn, g) / bnorm;
          if (total >= maxit) stop = true;
          ph = kCycleEnd;
          break;
        }
        case kCycleEnd:
          // y = H^{-1} g, x += Z y
          for (int i = k - 1; i >= 0; --i) {
            double acc = g[i];
            for (int c = i + 1; c < k; ++c) acc -= H[(size_t)i * m + c] * y[c];
            y[i] = acc / H[(size_t)i * m + i];
          }
          for (int i = 0; i < k; ++i) h->hbuf[i] = y[i];
          HIPCHK(h, hipMemcpyAsync(h->coef, h->hbuf, k * sizeof(double), hipMemcpyHostToDevice,
                                   h->stream));
          if ((rc = timed(h, 5, [&] {
                 return launch_multi_axpy(x, h->Zk, k, h->coef, 1.0, len, nullptr, h->stream);
               })))
            return rc;
          ph = stop ? kFinal : kCycle;
          break;
        case kFinal:
          // true residual (already known when the loop ended on it)
          rn = est * bnorm;
          if (converged) {
            ph = kFinish;
            break;
          }
          if ((rc = apply_sys(x, rhs, -1.0, 1.0, h->r))) return rc;
          if ((rc = dots(h, nullptr, 0, h->r, nullptr, len))) return rc;
          ph = kAfterFinal;
          return wait_coef(1);
        case kAfterFinal:
          rn = std::sqrt(h->hbuf[0]);
          ph = kFinish;
          break;
        case kFinish: {
          if (h->prof) drain(h);
          if (int rc2 = handoff_check(h)) return rc2;
          S = pitmg_stats{};
          S.fallback_at = -1;
          if (zero_rhs) {
            HIPCHK(h, hipStreamSynchronize(h->stream));
            S.converged = 1;
            status = PITMG_OK;
            ph = kDone;
            return kFinished;
          }
          S.iters = total;
          S.converged = converged ? 1 : 0;
          S.relres_est = est;
          S.relres_true = rn / bnorm;
          S.coarse_calls = coarse_calls;
          S.coarse_its_total = (int)coarse_its;
          S.ms_solve = std::chrono::duration<double, std::milli>(
                           std::chrono::steady_clock::now() - t0).count();
          S.net_calls = h->net_calls - net0;
          S.fallback_at = fallback_at;
          status = converged ? PITMG_OK : PITMG_NOT_CONVERGED;
          ph = kDone;
          return kFinished;
        }
        case kDone:
          return kFinished;
      }
    }
  }
};

// Run one solve to its end on the calling thread.
int run_to_end(FgmresRun& run) {
  for (;;) {
    const int rc = run.advance();
    if (rc < 0) {
      // an error that follows a failed hand-off is reported as that failure
      if (rc == PITMG_ERR_HIP) return rc;
      const int rh = handoff_check(run.h);
      return rh ? rh : rc;
    }
    if (rc == FgmresRun::kFinished) return run.status;
    if (run.h->prof) drain_ready(run.h);   // host work while the device is busy
    HIPCHK(run.h, hipStreamSynchronize(run.h->stream));
  }
}

}  // namespace

extern "C" {

void pitmg_default_options(pitmg_options* o) {
  if (!o) return;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->coarse_tol = 1e-3;
  o->coarse_maxit = 50;
  o->coarse_fixed_its = 0;
  o->restart = 30;
  o->maxit = 300;
  o->transfer_variant = 0;
  o->smoother_fp32 = 0;
  o->coarse_mode = 0;
  o->stall_ratio = 0.9;
  o->stall_steps = 2;
  o->vcycle_graph = 0;
  o->apply_from_sweep = 1;
  o->pair_sweeps = 2;
  o->omega = 0.5;
  o->mu_scale = 2.0;
  o->cycle = 0;
  o->smoother = 0;
  o->unlifted = 0;
  o->coarsen = 2;
}

int pitmg_autotune(pitmg_handle* h, int* cfg) {
  if (!h) return PITMG_ERR_INVALID;
  if (h->prof) return set_err(h, PITMG_ERR_INVALID, "turn profiling off before tuning");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  int rc = PITMG_OK;
  constexpr int kReps = 10;
  // a cycle that can chain its levels keeps the one-step kernel on every
  // level it applies to (the chained launches need it on all of them)
  const bool chain = chain_form(h->opt, h->L, 0) && jacobi_tiled_supported(h->p, h->q);
  for (int l = 0; l < h->L; ++l) {
    LevelBuf& B = h->lv[l];
    if (cfg) cfg[l] = 0;
    if (l == h->L - 1 || !B.y0 || !B.y1) continue;
    if (chain) {
      B.sweep_cfg = -1;
      if (cfg) cfg[l] = -1;
      continue;
    }
    B.sweep_cfg = 0;
    LevelView v = view(h, l);
    std::vector<int> cands;
    if (jacobi_shared_supported(v))
      cands = {1, 2, 3, 4};
    if (jacobi_tiled_supported(h->p, h->q)) cands.push_back(-1);
    if (cands.size() < 2) continue;
    HIPCHK(h, hipMemsetAsync(B.y0, 0, B.len * 8, h->stream));
    HIPCHK(h, hipMemsetAsync(B.y1, 0, B.len * 8, h->stream));
    float best = 1e30f;
    int pick = 0;
    // second output of a two-sweep launch (contents are scratch here)
    double* y2 = l == 0 ? h->r : B.out;
    for (int c : cands) {
      B.sweep_cfg = c;
      v = view(h, l);
      // a shape runs two sweeps per launch when the V-cycle would pair it:
      // time kReps sweeps either way
      const bool two = h->opt.pair_sweeps && y2 && jacobi_pair_supported(v, h->stream);
      const int launches = two ? kReps / 2 : kReps;
      for (int r = 0; r < launches + 2; ++r) {
        if (r == 2) HIPCHK(h, hipEventRecord(e0, h->stream));
        if (two)
          HIPCHK(h, sweep_pair(h, v, B.y1, B.y1, nullptr, B.y0, y2, nullptr, 0.0, 1.0));
        else
          HIPCHK(h, launch_jacobi(v, B.y1, B.y1, nullptr, h->opt.transfer_variant, B.y0,
                                  h->stream));
      }
      HIPCHK(h, hipEventRecord(e1, h->stream));
      HIPCHK(h, hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        pick = c;
      }
    }
    B.sweep_cfg = pick;
    if (cfg) cfg[l] = pick;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  drop_graph(h);
  // a timed two-sweep launch whose hand-off wait ran out fails the tuning
  if (int rh = handoff_check(h)) return rh;
  return rc;
}

int pitmg_set_handoff_wait(pitmg_handle* h, double seconds) {
  if (!h) return PITMG_ERR_INVALID;
  if (!(seconds >= 0.0) || !(seconds <= 60.0))
    return set_err(h, PITMG_ERR_INVALID, "the hand-off wait bound must be in [0, 60] s");
  h->hand_spin = (unsigned long long)(seconds * h->wall_hz);
  return PITMG_OK;
}

int pitmg_set_sweep_shapes(pitmg_handle* h, const int* cfg) {
  if (!h || !cfg) return PITMG_ERR_INVALID;
  for (int l = 0; l < h->L; ++l) {
    const int c = cfg[l];
    if (c == 0) continue;
    if (l == h->L - 1)
      return set_err(h, PITMG_ERR_INVALID, "the coarsest level has no sweep shape");
    LevelView v = view(h, l);
    v.sweep_cfg = 0;
    const bool ok = (c == -1 && jacobi_tiled_supported(h->p, h->q)) ||
                    (c >= 1 && c <= 4 && jacobi_shared_supported(v));
    if (!ok)
      return set_err(h, PITMG_ERR_INVALID,
                     "sweep shape " + std::to_string(c) + " is not available on level " +
                         std::to_string(l));
  }
  for (int l = 0; l < h->L; ++l) h->lv[l].sweep_cfg = cfg[l];
  drop_graph(h);
  return PITMG_OK;
}

int pitmg_coarse_net_attach(pitmg_handle* h, pitmg_net* net) {
  if (!h) return PITMG_ERR_INVALID;
  const int L = h->L - 1;
  if (net && !net_matches(net, 4 * h->p + h->q, h->lv[L].n))
    return set_err(h, PITMG_ERR_INVALID,
                   "the network's channels and steps must be 4p+q and the coarsest step count");
  h->net = net;
  return PITMG_OK;
}

int pitmg_coarse_pairs_arm(pitmg_handle* h, double* r, double* e, int cap) {
  if (!h || cap < 0) return PITMG_ERR_INVALID;
  if (cap > 0 && (!r || !e)) return set_err(h, PITMG_ERR_INVALID, "pair buffers are NULL");
  h->pair_r = r;
  h->pair_e = e;
  h->pair_cap = cap;
  h->pair_count = 0;
  return PITMG_OK;
}

int pitmg_coarse_pairs_count(const pitmg_handle* h) { return h ? h->pair_count : 0; }

int pitmg_setup(pitmg_handle** hp, const pitmg_problem* pb, const pitmg_options* opt,
                void* stream) {
  if (!hp) return PITMG_ERR_INVALID;
  *hp = nullptr;
  pitmg_handle* h = new pitmg_handle();
  h->stream = (hipStream_t)stream;
  pitmg_options o;
  pitmg_default_options(&o);
  if (opt) o = *opt;
  int rc = check_options(h, o);
  if (!rc) rc = check_problem(h, pb, o.coarsen);
  if (rc) {
    std::fprintf(stderr, "pitmg_setup: %s\n", h->err.c_str());
    delete h;
    return rc;
  }
  h->stream = (hipStream_t)stream;
  h->p = pb->p;
  h->q = pb->q;
  h->n = pb->n;
  h->L = pb->n_levels;
  h->opt = o;
  h->restart_cap = o.restart;
  h->maxit_cap = o.maxit;
  h->coarse_cap = o.coarse_fixed_its > 0 ? o.coarse_fixed_its : o.coarse_maxit;
  h->blocks_on_device = pb->blocks_on_device;
  h->lv.resize(h->L);
  const long long pp = (long long)h->p * h->p, pq = (long long)h->p * h->q;
  auto fail = [&](int code) {
    *hp = h;   // keep the handle so the caller can read the error, then destroy
    return code;
  };
  for (int l = 0; l < h->L; ++l) {
    LevelBuf& b = h->lv[l];
    b.n = l == 0 ? h->n : h->lv[l - 1].n / o.coarsen;
    b.len = (4LL * h->p + h->q) * b.n;
    if (!pb->blocks_on_device || o.unlifted) {
      // own copies: host blocks, or the scaled state blocks of the unlifted
      // system's lifted hierarchy
      const long long cN = (pb->N_stride ? b.n : 1) * pp, cV = (pb->V_stride ? b.n : 1) * pp,
                      cZ = (pb->Z_stride ? b.n : 1) * pq;
      if ((rc = dalloc(h, (void**)&b.N_own, cN * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.V_own, cV * 8))) return fail(rc);
      if (!pb->blocks_on_device && (rc = dalloc(h, (void**)&b.Z_own, cZ * 8))) return fail(rc);
    }
    const bool coarsest = l == h->L - 1;
    b.fp32 = l < o.smoother_fp32 && !coarsest;
    if (b.fp32) {
      const long long cN = (pb->N_stride ? b.n : 1) * pp, cV = (pb->V_stride ? b.n : 1) * pp,
                      cZ = (pb->Z_stride ? b.n : 1) * pq;
      if ((rc = dalloc(h, (void**)&b.N32, cN * 4))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.V32, cV * 4))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.Z32, cZ * 4))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.Gi32, (size_t)b.n * pp * 4))) return fail(rc);
      if (l == 0 && (rc = dalloc(h, (void**)&b.res, b.len * 8))) return fail(rc);
    } else {
      if ((rc = dalloc(h, (void**)&b.Gi, (size_t)b.n * pp * 8))) return fail(rc);
    }
    if ((rc = dalloc(h, (void**)&b.vzd, 2 * (size_t)h->p * 8))) return fail(rc);
    if (b.fp32 && (rc = dalloc(h, (void**)&b.vzd32, 2 * (size_t)h->p * 4))) return fail(rc);
    // W_k = G_k^{-1} N_k, used if V and Z~ turn out diagonal at factorisation
    if (!b.fp32 && h->p == h->q && (h->p == 64 || h->p == 128) && pb->V_stride == 0 &&
        pb->Z_stride == 0 && (rc = dalloc(h, (void**)&b.gin, (size_t)b.n * pp * 8)))
      return fail(rc);
    if (l > 0) {
      if ((rc = dalloc(h, (void**)&b.b, b.len * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.out, b.len * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.b2, b.len * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.e2, b.len * 8))) return fail(rc);
    }
    if (o.smoother != 0 && !coarsest) {
      double** gs[6] = {&b.gs_r, &b.gs_t, &b.gs_d, &b.gs_h, &b.hat_u, &b.hat_m};
      for (int i = 0; i < 6; ++i)
        if ((rc = dalloc(h, (void**)gs[i], b.len * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.Phi, (size_t)b.n * pp * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.PhiT, (size_t)b.n * pp * 8))) return fail(rc);
      // the chains write only the u (hat_u) or mu (hat_m) slots
      if (launch_fill(b.hat_u, 0.0, b.len, h->stream) != hipSuccess ||
          launch_fill(b.hat_m, 0.0, b.len, h->stream) != hipSuccess)
        return fail(set_err(h, PITMG_ERR_HIP, "fill of the Gauss-Seidel buffers failed"));
      if (l == 0 && (rc = dalloc(h, (void**)&h->gs_scr, (size_t)2 * b.n * pp * 8)))
        return fail(rc);
    }
    if (!coarsest) {
      if ((rc = dalloc(h, (void**)&b.y0, b.len * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.y1, b.len * 8))) return fail(rc);
    }
    // split sweep for large blocks whose V and Z~ are shared by every step
    if ((h->p == 256 || h->p == 512) && pb->V_stride == 0 && pb->Z_stride == 0) {
      const long long pn = (long long)h->p * b.n, qn = (long long)h->q * b.n;
      if ((rc = dalloc(h, (void**)&b.sp.Rm, (pn + h->p) * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.sp.U, pn * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.sp.Wz, qn * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.sp.Wv, pn * 8))) return fail(rc);
      if (b.fp32) {
        float** f32[6] = {&b.sp.Rm32, &b.sp.U32, &b.sp.L32, &b.sp.Wv32, &b.sp.Rz32, &b.sp.Wz32};
        for (int i = 0; i < 6; ++i)
          if ((rc = dalloc(h, (void**)f32[i], (i < 4 ? pn : qn) * 4))) return fail(rc);
      }
      b.split = true;
    }
  }
  const long long len = h->lv[0].len;
  const int m = h->restart_cap;
  if ((rc = dalloc(h, (void**)&h->Vk, (size_t)(m + 1) * len * 8))) return fail(rc);
  if ((rc = dalloc(h, (void**)&h->Zk, (size_t)m * len * 8))) return fail(rc);
  if ((rc = dalloc(h, (void**)&h->w, len * 8))) return fail(rc);
  if ((rc = dalloc(h, (void**)&h->r, len * 8))) return fail(rc);
  if (o.unlifted) {
    if ((rc = dalloc(h, (void**)&h->ul_in, len * 8))) return fail(rc);
    if ((rc = dalloc(h, (void**)&h->ul_out, len * 8))) return fail(rc);
  }
  const int nb = krylov_slices(len) > krylov_partial_blocks(len) ? krylov_slices(len)
                                                                   : krylov_partial_blocks(len);
  if ((rc = dalloc(h, (void**)&h->partial, (size_t)nb * (2 * m + 4) * 8))) return fail(rc);
  {
    int gmax = 1;
    for (int nbv = 1; nbv <= m + 1; ++nbv) gmax = std::max(gmax, krylov_groups(len, nbv));
    if (gmax > 1 &&
        (rc = dalloc(h, (void**)&h->upd, (size_t)gmax * 2 * len * 8)))
      return fail(rc);
  }
  const int ncoef = 2 * (m + 2) + 8;   // >= 2m+5: dot values and the step scalars
  if ((rc = dalloc(h, (void**)&h->coef, (size_t)ncoef * 8))) return fail(rc);
  if (hipHostMalloc((void**)&h->hbuf, (size_t)ncoef * 8, hipHostMallocDefault) != hipSuccess)
    return fail(set_err(h, PITMG_ERR_OOM, "hipHostMalloc failed"));
  const LevelBuf& lc = h->lv[h->L - 1];
  if ((rc = dalloc(h, (void**)&h->coarse_work,
                   coarse_work_doubles(h->p, h->q, lc.n, h->coarse_cap) * 8)))
    return fail(rc);
  {
    const long long lenc = lc.len;
    const long long ncp = (long long)lc.n * h->p;
    if ((rc = dalloc(h, (void**)&h->cst, coarse_state_doubles(h->coarse_cap) * 8))) return fail(rc);
    if ((rc = dalloc(h, (void**)&h->ist, 2 * sizeof(int)))) return fail(rc);
    h->coarse_fast = ncp <= 4096;
    if (h->coarse_fast) {
      double** vecs[6] = {&h->cC, &h->cA, &h->cD, &h->cY, &h->cY2, &h->czero};
      for (auto pp2 : vecs) {
        if ((rc = dalloc(h, (void**)pp2, lenc * 8))) return fail(rc);
        if (hipMemset(*pp2, 0, lenc * 8) != hipSuccess)
          return fail(set_err(h, PITMG_ERR_HIP, "hipMemset failed"));
      }
      if ((rc = dalloc(h, (void**)&h->Phi, (size_t)lc.n * pp * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&h->pscr, 2 * (size_t)lc.n * pp * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&h->Pf, (size_t)ncp * ncp * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&h->Qb, (size_t)ncp * ncp * 8))) return fail(rc);
      if (hipMemset(h->Pf, 0, (size_t)ncp * ncp * 8) != hipSuccess ||
          hipMemset(h->Qb, 0, (size_t)ncp * ncp * 8) != hipSuccess)
        return fail(set_err(h, PITMG_ERR_HIP, "hipMemset failed"));
      if ((h->p == 64 || h->p == 128) && h->p == h->q && lc.n + 1 <= 64) {
        const size_t nf = (size_t)sgs_fused_flags(lc.n, h->p);
        if ((rc = dalloc(h, (void**)&h->sgs_flag, nf * sizeof(unsigned long long))))
          return fail(rc);
        if (hipMemset(h->sgs_flag, 0, nf * sizeof(unsigned long long)) != hipSuccess)
          return fail(set_err(h, PITMG_ERR_HIP, "hipMemset failed"));
      }
    }
    if (hipHostMalloc((void**)&h->its_pinned, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess)
      return fail(set_err(h, PITMG_ERR_OOM, "hipHostMalloc failed"));
    h->its_pinned[0] = 1;
  }
  h->coarse_log_cap = h->maxit_cap + 64;
  if ((rc = dalloc(h, (void**)&h->coarse_its, (size_t)h->coarse_log_cap * sizeof(int))))
    return fail(rc);
  if ((rc = dalloc(h, (void**)&h->fail, sizeof(int)))) return fail(rc);
  if ((rc = dalloc(h, (void**)&h->vz_flags, 20 * sizeof(int)))) return fail(rc);
  if ((rc = dalloc(h, (void**)&h->zeros, 8 * sizeof(double)))) return fail(rc);
  if (launch_fill(h->zeros, 0.0, 8, h->stream) != hipSuccess)
    return fail(set_err(h, PITMG_ERR_HIP, "fill of the zero line failed"));
  if ((rc = dalloc(h, (void**)&h->hand_ticket, sizeof(unsigned long long))) ||
      (rc = dalloc(h, (void**)&h->hand_flag, (size_t)(2 * h->n + 2) * sizeof(unsigned long long))) ||
      (rc = dalloc(h, (void**)&h->hand_timeout, sizeof(int))))
    return fail(rc);
  if (hipMemsetAsync(h->hand_ticket, 0, sizeof(unsigned long long), h->stream) != hipSuccess ||
      hipMemsetAsync(h->hand_flag, 0, (size_t)(2 * h->n + 2) * sizeof(unsigned long long),
                     h->stream) != hipSuccess ||
      hipMemsetAsync(h->hand_timeout, 0, sizeof(int), h->stream) != hipSuccess)
    return fail(set_err(h, PITMG_ERR_HIP, "hipMemsetAsync failed"));
  {
    // resolve this GPU's static scratch (pitmg_coarse_solve_noalloc) while
    // setting up; a failure is reported by that entry point, which retries
    double* scr = nullptr;
    (void)noalloc_scratch(&scr);
    // the hand-off waits count ticks of the device's wall clock
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess &&
        khz > 0)
      h->wall_hz = 1e3 * khz;
    h->hand_spin = (unsigned long long)(2.0 * h->wall_hz);
  }
  rc = load_and_factor(h, pb);
  *hp = h;
  return rc;
}

int pitmg_refactor(pitmg_handle* h, const pitmg_problem* pb) {
  if (!h) return PITMG_ERR_INVALID;
  int rc = check_problem(h, pb, h->opt.coarsen);
  if (rc) return rc;
  if (pb->p != h->p || pb->q != h->q || pb->n != h->n || pb->n_levels != h->L ||
      pb->blocks_on_device != h->blocks_on_device)
    return set_err(h, PITMG_ERR_INVALID, "refactor needs the sizes and block placement of setup");
  if (!h->blocks_on_device && (pb->N_stride != h->lv[0].sN || pb->V_stride != h->lv[0].sV ||
                               pb->Z_stride != h->lv[0].sZ))
    return set_err(h, PITMG_ERR_INVALID, "refactor of host blocks needs the strides of setup");
  drop_graph(h);            // borrowed block pointers may have changed
  return load_and_factor(h, pb);
}

int pitmg_set_options(pitmg_handle* h, const pitmg_options* opt) {
  if (!h || !opt) return PITMG_ERR_INVALID;
  int rc = check_options(h, *opt);
  if (rc) return rc;
  const int cneed = opt->coarse_fixed_its > 0 ? opt->coarse_fixed_its : opt->coarse_maxit;
  if (opt->restart > h->restart_cap || cneed > h->coarse_cap)
    return set_err(h, PITMG_ERR_INVALID, "restart / coarse steps exceed the setup capacity");
  if (opt->smoother_fp32 != h->opt.smoother_fp32)
    return set_err(h, PITMG_ERR_INVALID, "smoother_fp32 is fixed at setup");
  if (opt->smoother != h->opt.smoother)
    return set_err(h, PITMG_ERR_INVALID, "smoother is fixed at setup");
  if (opt->unlifted != h->opt.unlifted)
    return set_err(h, PITMG_ERR_INVALID, "unlifted is fixed at setup");
  if (opt->coarsen != h->opt.coarsen)
    return set_err(h, PITMG_ERR_INVALID, "coarsen is fixed at setup");
  h->opt = *opt;
  drop_graph(h);            // the captured cycle depends on the options
  return PITMG_OK;
}

int pitmg_apply(pitmg_handle* h, int level, const double* x, double* y) {
  if (!h || !x || !y) return PITMG_ERR_INVALID;
  if (level < 0 || level >= h->L) return set_err(h, PITMG_ERR_INVALID, "bad level");
  LevelView v = view(h, level);
  return timed(h, 2, [&] { return launch_apply(v, x, nullptr, 1.0, 0.0, y, h->stream); });
}

int pitmg_unlifted_apply(pitmg_handle* h, const double* x, double* y) {
  if (!h || !x || !y) return PITMG_ERR_INVALID;
  if (!h->opt.unlifted)
    return set_err(h, PITMG_ERR_INVALID, "the handle was not set up with unlifted = 1");
  LevelView v = view(h, 0);
  return timed(h, 2, [&] {
    return launch_unlifted_apply(v, 1.0 / std::sqrt(2.0), x, nullptr, 1.0, 0.0, y, h->stream);
  });
}

int pitmg_unlifted_fgmres_solve(pitmg_handle* h, const double* rhs, double* x, double tol,
                                int use_x0, pitmg_stats* st) {
  if (!h) return PITMG_ERR_INVALID;
  if (!h->opt.unlifted)
    return set_err(h, PITMG_ERR_INVALID, "the handle was not set up with unlifted = 1");
  FgmresRun run;
  run.unl = true;
  int rc = run.start(h, rhs, x, tol, use_x0);
  if (rc) return rc;
  rc = run_to_end(run);
  if (rc >= 0 && st) *st = run.S;
  return rc;
}

int pitmg_jacobi_sweep(pitmg_handle* h, int level, const double* b, const double* y_in,
                       double* y_out) {
  if (!h || !b || !y_out) return PITMG_ERR_INVALID;
  if (level < 0 || level >= h->L) return set_err(h, PITMG_ERR_INVALID, "bad level");
  if (y_in == y_out) return set_err(h, PITMG_ERR_INVALID, "y_in and y_out must differ");
  LevelView v = view(h, level);
  return timed(h, 1, [&] {
    return launch_jacobi(v, b, y_in, nullptr, h->opt.transfer_variant, y_out, h->stream);
  });
}

int pitmg_coarse_solve(pitmg_handle* h, const double* b, double* x, int* its) {
  if (!h || !b || !x) return PITMG_ERR_INVALID;
  int rc = coarse_solve(h, b, x);
  if (rc) return rc;
  int hv = 0;
  HIPCHK(h, hipMemcpyAsync(&hv, h->coarse_its + ((h->coarse_calls - 1) % h->coarse_log_cap),
                           sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (its) *its = hv;
  return PITMG_OK;
}

int pitmg_coarse_solve_noalloc(pitmg_handle* h, const double* b, double* x, int* its) {
  if (!h || !b || !x) return PITMG_ERR_INVALID;
  const int l = h->L - 1;
  const long long len = h->lv[l].len;
  const int cap = h->coarse_cap;
  // layout: Krylov bases | GMRES state | 6 SGS work vectors | 3 ints
  const size_t nwork = coarse_work_doubles(h->p, h->q, h->lv[l].n, cap);
  const size_t nstate = coarse_state_doubles(cap);
  const size_t nvec = h->coarse_fast ? 6 * (size_t)len : 0;
  const size_t need = nwork + nstate + nvec + 2;
  if (need > kNoallocScratchDoubles)
    return set_err(h, PITMG_ERR_UNSUPPORTED,
                   "coarse solve needs " + std::to_string(need * 8) +
                       " bytes of scratch; the static scratch holds " +
                       std::to_string(kNoallocScratchDoubles * 8));
  double* base = nullptr;
  HIPCHK(h, noalloc_scratch(&base));
  double* vecs = base + nwork + nstate;
  int* ints = reinterpret_cast<int*>(vecs + nvec);          // {steps done, stop}, its
  CoarseWork cw{base, base + nwork, ints, nullptr, nullptr, nullptr, nullptr, nullptr,
                nullptr, ints + 2};
  if (h->coarse_fast) {
    double** slot[6] = {&cw.cC, &cw.cA, &cw.cD, &cw.cY, &cw.cY2, &cw.czero};
    for (int i = 0; i < 6; ++i) *slot[i] = vecs + (size_t)i * len;
    // the array keeps the last call's contents: the vectors whose unwritten
    // slots must read as zero are cleared
    HIPCHK(h, launch_fill(cw.cY, 0.0, 3 * len, h->stream));
  }
  int rc = coarse_solve_with(h, b, x, cw);
  if (rc) return rc;
  if (its) {
    HIPCHK(h, hipMemcpyAsync(its, cw.its, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  return PITMG_OK;
}

int pitmg_vcycle(pitmg_handle* h, const double* r, double* e) {
  if (!h || !r || !e) return PITMG_ERR_INVALID;
  if (r == e) return set_err(h, PITMG_ERR_INVALID, "r and e must differ");
  h->fell_back = false;
  const unsigned long long tickets = h->hand_tickets;
  const int rc = vcycle_top(h, r, e);
  // a two-sweep launch of this cycle whose hand-off wait ran out is this
  // call's error (the check synchronises; cycles without such launches,
  // e.g. under stream capture, stay asynchronous)
  if (h->hand_tickets != tickets) {
    const int rh = handoff_check(h);
    if (rh) return rh;
  }
  return rc;
}

int pitmg_fgmres_solve(pitmg_handle* h, const double* rhs, double* x, double tol, int use_x0,
                       pitmg_stats* st) {
  FgmresRun run;
  int rc = run.start(h, rhs, x, tol, use_x0);
  if (rc) return rc;
  rc = run_to_end(run);
  if (rc >= 0 && st) *st = run.S;
  return rc;
}

int pitmg_fgmres_solve_batch(pitmg_handle* const* hs, int count, const double* const* rhs,
                             double* const* x, double tol, int use_x0, pitmg_stats* st,
                             int* status) {
  if (!hs || !rhs || !x || count < 1) return PITMG_ERR_INVALID;
  for (int i = 0; i < count; ++i) {
    if (!hs[i]) return PITMG_ERR_INVALID;
    for (int k = 0; k < i; ++k)
      if (hs[k] == hs[i]) return set_err(hs[i], PITMG_ERR_INVALID, "a handle appears twice");
  }
  std::vector<FgmresRun> runs(count);
  std::vector<int> rcs(count, PITMG_OK), live(count, 1);
  int active = 0;
  for (int i = 0; i < count; ++i) {
    rcs[i] = runs[i].start(hs[i], rhs[i], x[i], tol, use_x0);
    if (rcs[i] < 0)
      live[i] = 0;
    else
      ++active;
  }
  std::vector<int> waiting(count, 0);
  while (active > 0) {
    // enqueue every live solve up to its next host wait ...
    for (int i = 0; i < count; ++i) {
      if (!live[i]) continue;
      int rc = runs[i].advance();
      waiting[i] = rc == FgmresRun::kWait;
      if (rc < 0 && rc != PITMG_ERR_HIP) {
        // an error that follows a failed hand-off is reported as that failure
        if (int rh = handoff_check(hs[i])) rc = rh;
      }
      if (rc != FgmresRun::kWait) {
        rcs[i] = rc < 0 ? rc : runs[i].status;
        live[i] = 0;
        --active;
      }
    }
    // ... then wait for each, while the others' work is in flight
    for (int i = 0; i < count; ++i)
      if (live[i] && waiting[i] && hs[i]->prof) drain_ready(hs[i]);
    for (int i = 0; i < count; ++i) {
      if (!live[i] || !waiting[i]) continue;
      const hipError_t e = hipStreamSynchronize(hs[i]->stream);
      if (e != hipSuccess) {
        rcs[i] = set_err(hs[i], PITMG_ERR_HIP, std::string("hipStreamSynchronize: ") +
                                                   hipGetErrorString(e));
        live[i] = 0;
        --active;
        continue;
      }
    }
  }
  int worst = PITMG_OK;
  for (int i = 0; i < count; ++i) {
    if (status) status[i] = rcs[i];
    if (st) st[i] = rcs[i] >= 0 ? runs[i].S : pitmg_stats{};
    if (rcs[i] < 0 && worst >= 0) worst = rcs[i];
    if (rcs[i] == PITMG_NOT_CONVERGED && worst == PITMG_OK) worst = PITMG_NOT_CONVERGED;
  }
  return worst;
}

int pitmg_profile_enable(pitmg_handle* h, int on) {
  if (!h) return PITMG_ERR_INVALID;
  if (on < 0 || on > 2) return set_err(h, PITMG_ERR_INVALID, "profiling level must be 0, 1 or 2");
  if (h->prof) drain(h);
  h->prof = on;
  return PITMG_OK;
}

int pitmg_profile_sample(pitmg_handle* h, int every) {
  if (!h || every < 1) return PITMG_ERR_INVALID;
  h->prof_every = every;
  return PITMG_OK;
}

int pitmg_profile_read(pitmg_handle* h, int cls, int* launches, double* ms, double* bytes) {
  if (!h || cls < 0 || cls >= kNumClasses) return PITMG_ERR_INVALID;
  drain(h);
  if (launches) *launches = h->prof_launches[cls];
  if (ms) *ms = h->prof_ms[cls];
  if (bytes) *bytes = 0.0;
  return PITMG_OK;
}

int pitmg_profile_reset(pitmg_handle* h) {
  if (!h) return PITMG_ERR_INVALID;
  drain(h);
  for (int c = 0; c < kNumClasses; ++c) {
    h->prof_launches[c] = 0;
    h->prof_ms[c] = 0.0;
  }
  return PITMG_OK;
}

int pitmg_failed_block(const pitmg_handle* h, int* level, int* k) {
  if (!h) return PITMG_ERR_INVALID;
  if (h->fail_code == INT_MAX) {
    if (level) *level = -1;
    if (k) *k = -1;
    return PITMG_OK;
  }
  if (level) *level = h->fail_code >> 20;
  if (k) *k = (h->fail_code & 0xFFFFF) + 1;
  return PITMG_OK;
}

long long pitmg_device_bytes(const pitmg_handle* h) { return h ? h->dev_bytes : 0; }

int pitmg_level_info(const pitmg_handle* h, int level, int* n, int* flags) {
  if (!h || level < 0 || level >= h->L) return PITMG_ERR_INVALID;
  const LevelBuf& b = h->lv[level];
  if (n) *n = b.n;
  if (flags)
    *flags = (b.fp32 ? PITMG_LEVEL_FP32 : 0) | (b.vz_diag ? PITMG_LEVEL_DIAG_VZ : 0) |
             (b.gn ? PITMG_LEVEL_GIN : 0);
  return PITMG_OK;
}

const char* pitmg_status_string(int code) {
  switch (code) {
    case PITMG_OK: return "ok";
    case PITMG_NOT_CONVERGED: return "not converged";
    case PITMG_ERR_INVALID: return "invalid argument";
    case PITMG_ERR_SINGULAR: return "singular time-step block";
    case PITMG_ERR_NONFINITE: return "non-finite value";
    case PITMG_ERR_HIP: return "HIP runtime error";
    case PITMG_ERR_OOM: return "out of device memory";
    case PITMG_ERR_UNSUPPORTED: return "unsupported size";
    default: return "unknown status";
  }
}

const char* pitmg_last_error(const pitmg_handle* h) { return h ? h->err.c_str() : ""; }

void pitmg_destroy(pitmg_handle* h) {
  if (!h) return;
  // teardown: nothing is left to report to, so failed calls are ignored
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  auto release = [](void* ptr) {
    if (ptr) (void)hipFree(ptr);
  };
  drain(h);
  drop_graph(h);
  release(h->g_in);
  release(h->g_out);
  release(h->upd);
  for (auto& b : h->lv) {
    void* sp[] = {b.sp.Rm, b.sp.U, b.sp.Wz, b.sp.Wv, b.sp.Rm32, b.sp.Rz32,
                  b.sp.U32, b.sp.L32, b.sp.Wz32, b.sp.Wv32};
    for (void* ptr : sp) release(ptr);
  }
  for (auto e : h->pool) (void)hipEventDestroy(e);
  for (auto& b : h->lv) {
    release(b.N_own);
    release(b.V_own);
    release(b.Z_own);
    release(b.Gi);
    release(b.b);
    release(b.y0);
    release(b.y1);
    release(b.out);
    release(b.res);
    release(b.vzd);
    release(b.vzd32);
    release(b.gin);
    release(b.b2);
    release(b.e2);
    release(b.Phi);
    release(b.PhiT);
    release(b.gs_r);
    release(b.gs_t);
    release(b.gs_d);
    release(b.gs_h);
    release(b.hat_u);
    release(b.hat_m);
    release(b.N32);
    release(b.V32);
    release(b.Z32);
    release(b.Gi32);
  }
  release(h->gs_scr);
  release(h->ul_in);
  release(h->ul_out);
  release(h->Vk);
  release(h->Zk);
  release(h->w);
  release(h->r);
  release(h->partial);
  release(h->coef);
  if (h->hbuf) (void)hipHostFree(h->hbuf);
  release(h->coarse_work);
  release(h->coarse_its);
  release(h->cst);
  release(h->ist);
  release(h->cC);
  release(h->cA);
  release(h->cD);
  release(h->cY);
  release(h->cY2);
  release(h->czero);
  release(h->Phi);
  release(h->pscr);
  release(h->Pf);
  release(h->sgs_flag);
  release(h->Qb);
  if (h->its_pinned) (void)hipHostFree(h->its_pinned);
  release(h->fail);
  release(h->vz_flags);
  release(h->zeros);
  release(h->hand_ticket);
  release(h->hand_flag);
  release(h->hand_timeout);
  delete h;
}

}  // extern "C"
