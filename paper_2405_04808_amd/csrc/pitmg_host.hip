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
#include <string>
#include <vector>

using namespace pitmg;

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
};

struct ProfRec {
  int cls;
  hipEvent_t a, b;
};

constexpr int kNumClasses = 6;

}  // namespace

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
  double* coef = nullptr;            // device scalars, 2*(restart+1)+4
  double* hbuf = nullptr;            // pinned host mirror of coef
  double* coarse_work = nullptr;
  int* coarse_its = nullptr;         // device log of coarse step counts
  int coarse_log_cap = 0;
  int coarse_calls = 0;
  int* fail = nullptr;
  int fail_code = INT_MAX;
  long long dev_bytes = 0;
  std::string err;
  bool prof = false;
  std::vector<ProfRec> pending;
  std::vector<hipEvent_t> pool;
  int prof_launches[kNumClasses] = {0};
  double prof_ms[kNumClasses] = {0};
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
  hipEventCreate(&e);
  return e;
}

// Accumulate the elapsed time of every recorded launch (waits for them).
void drain(pitmg_handle* h) {
  for (auto& r : h->pending) {
    hipEventSynchronize(r.b);
    float ms = 0.f;
    hipEventElapsedTime(&ms, r.a, r.b);
    h->prof_ms[r.cls] += ms;
    h->prof_launches[r.cls] += 1;
    h->pool.push_back(r.a);
    h->pool.push_back(r.b);
  }
  h->pending.clear();
}

template <class F>
int timed(pitmg_handle* h, int cls, F&& launch) {
  if (!h->prof) {
    HIPCHK(h, launch());
    return PITMG_OK;
  }
  ProfRec r{cls, take_event(h), take_event(h)};
  HIPCHK(h, hipEventRecord(r.a, h->stream));
  HIPCHK(h, launch());
  HIPCHK(h, hipEventRecord(r.b, h->stream));
  h->pending.push_back(r);
  if (h->pending.size() > 4096) drain(h);
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
  return PITMG_OK;
}

int check_problem(pitmg_handle* h, const pitmg_problem* pb) {
  if (!pb) return set_err(h, PITMG_ERR_INVALID, "problem is NULL");
  if (pb->p < 1 || pb->q < 1 || pb->n < 1 || pb->n_levels < 1)
    return set_err(h, PITMG_ERR_INVALID, "p, q, n and n_levels must be >= 1");
  if (pb->n_levels > 20) return set_err(h, PITMG_ERR_INVALID, "n_levels must be <= 20");
  if (pb->n >= (1 << 20)) return set_err(h, PITMG_ERR_UNSUPPORTED, "n must be < 2^20");
  const long long div = 1LL << (pb->n_levels - 1);
  if (pb->n % div != 0)
    return set_err(h, PITMG_ERR_INVALID, "n must be divisible by 2^(n_levels-1)");
  if (pb->p > 256 || pb->q > 256)
    return set_err(h, PITMG_ERR_UNSUPPORTED, "this build supports p, q <= 256");
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
  }
  const int big = INT_MAX;
  HIPCHK(h, hipMemcpyAsync(h->fail, &big, sizeof(int), hipMemcpyHostToDevice, h->stream));
  for (int l = 0; l < h->L; ++l) {
    LevelView v = view(h, l);
    int rc = timed(h, 0, [&] { return launch_factor(v, h->lv[l].Gi, l, h->fail, h->stream); });
    if (rc) return rc;
  }
  int code = INT_MAX;
  HIPCHK(h, hipMemcpyAsync(&code, h->fail, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->fail_code = code;
  if (code != INT_MAX)
    return set_err(h, PITMG_ERR_SINGULAR,
                   "S_k not positive definite at level " + std::to_string(code >> 20) +
                       ", step " + std::to_string((code & 0xFFFFF) + 1));
  return PITMG_OK;
}

// MG_l(b) -> out (Alg. 1 recursed; zero initial guess on every level).
int vcycle_level(pitmg_handle* h, int l, const double* b, double* out) {
  const pitmg_options& o = h->opt;
  const int var = o.transfer_variant;
  LevelView v = view(h, l);
  if (l == h->L - 1) {
    int* its = h->coarse_its + (h->coarse_calls % h->coarse_log_cap);
    h->coarse_calls++;
    return timed(h, 4, [&] {
      return launch_coarse(v, b, out, o.coarse_tol, o.coarse_maxit, o.coarse_fixed_its,
                           h->coarse_work, its, h->stream);
    });
  }
  LevelBuf& B = h->lv[l];
  LevelBuf& C = h->lv[l + 1];
  double* bufs[2] = {B.y0, B.y1};
  const double* yprev = nullptr;
  double* ycur = nullptr;
  int rc;
  for (int s = 0; s < o.nu_pre; ++s) {
    double* dst = bufs[s & 1];
    const double* yo = ycur;
    rc = timed(h, 1, [&] { return launch_jacobi(v, b, yo, nullptr, var, dst, h->stream); });
    if (rc) return rc;
    yprev = ycur;
    ycur = dst;
  }
  if (ycur == nullptr)
    rc = timed(h, 3, [&] { return launch_restrict(h->p, h->q, v.n, b, var, C.b, h->stream); });
  else
    rc = timed(h, 3, [&] {
      return launch_restrict_delta(h->p, h->q, v.n, yprev, ycur, var, C.b, h->stream);
    });
  if (rc) return rc;
  rc = vcycle_level(h, l + 1, C.b, C.out);
  if (rc) return rc;
  if (o.nu_post == 0) {
    if (ycur)
      HIPCHK(h, hipMemcpyAsync(out, ycur, B.len * 8, hipMemcpyDeviceToDevice, h->stream));
    else
      HIPCHK(h, hipMemsetAsync(out, 0, B.len * 8, h->stream));
    return timed(h, 3, [&] {
      return launch_interp_add(h->p, h->q, v.n, C.out, var, out, h->stream);
    });
  }
  for (int s = 0; s < o.nu_post; ++s) {
    double* dst = (s == o.nu_post - 1) ? out : (ycur == bufs[0] ? bufs[1] : bufs[0]);
    const double* yo = ycur;
    const double* ec = s == 0 ? C.out : nullptr;
    rc = timed(h, 1, [&] { return launch_jacobi(v, b, yo, ec, var, dst, h->stream); });
    if (rc) return rc;
    ycur = dst;
  }
  return PITMG_OK;
}

// dots of w against nvec basis vectors (and w . w when with_self) -> device
// coef[off .. off + nvec + with_self)
int multidot(pitmg_handle* h, const double* basis, int nvec, int with_self, const double* w,
             long long len, int off) {
  const int nb = krylov_partial_blocks(len);
  int rc = timed(h, 5, [&] {
    return launch_multidot(basis, nvec, with_self, w, len, h->partial, h->stream);
  });
  if (rc) return rc;
  return timed(h, 5, [&] {
    return launch_reduce_partials(h->partial, nb, nvec + with_self, h->coef + off, h->stream);
  });
}

int device_norm(pitmg_handle* h, const double* x, long long len, double* out) {
  int rc = multidot(h, x, 1, 0, x, len, 0);
  if (rc) return rc;
  HIPCHK(h, hipMemcpyAsync(h->hbuf, h->coef, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  *out = std::sqrt(h->hbuf[0]);
  return PITMG_OK;
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
}

int pitmg_setup(pitmg_handle** hp, const pitmg_problem* pb, const pitmg_options* opt,
                void* stream) {
  if (!hp) return PITMG_ERR_INVALID;
  *hp = nullptr;
  pitmg_handle* h = new pitmg_handle();
  int rc = check_problem(h, pb);
  pitmg_options o;
  pitmg_default_options(&o);
  if (opt) o = *opt;
  if (!rc) rc = check_options(h, o);
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
    b.n = h->n >> l;
    b.len = (4LL * h->p + h->q) * b.n;
    if (!pb->blocks_on_device) {
      const long long cN = (pb->N_stride ? b.n : 1) * pp, cV = (pb->V_stride ? b.n : 1) * pp,
                      cZ = (pb->Z_stride ? b.n : 1) * pq;
      if ((rc = dalloc(h, (void**)&b.N_own, cN * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.V_own, cV * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.Z_own, cZ * 8))) return fail(rc);
    }
    if ((rc = dalloc(h, (void**)&b.Gi, (size_t)b.n * pp * 8))) return fail(rc);
    const bool coarsest = l == h->L - 1;
    if (l > 0) {
      if ((rc = dalloc(h, (void**)&b.b, b.len * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.out, b.len * 8))) return fail(rc);
    }
    if (!coarsest) {
      if ((rc = dalloc(h, (void**)&b.y0, b.len * 8))) return fail(rc);
      if ((rc = dalloc(h, (void**)&b.y1, b.len * 8))) return fail(rc);
    }
  }
  const long long len = h->lv[0].len;
  const int m = h->restart_cap;
  if ((rc = dalloc(h, (void**)&h->Vk, (size_t)(m + 1) * len * 8))) return fail(rc);
  if ((rc = dalloc(h, (void**)&h->Zk, (size_t)m * len * 8))) return fail(rc);
  if ((rc = dalloc(h, (void**)&h->w, len * 8))) return fail(rc);
  if ((rc = dalloc(h, (void**)&h->r, len * 8))) return fail(rc);
  const int nb = krylov_partial_blocks(len);
  if ((rc = dalloc(h, (void**)&h->partial, (size_t)nb * (m + 2) * 8))) return fail(rc);
  const int ncoef = 2 * (m + 2) + 8;
  if ((rc = dalloc(h, (void**)&h->coef, (size_t)ncoef * 8))) return fail(rc);
  if (hipHostMalloc((void**)&h->hbuf, (size_t)ncoef * 8, hipHostMallocDefault) != hipSuccess)
    return fail(set_err(h, PITMG_ERR_OOM, "hipHostMalloc failed"));
  const LevelBuf& lc = h->lv[h->L - 1];
  if ((rc = dalloc(h, (void**)&h->coarse_work,
                   coarse_work_doubles(h->p, h->q, lc.n, h->coarse_cap) * 8)))
    return fail(rc);
  h->coarse_log_cap = h->maxit_cap + 64;
  if ((rc = dalloc(h, (void**)&h->coarse_its, (size_t)h->coarse_log_cap * sizeof(int))))
    return fail(rc);
  if ((rc = dalloc(h, (void**)&h->fail, sizeof(int)))) return fail(rc);
  rc = load_and_factor(h, pb);
  *hp = h;
  return rc;
}

int pitmg_refactor(pitmg_handle* h, const pitmg_problem* pb) {
  if (!h) return PITMG_ERR_INVALID;
  int rc = check_problem(h, pb);
  if (rc) return rc;
  if (pb->p != h->p || pb->q != h->q || pb->n != h->n || pb->n_levels != h->L ||
      pb->blocks_on_device != h->blocks_on_device)
    return set_err(h, PITMG_ERR_INVALID, "refactor needs the sizes and block placement of setup");
  if (!h->blocks_on_device && (pb->N_stride != h->lv[0].sN || pb->V_stride != h->lv[0].sV ||
                               pb->Z_stride != h->lv[0].sZ))
    return set_err(h, PITMG_ERR_INVALID, "refactor of host blocks needs the strides of setup");
  return load_and_factor(h, pb);
}

int pitmg_set_options(pitmg_handle* h, const pitmg_options* opt) {
  if (!h || !opt) return PITMG_ERR_INVALID;
  int rc = check_options(h, *opt);
  if (rc) return rc;
  const int cneed = opt->coarse_fixed_its > 0 ? opt->coarse_fixed_its : opt->coarse_maxit;
  if (opt->restart > h->restart_cap || cneed > h->coarse_cap)
    return set_err(h, PITMG_ERR_INVALID, "restart / coarse steps exceed the setup capacity");
  h->opt = *opt;
  return PITMG_OK;
}

int pitmg_apply(pitmg_handle* h, int level, const double* x, double* y) {
  if (!h || !x || !y) return PITMG_ERR_INVALID;
  if (level < 0 || level >= h->L) return set_err(h, PITMG_ERR_INVALID, "bad level");
  LevelView v = view(h, level);
  return timed(h, 2, [&] { return launch_apply(v, x, nullptr, 1.0, 0.0, y, h->stream); });
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
  int rc = vcycle_level(h, h->L - 1, b, x);
  if (rc) return rc;
  int hv = 0;
  HIPCHK(h, hipMemcpyAsync(&hv, h->coarse_its + ((h->coarse_calls - 1) % h->coarse_log_cap),
                           sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (its) *its = hv;
  return PITMG_OK;
}

int pitmg_vcycle(pitmg_handle* h, const double* r, double* e) {
  if (!h || !r || !e) return PITMG_ERR_INVALID;
  if (r == e) return set_err(h, PITMG_ERR_INVALID, "r and e must differ");
  return vcycle_level(h, 0, r, e);
}

int pitmg_fgmres_solve(pitmg_handle* h, const double* rhs, double* x, double tol, int use_x0,
                       pitmg_stats* st) {
  if (!h || !rhs || !x) return PITMG_ERR_INVALID;
  if (!(tol >= 0.0)) return set_err(h, PITMG_ERR_INVALID, "tol must be >= 0");
  const auto t0 = std::chrono::steady_clock::now();
  const long long len = h->lv[0].len;
  const int m = h->opt.restart, maxit = h->opt.maxit;
  const int calls0 = h->coarse_calls;
  LevelView v0 = view(h, 0);
  int rc;
  double bnorm = 0.0;
  if ((rc = device_norm(h, rhs, len, &bnorm))) return rc;
  if (!std::isfinite(bnorm)) return set_err(h, PITMG_ERR_NONFINITE, "right-hand side not finite");
  pitmg_stats S{};
  if (bnorm == 0.0) {
    HIPCHK(h, hipMemsetAsync(x, 0, len * 8, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    S.converged = 1;
    if (st) *st = S;
    return PITMG_OK;
  }
  if (!use_x0) HIPCHK(h, hipMemsetAsync(x, 0, len * 8, h->stream));
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  int total = 0;
  bool converged = false, started_from_zero = !use_x0;
  double est = 1.0;
  for (;;) {
    double beta;
    if (started_from_zero && total == 0) {
      beta = bnorm;
      if ((rc = timed(h, 5, [&] { return launch_scale(h->Vk, rhs, 1.0 / beta, len, h->stream); })))
        return rc;
    } else {
      if ((rc = timed(h, 2, [&] { return launch_apply(v0, x, rhs, -1.0, 1.0, h->r, h->stream); })))
        return rc;
      if ((rc = device_norm(h, h->r, len, &beta))) return rc;
      if (!std::isfinite(beta)) return set_err(h, PITMG_ERR_NONFINITE, "residual not finite");
      est = beta / bnorm;
      if (beta <= tol * bnorm) {
        converged = true;
        break;
      }
      if (total >= maxit) break;
      if ((rc = timed(h, 5, [&] { return launch_scale(h->Vk, h->r, 1.0 / beta, len, h->stream); })))
        return rc;
    }
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    bool stop = false;
    for (int j = 0; j < m; ++j) {
      double* vj = h->Vk + (size_t)j * len;
      double* zj = h->Zk + (size_t)j * len;
      if ((rc = vcycle_level(h, 0, vj, zj))) return rc;
      if ((rc = timed(h, 2, [&] { return launch_apply(v0, zj, nullptr, 1.0, 0.0, h->w, h->stream); })))
        return rc;
      // classical Gram-Schmidt, twice: h1 = V^T w (with ||w||^2), w -= V h1,
      // h2 = V^T w, w -= V h2 (with the new ||w||^2)
      const int nv = j + 1;
      const int nb = krylov_partial_blocks(len);
      const int o2 = m + 2, on = 2 * (m + 2);
      if ((rc = multidot(h, h->Vk, nv, 1, h->w, len, 0))) return rc;
      if ((rc = timed(h, 5, [&] {
             return launch_multi_axpy(h->w, h->Vk, nv, h->coef, -1.0, len, nullptr, h->stream);
           })))
        return rc;
      if ((rc = multidot(h, h->Vk, nv, 0, h->w, len, o2))) return rc;
      if ((rc = timed(h, 5, [&] {
             return launch_multi_axpy(h->w, h->Vk, nv, h->coef + o2, -1.0, len, h->partial,
                                      h->stream);
           })))
        return rc;
      if ((rc = timed(h, 5, [&] {
             return launch_reduce_partials(h->partial, nb, 1, h->coef + on, h->stream);
           })))
        return rc;
      HIPCHK(h, hipMemcpyAsync(h->hbuf, h->coef, (on + 1) * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      if (h->prof) drain(h);
      const double w0 = std::sqrt(h->hbuf[nv]);
      const double hn = std::sqrt(h->hbuf[on]);
      if (!std::isfinite(hn) || !std::isfinite(w0))
        return set_err(h, PITMG_ERR_NONFINITE, "Krylov vector not finite");
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h->hbuf[i] + h->hbuf[o2 + i];
      H[(size_t)(j + 1) * m + j] = hn;
      for (int i = 0; i < j; ++i) {
        const double a0 = H[(size_t)i * m + j], a1 = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a0 + sn[i] * a1;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a0 + cs[i] * a1;
      }
      const double a0 = H[(size_t)j * m + j];
      const double rr = std::hypot(a0, hn);
      cs[j] = rr > 0.0 ? a0 / rr : 1.0;
      sn[j] = rr > 0.0 ? hn / rr : 0.0;
      H[(size_t)j * m + j] = rr;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      total++;
      est = std::fabs(g[j + 1]) / bnorm;
      // the estimate (or a breakdown) ends the cycle; the true residual,
      // computed at the top of the next pass, decides convergence
      if (std::fabs(g[j + 1]) <= tol * bnorm || hn <= 1e-14 * w0) break;
      if (total >= maxit) {
        stop = true;
        break;
      }
      double* vn = h->Vk + (size_t)(j + 1) * len;
      if ((rc = timed(h, 5, [&] { return launch_scale(vn, h->w, 1.0 / hn, len, h->stream); })))
        return rc;
    }
    // y = H^{-1} g, x += Z y
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[i];
      for (int c = i + 1; c < k; ++c) acc -= H[(size_t)i * m + c] * y[c];
      y[i] = acc / H[(size_t)i * m + i];
    }
    for (int i = 0; i < k; ++i) h->hbuf[i] = y[i];
    HIPCHK(h, hipMemcpyAsync(h->coef, h->hbuf, k * sizeof(double), hipMemcpyHostToDevice,
                             h->stream));
    if ((rc = timed(h, 5, [&] { return launch_multi_axpy(x, h->Zk, k, h->coef, 1.0, len, nullptr, h->stream); })))
      return rc;
    started_from_zero = false;
    if (stop) break;
  }
  // true residual (already known when the loop ended on it)
  double rn = est * bnorm;
  if (!converged) {
    if ((rc = timed(h, 2, [&] { return launch_apply(v0, x, rhs, -1.0, 1.0, h->r, h->stream); })))
      return rc;
    if ((rc = device_norm(h, h->r, len, &rn))) return rc;
  }
  if (h->prof) drain(h);
  // coarse statistics
  const int ncalls = h->coarse_calls - calls0;
  long long cits = 0;
  if (ncalls > 0) {
    std::vector<int> log(h->coarse_log_cap);
    HIPCHK(h, hipMemcpy(log.data(), h->coarse_its, h->coarse_log_cap * sizeof(int),
                        hipMemcpyDeviceToHost));
    for (int c = calls0; c < h->coarse_calls; ++c) cits += log[c % h->coarse_log_cap];
  }
  S.iters = total;
  S.converged = converged ? 1 : 0;
  S.relres_est = est;
  S.relres_true = rn / bnorm;
  S.coarse_calls = ncalls;
  S.coarse_its_total = (int)cits;
  S.ms_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = S;
  return converged ? PITMG_OK : PITMG_NOT_CONVERGED;
}

int pitmg_profile_enable(pitmg_handle* h, int on) {
  if (!h) return PITMG_ERR_INVALID;
  if (!on && h->prof) drain(h);
  h->prof = on != 0;
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
  if (h->stream) hipStreamSynchronize(h->stream);
  else hipDeviceSynchronize();
  drain(h);
  for (auto e : h->pool) hipEventDestroy(e);
  for (auto& b : h->lv) {
    hipFree(b.N_own);
    hipFree(b.V_own);
    hipFree(b.Z_own);
    hipFree(b.Gi);
    hipFree(b.b);
    hipFree(b.y0);
    hipFree(b.y1);
    hipFree(b.out);
  }
  hipFree(h->Vk);
  hipFree(h->Zk);
  hipFree(h->w);
  hipFree(h->r);
  hipFree(h->partial);
  hipFree(h->coef);
  if (h->hbuf) hipHostFree(h->hbuf);
  hipFree(h->coarse_work);
  hipFree(h->coarse_its);
  hipFree(h->fail);
  delete h;
}

}  // extern "C"
