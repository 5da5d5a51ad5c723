// Host-side checks of the C ABI under AddressSanitizer and UBSan, with no
// GPU: option and problem validation, every entry point's NULL-handle path,
// the status strings, and a setup that gets past validation on a machine
// whose device calls fail (the partially built handle is kept for its error
// message and then destroyed).  Exits 0 when every return code is the one
// the header states; the sanitizers abort on any host memory or UB error.
#include "../include/pitmg.h"

#include <cstdio>
#include <cstring>
#include <vector>

static int failures = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

int main() {
  pitmg_options o;
  pitmg_default_options(&o);
  pitmg_default_options(nullptr);
  expect(o.nu_pre == 2 && o.nu_post == 2 && o.coarsen == 2 && o.cycle == 0, "defaults");
  for (int c = -8; c <= 2; ++c) expect(pitmg_status_string(c) != nullptr, "status string");
  pitmg_destroy(nullptr);
  expect(pitmg_last_error(nullptr) != nullptr, "last_error(NULL)");

  // a valid-looking problem on host blocks
  const int p = 3, q = 2, n = 16, L = 3;
  std::vector<std::vector<double>> N(L), V(L), Z(L);
  std::vector<const double*> pN(L), pV(L), pZ(L);
  for (int l = 0; l < L; ++l) {
    const int nl = n >> l;
    N[l].assign((size_t)nl * p * p, 0.5);
    V[l].assign((size_t)p * p, -1.0);
    Z[l].assign((size_t)p * q, 0.25);
    pN[l] = N[l].data();
    pV[l] = V[l].data();
    pZ[l] = Z[l].data();
  }
  auto base = [&]() {
    pitmg_problem pb;
    std::memset(&pb, 0, sizeof pb);
    pb.p = p;
    pb.q = q;
    pb.n = n;
    pb.n_levels = L;
    pb.N = pN.data();
    pb.V = pV.data();
    pb.Z = pZ.data();
    pb.N_stride = (long long)p * p;
    pb.V_stride = 0;
    pb.Z_stride = 0;
    pb.blocks_on_device = 0;
    return pb;
  };
  auto setup_fails = [&](const pitmg_problem* pb, const pitmg_options* opt, int want,
                         const char* what) {
    pitmg_handle* h = reinterpret_cast<pitmg_handle*>(0x1);
    const int rc = pitmg_setup(&h, pb, opt, nullptr);
    expect(rc == want, what);
    expect(h == nullptr, "no handle after a validation error");
  };

  // problem validation
  setup_fails(nullptr, &o, PITMG_ERR_INVALID, "NULL problem");
  {
    pitmg_problem pb = base();
    pb.p = 0;
    setup_fails(&pb, &o, PITMG_ERR_INVALID, "p = 0");
  }
  {
    pitmg_problem pb = base();
    pb.n = 10;                       // 10 % 2^(3-1) != 0
    setup_fails(&pb, &o, PITMG_ERR_INVALID, "n not divisible");
  }
  {
    pitmg_problem pb = base();
    pb.n_levels = 25;
    setup_fails(&pb, &o, PITMG_ERR_INVALID, "too many levels");
  }
  {
    pitmg_problem pb = base();
    pb.p = 600;
    pb.N_stride = 600LL * 600;
    setup_fails(&pb, &o, PITMG_ERR_UNSUPPORTED, "p > 512");
  }
  {
    pitmg_problem pb = base();
    pb.N_stride = 5;
    setup_fails(&pb, &o, PITMG_ERR_INVALID, "bad N stride");
  }
  {
    pitmg_problem pb = base();
    std::vector<const double*> bad = pN;
    bad[1] = nullptr;
    pb.N = bad.data();
    setup_fails(&pb, &o, PITMG_ERR_INVALID, "NULL level pointer");
  }
  {
    pitmg_problem pb = base();
    pb.blocks_on_device = 7;
    setup_fails(&pb, &o, PITMG_ERR_INVALID, "blocks_on_device");
  }
  // option validation
  struct BadOpt {
    const char* what;
    void (*set)(pitmg_options&);
  };
  const BadOpt bad_opts[] = {
      {"omega 0", [](pitmg_options& x) { x.omega = 0.0; }},
      {"mu_scale < 0", [](pitmg_options& x) { x.mu_scale = -1.0; }},
      {"cycle 5", [](pitmg_options& x) { x.cycle = 5; }},
      {"smoother 9", [](pitmg_options& x) { x.smoother = 9; }},
      {"GS with FP32", [](pitmg_options& x) { x.smoother = 1; x.smoother_fp32 = 1; }},
      {"unlifted 2", [](pitmg_options& x) { x.unlifted = 2; }},
      {"coarsen 3", [](pitmg_options& x) { x.coarsen = 3; }},
      {"coarsen 4 variant 1", [](pitmg_options& x) { x.coarsen = 4; x.transfer_variant = 1; }},
      {"nu_pre < 0", [](pitmg_options& x) { x.nu_pre = -1; }},
      {"restart 0", [](pitmg_options& x) { x.restart = 0; }},
  };
  for (const BadOpt& b : bad_opts) {
    pitmg_options x = o;
    b.set(x);
    pitmg_problem pb = base();
    setup_fails(&pb, &x, PITMG_ERR_INVALID, b.what);
  }
  {
    pitmg_options x = o;
    x.coarsen = 4;                   // 16 % 4^2 == 0, but the level sizes follow c
    pitmg_problem pb = base();
    pb.n = 8;                        // 8 % 16 != 0
    setup_fails(&pb, &x, PITMG_ERR_INVALID, "n not divisible by coarsen^(L-1)");
  }

  // every entry point with a NULL handle
  double v[8] = {0};
  int its = 0, cfg[4] = {0};
  pitmg_stats st;
  expect(pitmg_refactor(nullptr, nullptr) < 0, "refactor NULL");
  expect(pitmg_set_options(nullptr, &o) < 0, "set_options NULL");
  expect(pitmg_apply(nullptr, 0, v, v) < 0, "apply NULL");
  expect(pitmg_jacobi_sweep(nullptr, 0, v, v, v) < 0, "sweep NULL");
  expect(pitmg_coarse_solve(nullptr, v, v, &its) < 0, "coarse NULL");
  expect(pitmg_coarse_solve_noalloc(nullptr, v, v, &its) < 0, "coarse noalloc NULL");
  expect(pitmg_vcycle(nullptr, v, v) < 0, "vcycle NULL");
  expect(pitmg_fgmres_solve(nullptr, v, v, 1e-10, 0, &st) < 0, "solve NULL");
  expect(pitmg_unlifted_apply(nullptr, v, v) < 0, "unlifted apply NULL");
  expect(pitmg_unlifted_fgmres_solve(nullptr, v, v, 1e-10, 0, &st) < 0, "unlifted solve NULL");
  expect(pitmg_autotune(nullptr, cfg) < 0, "autotune NULL");
  expect(pitmg_set_sweep_shapes(nullptr, cfg) < 0, "shapes NULL");
  expect(pitmg_set_handoff_wait(nullptr, 1.0) < 0, "handoff NULL");
  expect(pitmg_profile_enable(nullptr, 1) < 0, "profile NULL");
  int lev = 0, k = 0;
  expect(pitmg_failed_block(nullptr, &lev, &k) < 0, "failed_block NULL");
  int nl = 0, fl = 0;
  expect(pitmg_level_info(nullptr, 0, &nl, &fl) < 0, "level_info NULL");

  // the Burgers dogleg's validation (before any device work)
  {
    double w0[16] = {0};
    pitmg_burgers bp{16, 10, 3, 1.0, 1e5, w0};       // 10 steps, 3 levels: 10 % 4 != 0
    pitmg_dogleg_params dp;
    pitmg_default_dogleg_params(&dp);
    expect(dp.lin_tol == 1e-6 && dp.maxit == 50, "dogleg defaults");
    pitmg_dogleg_stats ds[2];
    const double nus[2] = {0.1, 0.0};
    expect(pitmg_burgers_dogleg(&bp, &o, nus, 2, v, &dp, ds, nullptr) == PITMG_ERR_INVALID,
           "dogleg: n not divisible");
    bp.n = 12;
    expect(pitmg_burgers_dogleg(&bp, &o, nullptr, 2, v, &dp, ds, nullptr) == PITMG_ERR_INVALID,
           "dogleg: NULL viscosities");
    const double bad[1] = {-1.0};
    expect(pitmg_burgers_dogleg(&bp, &o, bad, 1, v, &dp, ds, nullptr) == PITMG_ERR_INVALID,
           "dogleg: negative viscosity");
    bp.gamma = 0.0;
    expect(pitmg_burgers_residual(&bp, 0.1, v, v, nullptr) == PITMG_ERR_INVALID,
           "residual: gamma 0");
    expect(pitmg_burgers_residual(nullptr, 0.1, v, v, nullptr) == PITMG_ERR_INVALID,
           "residual: NULL problem");
    expect(std::strlen(pitmg_burgers_last_error()) > 0, "dogleg message");
  }

  // past validation: device calls fail without a GPU; the handle is kept
  // for its message and destroyed
  {
    pitmg_problem pb = base();
    pitmg_handle* h = nullptr;
    const int rc = pitmg_setup(&h, &pb, &o, nullptr);
    if (rc == PITMG_OK) {
      std::fprintf(stderr, "note: a device is present; setup succeeded\n");
    } else {
      expect(rc == PITMG_ERR_HIP || rc == PITMG_ERR_OOM, "setup error without a device");
      if (h) expect(std::strlen(pitmg_last_error(h)) > 0, "error message");
    }
    pitmg_destroy(h);
  }
  std::printf("host sanitizer driver: %d failure(s)\n", failures);
  return failures == 0 ? 0 : 1;
}
