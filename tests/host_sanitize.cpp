// Host-side checks of the library's argument validation and host coefficient
// code, built with AddressSanitizer and UndefinedBehaviorSanitizer on the host
// code (the device code is the library's ordinary build).  Every call below
// must fail with HSDC_EINVAL before any device work, or compute on the host
// only; a sanitizer report or a failed expectation ends the process with a
// non-zero status.  No GPU is needed.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "hsdc.h"

static int failures = 0;

static void expect(bool ok, const char *what, int line) {
  if (!ok) {
    std::printf("FAILED line %d: %s\n", line, what);
    ++failures;
  }
}
#define EXPECT(cond) expect((cond), #cond, __LINE__)

static hsdc_problem problem(int dim, int nx, int ny, int nz) {
  hsdc_problem p;
  std::memset(&p, 0, sizeof p);
  p.dim = dim;
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.dx = 0.025;
  p.sigma[0] = p.sigma[1] = p.sigma[2] = 1.0;
  p.chi = 1400.0;
  p.Cm = 1.0;
  p.g_scale[0] = p.g_scale[1] = p.g_scale[2] = 1.0;
  p.stim_amp = 50.0;
  p.stim_dur = 1.0;
  return p;
}

static hsdc_method method() {
  hsdc_method m;
  std::memset(&m, 0, sizeof m);
  m.levels = 1;
  m.M[0] = 6;
  m.M[1] = 3;
  m.space_coarsen = 1;
  m.P = 1;
  m.dt = 0.05;
  m.max_iter = 6;
  m.cg_rtol = 1e-12;
  m.cg_maxit = 100;
  return m;
}

static bool rejected_init(const hsdc_problem &p, const hsdc_method &m) {
  hsdc_ctx *ctx = reinterpret_cast<hsdc_ctx *>(0x1);
  const hsdc_status st = hsdc_init_state(&p, &m, nullptr, nullptr, &ctx);
  const char *msg = hsdc_last_error(nullptr);
  return st == HSDC_EINVAL && ctx == nullptr && msg && std::strlen(msg) > 0;
}

int main() {
  // collocation coefficients on the host: Radau IIA nodes in (0, 1], increasing, c_M = 1
  for (int M = 1; M <= HSDC_MAX_M; ++M) {
    double c[HSDC_MAX_M + 1];
    for (double &v : c) v = -1.0;
    EXPECT(hsdc_colloc_coefficients(M, 0, nullptr, nullptr, c, nullptr) == HSDC_OK);
    for (int i = 0; i < M; ++i) EXPECT(c[i] > 0.0 && c[i] <= 1.0);
    for (int i = 1; i < M; ++i) EXPECT(c[i] > c[i - 1]);
    EXPECT(std::fabs(c[M - 1] - 1.0) < 1e-15);
    EXPECT(c[M] == -1.0);  // nothing written past M
  }
  EXPECT(hsdc_colloc_coefficients(0, 0, nullptr, nullptr, nullptr, nullptr) == HSDC_EINVAL);
  EXPECT(hsdc_colloc_coefficients(HSDC_MAX_M + 1, 0, nullptr, nullptr, nullptr, nullptr) == HSDC_EINVAL);
  EXPECT(hsdc_colloc_coefficients(4, 8, nullptr, nullptr, nullptr, nullptr) == HSDC_EINVAL);

  // problems the library must reject
  const hsdc_method m = method();
  {
    hsdc_problem p;
    const double nan = std::nan("");
    struct Bad { int dim, nx, ny, nz; double dx, sigma0, chi, Cm, gs0, stim_dur; } bad[] = {
        {0, 16, 1, 1, 0.025, 1, 1400, 1, 1, 1},   {4, 16, 1, 1, 0.025, 1, 1400, 1, 1, 1},
        {1, 0, 1, 1, 0.025, 1, 1400, 1, 1, 1},    {1, 16, 2, 1, 0.025, 1, 1400, 1, 1, 1},
        {2, 16, 16, 2, 0.025, 1, 1400, 1, 1, 1},  {1, 16, 1, 1, 0.0, 1, 1400, 1, 1, 1},
        {1, 16, 1, 1, nan, 1, 1400, 1, 1, 1},     {1, 16, 1, 1, 0.025, -1, 1400, 1, 1, 1},
        {1, 16, 1, 1, 0.025, nan, 1400, 1, 1, 1}, {1, 16, 1, 1, 0.025, 1, 0, 1, 1, 1},
        {1, 16, 1, 1, 0.025, 1, 1400, 0, 1, 1},   {1, 16, 1, 1, 0.025, 1, 1400, 1, INFINITY, 1},
        {1, 16, 1, 1, 0.025, 1, 1400, 1, 1, -1},  {3, 2000, 2000, 2000, 0.025, 1, 1400, 1, 1, 1},
        {1, -5, 1, 1, 0.025, 1, 1400, 1, 1, 1},
    };
    p = problem(2, 16, 16, 1);
    p.fd_order = 3;
    EXPECT(rejected_init(p, m));
    for (const Bad &b : bad) {
      p = problem(b.dim, b.nx, b.ny, b.nz);
      p.dx = b.dx;
      p.sigma[0] = b.sigma0;
      p.chi = b.chi;
      p.Cm = b.Cm;
      p.g_scale[0] = b.gs0;
      p.stim_dur = b.stim_dur;
      EXPECT(rejected_init(p, m));
    }
    EXPECT(hsdc_init_state(nullptr, &m, nullptr, nullptr, nullptr) == HSDC_EINVAL);
  }

  // methods the library must reject
  {
    const hsdc_problem p = problem(3, 8, 6, 4);
    const hsdc_problem podd = problem(2, 15, 16, 1);
    hsdc_problem p4 = problem(2, 16, 16, 1);
    p4.fd_order = 4;
    for (int k = 0; k < 22; ++k) {
      hsdc_method b = method();
      const hsdc_problem *pp = &p;
      switch (k) {
        case 0: b.levels = 0; break;
        case 1: b.levels = 3; break;
        case 2: b.M[0] = 0; break;
        case 3: b.M[0] = HSDC_MAX_M + 1; break;
        case 4: b.levels = 2; b.P = 2; b.M[1] = 0; break;
        case 5: b.levels = 2; b.P = 2; b.space_coarsen = 3; break;
        case 6: b.levels = 2; b.P = 2; b.space_coarsen = 2; pp = &podd; break;
        case 7: b.P = 0; break;
        case 8: b.P = 5000; break;
        case 9: b.dt = 0.0; break;
        case 10: b.dt = INFINITY; break;
        case 11: b.max_iter = 0; break;
        case 12: b.tol = std::nan(""); break;
        case 13: b.cg_rtol = 0.0; break;
        case 14: b.cg_rtol = 1.0; break;
        case 15: b.cg_maxit = 0; break;
        case 16: b.levels = 2; b.P = 2; b.coarse_fp32 = 2; break;
        case 17: b.solver = 4; break;
        case 18: b.coarse_cg_rtol = 2.0; break;
        case 19: b.residual_norm = 2; break;
        case 20: b.solver = 3; b.levels = 2; b.P = 2; b.coarse_fp32 = 1; break;
        case 21: b.solver = 0; pp = &p4; break;  // the fourth-order stencil needs DCT-II
      }
      EXPECT(rejected_init(*pp, b));
    }
  }

  // batches the library must reject
  {
    hsdc_problem probs[2] = {problem(2, 12, 10, 1), problem(2, 8, 14, 1)};
    hsdc_ctx *ctx = nullptr;
    EXPECT(hsdc_init_batch(nullptr, 0, &m, nullptr, nullptr, &ctx) == HSDC_EINVAL && !ctx);
    EXPECT(hsdc_init_batch(probs, -1, &m, nullptr, nullptr, &ctx) == HSDC_EINVAL && !ctx);
    probs[1].dx = 0.03;
    EXPECT(hsdc_init_batch(probs, 2, &m, nullptr, nullptr, &ctx) == HSDC_EINVAL && !ctx);
    probs[1].dx = 0.025;
    probs[1].sigma[0] = 2.0;
    EXPECT(hsdc_init_batch(probs, 2, &m, nullptr, nullptr, &ctx) == HSDC_EINVAL && !ctx);
    hsdc_method pf = method();
    pf.levels = 2;
    pf.P = 2;
    probs[1].sigma[0] = 1.0;
    EXPECT(hsdc_init_batch(probs, 2, &pf, nullptr, nullptr, &ctx) == HSDC_EINVAL && !ctx);
  }

  // calls on a NULL context or adjoint handle
  {
    double res[4];
    int32_t conv = 0;
    hsdc_stats st;
    EXPECT(hsdc_advance(nullptr, 1) == HSDC_EINVAL);
    EXPECT(hsdc_sdc_sweep(nullptr, 0, 0, 1) == HSDC_EINVAL);
    EXPECT(hsdc_pfasst_iter(nullptr, res, &conv) == HSDC_EINVAL);
    EXPECT(hsdc_residual(nullptr, 0, res) == HSDC_EINVAL);
    EXPECT(hsdc_current_step(nullptr) == -1);
    EXPECT(hsdc_tune(nullptr, 512, -1) == HSDC_EINVAL);
    EXPECT(hsdc_use_graph(nullptr, 1) == HSDC_EINVAL);
    EXPECT(hsdc_get_stats(nullptr, &st) == HSDC_EINVAL);
    EXPECT(hsdc_profile_enable(nullptr, 1) == HSDC_EINVAL);
    hsdc_destroy(nullptr);
    EXPECT(hsdc_misfit_backward(nullptr, nullptr, nullptr, nullptr) == HSDC_EINVAL);
    hsdc_adj_destroy(nullptr);
  }

  // stateless entry points with malformed arguments
  {
    const hsdc_problem p = problem(2, 16, 16, 1);
    hsdc_problem bad = p;
    bad.nx = 0;
    double d = 0.0;
    EXPECT(hsdc_phi(-1, nullptr, 1, nullptr, nullptr) == HSDC_EINVAL);
    EXPECT(hsdc_phi(10, nullptr, 0, nullptr, nullptr) == HSDC_EINVAL);
    EXPECT(hsdc_phi(10, &d, HSDC_MAX_M + 1, &d, nullptr) == HSDC_EINVAL);
    EXPECT(hsdc_ionic_eval(-1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
           HSDC_EINVAL);
    EXPECT(hsdc_ionic_eval(4, nullptr, nullptr, &d, &d, &d, &d, nullptr) == HSDC_EINVAL);
    EXPECT(hsdc_apply_diffusion(&bad, &d, &d, nullptr) == HSDC_EINVAL);
    EXPECT(hsdc_apply_diffusion(nullptr, &d, &d, nullptr) == HSDC_EINVAL);
    EXPECT(hsdc_diffusion_solve(&bad, 0.01, &d, &d, 1e-12, 100, nullptr, nullptr) == HSDC_EINVAL);
    EXPECT(hsdc_diffusion_solve(&p, 0.01, &d, &d, 0.0, 100, nullptr, nullptr) == HSDC_EINVAL);
    EXPECT(hsdc_diffusion_solve(&p, 0.01, &d, &d, 1e-12, 0, nullptr, nullptr) == HSDC_EINVAL);
    EXPECT(hsdc_diffusion_solve(&p, -1.0, &d, &d, 1e-12, 10, nullptr, nullptr) == HSDC_EINVAL);
    EXPECT(hsdc_diffusion_solve_noalloc(&p, 0.01, nullptr, &d, 1e-12, 10, nullptr, nullptr) ==
           HSDC_EINVAL);
    const hsdc_problem big = problem(2, 1024, 513, 1);
    EXPECT(hsdc_diffusion_solve_noalloc(&big, 0.01, &d, &d, 1e-12, 100, nullptr, nullptr) ==
           HSDC_EINVAL);
    EXPECT(std::strstr(hsdc_last_error(nullptr), "HSDC_NOALLOC_MAX_NODES") != nullptr);
    hsdc_adj *adj = reinterpret_cast<hsdc_adj *>(0x1);
    const int64_t probe = 3;
    double loss = 0.0;
    EXPECT(hsdc_misfit_forward(&p, &m, nullptr, 0, 1, 1, &probe, &d, &loss, &adj, nullptr) ==
           HSDC_EINVAL);
    EXPECT(adj == nullptr);
    EXPECT(hsdc_misfit_forward(&p, &m, nullptr, 4, 1, 1, nullptr, &d, &loss, &adj, nullptr) ==
           HSDC_EINVAL);
    hsdc_method pf = method();
    pf.levels = 2;
    pf.P = 2;
    EXPECT(hsdc_misfit_forward(&p, &pf, nullptr, 4, 1, 1, &probe, &d, &loss, &adj, nullptr) ==
           HSDC_EINVAL);
  }

  if (failures) {
    std::printf("%d host checks failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
