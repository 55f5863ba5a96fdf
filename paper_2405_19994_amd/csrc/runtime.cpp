// runtime.cpp -- host runtime of libhsdc: context, workspace, the HSDC sweep
// driver (Sec. 3.1.3), serial stepping, two-level PFASST (Sec. 3.2,
// Algorithm 1) and the C ABI of include/hsdc.h.
//
// Sweep in node-to-node form.  With R_i = (P_i - C_i)(y^k) + u + tau_i the
// right-hand side of eq. prec_picard, the forward substitution with P of
// eq. def_P reads, node by node,
//     (I - dt d_i f_I) y^{k+1}_i = y^{k+1}_{i-1} + (R_i - R_{i-1})
//         + dt d_i [ f_E(y^{k+1}_{i-1}) + phi_1(d_i dt Lambda(u)) (f_e(y^{k+1}_{i-1})
//                    + Lambda(u)(u - y^{k+1}_{i-1})) ]
// where R_i - R_{i-1} = dt sum_j (a_ij - a_{i-1,j}) g_j(y^k) - dt d_i Phi_i(y^k)
// + tau_i - tau_{i-1} uses only the previous iterate (kernel k_assemble) and
// the implicit part acts on V only (a CG solve).  Both sides use the start value
// u of the new iterate as anchor: y^k enters with y^k_{n,0} replaced by u.
//
// FP32 coarse level (coarse_fp32): the cell model, its stored terms (G,
// Lambda) and the CG work vectors are FP32, while states, K V, the assembled
// right-hand side and the CG solution accumulate in FP64.  An FP32 term enters
// both sides of a sweep from identical inputs at the fixed point and cancels
// there, and the coarse CG solves the warm-start correction to a relative
// accuracy, so FP32 rounding shrinks with the PFASST defect instead of
// setting a floor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "hsdc_internal.h"

namespace hsdc {
bool make_colloc(int M, double dt, Colloc &co);
void transfer_matrix(int Mfrom, const double *c_from, int Mto, const double *c_to, double *out);
}  // namespace hsdc

using namespace hsdc;

namespace hsdc {
// Serial steps of a 1D mesh of at most 256 nodes in one launch of one
// workgroup (hsdc_small.hip): y_n in stage 0 of st, y_{n+nsteps} left there;
// *steps_done receives the steps completed, negated when the last of them
// turned a state non-finite (the launch stops after that step).
hipError_t launch_small_steps(hipStream_t s, const Grid &g, const Stages &st, const Colloc &co,
                              const Stim &stim, double gs0, double gs1, double gs2, int K,
                              int nsteps, int *steps_done);

int default_cg_tile(int nx, int ny) {
  for (int t : {8, 7, 5})  // register tiles 48 x 32, 48 x 24, 48 x 16
    if (cg_start_tiles_of(nx, ny, t) >= 192) return t;
  return 6;  // 48 x 8
}
}  // namespace hsdc

namespace {

thread_local std::string g_free_error;

struct HipFail {
  hipError_t e;
  const char *what;
};

// A failed status raised inside a level callback (the message is already set).
struct StatusFail {
  hsdc_status st;
};

#define HIPC(call)                                  \
  do {                                              \
    hipError_t e_ = (call);                         \
    if (e_ != hipSuccess) throw HipFail{e_, #call}; \
  } while (0)

// One level's workspace; T is the type of its cell-model terms and CG work
// vectors (float only on an FP32 coarse level); states are FP64 on every level.
template <class T>
struct LevelT {
  Grid g{};
  Colloc co{};
  StagesT<T> st{};
  int P = 0;
  double *stim_w = nullptr;
  double *kface[3] = {nullptr, nullptr, nullptr};
  // CG workspace
  T *cg_r[2] = {nullptr, nullptr}, *cg_w[2] = {nullptr, nullptr};
  T *cg_s[2] = {nullptr, nullptr}, *cg_p = nullptr;
  double *cg_part = nullptr;
  // Chebyshev steps (FP64 levels with solver 0 or 1): second iterate buffer and
  // the parameters of every (slice, collocation node) operator
  double *cheb_x = nullptr;      // [P][Np]
  ChebTab *cheb_tab = nullptr;   // [P][M]
  // DCT-II solves (solver 3): transforms and eigenvalues of the level's mesh
  DctPlan dct{};
  bool direct = false;
  CgScalars *cg_sc = nullptr;       // [P][2]
  CgScalars *cg_sc_host = nullptr;  // [P][2]
  int cg_nblk = 0;
  int64_t cg_pstride = 0;
  bool tiled_start = false;  // CG starts with the tiled Chebyshev launch (2D meshes)
  // residual
  double *res_part = nullptr, *res_out = nullptr, *res_out_host = nullptr;
  int res_nblk = 0;
  // PFASST
  double *U = nullptr;    // [P][NF][Np] start values of a Q sweep
  double *Sz = nullptr;   // coarse: copy of the restricted fine iterate
  double *RI = nullptr;   // fine: time-restricted integrals [P][Mc][NF][Np]; coarse: FAS term
  double *y0c = nullptr;  // coarse: restricted block start value [NF][Np]
  // middle level of three: S (I + tau) restricted in time to the coarsest
  // level's nodes [P][M_2][NF][Np] (tau of the coarsest level before its own part)
  double *RI2 = nullptr;
  int cg_pred[16][MAXM];  // iteration budget per (sweep index, node)
  int cg_umax[16][MAXM];  // most iterations used since the last relaxation (graph mode;
                          // -1: no solve checked since)
};
using Level = LevelT<double>;

// A diffusion solve whose outcome is checked later (budgeted mode).
struct CgLogEntry {
  int lev, s0, ns, i, row, parity, off, budget;
  bool cheb;
  int margin;  // spare launches of the solve's budget
};

}  // namespace

namespace {
enum ProfClass { PC_NODE, PC_ASSEMBLE, PC_CGINIT, PC_CGITER, PC_EVAL, PC_SPMV, PC_RESIDUAL,
                 PC_TRANSFER, PC_COPY, PC_FAS, PC_CHEB, PC_DCT, PC_COUNT };
const char *kProfNames[PC_COUNT] = {"node_update", "assemble", "cg_init", "cg_iter", "eval_stages",
                                    "spmv", "residual", "transfer", "copy", "fas_integrals",
                                    "cheb_iter", "dct_solve"};
struct ProfPending {
  int cls;
  int launches;
  double bytes;
  hipEvent_t e0, e1;
};
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<ProfPending> pending;
  int64_t launches[PC_COUNT] = {};
  double ms[PC_COUNT] = {};
  double bytes[PC_COUNT] = {};
};
}  // namespace

struct hsdc_ctx {
  hipStream_t s = nullptr;
  hsdc_problem prob{};
  hsdc_method meth{};
  Level L[3];             // fine level, (FP64) coarse or middle level, coarsest level
  LevelT<float> Lf;       // coarse level when coarse_fp32
  bool cf32 = false;
  // ragged batch of independent tissues (one per slice of a serial context)
  bool batch = false;
  std::vector<int64_t> tissue_N;  // nodes per slice (batch)
  int32_t *rag = nullptr;         // device [P][RAG] tissue dimensions and divisors
  std::vector<std::pair<int, int>> tissue_dims;  // nx, ny per slice (batch)
  int nlev = 1;
  double *y0blk = nullptr;  // block (or step) start value [NF][Np_f]
  double *Rt = nullptr, *Tt = nullptr;  // device transfer matrices, levels 0 and 1
  double *Rt2 = nullptr, *Tt2 = nullptr;  // levels 1 and 2 (three levels)
  // PFASST with prefix_stop: slices 0..a0-1 have stopped iterating; the last
  // residual of every slice
  int a0 = 0;
  std::vector<double> rel_last;
  int64_t step = 0;
  int64_t *d_step = nullptr;  // device copy of step, read by the kernels
  int sweeps_done = 0;  // serial: sweeps applied to the current step
  int sweep_index = 0;
  bool pfasst = false;
  bool block_ready = false;
  bool ri_fresh = false;  // fine RI holds the restricted integrals of the current iterate
  // serial mode: stages 1..M of the current step are the spread of stage 0 and
  // only their V (the CG warm starts) is stored; the first sweep reads stage 0
  bool spread_pending = false;
  hsdc_stats stats{};
  std::string err;
  std::vector<void *> allocs;
  std::vector<void *> host_allocs;
  Stim stim[3]{};
  // budgeted CG: solves enqueued without a host synchronisation, verified in
  // bulk at the end of a step; a step with an unconverged solve is recomputed
  bool safe_cg = true;
  CgScalars *cg_log = nullptr;   // pinned host copy of cg_dlog
  CgScalars *cg_dlog = nullptr;  // device: final scalars of every budgeted solve
  int cg_log_cap = 0, cg_log_used = 0;
  int cg_fails = 0;  // unconverged budgeted solves found by flush_cg_log
  // when set, flush_cg_log appends the CG launches each fine-level solve used
  // (in the order the solves were enqueued): the misfit forward's record,
  // which its backward run's recomputed steps take as their budgets
  std::vector<int> *cg_record = nullptr;
  bool nonfinite = false;  // a solve met a NaN or Inf (reset by every stepping call)
  std::vector<CgLogEntry> cg_pending;
  Profiler prof;
  // graph replay of serial steps (hsdc_use_graph): one captured step, replayed
  // while the CG budgets it was captured with stay in force
  bool graph_on = false;
  // serial steps of a small 1D mesh in one single-workgroup launch (hsdc_single_block)
  bool single_block = true;
  int *d_small = nullptr;  // device: steps the last such launch completed
  bool graph_dirty = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<CgLogEntry> graph_pending;
  int graph_log_used = 0;
  int64_t graph_sweeps = 0, graph_ionic = 0;  // counters of one captured step
  int64_t graph_steps = 0;
  double *ybak = nullptr;  // [P][NF][Np] start value of the step being replayed
  hsdc_stats graph_delta{};  // PFASST: counters of one captured coarse part
  int64_t coarse_redo = 0;   // PFASST coarse parts run again (a missed budgeted solve)
  // launch tuning (hsdc_tune): CG block cap and iteration-budget margin
  int tune_cg_blocks = 512;
  int tune_cg_margin = -1;  // < 0: the default of each level (cg_margin())
};

namespace {

hsdc_status fail(hsdc_ctx *c, hsdc_status st, const std::string &msg) {
  if (c)
    c->err = msg;
  else
    g_free_error = msg;
  return st;
}

// Calls fn with the coarse level in its storage type.
template <class Fn>
void with_coarse(hsdc_ctx *c, Fn &&fn) {
  if (c->cf32)
    fn(c->Lf);
  else
    fn(c->L[1]);
}

// Mesh nodes of slices [s0, s0+ns) of level L (a batch's tissues differ).
template <class T>
double slice_nodes(const hsdc_ctx *c, const LevelT<T> &L, int s0, int ns) {
  if (!c->batch) return (double)L.g.N * ns;
  double n = 0.0;
  for (int k = s0; k < s0 + ns; ++k) n += (double)c->tissue_N[k];
  return n;
}

// Relative tolerance of the diffusion solves on level lev (an FP32 coarse level
// measures it against the warm start's residual).
double level_rtol(const hsdc_ctx *c, int lev) {
  if (lev == 0) return c->meth.cg_rtol;
  if (c->meth.coarse_cg_rtol > 0) return c->meth.coarse_cg_rtol;
  return c->cf32 ? 1e-5 : c->meth.cg_rtol;
}

// Spare launches of a budget: the tuned margin, or by default none after the
// tiled start (whose solves have needed no CG iteration) and one otherwise.
int cg_margin(const hsdc_ctx *c, bool tiled) {
  return c->tune_cg_margin >= 0 ? c->tune_cg_margin : (tiled ? 0 : 1);
}

int (&pred_table(hsdc_ctx *c, int lev))[16][MAXM] {
  return (lev == 1 && c->cf32) ? c->Lf.cg_pred : c->L[lev].cg_pred;
}
int (&umax_table(hsdc_ctx *c, int lev))[16][MAXM] {
  return (lev == 1 && c->cf32) ? c->Lf.cg_umax : c->L[lev].cg_umax;
}
// The level whose budgeted solves a graph replays: the fine level of a serial
// step, the coarse level of a PFASST iteration's coarse part.
int graph_level(const hsdc_ctx *c) { return c->pfasst ? 1 : 0; }

// ---- kernel timing -----------------------------------------------------------
void prof_harvest(hsdc_ctx *c) {
  Profiler &P = c->prof;
  if (P.pending.empty()) return;
  HIPC(hipStreamSynchronize(c->s));
  for (ProfPending &q : P.pending) {
    float ms = 0.0f;
    HIPC(hipEventElapsedTime(&ms, q.e0, q.e1));
    P.launches[q.cls] += q.launches;
    P.ms[q.cls] += ms;
    P.bytes[q.cls] += q.bytes;
    P.pool.push_back(q.e0);
    P.pool.push_back(q.e1);
  }
  P.pending.clear();
}

hipEvent_t prof_event(hsdc_ctx *c) {
  Profiler &P = c->prof;
  if (P.pool.empty()) {
    hipEvent_t e;
    HIPC(hipEventCreate(&e));
    return e;
  }
  hipEvent_t e = P.pool.back();
  P.pool.pop_back();
  return e;
}

// Brackets one launch with events when timing is enabled.
struct ProfScope {
  hsdc_ctx *c;
  int cls;
  double bytes;
  hipEvent_t e0 = nullptr;
  ProfScope(hsdc_ctx *c_, int cls_, double bytes_) : c(c_), cls(cls_), bytes(bytes_) {
    if (c->prof.on) {
      if (c->prof.pending.size() >= 4096) prof_harvest(c);
      e0 = prof_event(c);
      HIPC(hipEventRecord(e0, c->s));
    }
  }
  // nlaunch > 1: the bracket holds a run of back-to-back launches of one class
  void end(int nlaunch = 1) {
    if (!e0) return;
    hipEvent_t e1 = prof_event(c);
    HIPC(hipEventRecord(e1, c->s));
    c->prof.pending.push_back(ProfPending{cls, nlaunch, bytes, e0, e1});
    e0 = nullptr;
  }
};

#define PLAUNCH(ctx, cls, bytes, call) \
  do {                                 \
    ProfScope ps_((ctx), (cls), (bytes)); \
    HIPC(call);                        \
    ps_.end();                         \
  } while (0)

template <class T>
T *dalloc(hsdc_ctx *c, size_t n) {
  void *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw HipFail{e, "hipMalloc"};
  c->allocs.push_back(p);
  HIPC(hipMemsetAsync(p, 0, n * sizeof(T), c->s));
  return (T *)p;
}

template <class T>
T *halloc(hsdc_ctx *c, size_t n) {
  void *p = nullptr;
  hipError_t e = hipHostMalloc(&p, n * sizeof(T), hipHostMallocDefault);
  if (e != hipSuccess) throw HipFail{e, "hipHostMalloc"};
  c->host_allocs.push_back(p);
  return (T *)p;
}

int64_t pad64(int64_t n) { return (n + 63) / 64 * 64; }

bool check_problem(const hsdc_problem *p, std::string &why) {
  if (!p) return why = "problem is NULL", false;
  if (p->dim < 1 || p->dim > 3) return why = "dim must be 1, 2 or 3", false;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return why = "nx, ny, nz must be >= 1", false;
  if (p->dim < 2 && p->ny != 1) return why = "ny must be 1 for dim < 2", false;
  if (p->dim < 3 && p->nz != 1) return why = "nz must be 1 for dim < 3", false;
  if (!(p->dx > 0) || !std::isfinite(p->dx)) return why = "dx must be > 0", false;
  if (!(p->chi > 0) || !(p->Cm > 0)) return why = "chi and Cm must be > 0", false;
  for (int a = 0; a < 3; ++a)
    if (!(p->sigma[a] >= 0) || !std::isfinite(p->sigma[a])) return why = "sigma must be >= 0", false;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->g_scale[a])) return why = "g_scale must be finite", false;
  if (!std::isfinite(p->stim_amp) || !std::isfinite(p->stim_t0) || !(p->stim_dur >= 0))
    return why = "stimulus parameters must be finite, stim_dur >= 0", false;
  if (p->fd_order != 0 && p->fd_order != 2 && p->fd_order != 4)
    return why = "fd_order must be 2 (or 0) or 4", false;
  if (p->fd_order == 4 && p->sigma_node)
    return why = "fd_order 4 takes a uniform sigma (sigma_node NULL)", false;
  const double N = (double)p->nx * p->ny * p->nz;
  if (N > 2.0e9) return why = "mesh too large", false;
  return true;
}

bool check_method(const hsdc_method *m, const hsdc_problem *p, std::string &why) {
  if (!m) return why = "method is NULL", false;
  if (m->levels < 1 || m->levels > 3) return why = "levels must be 1, 2 or 3", false;
  for (int l = 0; l < m->levels; ++l)
    if (m->M[l] < 1 || m->M[l] > HSDC_MAX_M) return why = "M must be in 1..8", false;
  if (m->levels >= 2 && m->space_coarsen != 1 && m->space_coarsen != 2)
    return why = "space_coarsen must be 1 or 2", false;
  if (m->levels >= 2 && m->space_coarsen == 2) {
    // every coarsening halves each axis with more than one node
    const int q = m->levels == 3 ? 4 : 2;
    if ((p->nx > 1 && p->nx % q) || (p->ny > 1 && p->ny % q) || (p->nz > 1 && p->nz % q))
      return why = m->levels == 3 ? "space_coarsen 2 with three levels needs mesh sizes divisible by 4"
                                  : "space_coarsen 2 needs even mesh sizes",
             false;
    if (p->sigma_node) return why = "space_coarsen 2 needs a uniform sigma", false;
  }
  if (m->levels == 3 && m->coarse_fp32)
    return why = "three levels run in FP64 (coarse_fp32 0)", false;
  if (m->prefix_stop != 0 && m->prefix_stop != 1) return why = "prefix_stop must be 0 or 1", false;
  if (m->prefix_stop && m->levels != 2) return why = "prefix_stop is for two levels", false;
  if (m->P < 1 || m->P > 4096) return why = "P must be in 1..4096", false;
  if (!(m->dt > 0) || !std::isfinite(m->dt)) return why = "dt must be > 0", false;
  if (m->max_iter < 1) return why = "max_iter must be >= 1", false;
  if (!std::isfinite(m->tol)) return why = "tol must be finite", false;
  if (!(m->cg_rtol > 0) || !(m->cg_rtol < 1)) return why = "cg_rtol must be in (0, 1)", false;
  if (m->cg_maxit < 1) return why = "cg_maxit must be >= 1", false;
  if (m->coarse_fp32 != 0 && m->coarse_fp32 != 1) return why = "coarse_fp32 must be 0 or 1", false;
  if (m->solver < 0 || m->solver > 3)
    return why = "solver must be 0 (CG), 1 (Chebyshev), 2 (CG from the warm start) or 3 (DCT-II)",
           false;
  if (m->solver == 3 && p->sigma_node)
    return why = "solver 3 (DCT-II) needs a uniform sigma", false;
  if (m->solver == 3 && m->levels == 2 && m->coarse_fp32)
    return why = "solver 3 (DCT-II) needs FP64 levels (coarse_fp32 0)", false;
  if (p->fd_order == 4 && m->solver != 3)
    return why = "fd_order 4 is solved by solver 3 (DCT-II)", false;
  if (!std::isfinite(m->coarse_cg_rtol) || !(m->coarse_cg_rtol < 1))
    return why = "coarse_cg_rtol must be finite and < 1", false;
  if (m->residual_norm != 0 && m->residual_norm != 1)
    return why = "residual_norm must be 0 (over all fields) or 1 (per field)", false;
  return true;
}

Grid make_grid(const hsdc_problem &p, int nx, int ny, int nz, double dx) {
  Grid g{};
  g.dim = p.dim;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.N = (int64_t)nx * ny * nz;
  g.Np = pad64(g.N);
  g.fx = make_fastdiv((uint32_t)nx);
  g.fy = make_fastdiv((uint32_t)ny);
  g.nub = kDefaultNodeBlock;
  g.ctile = default_cg_tile(nx, ny);
  g.ptile = 0;
  g.order = p.fd_order == 4 ? 4 : 2;
  const double s = 1.0 / (dx * dx * p.chi * p.Cm);
  g.cx = p.sigma[0] * s;
  g.cy = p.sigma[1] * s;
  g.cz = p.sigma[2] * s;
  return g;
}

// Per-node conductivity: face coefficient between p and p + e_axis is the
// harmonic mean of the two node values over dx^2 chi Cm (0 on the last layer).
// Face coefficients along axis a of an nx x ny x nz mesh from host sigma.
std::vector<double> face_coeffs(int a, int nx, int ny, int nz, const std::vector<double> &s,
                                double sc) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t strides[3] = {1, nx, (int64_t)nx * ny};
  const int sizes[3] = {nx, ny, nz};
  std::vector<double> k(N, 0.0);
  for (int64_t p = 0; p < N; ++p) {
    const int coord = (int)((p / strides[a]) % sizes[a]);
    if (coord < sizes[a] - 1) {
      const double sp = s[p], sq = s[p + strides[a]];
      k[p] = (sp + sq > 0) ? 2.0 * sp * sq / (sp + sq) * sc : 0.0;
    }
  }
  return k;
}

// Gershgorin bound on the spectrum of -K (symmetric, positive semidefinite):
// twice the largest sum of the face coefficients around a node.
double lam_uniform(int dim, int nx, int ny, int nz, double cx, double cy, double cz) {
  const int n[3] = {nx, ny, nz};
  const double k[3] = {cx, cy, cz};
  double row = 0.0;
  for (int a = 0; a < dim; ++a) row += k[a] * std::min(2, n[a] - 1);
  return 2.0 * row;
}

double lam_faces(int dim, int nx, int ny, int nz, const std::vector<double> *k) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t strides[3] = {1, nx, (int64_t)nx * ny};
  const int sizes[3] = {nx, ny, nz};
  double best = 0.0;
  for (int64_t p = 0; p < N; ++p) {
    double row = 0.0;
    for (int a = 0; a < dim; ++a) {
      row += k[a][p];  // face p -> p + e_a (0 on the last layer)
      if ((p / strides[a]) % sizes[a] > 0) row += k[a][p - strides[a]];
    }
    best = std::max(best, row);
  }
  return 2.0 * best;
}

// Chebyshev parameters of I - a K with lam bounding the spectrum of -K.
ChebTab cheb_entry(double a, double lam) {
  ChebTab t{};
  const double delta = 0.5 * a * lam, theta = 1.0 + delta;
  t.inv_theta = 1.0 / theta;
  t.sigma = delta > 0.0 ? theta / delta : 0.0;
  t.s = delta > 0.0 ? std::acosh(t.sigma) : 0.0;
  for (int k = 1; k <= CHEB_KT; ++k)
    t.omega[k - 1] = t.s == 0.0 ? 1.0
                                : 2.0 * t.sigma * std::exp(-t.s) * (1.0 + std::exp(-2.0 * k * t.s)) /
                                      (1.0 + std::exp(-2.0 * (k + 1) * t.s));
  return t;
}

// Per-slice spectral bounds -> the level's Chebyshev table (levels running
// Chebyshev; a = dt d_i for collocation node i).
template <class T>
void set_lam(hsdc_ctx *c, LevelT<T> &L, const std::vector<double> &lam) {
  if (!L.cheb_tab) return;
  const int M = L.co.M;
  std::vector<ChebTab> tab((size_t)L.P * M);
  for (int n = 0; n < L.P; ++n)
    for (int i = 0; i < M; ++i) tab[(size_t)n * M + i] = cheb_entry(L.co.dt * L.co.d[i], lam[n]);
  HIPC(hipMemcpyAsync(L.cheb_tab, tab.data(), tab.size() * sizeof(ChebTab), hipMemcpyHostToDevice,
                      c->s));
  HIPC(hipStreamSynchronize(c->s));
}

template <class T>
void build_faces(hsdc_ctx *c, LevelT<T> &L, const double *sigma_node_dev) {
  const Grid &g = L.g;
  std::vector<double> s(g.N);
  HIPC(hipMemcpyAsync(s.data(), sigma_node_dev, g.N * sizeof(double), hipMemcpyDeviceToHost, c->s));
  HIPC(hipStreamSynchronize(c->s));
  const double sc = 1.0 / (c->prob.dx * c->prob.dx * c->prob.chi * c->prob.Cm);
  std::vector<double> kh[3];
  for (int a = 0; a < g.dim; ++a) {
    kh[a] = face_coeffs(a, g.nx, g.ny, g.nz, s, sc);
    L.kface[a] = dalloc<double>(c, g.N);
    HIPC(hipMemcpyAsync(L.kface[a], kh[a].data(), g.N * sizeof(double), hipMemcpyHostToDevice, c->s));
  }
  HIPC(hipStreamSynchronize(c->s));
  set_lam(c, L, std::vector<double>(L.P, lam_faces(g.dim, g.nx, g.ny, g.nz, kh)));
  L.g.kx = L.kface[0];
  L.g.ky = g.dim >= 2 ? L.kface[1] : nullptr;
  L.g.kz = g.dim >= 3 ? L.kface[2] : nullptr;
}

// ---------------------------------------------------------------------------
// diffusion solve for node i of a sweep, slices [s0, s0+ns)
// ---------------------------------------------------------------------------
// Degree of the Chebyshev start of CG (solver 0): each step shrinks the
// residual bound by about 2 sigma (sigma = 1 + 2 / (a lam), 4 to 100 on these
// workloads) for one stencil launch without inner products, cheaper than a CG
// iteration.
constexpr int kChebStartDegree = 3;
// On 2D meshes the whole start is one tiled launch, where a step costs far less
// than a launch: more steps, fewer CG iterations.
// Degree 7: on the 512 x 512 slab no solve needed a CG iteration after it in
// 400 steps (degree 5: 0.1 iterations per solve, degree 6: 0.001), at 14 us
// per launch against 12 us for degree 5; its solves then get no CG launch.
constexpr int kChebStartDegreeTiled = 7;

// The most CG-start tiles of any tissue of a 2D batch for tile shape `tile`
// (0 for a context that is not a batch).
int batch_tiles(const hsdc_ctx *c, int tile) {
  int t = 0;
  for (const auto &d : c->tissue_dims) t = std::max(t, cg_start_tiles_of(d.first, d.second, tile));
  return t;
}

// Tiles per slice of the one-launch CG start on level L (0: none): FP64 levels
// whose solver starts CG from Chebyshev steps, on 2D meshes (a ragged batch:
// the most tiles of any tissue).
template <class T>
int level_start_tiles(const hsdc_ctx *c, const LevelT<T> &L) {
  if (!std::is_same<T, double>::value || c->meth.solver != 0) return 0;
  const int tiles = L.g.rag ? (L.g.dim == 2 ? batch_tiles(c, L.g.ctile) : 0)
                            : cg_start_tiles(L.g, kChebStartDegreeTiled);
  return (tiles > 0 && tiles <= L.cg_pstride) ? tiles : 0;
}

// DCT-II transforms and eigenvalues of K on mesh g (uniform sigma), computed in
// long double and rounded (DctPlan in hsdc_internal.h).
DctPlan make_dct_plan(hsdc_ctx *c, const Grid &g) {
  DctPlan d{};
  const int nn[3] = {g.nx, g.ny, g.nz};
  const double ca[3] = {g.cx, g.cy, g.cz};
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int ax = 0; ax < 3; ++ax) {
    const int n = nn[ax];
    std::vector<double> C((size_t)n * n), CT((size_t)n * n), lam(n);
    for (int k = 0; k < n; ++k) {
      const long double sk = std::sqrt((k == 0 ? 1.0L : 2.0L) / n);
      for (int q = 0; q < n; ++q) {
        const double v = (double)(sk * std::cos(pi * k * (2 * q + 1) / (2.0L * n)));
        C[(size_t)k * n + q] = v;
        CT[(size_t)q * n + k] = v;
      }
      const long double th = pi * k / n;
      const long double sym = g.order == 4
                                  ? (-30.0L + 32.0L * std::cos(th) - 2.0L * std::cos(2.0L * th)) / 12.0L
                                  : 2.0L * std::cos(th) - 2.0L;
      lam[k] = n > 1 ? (double)(ca[ax] * sym) : 0.0;
    }
    double *dC = dalloc<double>(c, C.size()), *dCT = dalloc<double>(c, CT.size());
    double *dl = dalloc<double>(c, lam.size());
    HIPC(hipMemcpyAsync(dC, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice, c->s));
    HIPC(hipMemcpyAsync(dCT, CT.data(), CT.size() * sizeof(double), hipMemcpyHostToDevice, c->s));
    HIPC(hipMemcpyAsync(dl, lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice, c->s));
    HIPC(hipStreamSynchronize(c->s));  // the host vectors go out of scope
    d.C[ax] = dC;
    d.CT[ax] = dCT;
    d.lam[ax] = dl;
  }
  // the fast transforms: every transformed axis (x, and y, z when longer than
  // one node) of a power-of-two length in [2, 2048]
  bool fast = true;
  for (int ax = 0; ax < 3; ++ax) {
    const int n = nn[ax];
    if (ax > 0 && n == 1) continue;
    fast = fast && n >= 2 && n <= 2048 && (n & (n - 1)) == 0;
  }
  d.fast = fast ? 1 : 0;
  if (fast) HIPC(fdct_setup(std::max(nn[0], std::max(nn[1], nn[2]))));
  if (fast)
    for (int ax = 0; ax < 3; ++ax) {
      const int n = nn[ax];
      if (ax > 0 && n == 1) continue;
      std::vector<double> t((size_t)5 * n);
      for (int k = 0; k < n / 2; ++k) {  // W_k = e^{-2 pi i k / n}
        t[2 * k] = (double)std::cos(2.0L * pi * k / n);
        t[2 * k + 1] = (double)-std::sin(2.0L * pi * k / n);
      }
      for (int k = 0; k < n; ++k) {  // E_k = e^{-i pi k / 2n}, s_k
        t[n + 2 * k] = (double)std::cos(pi * k / (2.0L * n));
        t[n + 2 * k + 1] = (double)-std::sin(pi * k / (2.0L * n));
        t[3 * n + k] = (double)std::sqrt((k == 0 ? 1.0L : 2.0L) / n);
        t[4 * n + k] = (double)std::sqrt(n / (k == 0 ? 1.0L : 2.0L));
      }
      double *dt = dalloc<double>(c, t.size());
      HIPC(hipMemcpyAsync(dt, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, c->s));
      HIPC(hipStreamSynchronize(c->s));
      d.ft[ax] = dt;
    }
  return d;
}

template <class T>
void alloc_level(hsdc_ctx *c, LevelT<T> &L, int M, int P, bool coarse_extras, int Mc_for_RI) {
  const int64_t Np = L.g.Np;
  L.P = P;
  L.st.Np = Np;
  L.st.M = M;
  L.st.Y = dalloc<double>(c, (size_t)P * L.st.sY());
  L.st.G = dalloc<T>(c, (size_t)P * L.st.sY());
  L.st.FV = dalloc<double>(c, (size_t)P * L.st.sFV());
  L.st.RH = dalloc<double>(c, (size_t)P * L.st.sRH());
  L.st.L0 = dalloc<T>(c, (size_t)P * L.st.sL());
  L.st.B = dalloc<double>(c, (size_t)P * Np);
  L.cg_nblk = cg_blocks(L.g, c->tune_cg_blocks);
  for (int k = 0; k < 2; ++k) {
    L.cg_r[k] = dalloc<T>(c, (size_t)P * Np);
    L.cg_w[k] = dalloc<T>(c, (size_t)P * Np);
    L.cg_s[k] = dalloc<T>(c, (size_t)P * Np);
  }
  L.cg_p = dalloc<T>(c, (size_t)P * Np);
  // partials sized for the largest block cap hsdc_tune accepts
  // (and the tiles of the CG start on a 2D mesh, or of any tissue of a batch)
  // (and the smallest node-update block and start tile hsdc_tune_shapes accepts)
  L.cg_pstride = std::max(cg_blocks(L.g, 2 * BLOCK), node_blocks_of(L.g, 64));
  if (L.g.dim == 2)
    for (int t = 0; t < kNumCgTiles; ++t)
      L.cg_pstride = std::max<int64_t>(
          L.cg_pstride, std::max(cg_start_tiles_of(L.g.nx, L.g.ny, t), batch_tiles(c, t)));
  // two sets, by the parity of the collocation node: a node update writes its
  // solve's set while the previous solve's set is still read (its log entry)
  L.cg_part = dalloc<double>(c, (size_t)2 * P * 5 * L.cg_pstride);
  L.cg_sc = dalloc<CgScalars>(c, (size_t)2 * P);
  L.cg_sc_host = halloc<CgScalars>(c, (size_t)2 * P);
  if (std::is_same<T, double>::value && c->meth.solver == 3) {
    L.dct = make_dct_plan(c, L.g);
    L.direct = true;
  }
  if (std::is_same<T, double>::value && (c->meth.solver == 0 || c->meth.solver == 1)) {
    L.cheb_x = dalloc<double>(c, (size_t)P * Np);
    L.cheb_tab = dalloc<ChebTab>(c, (size_t)P * M);
    set_lam(c, L, std::vector<double>(P, lam_uniform(L.g.dim, L.g.nx, L.g.ny, L.g.nz, L.g.cx,
                                                     L.g.cy, L.g.cz)));
  }
  if (!coarse_extras) {  // the residual is taken on the fine level only
    L.res_nblk = residual_blocks(L.g);
    L.res_part = dalloc<double>(c, (size_t)P * 2 * L.res_nblk);
    L.res_out = dalloc<double>(c, (size_t)2 * NF * P);
    L.res_out_host = halloc<double>(c, 2 * NF * P);
  }
  L.U = dalloc<double>(c, (size_t)P * NF * Np);
  if (Mc_for_RI > 0) L.RI = dalloc<double>(c, (size_t)P * Mc_for_RI * NF * Np);
  if (coarse_extras) {
    L.Sz = dalloc<double>(c, (size_t)P * L.st.sY());
    L.y0c = dalloc<double>(c, (size_t)NF * Np);
  }
  // first budgets: two launches after the tiled start (its solves have needed
  // none), eight otherwise; the predictor adjusts them from the first steps on
  L.tiled_start = level_start_tiles(c, L) > 0;
  for (auto &row : L.cg_pred)
    for (int &v : row) v = L.tiled_start ? 2 : 8;
  for (auto &row : L.cg_umax)
    for (int &v : row) v = -1;
}

template <class T>
CgBatchT<T> make_batch(hsdc_ctx *c, LevelT<T> &L, int lev, int s0, int ns, int i) {
  CgBatchT<T> cb{};
  const int64_t Np = L.g.Np;
  cb.x = L.st.Y + s0 * L.st.sY() + (int64_t)i * L.st.sS();
  cb.sx = L.st.sY();
  cb.b = L.st.B + s0 * Np;
  cb.sb = Np;
  for (int k = 0; k < 2; ++k) {
    cb.r[k] = L.cg_r[k] + s0 * Np;
    cb.w[k] = L.cg_w[k] + s0 * Np;
    cb.s[k] = L.cg_s[k] + s0 * Np;
  }
  cb.p = L.cg_p + s0 * Np;
  cb.pstride = L.cg_pstride;
  cb.part = L.cg_part + ((int64_t)(i & 1) * L.P + s0) * 5 * L.cg_pstride;
  cb.sc = L.cg_sc + 2 * s0;
  cb.log = nullptr;
  cb.last_k = -1;
  cb.slice0 = s0;
  cb.nslices = ns;
  cb.nblk = L.cg_nblk;
  cb.nblk0 = node_blocks(L.g);  // r_0 and its partials come from the node update
  cb.nblk_s = node_blocks_of(L.g, kDefaultNodeBlock);  // those of k_cg_start (3D meshes)
  cb.a = L.co.dt * L.co.d[i - 1];
  const double rt = level_rtol(c, lev);
  cb.tol2 = rt * rt;
  cb.maxit = c->meth.cg_maxit;
  // FP32 work vectors: solve the correction from the warm start to a relative
  // accuracy, so that the solve error shrinks with the defect
  cb.rel_r0 = (lev == 1 && c->cf32) ? 1 : 0;
  if (L.direct) {
    cb.direct = 1;
    cb.bout = L.st.B + s0 * Np;
  }
  if (L.cheb_x) {
    cb.xt = L.cheb_x + s0 * Np;
    cb.bout = L.st.B + s0 * Np;
    cb.tab = L.cheb_tab + (i - 1);
    cb.tab_stride = L.co.M;
    cb.cstart = c->meth.solver == 0 ? kChebStartDegree : 0;
    // on 2D meshes the whole start is one tiled launch; the node update then
    // also stores x_0 in p for it
    const int tiles = level_start_tiles(c, L);
    if (tiles > 0) {
      cb.cstart = kChebStartDegreeTiled;
      cb.nblk_s = tiles;
      cb.x0_to_p = 1;
    }
  }
  return cb;
}

// A finished solve met the tolerance (Chebyshev: gamma is the bound on the
// final ||r||^2 and bb the reference).
bool cg_ok(const CgScalars &sc, double tol2) {
  return sc.done && (sc.gamma <= tol2 * sc.bb || sc.gamma == 0.0);
}

// A solve whose residual or right-hand-side norm is NaN or Inf: the state it
// was given is not finite (no further iteration or recomputation helps).
bool cg_nonfinite(const CgScalars &sc) { return !std::isfinite(sc.gamma) || !std::isfinite(sc.bb); }

// Launches a solve needed, as the budget predictor counts them (the budget is
// this plus the margin): CG needs one launch per iteration (convergence is
// checked by the kernel that writes the log entry).  Chebyshev's launch k
// forms x_{k+1} and the node update x_1, so an even count m takes max(1, m -
// 1) launches; since m moves in steps of 2 it is counted as m (one spare launch
// more than CG).
int budget_use(const CgScalars &sc, bool cheb) { return sc.it; }

// Check every budgeted solve enqueued since the last check (one host
// synchronisation); slices whose solve missed cg_rtol are added to cg_fails.
void flush_cg_log(hsdc_ctx *c) {
  if (c->cg_pending.empty()) return;
  HIPC(hipMemcpyAsync(c->cg_log, c->cg_dlog, c->cg_log_used * sizeof(CgScalars),
                      hipMemcpyDeviceToHost, c->s));
  HIPC(hipStreamSynchronize(c->s));
  int fails = 0;
  for (const CgLogEntry &e : c->cg_pending) {
    const double rt = level_rtol(c, e.lev), tol2 = rt * rt;
    int used = 0;
    bool ok_all = true;
    for (int n = 0; n < e.ns; ++n) {
      const CgScalars &sc = c->cg_log[e.off + n];
      const bool ok = cg_ok(sc, tol2);
      if (cg_nonfinite(sc)) c->nonfinite = true;
      ok_all = ok_all && ok;
      used = std::max(used, budget_use(sc, e.cheb));
      c->stats.cg_iters += sc.it;
      c->stats.cg_solves += 1;
      if (!ok) ++fails;
    }
    // budget = launches needed + margin, lowered by at most one per check;
    // doubled after a miss (a spare no-op launch costs far less than a
    // recomputed step)
    if (c->cg_record && e.lev == 0) c->cg_record->push_back(ok_all ? used : -1);
    int &pred = pred_table(c, e.lev)[e.row & 15][e.i - 1];
    if (!ok_all)
      pred = std::min(c->meth.cg_maxit + 1, std::max(2 * e.budget, used + 4));
    else if (c->graph_on && !c->prof.on && e.lev == graph_level(c)) {
      // graph replay (profiled steps run eagerly): raise at once, lower only at
      // a relaxation
      pred = std::max(pred, used + e.margin);
      int &um = umax_table(c, e.lev)[e.row & 15][e.i - 1];
      um = std::max(um, used);
    } else
      pred = std::max(used + e.margin, pred - 1);
  }
  c->cg_pending.clear();
  c->cg_log_used = 0;
  c->cg_fails += fails;
}

// Chebyshev solve of node i (the node update stored b and x_1).  Budgeted mode
// enqueues the predicted number of launches (those past the count the first
// launch derives exit at once) and logs the outcome; safe mode launches until
// every slice is done, checking on the host.
void cheb_solve(hsdc_ctx *c, Level &L, int lev, int s0, int ns, int i, int pred_row, CgBatch cb) {
  const double nodes = slice_nodes(c, L, s0, ns);
  int &pred = L.cg_pred[pred_row & 15][i - 1];
  const int cap = std::max(1, cb.maxit);
  if (!c->safe_cg) {
    if (c->cg_log_used + ns > c->cg_log_cap) flush_cg_log(c);  // log full: verify now
    const int budget = std::max(1, std::min(pred, cap));
    cb.log = c->cg_dlog + c->cg_log_used;
    cb.last_k = budget;
    ProfScope ps(c, PC_CHEB, 32.0 * nodes * budget);
    for (int k = 1; k <= budget; ++k) HIPC(launch_cheb_iter(c->s, L.g, cb, k));
    ps.end(budget);
    c->cg_pending.push_back(
        CgLogEntry{lev, s0, ns, i, pred_row, 0, c->cg_log_used, budget, true, cg_margin(c, false)});
    c->cg_log_used += ns;
    return;
  }
  int k = 1;
  int batch = std::max(1, std::min(pred, cap));
  for (;;) {
    int nl = 0;
    ProfScope ps(c, PC_CHEB, 0.0);
    for (int q = 0; q < batch && k <= cap; ++q, ++k, ++nl) HIPC(launch_cheb_iter(c->s, L.g, cb, k));
    ps.bytes = 32.0 * nodes * nl;
    ps.end(nl);
    HIPC(hipMemcpyAsync(L.cg_sc_host + 2 * s0, L.cg_sc + 2 * s0, 2 * ns * sizeof(CgScalars),
                        hipMemcpyDeviceToHost, c->s));
    HIPC(hipStreamSynchronize(c->s));
    bool all = true;
    for (int n = 0; n < ns; ++n) all = all && L.cg_sc_host[2 * (s0 + n)].done;
    if (all || k > cap) break;
    batch = 2;
  }
  int used = 0;
  for (int n = 0; n < ns; ++n) {
    const CgScalars &sc = L.cg_sc_host[2 * (s0 + n)];
    used = std::max(used, budget_use(sc, true));
    c->stats.cg_iters += sc.it;
    c->stats.cg_solves += 1;
    if (!cg_ok(sc, cb.tol2)) c->stats.cg_unconverged += 1;
    if (cg_nonfinite(sc)) c->nonfinite = true;
  }
  pred = std::max(used + cg_margin(c, false), pred - 1);
}

// Diffusion solve of node i whose node update has run (cb: that update's batch).
// In budgeted mode the solve gets the predicted number of CG launches (none
// when the start is predicted to meet the tolerance) and is checked by a
// later kernel: the returned arguments name its log entry, to be passed to the
// next node update of the same slices or to launch_cg_log.  Otherwise (safe
// mode, Chebyshev) nothing is left to log.
template <class T>
CgLogArgs cg_solve(hsdc_ctx *c, LevelT<T> &L, int lev, int s0, int ns, int i, int pred_row,
                   CgBatchT<T> cb) {
  const double nodes = slice_nodes(c, L, s0, ns);
  CgLogArgs lg{};
  if constexpr (std::is_same<T, double>::value) {
    if (cb.direct) {
      // exact solve in the DCT-II eigenbasis: b to the stage's V, through two
      // [P][Np] work vectors.  Fast transforms: one launch per axis each way,
      // the last axis's two fused, each reading and writing 8 B per node; dense
      // transforms: 2 n FLOP per node and axis each way (the dct_solve class
      // then counts FLOPs where the others count bytes)
      const int64_t Np = L.g.Np;
      const int na = 1 + (L.g.ny > 1 ? 1 : 0) + (L.g.nz > 1 ? 1 : 0);
      const double fl = L.dct.fast
                            ? 16.0 * (2 * na - 1)
                            : 4.0 * (L.g.nx + (L.g.ny > 1 ? L.g.ny : 0) + (L.g.nz > 1 ? L.g.nz : 0));
      PLAUNCH(c, PC_DCT, fl * nodes,
              launch_dct_solve(c->s, L.g, L.dct, cb.a, cb.bout, Np, cb.x, cb.sx,
                               L.cg_r[0] + s0 * Np, L.cg_w[0] + s0 * Np, Np, ns));
      c->stats.cg_solves += ns;
      return lg;
    }
  }
  // first CG launch index: 1 after a Chebyshev start (its vectors have parity 1)
  int k0 = 0;
  if constexpr (std::is_same<T, double>::value) {
    if (cb.xt && !cb.cstart) {
      cheb_solve(c, L, lev, s0, ns, i, pred_row, cb);
      return lg;
    }
    if (cb.cstart) {
      if (cb.x0_to_p) {
        // one launch: x_1, x_0, b read (with the tiles' halos), x_D, r_D, w_D written
        PLAUNCH(c, PC_CGINIT, 48.0 * nodes, launch_cg_start_tiled(c->s, L.g, cb, cb.nblk_s));
      } else {
        // x_2 .. x_D (x_k, x_{k-1}, b read, x_{k+1} written); r_D and w_D (x_D
        // and b read, r, w and for D odd x written)
        PLAUNCH(c, PC_CGINIT, 32.0 * nodes * (cb.cstart - 1),
                launch_cheb_steps(c->s, L.g, cb, cb.cstart - 1));
        PLAUNCH(c, PC_CGINIT, (32.0 + 8.0 * (cb.cstart & 1)) * nodes,
                launch_cg_start(c->s, L.g, cb));
      }
      k0 = 1;
    }
  }
  if (k0 == 0) PLAUNCH(c, PC_CGINIT, 16.0 * nodes, launch_cg_init(c->s, L.g, cb));
  int &pred = L.cg_pred[pred_row & 15][i - 1];
  if (!c->safe_cg) {
    if (c->cg_log_used + ns > c->cg_log_cap) flush_cg_log(c);  // log full: verify now
    // budget = CG launches, each one iteration unless it finds convergence
    const int budget = std::max(0, std::min(pred, cb.maxit + 1));
    if (budget > 0) {
      ProfScope ps(c, PC_CGITER, 0.0);
      for (int k = k0; k < budget + k0; ++k) HIPC(launch_cg_iter(c->s, L.g, cb, k));
      ps.end(budget);
    }
    lg.part = cb.part;
    lg.pstride = cb.pstride;
    lg.sc = cb.sc;
    lg.log = c->cg_dlog + c->cg_log_used;
    lg.par = (k0 + budget) & 1;  // the last launch k0 + budget - 1 publishes parity (k + 1) & 1
    // the final residual's partials: a CG launch's, the start's, or (plain CG,
    // no launch) the node update's ||r_0||^2
    lg.ngamma = budget > 0 ? -1 : (k0 == 1 ? cb.nblk_s : cb.nblk0);
    lg.cg_nblk = cb.nblk;
    lg.nbb = cb.nblk0;
    lg.slice0 = s0;
    lg.tol2 = cb.tol2;
    lg.rel_r0 = cb.rel_r0;
    c->cg_pending.push_back(CgLogEntry{lev, s0, ns, i, pred_row, 0, c->cg_log_used, budget, false,
                                       cg_margin(c, cb.x0_to_p)});
    c->cg_log_used += ns;
    return lg;
  }
  // safe mode: iterate until every slice has converged, checking on the host
  const double tol2 = cb.tol2;
  int k = k0;
  int batch = std::max(1, std::min(pred, cb.maxit + 1));
  for (;;) {
    ProfScope ps(c, PC_CGITER, 0.0);
    int nl = 0;
    for (int q = 0; q < batch && k <= cb.maxit + k0; ++q, ++k, ++nl)
      HIPC(launch_cg_iter(c->s, L.g, cb, k));
    ps.end(nl);
    HIPC(hipMemcpyAsync(L.cg_sc_host + 2 * s0, L.cg_sc + 2 * s0, 2 * ns * sizeof(CgScalars),
                        hipMemcpyDeviceToHost, c->s));
    HIPC(hipStreamSynchronize(c->s));
    bool all = true;
    for (int n = 0; n < ns; ++n) all = all && L.cg_sc_host[2 * (s0 + n) + (k & 1)].done;
    if (all || k > cb.maxit + k0) break;
    batch = 2;
  }
  int used = 0;
  for (int n = 0; n < ns; ++n) {
    const CgScalars &sc = L.cg_sc_host[2 * (s0 + n) + (k & 1)];
    used = std::max(used, sc.it);
    c->stats.cg_iters += sc.it;
    c->stats.cg_solves += 1;
    if (!cg_ok(sc, tol2)) c->stats.cg_unconverged += 1;
    if (cg_nonfinite(sc)) c->nonfinite = true;
  }
  if (c->cg_record && lev == 0) c->cg_record->push_back(used);
  pred = std::max(used + cg_margin(c, cb.x0_to_p), pred - 1);
  return lg;
}

// Reaction terms, Lambda(y_{n,0}) and K V of every stage of slices [s0, s0+ns).
template <class T>
void evaluate_all(hsdc_ctx *c, LevelT<T> &L, int lev, int s0, int ns) {
  const hsdc_problem &p = c->prob;
  const int M = L.co.M;
  const double N = slice_nodes(c, L, s0, ns) / ns;
  PLAUNCH(c, PC_EVAL, 8.0 * (2 * NF + NG) * N * ns,
          launch_eval_stages<T>(c->s, L.g, L.st, L.co, c->stim[lev], p.g_scale[0], p.g_scale[1],
                             p.g_scale[2], s0, ns, 0, 1, L.st.L0, nullptr));
  PLAUNCH(c, PC_EVAL, 8.0 * (2 * NF + NG) * N * ns * M,
          launch_eval_stages<T>(c->s, L.g, L.st, L.co, c->stim[lev], p.g_scale[0], p.g_scale[1],
                             p.g_scale[2], s0, ns, 1, M, nullptr, L.st.L0));
  PLAUNCH(c, PC_SPMV, 16.0 * (M + 1) * N * ns,
          launch_spmv_stages<T>(c->s, L.g, L.st, s0, ns, 0, M + 1));
  c->stats.ionic_evals += (int64_t)(N * ns) * (M + 1);
}

// ---------------------------------------------------------------------------
// one sweep on slices [s0, s0+ns) of level L.
//   u_src: new start values [ns][NF][Np], or NULL to keep y_{n,0}.  With
//   u_src the start values are stored into stage 0 first and the reaction
//   terms, Lambda(y_{n,0}) and K V of every stage are evaluated afresh, so the
//   right-hand side (P - C)(y^k) is taken at the new start value.  Without it:
//   precondition G, FV and L0 hold those terms of the current iterate.
//   RI: FAS term of tau per unit dt (coarse level of PFASST), or NULL.
//   drop_terms: the caller discards the new iterate's reaction terms and K V
//   (last sweep of a serial step, every coarse and burn-in sweep); otherwise
//   the postcondition is the precondition for the new iterate.
// ---------------------------------------------------------------------------
template <class T>
void sweep(hsdc_ctx *c, LevelT<T> &L, int lev, int s0, int ns, const double *u_src, const double *RI,
           int pred_row, bool drop_terms = false, const double *yref = nullptr) {
  const Colloc &co = L.co;
  const hsdc_problem &p = c->prob;
  const int M = co.M;
  const double N = slice_nodes(c, L, s0, ns) / ns;
  const int64_t sRI = (int64_t)M * NF * L.g.Np;
  const int spread = (lev == 0 && c->spread_pending) ? 1 : 0;
  if (u_src) {
    PLAUNCH(c, PC_COPY, 16.0 * NF * N * ns,
            launch_copy_fields(c->s, L.g.Np, L.st.Y + s0 * L.st.sY(), L.st.sY(), u_src,
                               (int64_t)NF * L.g.Np, NF, ns));
    evaluate_all(c, L, lev, s0, ns);
  }
  {
    // G of every stage (stage 0 only after a spread), K V, Lambda_n and the
    // anchor's gate values read; RH written
    const double per = spread ? (NF + 1 + 2 * NG + M * NF)
                              : ((M + 1) * NF + M + 2 * NG + M * NF + (RI ? M * NF : 0));
    PLAUNCH(c, PC_ASSEMBLE, 8.0 * per * N * ns,
            launch_assemble(c->s, L.g, L.st, co, s0, ns, RI, sRI, spread, c->stim[lev]));
  }
  CgLogArgs pending{};  // the previous budgeted solve, logged by the next node update
  for (int i = 1; i <= M; ++i) {
    const CgBatchT<T> cb = make_batch(c, L, lev, s0, ns, i);
    // doubles per node: stage i-1, RH_i, Lambda_n, x_0 and K x_0 read; stage i
    // (but V), b, x_1 and (unless dropped) the reaction terms of stage i-1
    // written; node 1 reads the stored reaction terms of stage 0 instead
    const double per = ((i == 1) ? 90.0 : (drop_terms ? 71.0 : 90.0)) * sizeof(T) / 8.0 +
                       (cb.x0_to_p ? 1.0 : 0.0);
    PLAUNCH(c, PC_NODE, 8.0 * per * N * ns,
            launch_node_update(c->s, L.g, L.st, co, c->stim[lev], p.g_scale[0], p.g_scale[1],
                               p.g_scale[2], s0, ns, i, cb, drop_terms ? 0 : 1, spread,
                               std::is_same<T, double>::value ? nullptr : yref, pending));
    if (i > 1) c->stats.ionic_evals += (int64_t)(N * ns);
    pending = cg_solve(c, L, lev, s0, ns, i, pred_row, cb);
  }
  if (pending.log) PLAUNCH(c, PC_CGITER, 0.0, launch_cg_log(c->s, L.g, pending, ns));
  if (lev == 0) c->spread_pending = false;
  if (!drop_terms) {
    // reaction terms and K V of the new iterate's last stage, for the next
    // sweep or the residual (stages 1..M-1 were stored by the node updates)
    PLAUNCH(c, PC_EVAL, 8.0 * (2 * NF + NG) * N * ns,
            launch_eval_stages<T>(c->s, L.g, L.st, co, c->stim[lev], p.g_scale[0], p.g_scale[1],
                               p.g_scale[2], s0, ns, M, 1, nullptr, L.st.L0));
    c->stats.ionic_evals += (int64_t)(N * ns);
    PLAUNCH(c, PC_SPMV, 16.0 * M * N * ns, launch_spmv_stages<T>(c->s, L.g, L.st, s0, ns, 1, M));
  }
  if (lev == 0)
    c->stats.sweeps += ns;
  else
    c->stats.coarse_sweeps += ns;
}

// Serial step start: y^0 = 1 (x) y_n from Y[0][0].
// (every slice of a serial context: one, or the tissues of a batch)
void begin_serial_step(hsdc_ctx *c) {
  Level &L = c->L[0];
  const hsdc_problem &p = c->prob;
  const int P = L.P;
  const double N = slice_nodes(c, L, 0, P);
  PLAUNCH(c, PC_EVAL, 8.0 * (2 * NF + NG) * N,
          launch_eval_stages<double>(c->s, L.g, L.st, L.co, c->stim[0], p.g_scale[0],
                                     p.g_scale[1], p.g_scale[2], 0, P, 0, 1, L.st.L0,
                                     nullptr));
  PLAUNCH(c, PC_SPMV, 16.0 * N, launch_spmv_stages<double>(c->s, L.g, L.st, 0, P, 0, 1));
  PLAUNCH(c, PC_COPY, 8.0 * (1 + L.co.M) * N, launch_copy_V_to_stages(c->s, L.g, L.st, 0, P));
  c->spread_pending = true;
  c->stats.ionic_evals += (int64_t)N;
  c->sweeps_done = 0;
  c->sweep_index = 0;
}

// Store the spread of stage 0 in full (states, reaction terms, K V) when a
// caller needs the stage vector itself before the first sweep of a step.
void materialize(hsdc_ctx *c) {
  if (!c->spread_pending) return;
  Level &L = c->L[0];
  HIPC(launch_spread(c->s, L.g, L.st, L.co, c->stim[0], 0, L.P, true));
  c->spread_pending = false;
}

hsdc_status residual_pass(hsdc_ctx *c, double *res_host, bool want_RI, int s0 = 0) {
  materialize(c);
  Level &L = c->L[0];
  const int ns = L.P - s0;
  const double *yb = c->pfasst ? c->y0blk : nullptr;  // serial, batch: u = y_{n,0}
  const int Mc = c->nlev >= 2 ? c->meth.M[1] : 0;
  double *RI = (want_RI && c->nlev >= 2) ? L.RI : nullptr;
  {
    const double M = L.co.M;
    const double per = (M + 1) * NF + M * NF + M + NG + NF + (RI ? Mc * NF : 0);
    PLAUNCH(c, PC_RESIDUAL, 8.0 * per * slice_nodes(c, L, s0, ns),
            launch_residual(c->s, L.g, L.st, L.co, s0, ns, yb, L.res_part, L.res_nblk, L.res_out,
                            c->Rt, Mc, RI, (int64_t)Mc * NF * L.g.Np));
  }
  HIPC(hipMemcpyAsync(L.res_out_host, L.res_out, 2 * NF * ns * sizeof(double),
                      hipMemcpyDeviceToHost, c->s));
  HIPC(hipStreamSynchronize(c->s));
  bool finite = true;
  // res_out holds slices s0..P-1 from its start; res_host[n] is slice n
  for (int q = 0; q < ns; ++q) {
    const int n = q;
    // ||r_n||_inf / ||y_n||_inf over every field (Algorithm 1), or the largest
    // of the per-field ratios ||r_{n,f}||_inf / ||y_{n,f}||_inf
    double r = 0.0, y = 0.0, worst = 0.0;
    for (int f = 0; f < NF; ++f) {
      const double rf = L.res_out_host[2 * (q * NF + f)], yf = L.res_out_host[2 * (q * NF + f) + 1];
      if (!std::isfinite(rf) || !std::isfinite(yf)) finite = false;
      r = std::max(r, rf);
      y = std::max(y, yf);
      worst = std::max(worst, yf > 0 ? rf / yf : rf);
    }
    const double rel = c->meth.residual_norm == 1 ? worst : (y > 0 ? r / y : r);
    if (!std::isfinite(rel)) finite = false;
    if (res_host) res_host[s0 + n] = finite ? rel : NAN;
  }
  if (!finite) return fail(c, HSDC_ENONFINITE, "non-finite residual or state");
  return HSDC_OK;
}

// ---------------------------------------------------------------------------
// PFASST (two levels)
// ---------------------------------------------------------------------------
template <class T>
void restrict_stages_between(hsdc_ctx *c, Level &F, LevelT<T> &Cc, const double *Rt, int s0 = 0,
                             int ns = -1) {
  if (ns < 0) ns = F.P - s0;
  const double bytes = 8.0 * ns * NF * ((F.co.M + 1.0) * F.g.N + 2.0 * (Cc.co.M + 1.0) * Cc.g.N);
  PLAUNCH(c, PC_TRANSFER, bytes,
          launch_restrict_stages(c->s, F.g, Cc.g, c->meth.space_coarsen, F.st.Y + s0 * F.st.sY(),
                                 F.st.sY(), F.co.M, Rt, Cc.co.M, Cc.st.Y + s0 * Cc.st.sY(),
                                 Cc.st.sY(), Cc.Sz + s0 * Cc.st.sY(), ns));
}
template <class T>
void restrict_fine_to_coarse(hsdc_ctx *c, LevelT<T> &Cc, int s0 = 0, int ns = -1) {
  restrict_stages_between(c, c->L[0], Cc, c->Rt, s0, ns);
}

// Fine stages from stage i0 on take the coarse correction.  i0 = 1 where a
// fine sweep follows at once: it overwrites every slice's stage 0 with its
// start value before reading it.
template <class T>
void correct_between(hsdc_ctx *c, Level &F, LevelT<T> &Cc, const double *Tt, int i0, int s0 = 0,
                     int ns = -1) {
  if (ns < 0) ns = F.P - s0;
  // z_c - S z formed in S z (z_c and S z read, the difference written), then
  // read once at the coarse cells; fine stages i0..M read and written
  const double bytes =
      8.0 * ns * NF * (4.0 * (Cc.co.M + 1.0) * Cc.g.N + 2.0 * (F.co.M + 1.0 - i0) * F.g.N);
  PLAUNCH(c, PC_TRANSFER, bytes,
          launch_prolong_correct(c->s, F.g, Cc.g, c->meth.space_coarsen, Cc.st.Y + s0 * Cc.st.sY(),
                                 Cc.Sz + s0 * Cc.st.sY(), Cc.st.sY(), Cc.co.M, Tt, F.co.M, i0,
                                 F.st.Y + s0 * F.st.sY(), F.st.sY(), ns));
}
template <class T>
void coarse_correct_fine(hsdc_ctx *c, LevelT<T> &Cc, int i0, int s0 = 0, int ns = -1) {
  correct_between(c, c->L[0], Cc, c->Tt, i0, s0, ns);
}

// start values u_n of a sweep over slices [s0, s0+ns) from the stage-M values
// of slices n-1 (ends) and the block start value blk0 for n = 0
template <class T>
void gather_starts(hsdc_ctx *c, LevelT<T> &L, const double *blk0, int s0, int ns) {
  const int64_t sS = L.st.sS();
  int n = s0;
  const double per = 16.0 * NF * L.g.N;
  if (n == 0) {
    PLAUNCH(c, PC_COPY, per, launch_copy_fields(c->s, L.g.Np, L.U, sS, blk0, sS, NF, 1));
    ++n;
  }
  if (n < s0 + ns)
    PLAUNCH(c, PC_COPY, per * (s0 + ns - n),
            launch_copy_fields(c->s, L.g.Np, L.U + n * sS, sS,
                               L.st.Y + (n - 1) * L.st.sY() + (int64_t)L.co.M * sS,
                               L.st.sY(), NF, s0 + ns - n));
}

// Staggered coarse predictor: at stage s every slice n >= s takes one coarse
// sweep (tau = 0) from the end value slice n-1 held after stage s-1.
template <class T>
void burn_in(hsdc_ctx *c, LevelT<T> &Cc) {
  const int P = Cc.P;
  restrict_fine_to_coarse(c, Cc);
  for (int s = 0; s < P; ++s) {
    gather_starts(c, Cc, Cc.y0c, s, P - s);
    sweep(c, Cc, 1, s, P - s, Cc.U + s * Cc.st.sS(), nullptr, 15, true);
  }
  coarse_correct_fine(c, Cc, 0);
}

// Three levels: the staggered burn-in on the coarsest level, its correction
// carried to the middle and then the fine level (every stage).
void burn_in3(hsdc_ctx *c) {
  Level &F = c->L[0], &Mi = c->L[1], &C = c->L[2];
  const int P = C.P;
  restrict_stages_between(c, F, Mi, c->Rt);
  restrict_stages_between(c, Mi, C, c->Rt2);
  for (int s = 0; s < P; ++s) {
    gather_starts(c, C, C.y0c, s, P - s);
    sweep(c, C, 2, s, P - s, C.U + s * C.st.sS(), nullptr, 15, true);
  }
  correct_between(c, Mi, C, c->Tt2, 0);
  correct_between(c, F, Mi, c->Tt, 0);
}

void begin_block(hsdc_ctx *c) {
  Level &F = c->L[0];
  const int P = F.P;
  // spread y0 over every stage of every slice
  for (int j = 0; j <= F.co.M; ++j)
    HIPC(launch_copy_fields(c->s, F.g.Np, F.st.Y + (int64_t)j * F.st.sS(), F.st.sY(),
                            c->y0blk, 0, NF, P));
  if (c->nlev == 2) {
    with_coarse(c, [&](auto &Cc) {
      HIPC(launch_restrict_fields(c->s, F.g, Cc.g, c->meth.space_coarsen,
                                  c->y0blk, 0, Cc.y0c, 0, NF, 1));
      if (P > 1 && c->meth.burn_in) burn_in(c, Cc);
    });
  } else if (c->nlev == 3) {
    Level &Mi = c->L[1], &C = c->L[2];
    HIPC(launch_restrict_fields(c->s, F.g, Mi.g, c->meth.space_coarsen, c->y0blk, 0, Mi.y0c, 0,
                                NF, 1));
    HIPC(launch_restrict_fields(c->s, Mi.g, C.g, c->meth.space_coarsen, Mi.y0c, 0, C.y0c, 0, NF,
                                1));
    if (P > 1 && c->meth.burn_in) burn_in3(c);
  }
  evaluate_all(c, F, 0, 0, P);
  c->block_ready = true;
  c->ri_fresh = false;
  if (c->a0 != 0) c->graph_dirty = true;  // a captured coarse part covered slices a0..P-1
  c->a0 = 0;
  c->rel_last.assign(P, INFINITY);
}

void graph_release(hsdc_ctx *c) {
  if (c->gexec) hipGraphExecDestroy(c->gexec);
  if (c->graph) hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
}

void stats_add(hsdc_stats &a, const hsdc_stats &d, int sign) {
  a.steps += sign * d.steps;
  a.sweeps += sign * d.sweeps;
  a.coarse_sweeps += sign * d.coarse_sweeps;
  a.cg_solves += sign * d.cg_solves;
  a.cg_iters += sign * d.cg_iters;
  a.cg_unconverged += sign * d.cg_unconverged;
  a.pfasst_iters += sign * d.pfasst_iters;
  a.ionic_evals += sign * d.ionic_evals;
  a.cg_redo_steps += sign * d.cg_redo_steps;
}

// Capture part() (enqueued with budgeted solves) into the context's graph; the
// host-side counters and CG log entries it leaves are kept for the replays.
template <class Fn>
void capture_part(hsdc_ctx *c, Fn &&part) {
  graph_release(c);
  c->cg_pending.clear();
  c->cg_log_used = 0;
  const hsdc_stats before = c->stats;
  HIPC(hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
  try {
    c->safe_cg = false;
    part();
    c->safe_cg = true;
  } catch (...) {
    hipGraph_t g = nullptr;
    hipStreamEndCapture(c->s, &g);
    if (g) hipGraphDestroy(g);
    c->cg_pending.clear();
    c->cg_log_used = 0;
    c->stats = before;
    c->safe_cg = true;
    throw;
  }
  HIPC(hipStreamEndCapture(c->s, &c->graph));
  HIPC(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  c->graph_pending = c->cg_pending;
  c->graph_log_used = c->cg_log_used;
  c->cg_pending.clear();
  c->cg_log_used = 0;
  c->graph_delta = c->stats;
  stats_add(c->graph_delta, before, -1);
  c->stats = before;
  c->graph_dirty = false;
}

// The coarse part of a PFASST iteration (FAS restriction, coarse evaluations,
// the Q^seq chain) reads the fine level and writes the coarse level only, so
// it can run again from its start: its solves run at predicted budgets,
// verified once at its end, and a part with a missed solve runs again with
// every solve checked.  With graph replay on, the part is captured once and
// replayed while the budgets it was captured with stay in force (raised at
// once after a miss, lowered every 8 replays to the most iterations used).
template <class T, class Fn>
void run_coarse_part(hsdc_ctx *c, LevelT<T> &Cc, Fn &&part) {
  int pred0[16][MAXM];
  std::memcpy(pred0, Cc.cg_pred, sizeof(pred0));
  const bool graph = c->graph_on && !c->prof.on;
  c->cg_fails = 0;
  if (graph) {
    if (c->graph_dirty || !c->gexec) capture_part(c, part);
    c->cg_pending = c->graph_pending;
    c->cg_log_used = c->graph_log_used;
    HIPC(hipGraphLaunch(c->gexec, c->s));
    stats_add(c->stats, c->graph_delta, 1);
  } else {
    c->safe_cg = false;
    try {
      part();
    } catch (...) {
      c->safe_cg = true;
      throw;
    }
    c->safe_cg = true;
  }
  flush_cg_log(c);
  if (c->cg_fails > 0 && !c->nonfinite) {
    c->stats.cg_redo_steps += 1;
    c->cg_fails = 0;
    part();
  }
  if (graph) {
    c->graph_steps += 1;
    if (c->graph_steps % 8 == 0)
      for (int r = 0; r < 16; ++r)
        for (int i = 0; i < MAXM; ++i)
          if (Cc.cg_umax[r][i] >= 0) {
            Cc.cg_pred[r][i] = Cc.cg_umax[r][i] + cg_margin(c, Cc.tiled_start);
            Cc.cg_umax[r][i] = -1;
          }
    if (std::memcmp(pred0, Cc.cg_pred, sizeof(pred0)) != 0) c->graph_dirty = true;
  }
}

// The relative residuals of the fine level after an iteration (Algorithm 1's
// stop test); the restricted integrals for the next iteration come with them.
hsdc_status finish_iteration(hsdc_ctx *c, double *res_host, int32_t *conv) {
  Level &F = c->L[0];
  const int P = F.P;
  c->stats.pfasst_iters += 1;
  if ((int)c->rel_last.size() != P) c->rel_last.assign(P, INFINITY);
  // the residuals of the active slices (a stopped slice keeps its last one)
  hsdc_status st = residual_pass(c, c->rel_last.data(), c->nlev >= 2, c->a0);
  c->ri_fresh = (st == HSDC_OK && c->nlev >= 2);
  if (res_host)
    for (int n = 0; n < P; ++n) res_host[n] = c->rel_last[n];
  const double tol = c->meth.tol;
  bool all = tol > 0;
  for (int n = 0; n < P; ++n) all = all && c->rel_last[n] < tol;
  if (c->meth.prefix_stop && st == HSDC_OK) {
    const int a0 = c->a0;
    while (tol > 0 && c->a0 < P && c->rel_last[c->a0] < tol) ++c->a0;
    if (c->a0 != a0) c->graph_dirty = true;  // a captured coarse part covers slices a0..P-1
    all = c->a0 == P;
  }
  if (conv) *conv = all ? 1 : 0;
  return st;
}

// Algorithm 1 with three levels (FP64).  Down: level l = 1, 2 restricted from
// level l - 1 with its FAS term tau_l = D_l(S z_{l-1}) - S D_{l-1}(z_{l-1}) +
// S tau_{l-1}; the middle level sweeps once (Q^par), the coarsest runs Q^seq.
// Up: the middle level corrected and swept again (Q^par), then the fine level
// corrected and swept (Q^par); the residual of the fine level.  Rows i >= 1 of
// tau_l / dt are S (I_{l-1} + tau_{l-1} / dt) - I_l(S z), the rest cancels
// (restriction is linear and keeps node 0).
hsdc_status pfasst_iteration3(hsdc_ctx *c, double *res_host, int32_t *conv) {
  Level &F = c->L[0], &Mi = c->L[1], &C = c->L[2];
  const int P = F.P, M1 = Mi.co.M, M2 = C.co.M, f = c->meth.space_coarsen;
  if (!c->ri_fresh) {
    const hsdc_status st = residual_pass(c, nullptr, true);
    if (st != HSDC_OK) throw StatusFail{st};
  }
  // level 1: tau_1 / dt = S I_0(z_0) - I_1(S z_0), then one Q^par sweep from
  // the restricted iterate
  const int64_t sRI1 = (int64_t)M1 * NF * Mi.g.Np;
  PLAUNCH(c, PC_TRANSFER, 8.0 * P * M1 * NF * ((double)F.g.N + Mi.g.N),
          launch_restrict_fields(c->s, F.g, Mi.g, f, F.RI, (int64_t)M1 * NF * F.g.Np, Mi.RI,
                                 sRI1, M1 * NF, P));
  restrict_stages_between(c, F, Mi, c->Rt);
  evaluate_all(c, Mi, 1, 0, P);
  PLAUNCH(c, PC_FAS, 8.0 * (3.0 * M1 * NF + M1 + NG) * Mi.g.N * P,
          launch_fas_integrals(c->s, Mi.g, Mi.st, Mi.co, 0, P, Mi.RI, sRI1));
  gather_starts(c, Mi, Mi.y0c, 0, P);
  sweep(c, Mi, 1, 0, P, Mi.U, Mi.RI, 0, false);
  // level 2: tau_2 / dt = S (I_1(z_1) + tau_1 / dt) - I_2(S z_1), then Q^seq
  const int64_t sRI2 = (int64_t)M2 * NF * Mi.g.Np, sRIc = (int64_t)M2 * NF * C.g.Np;
  PLAUNCH(c, PC_RESIDUAL, 8.0 * ((2.0 * M1 + 1) * NF + M1 + NG + M2 * NF) * Mi.g.N * P,
          launch_residual(c->s, Mi.g, Mi.st, Mi.co, 0, P, Mi.y0c, Mi.res_part, Mi.res_nblk,
                          Mi.res_out, c->Rt2, M2, Mi.RI2, sRI2, Mi.RI, sRI1));
  PLAUNCH(c, PC_TRANSFER, 8.0 * P * M2 * NF * ((double)Mi.g.N + C.g.N),
          launch_restrict_fields(c->s, Mi.g, C.g, f, Mi.RI2, sRI2, C.RI, sRIc, M2 * NF, P));
  restrict_stages_between(c, Mi, C, c->Rt2);
  evaluate_all(c, C, 2, 0, P);
  PLAUNCH(c, PC_FAS, 8.0 * (3.0 * M2 * NF + M2 + NG) * C.g.N * P,
          launch_fas_integrals(c->s, C.g, C.st, C.co, 0, P, C.RI, sRIc));
  for (int n = 0; n < P; ++n) {
    gather_starts(c, C, C.y0c, n, 1);
    sweep(c, C, 2, n, 1, C.U + n * C.st.sS(), C.RI, n % 14, true);
  }
  // up
  correct_between(c, Mi, C, c->Tt2, 1);
  gather_starts(c, Mi, Mi.y0c, 0, P);
  sweep(c, Mi, 1, 0, P, Mi.U, Mi.RI, 1, true);
  correct_between(c, F, Mi, c->Tt, 1);
  gather_starts(c, F, c->y0blk, 0, P);
  sweep(c, F, 0, 0, P, F.U, nullptr, c->sweep_index++);
  return finish_iteration(c, res_host, conv);
}

hsdc_status pfasst_iteration(hsdc_ctx *c, double *res_host, int32_t *conv) {
  if (c->nlev == 3) return pfasst_iteration3(c, res_host, conv);
  Level &F = c->L[0];
  const int P = F.P;
  // the active slices a0..P-1 (all of them unless prefix_stop has stopped a prefix)
  const int a0 = c->a0, na = P - a0;
  if (c->nlev == 2) with_coarse(c, [&](auto &Cc) {
    const int Mc = Cc.co.M;
    // tau (Algorithm 1): its rows i >= 1 are dt (S (A G)_f(z) - (A G)_c(S z))_i,
    // the row-0 and H parts cancel; the fine integrals come with the residual
    if (!c->ri_fresh) {
      std::vector<double> rel(P);
      const hsdc_status st = residual_pass(c, rel.data(), true, a0);
      if (st != HSDC_OK) throw StatusFail{st};
    }
    const int64_t sRIc = (int64_t)Mc * NF * Cc.g.Np, sRIf = (int64_t)Mc * NF * F.g.Np;
    run_coarse_part(c, Cc, [&]() {
      PLAUNCH(c, PC_TRANSFER, 8.0 * na * Mc * NF * ((double)F.g.N + Cc.g.N),
              launch_restrict_fields(c->s, F.g, Cc.g, c->meth.space_coarsen, F.RI + a0 * sRIf,
                                     sRIf, Cc.RI + a0 * sRIc, sRIc, Mc * NF, na));
      restrict_fine_to_coarse(c, Cc, a0, na);
      evaluate_all(c, Cc, 1, a0, na);
      PLAUNCH(c, PC_FAS, 8.0 * (3.0 * Mc * NF + Mc + NG) * Cc.g.N * na,
              launch_fas_integrals(c->s, Cc.g, Cc.st, Cc.co, a0, na, Cc.RI, sRIc));
      for (int n = a0; n < P; ++n) {  // Q^seq: slice by slice with the new end values
        gather_starts(c, Cc, Cc.y0c, n, 1);
        // the right-hand side is evaluated at S z (kept in Sz until the
        // correction); budgets per slice (rows 0..13; the burn-in has row 15)
        sweep(c, Cc, 1, n, 1, Cc.U + n * Cc.st.sS(), Cc.RI, n % 14, true, Cc.Sz);
      }
    });
    coarse_correct_fine(c, Cc, 1, a0, na);
  });
  // Q^par on the fine level: start values from the (corrected) iterate
  gather_starts(c, F, c->y0blk, a0, na);
  sweep(c, F, 0, a0, na, F.U + a0 * F.st.sS(), nullptr, c->sweep_index++);
  return finish_iteration(c, res_host, conv);
}

}  // namespace

// ---------------------------------------------------------------------------
// graph replay of serial steps
// ---------------------------------------------------------------------------

// Capture one serial step from the state begin_serial_step leaves: save y_n,
// max_iter budgeted sweeps, y_{n+1} = y_{n,M}, advance the device step
// counter, begin the next step.  The host-side counters and the CG log
// entries of the step are kept for the replays.
void capture_serial_step(hsdc_ctx *c) {
  Level &F = c->L[0];
  graph_release(c);
  c->cg_pending.clear();
  c->cg_log_used = 0;
  const hsdc_stats before = c->stats;
  const int K = c->meth.max_iter;
  HIPC(hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
  try {
    HIPC(launch_copy_fields(c->s, F.g.Np, c->ybak, F.st.sS(), F.st.Y, F.st.sY(), NF, F.P));
    c->safe_cg = false;
    for (int k = 0; k < K; ++k)
      sweep(c, F, 0, 0, F.P, nullptr, nullptr, c->sweep_index++, k == K - 1);
    HIPC(launch_copy_fields(c->s, F.g.Np, F.st.Y, F.st.sY(), F.st.Y + (int64_t)F.co.M * F.st.sS(),
                            F.st.sY(), NF, F.P));
    HIPC(launch_step_add(c->s, c->d_step, 1));
    begin_serial_step(c);
  } catch (...) {
    hipGraph_t g = nullptr;
    hipStreamEndCapture(c->s, &g);
    if (g) hipGraphDestroy(g);
    c->cg_pending.clear();
    c->cg_log_used = 0;
    c->stats = before;
    throw;
  }
  HIPC(hipStreamEndCapture(c->s, &c->graph));
  HIPC(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  c->graph_pending = c->cg_pending;
  c->graph_log_used = c->cg_log_used;
  c->cg_pending.clear();
  c->cg_log_used = 0;
  c->graph_sweeps = c->stats.sweeps - before.sweeps;
  c->graph_ionic = c->stats.ionic_evals - before.ionic_evals;
  c->stats = before;
  c->graph_dirty = false;
}

// One serial step by graph replay; a step whose budgeted solve missed cg_rtol
// is recomputed from the saved y_n with every solve checked.
void graph_step(hsdc_ctx *c) {
  Level &F = c->L[0];
  if (c->graph_dirty || !c->gexec) capture_serial_step(c);
  c->cg_pending = c->graph_pending;
  c->cg_log_used = c->graph_log_used;
  c->cg_fails = 0;
  int pred0[16][MAXM];
  std::memcpy(pred0, F.cg_pred, sizeof(pred0));
  HIPC(hipGraphLaunch(c->gexec, c->s));
  c->stats.sweeps += c->graph_sweeps;
  c->stats.ionic_evals += c->graph_ionic;
  flush_cg_log(c);
  if (c->cg_fails > 0 && !c->nonfinite) {
    c->stats.cg_redo_steps += 1;
    c->cg_fails = 0;
    HIPC(launch_copy_fields(c->s, F.g.Np, F.st.Y, F.st.sY(), c->ybak, F.st.sS(), NF, F.P));
    HIPC(launch_step_set(c->s, c->d_step, c->step));
    c->safe_cg = true;
    begin_serial_step(c);
    while (c->sweeps_done < c->meth.max_iter) {
      const bool last = c->sweeps_done == c->meth.max_iter - 1;
      sweep(c, F, 0, 0, F.P, nullptr, nullptr, c->sweep_index++, last);
      c->sweeps_done += 1;
    }
    HIPC(launch_copy_fields(c->s, F.g.Np, F.st.Y, F.st.sY(), F.st.Y + (int64_t)F.co.M * F.st.sS(),
                            F.st.sY(), NF, F.P));
    HIPC(launch_step_add(c->s, c->d_step, 1));
    begin_serial_step(c);
  }
  // host flags as begin_serial_step leaves them (a replay does not rerun host code)
  c->spread_pending = true;
  c->sweeps_done = 0;
  c->sweep_index = 0;
  c->safe_cg = true;
  c->step += 1;
  c->stats.steps += 1;
  c->graph_steps += 1;
  if (c->graph_steps % 16 == 0) {
    // relaxation: budgets down to the most iterations used since the last one
    // (also to none: after a Chebyshev start most solves need no iteration)
    for (int r = 0; r < 16; ++r)
      for (int i = 0; i < MAXM; ++i)
        if (F.cg_umax[r][i] >= 0) {
          F.cg_pred[r][i] = F.cg_umax[r][i] + cg_margin(c, F.tiled_start);
          F.cg_umax[r][i] = -1;
        }
  }
  if (std::memcmp(pred0, F.cg_pred, sizeof(pred0)) != 0) c->graph_dirty = true;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
namespace {
template <class Fn>
hsdc_status run_guarded(hsdc_ctx *c, Fn &&fn) {
  try {
    return fn();
  } catch (const StatusFail &f) {
    return f.st;
  } catch (const HipFail &h) {
    std::string m = std::string("HIP error in ") + h.what + ": " + hipGetErrorString(h.e);
    if (h.e == hipErrorOutOfMemory || h.e == hipErrorMemoryAllocation) return fail(c, HSDC_ENOMEM, m);
    return fail(c, HSDC_EDEVICE, m);
  } catch (const std::exception &e) {
    return fail(c, HSDC_EDEVICE, e.what());
  }
}
}  // namespace

extern "C" {

hsdc_status hsdc_init_state(const hsdc_problem *prob, const hsdc_method *meth, const double *y0,
                            void *hip_stream, hsdc_ctx **out) {
  if (!out) return fail(nullptr, HSDC_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!check_problem(prob, why)) return fail(nullptr, HSDC_EINVAL, why);
  if (!check_method(meth, prob, why)) return fail(nullptr, HSDC_EINVAL, why);
  if (meth->levels == 1 && meth->P > 1)
    return fail(nullptr, HSDC_EINVAL, "P > 1 needs levels >= 2");
  hsdc_ctx *c = new hsdc_ctx();
  c->s = (hipStream_t)hip_stream;
  c->prob = *prob;
  c->meth = *meth;
  c->nlev = meth->levels;
  c->cf32 = meth->levels == 2 && meth->coarse_fp32 != 0;
  c->pfasst = !(meth->levels == 1 && meth->P == 1);
  hsdc_status st = run_guarded(c, [&]() -> hsdc_status {
    const int P = meth->P;
    Level &F = c->L[0];
    F.g = make_grid(*prob, prob->nx, prob->ny, prob->nz, prob->dx);
    if (!make_colloc(meth->M[0], meth->dt, F.co))
      return fail(c, HSDC_EINVAL, "Radau node computation failed");
    const int Mc = c->nlev >= 2 ? meth->M[1] : 0;
    alloc_level(c, F, meth->M[0], P, false, Mc);
    if (prob->sigma_node) build_faces(c, F, prob->sigma_node);
    c->y0blk = dalloc<double>(c, (size_t)NF * F.g.Np);
    c->d_step = dalloc<int64_t>(c, 1);  // step 0
    c->cg_log_cap = 8192;
    c->cg_log = halloc<CgScalars>(c, c->cg_log_cap);
    c->cg_dlog = dalloc<CgScalars>(c, c->cg_log_cap);
    if (prob->stim_w) {
      F.stim_w = dalloc<double>(c, F.g.Np);
      HIPC(hipMemcpyAsync(F.stim_w, prob->stim_w, F.g.N * sizeof(double),
                          hipMemcpyDeviceToDevice, c->s));
    }
    for (int l = 0; l < 3; ++l) {
      c->stim[l].step = c->d_step;
      c->stim[l].tn = 1;  // slice n is time step step + n
      c->stim[l].amp = prob->stim_amp;
      c->stim[l].t0 = prob->stim_t0;
      c->stim[l].dur = prob->stim_dur;
      c->stim[l].eps = 1e-9 * meth->dt;
      c->stim[l].Cm = prob->Cm;
    }
    c->stim[0].w = F.stim_w;
    if (c->nlev == 2) {
      const int f = meth->space_coarsen;
      const int cnx = prob->nx > 1 ? prob->nx / f : 1;
      const int cny = prob->ny > 1 ? prob->ny / f : 1;
      const int cnz = prob->nz > 1 ? prob->nz / f : 1;
      bool ok = true;
      with_coarse(c, [&](auto &Cc) {
        Cc.g = make_grid(*prob, cnx, cny, cnz, prob->dx * f);
        if (!make_colloc(meth->M[1], meth->dt, Cc.co)) {
          ok = false;
          return;
        }
        alloc_level(c, Cc, meth->M[1], P, true, Mc);
        if (prob->sigma_node) build_faces(c, Cc, prob->sigma_node);  // f == 1 only
        if (F.stim_w) {
          Cc.stim_w = dalloc<double>(c, Cc.g.Np);
          HIPC(launch_restrict_fields(c->s, F.g, Cc.g, f, F.stim_w, 0,
                                      Cc.stim_w, 0, 1, 1));
        }
        c->stim[1].w = Cc.stim_w;
      });
      if (!ok) return fail(c, HSDC_EINVAL, "Radau node computation failed");
      const Colloc &cco = c->cf32 ? c->Lf.co : c->L[1].co;
      std::vector<double> R((Mc + 1) * (meth->M[0] + 1)), T((meth->M[0] + 1) * (Mc + 1));
      transfer_matrix(meth->M[0], F.co.c, Mc, cco.c, R.data());
      transfer_matrix(Mc, cco.c, meth->M[0], F.co.c, T.data());
      c->Rt = dalloc<double>(c, R.size());
      c->Tt = dalloc<double>(c, T.size());
      HIPC(hipMemcpyAsync(c->Rt, R.data(), R.size() * sizeof(double), hipMemcpyHostToDevice, c->s));
      HIPC(hipMemcpyAsync(c->Tt, T.data(), T.size() * sizeof(double), hipMemcpyHostToDevice, c->s));
      HIPC(hipStreamSynchronize(c->s));  // R and T go out of scope
    }
    if (c->nlev == 3) {
      // levels 1 and 2, FP64, each on the mesh of the one above coarsened by f
      const int f = meth->space_coarsen;
      Level *up = &F;
      for (int l = 1; l < 3; ++l) {
        Level &L = c->L[l];
        const Grid &gu = up->g;
        L.g = make_grid(*prob, gu.nx > 1 ? gu.nx / f : 1, gu.ny > 1 ? gu.ny / f : 1,
                        gu.nz > 1 ? gu.nz / f : 1, prob->dx * (l == 1 ? f : f * f));
        if (!make_colloc(meth->M[l], meth->dt, L.co))
          return fail(c, HSDC_EINVAL, "Radau node computation failed");
        alloc_level(c, L, meth->M[l], P, true, meth->M[l]);
        if (prob->sigma_node) build_faces(c, L, prob->sigma_node);  // f == 1 only
        if (up->stim_w) {
          L.stim_w = dalloc<double>(c, L.g.Np);
          HIPC(launch_restrict_fields(c->s, gu, L.g, f, up->stim_w, 0, L.stim_w, 0, 1, 1));
        }
        c->stim[l].w = L.stim_w;
        std::vector<double> R((L.co.M + 1) * (up->co.M + 1)), T((up->co.M + 1) * (L.co.M + 1));
        transfer_matrix(up->co.M, up->co.c, L.co.M, L.co.c, R.data());
        transfer_matrix(L.co.M, L.co.c, up->co.M, up->co.c, T.data());
        double *dR = dalloc<double>(c, R.size()), *dT = dalloc<double>(c, T.size());
        HIPC(hipMemcpyAsync(dR, R.data(), R.size() * sizeof(double), hipMemcpyHostToDevice, c->s));
        HIPC(hipMemcpyAsync(dT, T.data(), T.size() * sizeof(double), hipMemcpyHostToDevice, c->s));
        HIPC(hipStreamSynchronize(c->s));
        (l == 1 ? c->Rt : c->Rt2) = dR;
        (l == 1 ? c->Tt : c->Tt2) = dT;
        up = &L;
      }
      // the middle level's residual pass restricts its integrals to level 2
      Level &Mi = c->L[1];
      Mi.RI2 = dalloc<double>(c, (size_t)P * meth->M[2] * NF * Mi.g.Np);
      Mi.res_nblk = residual_blocks(Mi.g);
      Mi.res_part = dalloc<double>(c, (size_t)P * 2 * Mi.res_nblk);
      Mi.res_out = dalloc<double>(c, (size_t)2 * NF * P);
    }
    // initial state
    if (y0) {
      for (int f = 0; f < NF; ++f)
        HIPC(hipMemcpyAsync(c->y0blk + f * F.g.Np, y0 + f * F.g.N, F.g.N * sizeof(double),
                            hipMemcpyDeviceToDevice, c->s));
    } else {
      HIPC(launch_fill_rest(c->s, F.g.N, F.g.Np, c->y0blk));
    }
    if (c->pfasst) {
      begin_block(c);
    } else {
      HIPC(launch_copy_fields(c->s, F.g.Np, F.st.Y, 0, c->y0blk, 0, NF, 1));
      begin_serial_step(c);
    }
    HIPC(hipStreamSynchronize(c->s));
    return HSDC_OK;
  });
  if (st != HSDC_OK) {
    g_free_error = c->err;
    hsdc_destroy(c);
    return st;
  }
  *out = c;
  return HSDC_OK;
}

hsdc_status hsdc_init_batch(const hsdc_problem *probs, int32_t count, const hsdc_method *meth,
                            const double *const *y0, void *hip_stream, hsdc_ctx **out) {
  if (!out) return fail(nullptr, HSDC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!probs || count < 1 || count > 4096)
    return fail(nullptr, HSDC_EINVAL, "count must be in 1..4096 and probs non-NULL");
  std::string why;
  for (int n = 0; n < count; ++n)
    if (!check_problem(&probs[n], why))
      return fail(nullptr, HSDC_EINVAL, "tissue " + std::to_string(n) + ": " + why);
  if (!check_method(meth, &probs[0], why)) return fail(nullptr, HSDC_EINVAL, why);
  if (meth->levels != 1 || meth->P != 1)
    return fail(nullptr, HSDC_EINVAL, "a batch takes levels = 1 and P = 1 (serial steps)");
  if (meth->solver == 3)
    return fail(nullptr, HSDC_EINVAL, "a batch solves by CG or Chebyshev (solver 0..2), not DCT-II");
  const hsdc_problem &p0 = probs[0];
  for (int n = 1; n < count; ++n) {
    const hsdc_problem &q = probs[n];
    bool same = q.dim == p0.dim && q.dx == p0.dx && q.chi == p0.chi && q.Cm == p0.Cm &&
                q.stim_amp == p0.stim_amp && q.stim_t0 == p0.stim_t0 &&
                q.stim_dur == p0.stim_dur && (q.sigma_node == nullptr) == (p0.sigma_node == nullptr) &&
                (q.stim_w == nullptr) == (p0.stim_w == nullptr);
    for (int a = 0; a < 3; ++a)
      same = same && q.sigma[a] == p0.sigma[a] && q.g_scale[a] == p0.g_scale[a];
    if (!same)
      return fail(nullptr, HSDC_EINVAL,
                  "tissue " + std::to_string(n) +
                      ": tissues of a batch differ only in nx, ny, nz, sigma_node and stim_w");
  }
  hsdc_ctx *c = new hsdc_ctx();
  c->s = (hipStream_t)hip_stream;
  c->prob = p0;
  c->meth = *meth;
  c->meth.P = count;
  c->nlev = 1;
  c->pfasst = false;
  c->batch = true;
  hsdc_status st = run_guarded(c, [&]() -> hsdc_status {
    Level &F = c->L[0];
    int big = 0;
    std::vector<int32_t> dims(RAG * count);
    for (int n = 0; n < count; ++n) {
      const hsdc_problem &q = probs[n];
      c->tissue_N.push_back((int64_t)q.nx * q.ny * q.nz);
      const FastDiv fx = make_fastdiv((uint32_t)q.nx), fy = make_fastdiv((uint32_t)q.ny);
      const int32_t row[RAG] = {q.nx, q.ny, q.nz, (int32_t)fx.m, fx.s1, fx.s2,
                                (int32_t)fy.m, fy.s1, fy.s2};
      for (int k = 0; k < RAG; ++k) dims[RAG * n + k] = row[k];
      if (c->tissue_N[n] > c->tissue_N[big]) big = n;
    }
    // rows padded to the largest tissue; slice n holds tissue n
    F.g = make_grid(p0, probs[big].nx, probs[big].ny, probs[big].nz, p0.dx);
    if (!make_colloc(meth->M[0], meth->dt, F.co))
      return fail(c, HSDC_EINVAL, "Radau node computation failed");
    for (int n = 0; n < count; ++n) c->tissue_dims.push_back({probs[n].nx, probs[n].ny});
    alloc_level(c, F, meth->M[0], count, false, 0);
    const int64_t Np = F.g.Np;
    c->rag = dalloc<int32_t>(c, dims.size());
    HIPC(hipMemcpyAsync(c->rag, dims.data(), dims.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                        c->s));
    F.g.rag = c->rag;
    // per-tissue spectral bounds (each tissue gets the bound of its own context)
    std::vector<double> lam(count);
    for (int n = 0; n < count; ++n)
      lam[n] = lam_uniform(p0.dim, probs[n].nx, probs[n].ny, probs[n].nz, F.g.cx, F.g.cy, F.g.cz);
    if (p0.sigma_node) {
      const double sc = 1.0 / (p0.dx * p0.dx * p0.chi * p0.Cm);
      for (int a = 0; a < p0.dim; ++a) F.kface[a] = dalloc<double>(c, (size_t)count * Np);
      for (int n = 0; n < count; ++n) {
        const hsdc_problem &q = probs[n];
        std::vector<double> s(c->tissue_N[n]);
        HIPC(hipMemcpyAsync(s.data(), q.sigma_node, s.size() * sizeof(double),
                            hipMemcpyDeviceToHost, c->s));
        HIPC(hipStreamSynchronize(c->s));
        std::vector<double> kh[3];
        for (int a = 0; a < p0.dim; ++a) {
          kh[a] = face_coeffs(a, q.nx, q.ny, q.nz, s, sc);
          HIPC(hipMemcpyAsync(F.kface[a] + n * Np, kh[a].data(), kh[a].size() * sizeof(double),
                              hipMemcpyHostToDevice, c->s));
        }
        lam[n] = lam_faces(p0.dim, q.nx, q.ny, q.nz, kh);
        HIPC(hipStreamSynchronize(c->s));
      }
      F.g.kx = F.kface[0];
      F.g.ky = p0.dim >= 2 ? F.kface[1] : nullptr;
      F.g.kz = p0.dim >= 3 ? F.kface[2] : nullptr;
    }
    set_lam(c, F, lam);
    c->d_step = dalloc<int64_t>(c, 1);  // step 0
    c->cg_log_cap = std::max(8192, 64 * count);
    c->cg_log = halloc<CgScalars>(c, c->cg_log_cap);
    c->cg_dlog = dalloc<CgScalars>(c, c->cg_log_cap);
    if (p0.stim_w) {
      F.stim_w = dalloc<double>(c, (size_t)count * Np);
      for (int n = 0; n < count; ++n)
        HIPC(hipMemcpyAsync(F.stim_w + n * Np, probs[n].stim_w, c->tissue_N[n] * sizeof(double),
                            hipMemcpyDeviceToDevice, c->s));
    }
    c->stim[0].w = F.stim_w;
    c->stim[0].sw = Np;
    c->stim[0].tn = 0;  // every tissue is at the same time step
    c->stim[0].step = c->d_step;
    c->stim[0].amp = p0.stim_amp;
    c->stim[0].t0 = p0.stim_t0;
    c->stim[0].dur = p0.stim_dur;
    c->stim[0].eps = 1e-9 * meth->dt;
    c->stim[0].Cm = p0.Cm;
    for (int n = 0; n < count; ++n) {
      double *Y0 = F.st.Y + n * F.st.sY();
      if (y0 && y0[n]) {
        for (int f = 0; f < NF; ++f)
          HIPC(hipMemcpyAsync(Y0 + f * Np, y0[n] + f * c->tissue_N[n],
                              c->tissue_N[n] * sizeof(double), hipMemcpyDeviceToDevice, c->s));
      } else {
        HIPC(launch_fill_rest(c->s, c->tissue_N[n], Np, Y0));
      }
    }
    begin_serial_step(c);
    HIPC(hipStreamSynchronize(c->s));
    return HSDC_OK;
  });
  if (st != HSDC_OK) {
    g_free_error = c->err;
    hsdc_destroy(c);
    return st;
  }
  *out = c;
  return HSDC_OK;
}

hsdc_status hsdc_tune(hsdc_ctx *c, int32_t cg_blocks_cap, int32_t cg_margin) {
  if (!c) return fail(nullptr, HSDC_EINVAL, "ctx is NULL");
  if (cg_blocks_cap > 2 * BLOCK) return fail(c, HSDC_EINVAL, "cg_blocks must be <= 1024");
  if (cg_margin > 64) return fail(c, HSDC_EINVAL, "cg_margin must be <= 64");
  if (cg_blocks_cap > 0) {
    c->tune_cg_blocks = cg_blocks_cap;
    for (int l = 0; l < c->nlev; ++l) {
      if (l == 1 && c->cf32)
        c->Lf.cg_nblk = cg_blocks(c->Lf.g, cg_blocks_cap);
      else
        c->L[l].cg_nblk = cg_blocks(c->L[l].g, cg_blocks_cap);
    }
  }
  if (cg_margin >= 0) c->tune_cg_margin = cg_margin;
  c->graph_dirty = true;
  return HSDC_OK;
}

hsdc_status hsdc_tune_shapes(hsdc_ctx *c, int32_t node_block, int32_t cg_tile,
                             int32_t prolong_tile) {
  if (!c) return fail(nullptr, HSDC_EINVAL, "ctx is NULL");
  if (node_block != 0 && node_block != 64 && node_block != 128 && node_block != 256 &&
      node_block != 512)
    return fail(c, HSDC_EINVAL, "node_block must be 0, 64, 128, 256 or 512");
  if (cg_tile < -1 || cg_tile >= kNumCgTiles)
    return fail(c, HSDC_EINVAL, "cg_tile must be -1 or 0..8");
  if (prolong_tile < -1 || prolong_tile >= kNumProlongTiles)
    return fail(c, HSDC_EINVAL, "prolong_tile must be -1 or 0..3");
  // FP64 levels; an FP32 coarse level keeps the default shapes
  for (int l = 0; l < c->nlev; ++l) {
    if (l == 1 && c->cf32) continue;
    Grid &g = c->L[l].g;
    if (node_block > 0) g.nub = node_block;
    if (cg_tile >= 0) g.ctile = cg_tile;
  }
  // the correction into the fine level
  if (prolong_tile >= 0) c->L[0].g.ptile = prolong_tile;
  for (int l = 0; l < c->nlev; ++l)
    if (!(l == 1 && c->cf32)) c->L[l].tiled_start = level_start_tiles(c, c->L[l]) > 0;
  c->graph_dirty = true;
  return HSDC_OK;
}

hsdc_status hsdc_use_graph(hsdc_ctx *c, int32_t on) {
  if (!c) return fail(nullptr, HSDC_EINVAL, "ctx is NULL");
  if (on && c->pfasst && c->nlev != 2)
    return fail(c, HSDC_EINVAL, "PFASST graph replay captures the coarse part of two levels");
  if (on && c->s == nullptr)
    return fail(c, HSDC_EINVAL, "graph replay needs a context created on a non-null stream");
  Level &F = c->L[0];
  const int64_t solves = c->pfasst ? (int64_t)c->meth.M[1] * F.P
                                   : (int64_t)c->meth.max_iter * F.co.M * F.P;
  if (on && solves > c->cg_log_cap)
    return fail(c, HSDC_EINVAL, "a captured part has more solves than the CG log holds");
  return run_guarded(c, [&]() -> hsdc_status {
    if (on && !c->ybak && !c->pfasst) c->ybak = dalloc<double>(c, (size_t)F.P * NF * F.g.Np);
    if (!on) graph_release(c);
    c->graph_on = on != 0;
    c->graph_dirty = true;
    return HSDC_OK;
  });
}

hsdc_status hsdc_single_block(hsdc_ctx *c, int32_t on) {
  if (!c) return fail(nullptr, HSDC_EINVAL, "ctx is NULL");
  c->single_block = on != 0;
  return HSDC_OK;
}

hsdc_status hsdc_sdc_sweep(hsdc_ctx *c, int32_t level, int32_t slice, int32_t nsweeps) {
  if (!c) return fail(nullptr, HSDC_EINVAL, "ctx is NULL");
  if (level != 0) return fail(c, HSDC_EINVAL, "level must be 0");
  if (slice < 0 || slice >= c->L[0].P) return fail(c, HSDC_EINVAL, "slice out of range");
  if (!c->pfasst && slice != 0)
    return fail(c, HSDC_EINVAL, "serial and batch contexts take slice 0 (a sweep covers every tissue)");
  if (nsweeps < 0) return fail(c, HSDC_EINVAL, "nsweeps must be >= 0");
  return run_guarded(c, [&]() -> hsdc_status {
    for (int k = 0; k < nsweeps; ++k) {
      if (c->pfasst)
        sweep(c, c->L[0], 0, slice, 1, nullptr, nullptr, 13);
      else  // serial and batch contexts: every slice (tissue) takes the sweep
        sweep(c, c->L[0], 0, 0, c->L[0].P, nullptr, nullptr, c->sweep_index++);
      if (!c->pfasst) c->sweeps_done += 1;
    }
    if (nsweeps > 0) c->ri_fresh = false;
    HIPC(hipGetLastError());
    return HSDC_OK;
  });
}

// Serial steps may run as one single-workgroup launch: a serial context (one
// tissue) on a 1D mesh of at most 256 nodes with the second-order stencil, CG
// or the Chebyshev iteration as its solver, between steps, without graph
// replay or kernel timing, unless hsdc_single_block turned it off.
static bool single_block_ok(const hsdc_ctx *c) {
  const Level &F = c->L[0];
  return c->single_block && !c->pfasst && c->nlev == 1 && F.P == 1 && F.g.dim == 1 &&
         F.g.nx <= 256 && F.g.rag == nullptr && F.g.order == 2 && c->meth.solver != 3 &&
         c->sweeps_done == 0 && !c->graph_on && !c->prof.on;
}

hsdc_status hsdc_advance(hsdc_ctx *c, int32_t nsteps) {
  if (!c) return fail(nullptr, HSDC_EINVAL, "ctx is NULL");
  if (nsteps < 0) return fail(c, HSDC_EINVAL, "nsteps must be >= 0");
  // the status describes this call: solves of earlier calls do not count
  const int64_t unconverged0 = c->stats.cg_unconverged;
  c->nonfinite = false;
  return run_guarded(c, [&]() -> hsdc_status {
    Level &F = c->L[0];
    if (single_block_ok(c) && nsteps > 0) {
      // the steps in launches of one workgroup (hsdc_small.hip), at most
      // kSmallChunk steps each (a launch of the 128-node cable: about 0.25 s)
      constexpr int kSmallChunk = 1024;
      if (!c->d_small) c->d_small = dalloc<int>(c, 1);
      const hsdc_problem &p = c->prob;
      const int K = c->meth.max_iter, M = F.co.M;
      for (int s0 = 0; s0 < nsteps && !c->nonfinite; s0 += kSmallChunk) {
        const int n = std::min(kSmallChunk, nsteps - s0);
        HIPC(launch_small_steps(c->s, F.g, F.st, F.co, c->stim[0], p.g_scale[0], p.g_scale[1],
                                p.g_scale[2], K, n, c->d_small));
        int flag = 0;
        HIPC(hipMemcpyAsync(&flag, c->d_small, sizeof(int), hipMemcpyDeviceToHost, c->s));
        HIPC(hipStreamSynchronize(c->s));
        const int done = flag < 0 ? -flag : flag;
        c->step += done;
        HIPC(launch_step_add(c->s, c->d_step, done));
        c->stats.steps += done;
        c->stats.sweeps += (int64_t)K * done;
        c->stats.cg_solves += (int64_t)K * M * done;  // direct solves: no CG iteration
        c->stats.ionic_evals += F.g.N * (int64_t)(1 + K * (M - 1) + (K - 1)) * done;
        c->nonfinite = flag < 0;
      }
      begin_serial_step(c);
      if (c->nonfinite) return fail(c, HSDC_ENONFINITE, "a step met a non-finite state");
      return HSDC_OK;
    }
    for (int s = 0; s < nsteps; ++s) {
      if (c->nonfinite) break;  // a non-finite state: no further step helps
      if (!c->pfasst && c->graph_on && !c->prof.on && c->sweeps_done == 0) {
        graph_step(c);
      } else if (!c->pfasst) {
        // budgeted solves, verified once per step; a step with a solve that
        // missed cg_rtol is recomputed from y_n with every solve checked
        c->safe_cg = false;
        c->cg_fails = 0;
        while (c->sweeps_done < c->meth.max_iter) {
          const bool last = c->sweeps_done == c->meth.max_iter - 1;
          sweep(c, F, 0, 0, F.P, nullptr, nullptr, c->sweep_index++, last);
          c->sweeps_done += 1;
        }
        flush_cg_log(c);
        c->safe_cg = true;
        if (c->cg_fails > 0 && !c->nonfinite) {
          c->stats.cg_redo_steps += 1;
          c->cg_fails = 0;
          begin_serial_step(c);
          while (c->sweeps_done < c->meth.max_iter) {
            const bool last = c->sweeps_done == c->meth.max_iter - 1;
            sweep(c, F, 0, 0, F.P, nullptr, nullptr, c->sweep_index++, last);
            c->sweeps_done += 1;
          }
        }
        // y_{n+1} = y_{n,M}
        HIPC(launch_copy_fields(c->s, F.g.Np, F.st.Y, F.st.sY(),
                                F.st.Y + (int64_t)F.co.M * F.st.sS(), F.st.sY(), NF, F.P));
        c->step += 1;
        HIPC(launch_step_add(c->s, c->d_step, 1));
        c->stats.steps += 1;
        begin_serial_step(c);
      } else {
        int32_t conv = 0;
        c->sweep_index = 0;
        for (int k = 0; k < c->meth.max_iter && !conv; ++k) {
          hsdc_status st = pfasst_iteration(c, nullptr, &conv);
          if (st != HSDC_OK) return st;
        }
        HIPC(launch_copy_fields(c->s, F.g.Np, c->y0blk, 0,
                                F.st.Y + (int64_t)(F.P - 1) * F.st.sY() +
                                    (int64_t)F.co.M * F.st.sS(),
                                0, NF, 1));
        c->step += F.P;
        HIPC(launch_step_add(c->s, c->d_step, F.P));
        c->stats.steps += F.P;
        begin_block(c);
      }
    }
    if (c->nonfinite) return fail(c, HSDC_ENONFINITE, "a diffusion solve met a non-finite state");
    if (c->stats.cg_unconverged > unconverged0)
      return fail(c, HSDC_ENOCONV, "a diffusion solve reached cg_maxit");
    return HSDC_OK;
  });
}

hsdc_status hsdc_pfasst_iter(hsdc_ctx *c, double *res_host, int32_t *all_converged) {
  if (!c) return fail(nullptr, HSDC_EINVAL, "ctx is NULL");
  if (!c->pfasst) return fail(c, HSDC_ESTATE, "context is in serial mode (levels = 1, P = 1)");
  return run_guarded(c, [&]() -> hsdc_status { return pfasst_iteration(c, res_host, all_converged); });
}

hsdc_status hsdc_residual(hsdc_ctx *c, int32_t level, double *res_host) {
  if (!c) return fail(nullptr, HSDC_EINVAL, "ctx is NULL");
  if (level != 0) return fail(c, HSDC_EINVAL, "level must be 0");
  if (!res_host) return fail(c, HSDC_EINVAL, "res_host is NULL");
  return run_guarded(c, [&]() -> hsdc_status { return residual_pass(c, res_host, false); });
}

static hsdc_status state_copy(hsdc_ctx *c, int32_t level, int32_t slice, int32_t node, double *dev,
                              bool get) {
  if (!c) return fail(nullptr, HSDC_EINVAL, "ctx is NULL");
  if (level < 0 || level >= c->nlev) return fail(c, HSDC_EINVAL, "level out of range");
  const int P = c->L[0].P;
  const int Ml = (level == 1 && c->cf32) ? c->Lf.co.M : c->L[level].co.M;
  if (slice < 0 || slice >= P) return fail(c, HSDC_EINVAL, "slice out of range");
  if (node < 0 || node > Ml) return fail(c, HSDC_EINVAL, "node out of range");
  if (!dev) return fail(c, HSDC_EINVAL, "buffer is NULL");
  return run_guarded(c, [&]() -> hsdc_status {
    if (node != 0 || !get) materialize(c);
    auto copy = [&](auto &L) {
      double *base = L.st.Y + slice * L.st.sY() + (int64_t)node * L.st.sS();
      const int64_t N = c->batch ? c->tissue_N[slice] : L.g.N;
      for (int f = 0; f < NF; ++f) {
        if (get)
          HIPC(hipMemcpyAsync(dev + f * N, base + f * L.g.Np, N * sizeof(double),
                              hipMemcpyDeviceToDevice, c->s));
        else
          HIPC(hipMemcpyAsync(base + f * L.g.Np, dev + f * N, N * sizeof(double),
                              hipMemcpyDeviceToDevice, c->s));
      }
      if (!get && c->pfasst) evaluate_all(c, L, level, slice, 1);
    };
    if (level == 1)
      with_coarse(c, copy);
    else
      copy(c->L[level]);
    if (!get) {
      c->ri_fresh = false;
      // keep the cached stage terms consistent with the new state
      Level &F = c->L[0];
      if (c->pfasst) {
        if (level == 0 && node == 0 && slice == 0) {
          for (int f = 0; f < NF; ++f)
            HIPC(hipMemcpyAsync(c->y0blk + f * F.g.Np, dev + f * F.g.N, F.g.N * sizeof(double),
                                hipMemcpyDeviceToDevice, c->s));
        }
      } else if (node == 0) {
        begin_serial_step(c);
      } else {
        evaluate_all(c, F, 0, slice, 1);
      }
    }
    HIPC(hipStreamSynchronize(c->s));
    return HSDC_OK;
  });
}

hsdc_status hsdc_get_state(const hsdc_ctx *c, int32_t level, int32_t slice, int32_t node,
                           double *dst) {
  return state_copy(const_cast<hsdc_ctx *>(c), level, slice, node, dst, true);
}

hsdc_status hsdc_set_state(hsdc_ctx *c, int32_t level, int32_t slice, int32_t node,
                           const double *src) {
  return state_copy(c, level, slice, node, const_cast<double *>(src), false);
}

int64_t hsdc_current_step(const hsdc_ctx *c) { return c ? c->step : -1; }

hsdc_status hsdc_get_stats(const hsdc_ctx *c, hsdc_stats *out) {
  if (!c || !out) return fail(const_cast<hsdc_ctx *>(c), HSDC_EINVAL, "NULL argument");
  *out = c->stats;
  return HSDC_OK;
}

hsdc_status hsdc_profile_enable(hsdc_ctx *c, int32_t on) {
  if (!c) return fail(nullptr, HSDC_EINVAL, "ctx is NULL");
  return run_guarded(c, [&]() -> hsdc_status {
    if (!on) prof_harvest(c);
    c->prof.on = on != 0;
    return HSDC_OK;
  });
}

hsdc_status hsdc_profile_read(hsdc_ctx *c, hsdc_kernel_profile *out, int32_t max, int32_t *count) {
  if (!c || (max > 0 && !out)) return fail(c, HSDC_EINVAL, "NULL argument");
  return run_guarded(c, [&]() -> hsdc_status {
    prof_harvest(c);
    Profiler &P = c->prof;
    int k = 0;
    for (int q = 0; q < PC_COUNT; ++q) {
      if (P.launches[q] == 0) continue;
      if (k < max) {
        hsdc_kernel_profile &o = out[k];
        std::memset(&o, 0, sizeof(o));
        std::strncpy(o.name, kProfNames[q], sizeof(o.name) - 1);
        o.launches = P.launches[q];
        o.total_ms = P.ms[q];
        o.bytes = P.bytes[q];
      }
      ++k;
      P.launches[q] = 0;
      P.ms[q] = 0.0;
      P.bytes[q] = 0.0;
    }
    if (count) *count = k;
    return HSDC_OK;
  });
}

void hsdc_destroy(hsdc_ctx *c) {
  if (!c) return;
  try {
    prof_harvest(c);
  } catch (...) {
  }
  for (hipEvent_t e : c->prof.pool) hipEventDestroy(e);
  graph_release(c);
  if (c->s) hipStreamSynchronize(c->s);
  else hipDeviceSynchronize();
  for (void *p : c->allocs) hipFree(p);
  for (void *p : c->host_allocs) hipHostFree(p);
  delete c;
}

const char *hsdc_last_error(const hsdc_ctx *c) {
  if (c) return c->err.c_str();
  return g_free_error.c_str();
}

// ---- exported building blocks ---------------------------------------------

hsdc_status hsdc_ionic_eval(int64_t n, const double *y, const double *g_scale_host3, double *I_ion,
                            double *h_a, double *lam, double *w_inf, void *hip_stream) {
  if (n < 0 || (n > 0 && (!y || !I_ion || !h_a || !lam || !w_inf)))
    return fail(nullptr, HSDC_EINVAL, "bad arguments");
  if (n == 0) return HSDC_OK;
  const double gs0 = g_scale_host3 ? g_scale_host3[0] : 1.0;
  const double gs1 = g_scale_host3 ? g_scale_host3[1] : 1.0;
  const double gs2 = g_scale_host3 ? g_scale_host3[2] : 1.0;
  hipError_t e = launch_ionic_test((hipStream_t)hip_stream, n, y, gs0, gs1, gs2, I_ion, h_a, lam, w_inf);
  if (e != hipSuccess) return fail(nullptr, HSDC_EDEVICE, hipGetErrorString(e));
  return HSDC_OK;
}

hsdc_status hsdc_phi(int64_t n, const double *x, int32_t kmax, double *out, void *hip_stream) {
  if (n < 0 || kmax < 1 || kmax > HSDC_MAX_M || (n > 0 && (!x || !out)))
    return fail(nullptr, HSDC_EINVAL, "bad arguments");
  if (n == 0) return HSDC_OK;
  hipError_t e = launch_phi_test((hipStream_t)hip_stream, n, x, kmax, out);
  if (e != hipSuccess) return fail(nullptr, HSDC_EDEVICE, hipGetErrorString(e));
  return HSDC_OK;
}

hsdc_status hsdc_apply_diffusion(const hsdc_problem *prob, const double *v, double *out,
                                 void *hip_stream) {
  std::string why;
  if (!check_problem(prob, why)) return fail(nullptr, HSDC_EINVAL, why);
  if (!v || !out) return fail(nullptr, HSDC_EINVAL, "NULL vector");
  hsdc_ctx tmp;
  tmp.s = (hipStream_t)hip_stream;
  tmp.prob = *prob;
  hsdc_status st = run_guarded(&tmp, [&]() -> hsdc_status {
    Level L;
    L.g = make_grid(*prob, prob->nx, prob->ny, prob->nz, prob->dx);
    if (prob->sigma_node) build_faces(&tmp, L, prob->sigma_node);
    HIPC(launch_apply_K(tmp.s, L.g, v, out));
    // the face coefficients of sigma_node are freed below, after the kernel
    if (!tmp.allocs.empty()) HIPC(hipStreamSynchronize(tmp.s));
    return HSDC_OK;
  });
  for (void *p : tmp.allocs) hipFree(p);
  tmp.allocs.clear();
  if (st != HSDC_OK) g_free_error = tmp.err;
  return st;
}

}  // extern "C"

namespace {
// One CG solve from the initial guess in cb.x, checked on the host every four
// launches (the building-block solves: no budget, no log).
void run_cg(hipStream_t s, const Grid &g, const CgBatch &cb, int *used, bool *conv) {
  HIPC(launch_cg_resid0(s, g, cb));
  HIPC(launch_cg_init(s, g, cb));
  CgScalars sc2[2];
  int k = 0;
  for (;;) {
    for (int q = 0; q < 4 && k <= cb.maxit; ++q, ++k) HIPC(launch_cg_iter(s, g, cb, k));
    HIPC(hipMemcpyAsync(sc2, cb.sc, sizeof(sc2), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (sc2[k & 1].done || k > cb.maxit) break;
  }
  const CgScalars &sc = sc2[k & 1];
  *used = sc.it;
  *conv = cg_ok(sc, cb.tol2);
}
}  // namespace

// ---- the diffusion solve without allocation -------------------------------
// Workspace of hsdc_diffusion_solve_noalloc, in doubles: the CG vectors r, w, s
// (two each) and p, then the face coefficients kx, ky, kz, each
// HSDC_NOALLOC_MAX_NODES long; then the 5 x kNaBlocks partial sums and the two
// CG scalars.  Each device holds its own copy at its own address; host code
// uses the address from hipGetSymbolAddress, never the name.
namespace {
constexpr int64_t kNaNodes = HSDC_NOALLOC_MAX_NODES;
constexpr int kNaBlocks = 2 * BLOCK;
constexpr size_t kNaVecs = 10;
constexpr size_t kNaDoubles = kNaVecs * (size_t)kNaNodes + 5 * (size_t)kNaBlocks +
                              2 * (sizeof(CgScalars) + 7) / 8;
static_assert(sizeof(CgScalars) % 8 == 0, "CG scalars are whole doubles");
constexpr int kNaMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kNaMaxDevices] = {};
}  // namespace

static __device__ __align__(256) double scratch[kNaDoubles];

namespace {
// Address of this device's scratch array, looked up on the first call on the
// device (with it current) and kept for the process.
hsdc_status scratch_address(double **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, HSDC_EDEVICE, hipGetErrorString(e));
  if (dev < 0 || dev >= kNaMaxDevices) return fail(nullptr, HSDC_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, HSDC_EDEVICE,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (double *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return HSDC_OK;
}
}  // namespace

extern "C" {

hsdc_status hsdc_diffusion_solve_noalloc(const hsdc_problem *prob, double a, const double *b,
                                         double *x, double rtol, int32_t maxit,
                                         int32_t *iters_host, void *hip_stream) {
  std::string why;
  if (!check_problem(prob, why)) return fail(nullptr, HSDC_EINVAL, why);
  if (!b || !x || !(rtol > 0) || maxit < 1 || !(a >= 0))
    return fail(nullptr, HSDC_EINVAL, "bad arguments");
  if ((int64_t)prob->nx * prob->ny * prob->nz > kNaNodes)
    return fail(nullptr, HSDC_EINVAL, "mesh larger than HSDC_NOALLOC_MAX_NODES");
  if (prob->fd_order == 4)
    return fail(nullptr, HSDC_EINVAL, "the no-allocation solve is CG on the second-order stencil");
  double *base = nullptr;
  hsdc_status st = scratch_address(&base);
  if (st != HSDC_OK) return st;
  const hipStream_t s = (hipStream_t)hip_stream;
  int used = 0;
  bool conv = false;
  try {
    Grid g = make_grid(*prob, prob->nx, prob->ny, prob->nz, prob->dx);
    double *vec[kNaVecs];
    for (size_t k = 0; k < kNaVecs; ++k) vec[k] = base + k * (size_t)kNaNodes;
    if (prob->sigma_node) {
      const double sc = 1.0 / (prob->dx * prob->dx * prob->chi * prob->Cm);
      HIPC(launch_faces(s, g, prob->sigma_node, sc, vec[7], vec[8], vec[9]));
      g.kx = vec[7];
      g.ky = g.dim >= 2 ? vec[8] : nullptr;
      g.kz = g.dim >= 3 ? vec[9] : nullptr;
    }
    CgBatch cb{};
    cb.x = x;
    cb.b = b;
    for (int k = 0; k < 2; ++k) {
      cb.r[k] = vec[k];
      cb.w[k] = vec[2 + k];
      cb.s[k] = vec[4 + k];
    }
    cb.p = vec[6];
    cb.nslices = 1;
    cb.nblk = cg_blocks(g);
    cb.nblk0 = cb.nblk;
    cb.pstride = cb.nblk;
    cb.part = base + kNaVecs * (size_t)kNaNodes;
    cb.sc = (CgScalars *)(cb.part + 5 * (size_t)kNaBlocks);
    cb.log = nullptr;
    cb.last_k = -1;
    cb.a = a;
    cb.tol2 = rtol * rtol;
    cb.maxit = maxit;
    // every partial and scalar is written before it is read (k_cg_resid0 and
    // k_cg_init write them): nothing of an earlier call has to be cleared
    run_cg(s, g, cb, &used, &conv);
  } catch (const HipFail &h) {
    return fail(nullptr, HSDC_EDEVICE, std::string("HIP error in ") + h.what + ": " +
                                           hipGetErrorString(h.e));
  }
  if (iters_host) *iters_host = used;
  if (!conv) return fail(nullptr, HSDC_ENOCONV, "CG reached maxit");
  return HSDC_OK;
}

hsdc_status hsdc_diffusion_solve(const hsdc_problem *prob, double a, const double *b, double *x,
                                 double rtol, int32_t maxit, int32_t *iters_host,
                                 void *hip_stream) {
  std::string why;
  if (!check_problem(prob, why)) return fail(nullptr, HSDC_EINVAL, why);
  if (!b || !x || !(rtol > 0) || maxit < 1 || !(a >= 0))
    return fail(nullptr, HSDC_EINVAL, "bad arguments");
  hsdc_ctx tmp;
  tmp.s = (hipStream_t)hip_stream;
  tmp.prob = *prob;
  tmp.meth.cg_rtol = rtol;
  tmp.meth.cg_maxit = maxit;
  int used = 0;
  bool conv = false;
  hsdc_status st = run_guarded(&tmp, [&]() -> hsdc_status {
    Level L;
    L.g = make_grid(*prob, prob->nx, prob->ny, prob->nz, prob->dx);
    if (prob->sigma_node) build_faces(&tmp, L, prob->sigma_node);
    const int64_t Np = L.g.Np;
    if (L.g.order == 4) {
      // the fourth-order stencil: the exact DCT-II solve (no iterations)
      const DctPlan d = make_dct_plan(&tmp, L.g);
      double *t1 = dalloc<double>(&tmp, Np), *t2 = dalloc<double>(&tmp, Np);
      HIPC(launch_dct_solve(tmp.s, L.g, d, a, b, Np, x, Np, t1, t2, Np, 1));
      HIPC(hipStreamSynchronize(tmp.s));  // the plan and work vectors are freed below
      conv = true;
      return HSDC_OK;
    }
    L.cg_nblk = cg_blocks(L.g);
    CgBatch cb{};
    cb.x = x;
    cb.sx = 0;
    cb.b = b;
    cb.sb = 0;
    for (int k = 0; k < 2; ++k) {
      cb.r[k] = dalloc<double>(&tmp, Np);
      cb.w[k] = dalloc<double>(&tmp, Np);
      cb.s[k] = dalloc<double>(&tmp, Np);
    }
    cb.p = dalloc<double>(&tmp, Np);
    cb.part = dalloc<double>(&tmp, 5 * L.cg_nblk);
    cb.sc = dalloc<CgScalars>(&tmp, 2);
    cb.log = nullptr;
    cb.last_k = -1;
    cb.nslices = 1;
    cb.nblk = L.cg_nblk;
    cb.nblk0 = L.cg_nblk;
    cb.pstride = L.cg_nblk;
    cb.a = a;
    cb.tol2 = rtol * rtol;
    cb.maxit = maxit;
    run_cg(tmp.s, L.g, cb, &used, &conv);
    return HSDC_OK;
  });
  for (void *p : tmp.allocs) hipFree(p);
  tmp.allocs.clear();
  if (iters_host) *iters_host = used;
  if (st != HSDC_OK) {
    g_free_error = tmp.err;
    return st;
  }
  if (!conv) return fail(nullptr, HSDC_ENOCONV, "CG reached maxit");
  return HSDC_OK;
}

hsdc_status hsdc_colloc_coefficients(int32_t M, int64_t n, const double *z, double *out,
                                     double *c_host, void *hip_stream) {
  if (M < 1 || M > HSDC_MAX_M || n < 0 || (n > 0 && (!z || !out)))
    return fail(nullptr, HSDC_EINVAL, "bad arguments");
  Colloc co;
  if (!make_colloc(M, 1.0, co)) return fail(nullptr, HSDC_EINVAL, "Radau node computation failed");
  if (c_host)
    for (int i = 0; i < M; ++i) c_host[i] = co.c[i];
  if (n == 0) return HSDC_OK;
  hipError_t e = launch_aij_test((hipStream_t)hip_stream, n, z, co, out);
  if (e != hipSuccess) return fail(nullptr, HSDC_EDEVICE, hipGetErrorString(e));
  return HSDC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// discrete adjoint of serial hybrid SDC: the gradient of a probe-voltage
// misfit L = sum over samples s and probes q of (V_q(t_s) - target_{s,q})^2
// with respect to the per-node conductivity, the G_Na, G_CaL, G_Kr scalings
// and the initial state.  The forward run keeps y_n before every step (the
// per-step checkpoints); the reverse run recomputes each step from its
// checkpoint with every sweep's iterate kept, and runs the step backwards
// (hsdc_adjoint.hip: the transposed sweep of eqs. prec_picard, def_P, def_C).
// ---------------------------------------------------------------------------
struct hsdc_adj {
  hsdc_ctx *c = nullptr;  // the forward's context; its workspace serves the recompute
  int nsteps = 0, every = 0, np = 0, nsamples = 0;
  double loss = 0.0;
  double *ckpt = nullptr;     // [nsteps + 1][NF][Np] y_n before step n, and the final state
  int64_t *probes = nullptr;  // [np]
  double *targets = nullptr;  // [nsamples][np]
  double *sigma = nullptr;    // [N] per-node sigma, or null
  double *work = nullptr;     // the reverse run's buffers (allocated on first use)
  // CG launches of the forward's budgeted solves, step n at cg_used[cg_off[n]..cg_off[n + 1])
  std::vector<int> cg_used;
  std::vector<int64_t> cg_off;
};

namespace {

// The adjoint of one step's sweeps; lam holds the adjoint of y_{n+1} on entry
// and receives that of y_n.  Xs must hold the step's iterates X^0 .. X^K.
struct AdjBuffers {
  double *Xs, *MU, *MUX, *RHO, *lam, *DYN, *DZ, *DLAM, *W, *dk, *PS, *gs_part, *gs_acc;
  double *bak;          // lam, dk and gs_acc before the step (a budgeted step run again)
  CgScalars *dlog;      // final scalars of the step's adjoint solves, [K][M]
  std::vector<int> *pred;  // CG launches per adjoint solve (sweep, node); -1: not yet known
};

// The adjoint diffusion solves of a step run at predicted numbers of CG
// launches without a host synchronisation; their final scalars go to dlog and
// are checked once per step (adjoint_verify).  In safe mode each solve is run
// to convergence with host checks, and its launches become the prediction.
// With the Chebyshev tables of the forward solves (solver 0 or 1), the CG
// starts from x_D, D Chebyshev steps from x_0 = b (a spectral interval of the
// operator is known, so they need no inner products).  Where the forward
// solves take the one-launch start (solver 0, 2D meshes), so do these: x_1
// with the partials of ||b||^2, then x_2 .. x_7, r_7, w_7 and their partials
// in one launch, and CG continues from launch k = 1.
constexpr int kAdjChebDegree = 8;  // even: x_D lands in x

void adjoint_solve(hsdc_ctx *c, const AdjBuffers &b, const CgBatch &cb0, int k, int i, bool safe) {
  Level &F = c->L[0];
  const hipStream_t s = c->s;
  const int M = F.co.M;
  CgBatch cb = cb0;
  const int tiles = F.cheb_x ? level_start_tiles(c, F) : 0;
  if (F.cheb_x) {
    CgBatch cs = cb;
    cs.xt = F.cheb_x;
    cs.tab = F.cheb_tab + (i - 1);
    cs.tab_stride = M;
    if (tiles > 0) {
      // x_0 = b: the start reads it from p (and only reads p) and writes x_7 to x
      cs.p = const_cast<double *>(cb.b);
      cs.cstart = kChebStartDegreeTiled;
      cs.x0_to_p = 1;
      HIPC(launch_adj_cheb_x1(s, F.g, cb.b, cb.b, cb.a, cs.tab, cs.xt, cb.part + 4 * cb.pstride));
      HIPC(launch_cg_start_tiled(s, F.g, cs, tiles));
      cb.cstart = kChebStartDegreeTiled;
      cb.nblk_s = tiles;
      cb.nblk0 = (int)((F.g.N + kAdjBlock - 1) / kAdjBlock);
    } else {
      HIPC(launch_adj_cheb_x1(s, F.g, cb.x, cb.b, cb.a, cs.tab, cs.xt, nullptr));
      HIPC(launch_cheb_steps(s, F.g, cs, kAdjChebDegree - 1));
    }
  }
  int &pred = (*b.pred)[(k - 1) * M + (i - 1)];
  if (safe) {
    int used = 0;
    bool conv = false;
    run_cg(s, F.g, cb0, &used, &conv);  // from the start's x_D
    if (!conv) {
      fail(c, HSDC_ENOCONV, "an adjoint diffusion solve reached cg_maxit");
      throw StatusFail{HSDC_ENOCONV};
    }
    c->stats.cg_iters += used;
    c->stats.cg_solves += 1;
    pred = used + 2;
    return;
  }
  const int budget = std::max(1, std::min(pred, cb.maxit + 1));
  const int k0 = tiles > 0 ? 1 : 0;  // the one-launch start's vectors have parity 1
  if (k0 == 0) {
    HIPC(launch_cg_resid0(s, F.g, cb));
    HIPC(launch_cg_init(s, F.g, cb));
  }
  for (int q = k0; q < budget + k0; ++q) HIPC(launch_cg_iter(s, F.g, cb, q));
  HIPC(hipMemcpyAsync(b.dlog + (int64_t)(k - 1) * M + (i - 1), cb.sc + ((budget + k0) & 1),
                      sizeof(CgScalars), hipMemcpyDeviceToDevice, s));
}

// One host synchronisation: did every adjoint solve of the step converge?
// Predictions follow the iterations used plus two launches, lowered by at
// most one per step, raised at once.
bool adjoint_verify(hsdc_ctx *c, const AdjBuffers &b) {
  Level &F = c->L[0];
  const int n = c->meth.max_iter * F.co.M;
  std::vector<CgScalars> h(n);
  HIPC(hipMemcpyAsync(h.data(), b.dlog, n * sizeof(CgScalars), hipMemcpyDeviceToHost, c->s));
  HIPC(hipStreamSynchronize(c->s));
  const double tol2 = c->meth.cg_rtol * c->meth.cg_rtol;
  bool ok = true;
  for (int q = 0; q < n; ++q) {
    int &pred = (*b.pred)[q];
    if (!cg_ok(h[q], tol2)) {
      ok = false;
      continue;
    }
    c->stats.cg_iters += h[q].it;
    c->stats.cg_solves += 1;
    pred = std::max(h[q].it + 2, pred - 1);
  }
  return ok;
}

void adjoint_step(hsdc_ctx *c, const AdjBuffers &b, bool safe) {
  Level &F = c->L[0];
  const int M = F.co.M, K = c->meth.max_iter;
  const int64_t Np = F.g.Np, sS = (int64_t)NF * Np, sY = (int64_t)(M + 1) * sS;
  const hipStream_t s = c->s;
  double *MU = b.MU, *MUX = b.MUX;
  HIPC(hipMemsetAsync(MU, 0, sY * sizeof(double), s));
  HIPC(hipMemsetAsync(b.DYN, 0, sS * sizeof(double), s));
  HIPC(hipMemsetAsync(b.DZ, 0, (size_t)NG * Np * sizeof(double), s));
  HIPC(hipMemsetAsync(b.DLAM, 0, (size_t)NG * Np * sizeof(double), s));
  HIPC(hipMemcpyAsync(MU + (int64_t)M * sS, b.lam, sS * sizeof(double), hipMemcpyDeviceToDevice, s));
  AdjArgs a{};
  a.N = F.g.N;
  a.Np = Np;
  a.co = F.co;
  for (int q = 0; q < 3; ++q) a.gs[q] = c->prob.g_scale[q];
  a.L0 = F.st.L0;
  a.RHO = b.RHO;
  a.DYN = b.DYN;
  a.DZ = b.DZ;
  a.DLAM = b.DLAM;
  a.W = b.W;
  a.PS = b.PS;
  a.gs_part = b.gs_part;
  a.gs_acc = b.gs_acc;
  double *dkx = b.dk, *dky = b.dk + Np, *dkz = b.dk + 2 * Np;
  for (int k = K; k >= 1; --k) {
    const double *X = b.Xs + (int64_t)(k - 1) * sY, *Z = b.Xs + (int64_t)k * sY;
    HIPC(hipMemsetAsync(MUX, 0, sY * sizeof(double), s));
    a.X = X;
    a.Z = Z;
    a.MU = MU;
    a.MUX = MUX;
    for (int i = M; i >= 1; --i) {
      // beta_i^V = (I - dt d_i K)^-1 MU_i^V (the operator is symmetric)
      CgBatch cb{};
      cb.x = b.RHO + (int64_t)i * sS;
      cb.b = MU + (int64_t)i * sS;
      HIPC(hipMemcpyAsync(cb.x, cb.b, Np * sizeof(double), hipMemcpyDeviceToDevice, s));
      for (int q = 0; q < 2; ++q) {
        cb.r[q] = F.cg_r[q];
        cb.w[q] = F.cg_w[q];
        cb.s[q] = F.cg_s[q];
      }
      cb.p = F.cg_p;
      cb.part = F.cg_part;
      cb.pstride = F.cg_pstride;
      cb.sc = F.cg_sc;
      cb.log = nullptr;
      cb.last_k = -1;
      cb.nslices = 1;
      cb.nblk = cg_blocks(F.g);
      cb.nblk0 = cb.nblk;
      cb.a = F.co.dt * F.co.d[i - 1];
      cb.tol2 = c->meth.cg_rtol * c->meth.cg_rtol;
      cb.maxit = c->meth.cg_maxit;
      adjoint_solve(c, b, cb, k, i, safe);
      HIPC(launch_adj_faces(s, F.g, cb.x, Z + (int64_t)i * sS, cb.a, dkx, dky, dkz));
      HIPC(launch_adj_backsub(s, a, i));
    }
    HIPC(launch_adj_assemble(s, a));
    for (int j = 1; j <= M; ++j) {
      HIPC(launch_adj_spmv_add(s, F.g, b.W + (int64_t)j * Np, 1.0, MUX + (int64_t)j * sS));
      HIPC(launch_adj_faces(s, F.g, b.W + (int64_t)j * Np, X + (int64_t)j * sS, 1.0, dkx, dky, dkz));
    }
    if (k > 1) {
      std::swap(MU, MUX);  // the previous sweep's result is this sweep's X
    } else {
      for (int j = 1; j <= M; ++j)  // X^0 = 1 (x) y_n
        HIPC(launch_adj_axpy(s, b.DYN, MUX + (int64_t)j * sS, sS));
    }
  }
  a.Z = b.Xs;  // stage 0: y_n
  HIPC(launch_adj_anchor(s, a));
  HIPC(hipMemcpyAsync(b.lam, b.DYN, sS * sizeof(double), hipMemcpyDeviceToDevice, s));
}

// Recompute step n from its checkpoint, keeping every sweep's iterate.  The
// solves run at budgets, verified once at the end (flush_cg_log); a step with
// a solve that missed cg_rtol is recomputed with every solve checked.
void recompute_step(hsdc_ctx *c, const hsdc_adj *adj, int n, double *Xs, bool safe = false) {
  Level &F = c->L[0];
  const int M = F.co.M, K = c->meth.max_iter;
  const int64_t sY = F.st.sY();
  c->step = n;
  HIPC(launch_step_set(c->s, c->d_step, n));
  HIPC(launch_copy_fields(c->s, F.g.Np, F.st.Y, 0, adj->ckpt + (int64_t)n * NF * F.g.Np, 0, NF, 1));
  begin_serial_step(c);
  materialize(c);
  // the forward's own launches as budgets: the recomputation repeats its work
  if (!safe && (int64_t)adj->cg_off.size() > n + 1 &&
      adj->cg_off[n + 1] - adj->cg_off[n] == (int64_t)K * M) {
    const int *u = adj->cg_used.data() + adj->cg_off[n];
    bool known = true;
    for (int q = 0; q < K * M; ++q) known = known && u[q] >= 0;
    if (known)
      for (int k = 0; k < K; ++k)
        for (int i = 1; i <= M; ++i) F.cg_pred[k & 15][i - 1] = u[k * M + (i - 1)];
  }
  c->safe_cg = safe;
  c->cg_fails = 0;
  HIPC(launch_copy_fields(c->s, F.g.Np, Xs, 0, F.st.Y, 0, (M + 1) * NF, 1));
  for (int k = 1; k <= K; ++k) {
    sweep(c, F, 0, 0, 1, nullptr, nullptr, k - 1, false);
    HIPC(launch_copy_fields(c->s, F.g.Np, Xs + (int64_t)k * sY, 0, F.st.Y, 0, (M + 1) * NF, 1));
  }
  if (safe) return;
  flush_cg_log(c);
  c->safe_cg = true;
  if (c->nonfinite) {
    fail(c, HSDC_ENONFINITE, "non-finite state in the recomputed step");
    throw StatusFail{HSDC_ENONFINITE};
  }
  if (c->cg_fails > 0) {
    c->stats.cg_redo_steps += 1;
    c->cg_fails = 0;
    recompute_step(c, adj, n, Xs, true);
  }
}

}  // namespace

extern "C" {

hsdc_status hsdc_misfit_forward(const hsdc_problem *prob, const hsdc_method *meth, const double *y0,
                                int32_t nsteps, int32_t sample_every, int32_t nprobes,
                                const int64_t *probes, const double *targets, double *loss_host,
                                hsdc_adj **out, void *hip_stream) {
  if (!out) return fail(nullptr, HSDC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!prob || !meth) return fail(nullptr, HSDC_EINVAL, "problem or method is NULL");
  if (meth->levels != 1 || meth->P != 1)
    return fail(nullptr, HSDC_EINVAL, "the adjoint is of serial hybrid SDC (levels = 1, P = 1)");
  if (meth->M[0] > 6) return fail(nullptr, HSDC_EINVAL, "the adjoint takes M <= 6");
  if (prob->fd_order == 4 || meth->solver == 3)
    return fail(nullptr, HSDC_EINVAL,
                "the adjoint takes the second-order stencil and an iterative solver (0..2)");
  if (nsteps < 1 || sample_every < 1 || nprobes < 1 || !probes || !targets)
    return fail(nullptr, HSDC_EINVAL, "nsteps, sample_every, nprobes >= 1 and probes, targets needed");
  hsdc_ctx *c = nullptr;
  hsdc_status st = hsdc_init_state(prob, meth, y0, hip_stream, &c);
  if (st != HSDC_OK) return st;
  // the recomputation in the reverse run repeats the per-launch kernels' steps
  c->single_block = false;
  hsdc_adj *adj = new hsdc_adj();
  adj->c = c;
  adj->nsteps = nsteps;
  adj->every = sample_every;
  adj->np = nprobes;
  adj->nsamples = nsteps / sample_every;
  st = run_guarded(c, [&]() -> hsdc_status {
    Level &F = c->L[0];
    const int64_t N = F.g.N, Np = F.g.Np;
    std::vector<int64_t> hp(nprobes);
    HIPC(hipMemcpyAsync(hp.data(), probes, nprobes * sizeof(int64_t), hipMemcpyDeviceToHost, c->s));
    HIPC(hipStreamSynchronize(c->s));
    std::vector<int64_t> sorted(hp);
    std::sort(sorted.begin(), sorted.end());
    for (int q = 0; q < nprobes; ++q)
      if (sorted[q] < 0 || sorted[q] >= N || (q > 0 && sorted[q] == sorted[q - 1]))
        return fail(c, HSDC_EINVAL, "probes must be distinct node indices in [0, N)");
    adj->probes = dalloc<int64_t>(c, nprobes);
    HIPC(hipMemcpyAsync(adj->probes, hp.data(), nprobes * sizeof(int64_t), hipMemcpyHostToDevice, c->s));
    const int ns = adj->nsamples;
    adj->targets = dalloc<double>(c, (size_t)std::max(1, ns) * nprobes);
    if (ns > 0)
      HIPC(hipMemcpyAsync(adj->targets, targets, (size_t)ns * nprobes * sizeof(double),
                          hipMemcpyDeviceToDevice, c->s));
    if (prob->sigma_node) {
      adj->sigma = dalloc<double>(c, N);
      HIPC(hipMemcpyAsync(adj->sigma, prob->sigma_node, N * sizeof(double), hipMemcpyDeviceToDevice, c->s));
    }
    adj->ckpt = dalloc<double>(c, (size_t)(nsteps + 1) * NF * Np);
    double *sq = dalloc<double>(c, (size_t)std::max(1, ns) * nprobes);
    adj->cg_off.assign(1, 0);
    for (int n = 0; n < nsteps; ++n) {
      HIPC(launch_copy_fields(c->s, Np, adj->ckpt + (int64_t)n * NF * Np, 0, F.st.Y, 0, NF, 1));
      c->cg_record = &adj->cg_used;
      const hsdc_status sa = hsdc_advance(c, 1);
      c->cg_record = nullptr;
      // a step run again with checked solves: its own solves come last
      const int64_t per = (int64_t)c->meth.max_iter * F.co.M, got = (int64_t)adj->cg_used.size() - adj->cg_off.back();
      if (got > per)
        adj->cg_used.erase(adj->cg_used.begin() + adj->cg_off.back(), adj->cg_used.end() - per);
      adj->cg_off.push_back((int64_t)adj->cg_used.size());
      if (sa != HSDC_OK) return sa;
      if ((n + 1) % sample_every == 0) {
        const int smp = (n + 1) / sample_every - 1;
        HIPC(launch_adj_probes(c->s, F.st.Y, adj->probes, adj->targets + (int64_t)smp * nprobes,
                               nprobes, sq + (int64_t)smp * nprobes, nullptr));
      }
    }
    HIPC(launch_copy_fields(c->s, Np, adj->ckpt + (int64_t)nsteps * NF * Np, 0, F.st.Y, 0, NF, 1));
    std::vector<double> hs((size_t)std::max(1, ns) * nprobes, 0.0);
    HIPC(hipMemcpyAsync(hs.data(), sq, hs.size() * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPC(hipStreamSynchronize(c->s));
    double L = 0.0;
    for (int k = 0; k < ns * nprobes; ++k) L += hs[k];
    adj->loss = L;
    if (!std::isfinite(L)) return fail(c, HSDC_ENONFINITE, "non-finite misfit");
    return HSDC_OK;
  });
  if (st != HSDC_OK) {
    g_free_error = c->err;
    hsdc_adj_destroy(adj);
    return st;
  }
  if (loss_host) *loss_host = adj->loss;
  *out = adj;
  return HSDC_OK;
}

hsdc_status hsdc_misfit_backward(hsdc_adj *adj, double *grad_sigma, double *grad_gscale_host,
                                 double *grad_y0) {
  if (!adj || !adj->c) return fail(nullptr, HSDC_EINVAL, "adjoint handle is NULL");
  hsdc_ctx *c = adj->c;
  if (grad_sigma && !adj->sigma)
    return fail(c, HSDC_EINVAL, "grad_sigma needs a problem with sigma_node");
  return run_guarded(c, [&]() -> hsdc_status {
    Level &F = c->L[0];
    const int M = F.co.M, K = c->meth.max_iter;
    const int64_t N = F.g.N, Np = F.g.Np, sS = (int64_t)NF * Np, sY = (int64_t)(M + 1) * sS;
    const int64_t nbl = (M + 1) * ((N + 255) / 256);  // blocks of the transposed assembly
    const int64_t nlog = (int64_t)K * M * (int64_t)((sizeof(CgScalars) + 7) / 8);
    const int64_t sizes[] = {(K + 1) * sY, sY, sY, sY, sS, sS, (int64_t)NG * Np, (int64_t)NG * Np,
                             (int64_t)(M + 1) * Np, 3 * Np, (int64_t)(M + 1) * 3 * NG * Np,
                             3 * nbl, 8, sS + 3 * Np + 8, nlog};
    int64_t total = 0;
    for (int64_t v : sizes) total += v;
    if (!adj->work) adj->work = dalloc<double>(c, total);
    double *w = adj->work;
    AdjBuffers b{};
    double *dlog = nullptr;
    double **slots[] = {&b.Xs, &b.MU, &b.MUX, &b.RHO, &b.lam, &b.DYN, &b.DZ, &b.DLAM, &b.W, &b.dk,
                        &b.PS, &b.gs_part, &b.gs_acc, &b.bak, &dlog};
    for (int q = 0; q < 15; ++q) {
      *slots[q] = w;
      w += sizes[q];
    }
    b.dlog = reinterpret_cast<CgScalars *>(dlog);
    std::vector<int> pred((size_t)K * M, -1);
    b.pred = &pred;
    HIPC(hipMemsetAsync(b.lam, 0, sS * sizeof(double), c->s));
    HIPC(hipMemsetAsync(b.dk, 0, 3 * Np * sizeof(double), c->s));
    HIPC(hipMemsetAsync(b.gs_acc, 0, 8 * sizeof(double), c->s));
    const int every = adj->every, np = adj->np;
    // the last sample is taken on y_nsteps (kept with the checkpoints)
    if (adj->nsteps % every == 0)
      HIPC(launch_adj_probes(c->s, adj->ckpt + (int64_t)adj->nsteps * NF * Np, adj->probes,
                             adj->targets + (int64_t)(adj->nsteps / every - 1) * np, np, nullptr, b.lam));
    for (int n = adj->nsteps - 1; n >= 0; --n) {
      recompute_step(c, adj, n, b.Xs);
      // budgeted adjoint solves once every solve has a prediction
      const bool safe = *std::min_element(pred.begin(), pred.end()) < 0;
      if (!safe) {
        HIPC(hipMemcpyAsync(b.bak, b.lam, sS * sizeof(double), hipMemcpyDeviceToDevice, c->s));
        HIPC(hipMemcpyAsync(b.bak + sS, b.dk, 3 * Np * sizeof(double), hipMemcpyDeviceToDevice, c->s));
        HIPC(hipMemcpyAsync(b.bak + sS + 3 * Np, b.gs_acc, 8 * sizeof(double),
                            hipMemcpyDeviceToDevice, c->s));
      }
      adjoint_step(c, b, safe);
      if (!safe && !adjoint_verify(c, b)) {
        // a solve missed cg_rtol: restore what the step accumulates, run it safe
        c->stats.cg_redo_steps += 1;
        HIPC(hipMemcpyAsync(b.lam, b.bak, sS * sizeof(double), hipMemcpyDeviceToDevice, c->s));
        HIPC(hipMemcpyAsync(b.dk, b.bak + sS, 3 * Np * sizeof(double), hipMemcpyDeviceToDevice, c->s));
        HIPC(hipMemcpyAsync(b.gs_acc, b.bak + sS + 3 * Np, 8 * sizeof(double),
                            hipMemcpyDeviceToDevice, c->s));
        adjoint_step(c, b, true);
      }
      if (n > 0 && n % every == 0)
        HIPC(launch_adj_probes(c->s, adj->ckpt + (int64_t)n * NF * Np, adj->probes,
                               adj->targets + (int64_t)(n / every - 1) * np, np, nullptr, b.lam));
    }
    if (grad_y0)
      for (int f = 0; f < NF; ++f)
        HIPC(hipMemcpyAsync(grad_y0 + f * N, b.lam + f * Np, N * sizeof(double),
                            hipMemcpyDeviceToDevice, c->s));
    if (grad_sigma) {
      const double sc = 1.0 / (c->prob.dx * c->prob.dx * c->prob.chi * c->prob.Cm);
      HIPC(launch_adj_sigma(c->s, F.g, adj->sigma, sc, b.dk, b.dk + Np, b.dk + 2 * Np, grad_sigma));
    }
    double gs[8];
    HIPC(hipMemcpyAsync(gs, b.gs_acc, sizeof(gs), hipMemcpyDeviceToHost, c->s));
    HIPC(hipStreamSynchronize(c->s));
    if (grad_gscale_host)
      for (int q = 0; q < 3; ++q) grad_gscale_host[q] = gs[q];
    return HSDC_OK;
  });
}

void hsdc_adj_destroy(hsdc_adj *adj) {
  if (!adj) return;
  hsdc_destroy(adj->c);
  delete adj;
}

}  // extern "C"
