// hsdc_internal.h -- declarations shared by the host runtime and the HIP
// kernels of libhsdc (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hsdc.h"

namespace hsdc {

constexpr int NF = HSDC_NFIELDS;
constexpr int NG = HSDC_NGATES;
constexpr int GATE0 = 7;  // first gate field
constexpr int MAXM = HSDC_MAX_M;
constexpr int BLOCK = 512;

// Division of a 32-bit unsigned value by a divisor d fixed per mesh, as a
// multiply-high, a subtraction and two shifts (Granlund and Montgomery,
// division by invariant integers using multiplication, 1994):
//   n / d = (t + ((n - t) >> s1)) >> s2,  t = hi32(m n),  l = ceil(log2 d),
//   m = floor(2^32 (2^l - d) / d) + 1,  s1 = min(l, 1),  s2 = max(l - 1, 0),
// exact for every n < 2^32.  Node indices are below 2^31, so the mesh
// coordinates of a node cost a few instructions instead of 64-bit divisions.
struct FastDiv {
  uint32_t m;
  int32_t s1, s2;
};
inline FastDiv make_fastdiv(uint32_t d) {
  int l = 0;
  while ((1ull << l) < d) ++l;
  FastDiv f;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  f.s1 = l < 1 ? l : 1;
  f.s2 = l > 1 ? l - 1 : 0;
  return f;
}
__host__ __device__ inline uint32_t fastdiv(uint32_t n, FastDiv f) {
  const uint32_t t = (uint32_t)(((uint64_t)f.m * n) >> 32);
  return (t + ((n - t) >> f.s1)) >> f.s2;
}

// Mesh and diffusion operator K = (chi Cm)^-1 A (cell-centred, no-flux).
// A ragged batch of independent tissues (one per slice) sets rag: slice n then
// has the dimensions rag[RAG * n + 0..2] (N <= Np) and the divisors of nx and
// ny at rag[RAG * n + 3..8] (m, s1, s2 each), and its face coefficients start
// at kx + n Np (likewise ky, kz).
constexpr int RAG = 9;
struct Grid {
  int dim, nx, ny, nz;
  FastDiv fx, fy;  // division by nx and by ny
  int64_t N;    // nodes (largest tissue of a batch)
  int64_t Np;   // padded row length (multiple of 64 doubles)
  double cx, cy, cz;           // sigma_axis / (dx^2 chi Cm) for uniform sigma
  const double *kx, *ky, *kz;  // per-node face coefficients (face p -> p+e_axis), or null
  const int32_t *rag;          // device [P][RAG] tissue dimensions and divisors, or null
  // launch shapes (tunable per level): node-update block size (64, 128, 256 or
  // 512 threads), tile of the one-launch CG start (an index into kCgTiles),
  // tile of the coarse-to-fine correction on this mesh as the fine level (an
  // index into kProlongTiles2D / 3D)
  int nub, ctile, ptile;
  int order;  // finite-difference order of K: 2, or 4 (uniform sigma; hsdc_dct.hip)
};

// Tiles of the one-launch CG start (x by y nodes, threads per block): 0..4
// with the iterates in LDS, 5..8 in registers (64-column blocks).
struct TileShape {
  int tx, ty, threads;
};
constexpr int kNumCgTiles = 9;
constexpr TileShape kCgTiles[kNumCgTiles] = {
    {64, 16, 1024}, {32, 32, 1024}, {32, 16, 512}, {32, 8, 256}, {16, 16, 256},
    {48, 16, 512},  {48, 8, 512},   {48, 24, 512}, {48, 32, 512}};
// The default tile on an nx x ny mesh: the tallest register tile that still
// gives 192 tiles (three quarters of the compute units), else the one with
// the most tiles (48 x 8); on 256^2 to 1024^2 slabs the fastest or within 1%
// of it, where the LDS tile 64 x 16 takes 4% to 7% longer.
int default_cg_tile(int nx, int ny);
// Tiles of the coarse-to-fine correction (fine nodes x, y, z; 256 threads).
constexpr int kNumProlongTiles = 4;
constexpr int kProlongTiles3D[kNumProlongTiles][3] = {{32, 4, 2}, {64, 2, 2}, {16, 8, 2}, {16, 4, 4}};
constexpr int kProlongTiles2D[kNumProlongTiles][2] = {{32, 8}, {64, 4}, {16, 16}, {128, 2}};
constexpr int kDefaultNodeBlock = 256;

// Collocation data of one level (host-computed in FP64, passed by value).
struct Colloc {
  int M;
  double dt;
  double c[MAXM];           // c_1..c_M
  double d[MAXM];           // d_1..d_M
  double W[MAXM][MAXM];     // W[k][j] = l_j^{(k)}(0)
  double Q[MAXM][MAXM];     // a_ij(0)
  double cpow[MAXM][MAXM + 1];  // c_i^k
  double invfact[MAXM + 10];    // 1/k!, k = 0..MAXM+9
};

// Strided view of a set of stage vectors on one level.  States, K V, the
// assembled right-hand side and the diffusion right-hand side are FP64 on every
// level; the cell-model terms (G, Lambda) are stored and computed in T (float
// on an FP32 coarse level).  Every T-valued term enters both sides of a sweep
// from the same inputs, so its rounding cancels at the fixed point.
template <class T>
struct StagesT {
  double *Y;   // [P][M+1][NF][Np]
  T *G;        // [P][M+1][NF][Np]  reaction part of g at each stage
  double *FV;  // [P][M+1][Np]      K V at each stage
  double *RH;  // [P][M][NF][Np]    assembled right-hand-side differences
  T *L0;       // [P][NG][Np]       Lambda(y_{n,0}) of the current iterate
  double *B;   // [P][Np]           diffusion right-hand side
  int64_t Np;
  int M;
  __host__ __device__ int64_t sY() const { return (int64_t)(M + 1) * NF * Np; }
  __host__ __device__ int64_t sS() const { return (int64_t)NF * Np; }
  __host__ __device__ int64_t sFV() const { return (int64_t)(M + 1) * Np; }
  __host__ __device__ int64_t sRH() const { return (int64_t)M * NF * Np; }
  __host__ __device__ int64_t sL() const { return (int64_t)NG * Np; }
};
using Stages = StagesT<double>;

// Also carries the time of slice n: step (step0 + n tn), tn = 1 for the
// consecutive time slices of PFASST, 0 for the tissues of a batch.
struct Stim {
  const double *w;  // [Np] (shared by the slices, sw = 0) or [P][Np] (sw = Np), or null
  int64_t sw;
  int64_t tn;
  const int64_t *step;  // device: the current step (slice 0), read by the kernels
  double amp, t0, dur, eps;
  double Cm;
};

// Per-slice CG scalars, double-buffered by iteration parity; written only by
// block 0 of the kernel that computes them and read by the next kernel.
struct CgScalars {
  double bb;      // ||b||^2
  double gamma;   // (r_k, r_k) of the last iteration started
  double alpha;   // alpha of that iteration
  int32_t it;     // iterations completed
  int32_t done;   // 1: converged (or maxit reached) -- x is final
};

// ---- kernel launch wrappers (defined in hsdc_kernels.hip) -------------------
// Kernels templated on T run on both storage types; arithmetic follows the
// storage type except where noted (collocation integrals, phi functions and
// reductions are FP64 throughout).
template <class T>
hipError_t launch_eval_stages(hipStream_t s, const Grid &g, const StagesT<T> &st, const Colloc &co,
                              const Stim &stim, double gs0, double gs1, double gs2, int slice0,
                              int nslices, int stage0, int nstages, T *L_anchor_out,
                              const T *L_anchor_in);
template <class T>
hipError_t launch_spmv_stages(hipStream_t s, const Grid &g, const StagesT<T> &st, int slice0,
                              int nslices, int stage0, int nstages);
hipError_t launch_spread(hipStream_t s, const Grid &g, const Stages &st, const Colloc &co,
                         const Stim &stim, int slice0, int nslices, bool copy_Y_from_stage0);
// spread != 0: stages 1..M are the spread of stage 0 (y^0 = 1 (x) y_n) and are
// read from stage 0 (the stimulus part of the V reaction term follows t_{n,j}).
template <class T>
hipError_t launch_assemble(hipStream_t s, const Grid &g, const StagesT<T> &st, const Colloc &co,
                           int slice0, int nslices, const double *RI, int64_t sRI, int spread,
                           const Stim &stim);
// RI[n][i][f] -= (A G)_i of the stage vector held by st (coarse FAS term of tau).
template <class T>
hipError_t launch_fas_integrals(hipStream_t s, const Grid &g, const StagesT<T> &st,
                                const Colloc &co, int slice0, int nslices, double *RI,
                                int64_t sRI);
// The node update also forms the CG start residual r_0 = b - x_0 + a K x_0 from
// the cached K x_0 (x_0 = V^k_i) and writes the partials of ||b||^2, ||r_0||^2.
template <class T>
struct CgBatchT;
// store_g = 0 skips storing the reaction term (its caller discards it);
// spread != 0 takes K x_0 from stage 0 (first sweep after a spread).
// yref (T = float only; null elsewhere): stage vectors [P][M+1][NF][Np] of the
// iterate the right-hand side was evaluated at; the FP32 cell model is then
// evaluated at fl(yref) + fl(y - yref).
// lg: the previous solve of the same slices to log (lg.log null: none); block 0
// of each slice writes its entry before its own work.
struct CgLogArgs;
template <class T>
hipError_t launch_node_update(hipStream_t s, const Grid &g, const StagesT<T> &st,
                              const Colloc &co, const Stim &stim, double gs0, double gs1,
                              double gs2, int slice0, int nslices, int i,
                              const CgBatchT<T> &cb, int store_g, int spread, const double *yref,
                              const CgLogArgs &lg);
hipError_t launch_copy_V_to_stages(hipStream_t s, const Grid &g, const Stages &st, int slice0,
                                   int nslices);
// Blocks of a node-update launch of g.nub threads, and of any launch of nb
// threads per node block (XCD-padded unless the slices are a ragged batch).
int node_blocks(const Grid &g);
int node_blocks_of(const Grid &g, int nb);
// out2[2 (n NF + f)] = max |r_{n,f}|, out2[2 (n NF + f) + 1] = max |y_{n,f}| per
// slice n and field f.  With RI: the collocation integrals of rows 1..M (plus
// RIadd, a level's own FAS term, when given) restricted in time by Rt to the
// Mc nodes of the next coarser level.
hipError_t launch_residual(hipStream_t s, const Grid &g, const Stages &st, const Colloc &co,
                           int slice0, int nslices, const double *y_block0, double *part,
                           int nblk, double *out2, const double *Rt, int Mc, double *RI,
                           int64_t sRI, const double *RIadd = nullptr, int64_t sRIadd = 0);
int residual_blocks(const Grid &g);
hipError_t launch_copy_fields(hipStream_t s, int64_t Np, double *dst, int64_t sdst,
                              const double *src, int64_t ssrc, int nf, int nslices);

// Chebyshev parameters of one diffusion operator I - a K whose spectrum lies in
// [1, 1 + a lam] (lam bounds the spectrum of -K): theta and delta are the
// centre and half-width of that interval, sigma = theta / delta, s =
// acosh(sigma) (s = 0 when delta = 0, A = I), and omega[k - 1] =
// omega_{k+1} = 2 sigma T_k(sigma) / T_{k+1}(sigma) for k = 1..CHEB_KT
// (host-computed per slice and collocation node).
constexpr int CHEB_KT = 61;
struct ChebTab {
  double inv_theta, sigma, s;
  double omega[CHEB_KT];
};

// CG on (I - a K) x = b, batched over slices with strided vectors
// (Chronopoulos-Gear single-reduction form: one stencil kernel per iteration).
// The solution and right-hand side are FP64; the work vectors are stored in T;
// scalars, stencil sums and reductions are FP64.  rel_r0 = 1 stops on
// ||r_k|| <= rtol ||r_0|| (a correction solved to relative accuracy), else on
// ||r_k|| <= rtol ||b||.
template <class T>
struct CgBatchT {
  double *x; int64_t sx;        // solution (in place), slice stride
  const double *b; int64_t sb;
  T *r[2], *w[2], *s[2];        // ping-pong [nslices][Np]
  T *p;                         // [nslices][Np]
  double *part;                 // [nslices][5][pstride] partial sums:
                                //   gamma par0 | delta par0 | gamma par1 | delta par1 | bb
  int64_t pstride;
  CgScalars *sc;                // [nslices][2] by parity
  CgScalars *log;               // [nslices] final scalars (written by the kernel k == last_k) or null
  int last_k;
  int slice0;                   // absolute index of the batch's first slice
  int nslices, nblk;            // blocks of the CG kernels (<= 512)
  int nblk0;                    // partials of gamma_0 and bb (written by the producer of r_0)
  double a, tol2;
  int maxit;
  int rel_r0;
  // Chebyshev iteration (FP64 levels; xt == null selects CG): the node update
  // stores b in bout and x_1 = x_0 + r_0 / theta in xt, x_0 staying in x;
  // iterate k overwrites x_{k-1} with x_{k+1}, so x_k alternates between x (k
  // even) and xt (k odd) and the iteration count is rounded up to even.
  double *xt;                   // [nslices][Np]
  double *bout;                 // [nslices][Np] (the memory b points to)
  const struct ChebTab *tab;    // this node's entry of absolute slice n: tab[n * tab_stride]
  int tab_stride;
  // cstart = D >= 2 (with xt set): CG from the Chebyshev iterate x_D.  The node
  // update stores b and x_1 as above, D - 1 Chebyshev launches form x_2 .. x_D,
  // and launch_cg_start forms r_D = b - A x_D and w_D = A r_D in the parity-1
  // vectors (and x_D in x), so the CG launches run k = 1, 2, ...
  int cstart;
  // direct = 1: the level solves by DCT-II (hsdc_dct.hip); the node update only
  // stores b in bout
  int direct;
  // partials of (r_D, r_D) and (w_D, r_D) written by the start (first CG
  // launch); x0_to_p = 1: the node update also stores the warm start x_0 in p,
  // where the tiled start (launch_cg_start_tiled) reads it, so that the start
  // can write x_D into x while other tiles still read x_0
  int nblk_s;
  int x0_to_p;
};

// A budgeted solve whose outcome a later kernel writes to the solve log (the
// next node update of the same slices, or launch_cg_log): the final scalars
// when a CG launch found convergence, else the residual reduced from the
// partial sums of the last writer (the start, or a CG launch that iterated).
struct CgLogArgs {
  const double *part;   // the solve's partial sums [nslices][5][pstride]
  int64_t pstride;
  const CgScalars *sc;  // the solve's scalars [nslices][2]
  CgScalars *log;       // [nslices] log entries, or null (nothing to log)
  int par;              // parity of the scalars and partials holding the final state
  int ngamma;           // partials of the final (r, r) (start tiles or blocks, or
                        // node-update blocks); -1: the CG blocks active for the mesh
  int cg_nblk;          // blocks of the solve's CG launches
  int nbb;              // partials of ||b||^2 (node-update blocks)
  int slice0;
  double tol2;
  int rel_r0;
};
// Writes the log entries of lg (one block per slice).
hipError_t launch_cg_log(hipStream_t s, const Grid &g, const CgLogArgs &lg, int nslices);
using CgBatch = CgBatchT<double>;
int cg_blocks(const Grid &g, int cap = 512);
template <class T>
hipError_t launch_cg_init(hipStream_t s, const Grid &g, const CgBatchT<T> &cb);
template <class T>
hipError_t launch_cg_resid0(hipStream_t s, const Grid &g, const CgBatchT<T> &cb);
template <class T>
hipError_t launch_cg_iter(hipStream_t s, const Grid &g, const CgBatchT<T> &cb, int k);
hipError_t launch_apply_K(hipStream_t s, const Grid &g, const double *v, double *out);
// Chebyshev iterate k >= 1 (one launch per k; launch k = 1 also derives the
// iteration count from the node update's partials of ||r_0||^2 and ||b||^2).
hipError_t launch_cheb_iter(hipStream_t s, const Grid &g, const CgBatch &cb, int k);
// Chebyshev steps k = 1 .. kmax alone, x_{k+1} = x_{k-1} + omega_{k+1} (x_k -
// x_{k-1} + (b - A x_k) / theta) (no iteration count derived or checked).
hipError_t launch_cheb_steps(hipStream_t s, const Grid &g, const CgBatch &cb, int kmax);
// CG start from x_D (cstart = D): r_D, w_D, the partials of (r_D, r_D) and
// (w_D, r_D), the parity-1 scalars, and x_D in x.
hipError_t launch_cg_start(hipStream_t s, const Grid &g, const CgBatch &cb);
// The whole CG start of degree D = cb.cstart (7) in one launch on 2D meshes
// (x_2 .. x_D, r_D, w_D on tiles of kCgTiles[g.ctile] with a halo of D + 1,
// the iterates in LDS or in registers); x_0 is read from p (cb.x0_to_p) and
// x_D written to x.
// cg_start_tiles(g, D) = its tiles per slice on a mesh that is not a ragged
// batch (0: not applicable); ntiles = the launch's tiles per slice (a ragged
// batch: the most of any tissue, cg_start_tiles_of).
int cg_start_tiles(const Grid &g, int degree);
int cg_start_tiles_of(int nx, int ny, int tile);
hipError_t launch_cg_start_tiled(hipStream_t s, const Grid &g, const CgBatch &cb, int ntiles);

// DCT-II data of a mesh with uniform sigma (hsdc_dct.hip): per axis the
// orthonormal DCT-II matrix C[k][p] = s_k cos(pi k (p + 1/2) / n) and its
// transpose CT, row-major n x n, and the eigenvalue of K for each mode,
// lam[k] = sigma_axis / (dx^2 chi Cm) times the stencil's symbol at
// theta = pi k / n (one entry 0 for an axis of one node).
struct DctPlan {
  const double *C[3], *CT[3], *lam[3];
  // fast: every transformed axis has a power-of-two length in [2, 2048]; ft
  // holds per axis the twiddles W (n/2 complex), E (n complex), s and 1/s (n)
  int fast;
  const double *ft[3];
};
// x = (I - a K)^-1 b for nslices slices (slice strides sb, sx; t1, t2 scratch
// [nslices][st]); g uniform, not a batch.
// allows the fast transforms' LDS for lines up to nmax long (once per process)
hipError_t fdct_setup(int nmax);
hipError_t launch_dct_solve(hipStream_t s, const Grid &g, const DctPlan &d, double a,
                            const double *b, int64_t sb, double *x, int64_t sx, double *t1,
                            double *t2, int64_t st, int nslices);
// K V with the fourth-order stencil (g.order 4): stages stage0.. of slices
// slice0.. of Y into FV (strides as StagesT), or one vector v into out.
hipError_t launch_spmv4_stages(hipStream_t s, const Grid &g, const double *Y, int64_t sY,
                               int64_t sS, double *FV, int64_t sFV, int slice0, int nslices,
                               int stage0, int nstages);
hipError_t launch_apply_K4(hipStream_t s, const Grid &g, const double *v, double *out);

// transfers (space coarsening 2x or identity) between a fine and a coarse level
hipError_t launch_restrict_stages(hipStream_t s, const Grid &gf, const Grid &gc, int sc_factor,
                                  const double *Yf, int64_t sYf, int Mf, const double *Rt,
                                  int Mc, double *Yc, int64_t sYc, double *Yc_copy, int nslices);
hipError_t launch_restrict_fields(hipStream_t s, const Grid &gf, const Grid &gc, int sc_factor,
                                  const double *src, int64_t ssrc, double *dst, int64_t sdst,
                                  int nrows, int nslices);
// Yf += T (P_space (Yc - Sz)) on fine stages i0..Mf; Sz is overwritten with
// Yc - Sz.
hipError_t launch_prolong_correct(hipStream_t s, const Grid &gf, const Grid &gc, int sc_factor,
                                  const double *Yc, double *Sz, int64_t sYc, int Mc,
                                  const double *Tt, int Mf, int i0, double *Yf, int64_t sYf,
                                  int nslices);

// ---- discrete adjoint of a serial step (hsdc_adjoint.hip) -------------------
// Buffers of one slice: stage vectors [M+1][NF][Np], fields [NF][Np], gate
// rows [NG][Np].  X: the sweep's previous iterate, Z: its result (stage 0 of
// both is the anchor u = y_n); MU, MUX: adjoints of Z and X; RHO: the
// adjoints of the right-hand sides b_i (V row from the adjoint solves); DYN:
// adjoint of y_n; DZ, DLAM: adjoints of z = dt Lambda_n and of Lambda_n where
// it enters explicitly; W: [M+1][Np] adjoints of K X_j^V (rows 1..M); L0:
// Lambda_n; gs_part: per-block partials of the scaling gradient, summed into
// gs_acc[3] after every launch.
struct AdjArgs {
  int64_t N, Np;
  Colloc co;
  double gs[3];
  const double *X, *Z, *L0;
  double *MU, *MUX, *RHO, *DYN, *DZ, *DLAM, *W;
  double *PS;  // (M + 1) x 3 NG x Np: per-stage terms of the transposed assembly
  double *gs_part, *gs_acc;  // gs_part: 3 per block of 256 nodes and stage
};
hipError_t launch_adj_backsub(hipStream_t s, const AdjArgs &a, int i);
hipError_t launch_adj_assemble(hipStream_t s, const AdjArgs &a);  // M <= 6
hipError_t launch_adj_anchor(hipStream_t s, const AdjArgs &a);
hipError_t launch_adj_faces(hipStream_t s, const Grid &g, const double *u, const double *v,
                            double scale, double *dkx, double *dky, double *dkz);
hipError_t launch_adj_spmv_add(hipStream_t s, const Grid &g, const double *v, double scale,
                               double *out);
// x1 = x0 + (b - (I - a K) x0) * tab->inv_theta (the first Chebyshev step);
// bpart (or null): the partials of ||b||^2, one per block of kAdjBlock nodes
constexpr int kAdjBlock = 256;
hipError_t launch_adj_cheb_x1(hipStream_t s, const Grid &g, const double *x0, const double *b,
                              double a, const ChebTab *tab, double *x1, double *bpart);
hipError_t launch_adj_sigma(hipStream_t s, const Grid &g, const double *sig, double sc,
                            const double *dkx, const double *dky, const double *dkz, double *dsig);
hipError_t launch_adj_probes(hipStream_t s, const double *y, const int64_t *probes,
                             const double *target, int np, double *out_sq, double *lambda);
hipError_t launch_adj_axpy(hipStream_t s, double *y, const double *x, int64_t n);

// building blocks exported for tests
hipError_t launch_ionic_test(hipStream_t s, int64_t n, const double *y, double gs0, double gs1,
                             double gs2, double *I_ion, double *ha, double *lam, double *winf);
hipError_t launch_phi_test(hipStream_t s, int64_t n, const double *x, int kmax, double *out);
hipError_t launch_aij_test(hipStream_t s, int64_t n, const double *z, const Colloc &co,
                           double *out);
hipError_t launch_fill_rest(hipStream_t s, int64_t N, int64_t Np, double *y);
// face coefficients kx, ky (dim >= 2), kz (dim 3) of a per-node sigma field on
// the device: harmonic mean of the two nodes times sc, 0 on the last layer
hipError_t launch_faces(hipStream_t s, const Grid &g, const double *sigma_node, double sc,
                        double *kx, double *ky, double *kz);
// device step counter: *step = value, or *step += add
hipError_t launch_step_set(hipStream_t s, int64_t *step, int64_t value);
hipError_t launch_step_add(hipStream_t s, int64_t *step, int64_t add);

}  // namespace hsdc
