// hsdc_kernels.hip -- gfx950 kernels of the hybrid SDC / PFASST hot path.
//
// One lane per mesh node, states field-major (SoA) so every field load is a
// coalesced 64-lane FP64 row.  Nothing here is a dense contraction, so no MFMA:
// the cell model is bound by FP64 VALU work (exp/log/div sequences), the
// stencil, CG vector updates, assembly, residual and transfers by HBM bytes.
#include <hip/hip_runtime.h>
#include <type_traits>

#include "hsdc_device.h"
#include "hsdc_internal.h"
#include "ttp06_device.h"

namespace hsdc {

// ---------------------------------------------------------------------------
// cell model at stages: G_j = f_E + f_e + Lambda(u)(u - y_j) (reaction part of g)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double stim_value(const Stim &st, double t, int n, int64_t p) {
  if (st.w == nullptr) return 0.0;
  const bool on = (t > st.t0 + st.eps) && (t <= st.t0 + st.dur + st.eps);
  return on ? st.amp * st.w[n * st.sw + p] : 0.0;
}

template <class T>
__global__ void __launch_bounds__(BLOCK)
k_eval_stages(Grid g0, StagesT<T> st, Colloc co, Stim stim, double gs0, double gs1, double gs2,
              int slice0, int stage0, T *Lout, const T *Lin) {
  const int64_t step0 = *stim.step;
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int n = slice0 + blockIdx.z;
  const Grid g = slice_grid(g0, n);
  if (p >= g.N) return;
  const int j = stage0 + blockIdx.y;
  const int64_t Np = st.Np;
  const double *y = st.Y + n * st.sY() + j * st.sS();
  T *G = st.G + n * st.sY() + j * st.sS();
  T yv[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) yv[f] = T(y[f * Np + p]);
  const double cj = (j == 0) ? 0.0 : co.c[j - 1];
  const double t = ((double)(step0 + n * stim.tn) + cj) * co.dt;
  // stage 0 is the anchor itself (its Lambda is the anchor's); later stages
  // read Lambda_n
  const T *La = (j == 0) ? nullptr : Lin + n * st.sL();
  T *Lo = (j == 0 && Lout) ? Lout + n * st.sL() : nullptr;
  // gate rows without the anchor part: f_e(w) - Lambda_n w (software-pipelined
  // by one gate: Lambda_n of gate k + 1 is loaded when gate k is stored)
  T nla = La ? La[p] : T(0);
  ttp06::gates<T>(yv[0], yv[3], [&](int k, T inf, T rate) {
    const T lam = -rate;
    const T la = La ? nla : lam;
    if (La && k + 1 < NG) nla = La[(k + 1) * Np + p];
    const T w = yv[GATE0 + k];
    G[(GATE0 + k) * Np + p] = lam * (w - inf) - la * w;
    if (Lo) Lo[k * Np + p] = lam;
  });
  T I_ion, ha[6];
  ttp06::currents<T>(yv, T(gs0), T(gs1), T(gs2), I_ion, ha);
  G[p] = (T(stim_value(stim, t, n, p)) - T(stim.Cm) * I_ion) / T(stim.Cm);
#pragma unroll
  for (int k = 0; k < 6; ++k) G[(1 + k) * Np + p] = ha[k];
}

template <class T>
hipError_t launch_eval_stages(hipStream_t s, const Grid &g, const StagesT<T> &st, const Colloc &co,
                              const Stim &stim, double gs0, double gs1, double gs2, int slice0,
                              int nslices, int stage0, int nstages, T *L_anchor_out,
                              const T *L_anchor_in) {
  if (nslices <= 0 || nstages <= 0) return hipSuccess;
  dim3 grid(nblocks(g.N), nstages, nslices);
  hipLaunchKernelGGL(k_eval_stages<T>, grid, dim3(BLOCK), 0, s, g, st, co, stim, gs0, gs1, gs2,
                     slice0, stage0, L_anchor_out, L_anchor_in);
  return hipGetLastError();
}

// FV_j = K V_j at stages.
template <int DIM, bool PN, class T>
__global__ void __launch_bounds__(BLOCK) k_spmv_stages(Grid g0, StagesT<T> st, int slice0,
                                                       int stage0) {
  const int64_t p = stencil_node_block(g0, blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  const int n = slice0 + blockIdx.z;
  const Grid g = slice_grid(g0, n);
  if (p >= g.N) return;
  const int j = stage0 + blockIdx.y;
  const double *v = st.Y + n * st.sY() + j * st.sS();
  const Ijk c = ijk(g, p);
  const double vc = v[p];
  st.FV[n * st.sFV() + j * st.Np + p] =
      applyK<DIM, PN>(g, p, c, vc, [&](int64_t k) { return v[k]; });
}

template <class T>
hipError_t launch_spmv_stages(hipStream_t s, const Grid &g, const StagesT<T> &st, int slice0,
                              int nslices, int stage0, int nstages) {
  if (nslices <= 0 || nstages <= 0) return hipSuccess;
  if (g.order == 4) {  // fourth-order stencil: FP64 levels with uniform sigma
    if constexpr (std::is_same<T, double>::value)
      return launch_spmv4_stages(s, g, st.Y, st.sY(), st.sS(), st.FV, st.sFV(), slice0, nslices,
                                 stage0, nstages);
    return hipErrorInvalidValue;
  }
  dim3 grid(g.rag ? nblocks(g.N) : nblocks_xcd(g.N), nstages, nslices);
  HSDC_DISPATCH_OP(g, hipLaunchKernelGGL((k_spmv_stages<DIM, PN, T>), grid, dim3(BLOCK), 0, s, g,
                                         st, slice0, stage0));
  return hipGetLastError();
}

// Spread stage 0 (Y optionally, G, FV) to stages 1..M; the stimulus part of the
// V entry of G follows the stage time.
__global__ void __launch_bounds__(BLOCK)
k_spread(Grid g0, Stages st, Colloc co, Stim stim, int slice0, int copyY) {
  const int64_t step0 = *stim.step;
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int n = slice0 + blockIdx.z;
  if (p >= slice_grid(g0, n).N) return;
  const int64_t Np = st.Np;
  double *Y = st.Y + n * st.sY();
  double *G = st.G + n * st.sY();
  double *FV = st.FV + n * st.sFV();
  const double t0 = ((double)(step0 + n * stim.tn)) * co.dt;
  const double s0 = stim_value(stim, t0, n, p);
  const double fv = FV[p];
  for (int j = 1; j <= st.M; ++j) {
    const double tj = ((double)(step0 + n * stim.tn) + co.c[j - 1]) * co.dt;
    const double sj = stim_value(stim, tj, n, p);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      double gv = G[f * Np + p];
      if (f == 0 && sj != s0) gv += (sj - s0) / stim.Cm;
      G[j * st.sS() + f * Np + p] = gv;
      if (copyY) Y[j * st.sS() + f * Np + p] = Y[f * Np + p];
    }
    FV[j * Np + p] = fv;
  }
}

hipError_t launch_spread(hipStream_t s, const Grid &g, const Stages &st, const Colloc &co,
                         const Stim &stim, int slice0, int nslices, bool copy_Y_from_stage0) {
  dim3 grid(nblocks(g.N), 1, nslices);
  hipLaunchKernelGGL(k_spread, grid, dim3(BLOCK), 0, s, g, st, co, stim, slice0,
                     copy_Y_from_stage0 ? 1 : 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sweep right-hand side: RH_i = R_i - R_{i-1} of eq. prec_picard in node-to-node
// form,  dt (I_i - I_{i-1}) - dt d_i Phi_i(y^k), where I are the collocation
// integrals of the iterate; on the coarse level of PFASST the FAS term of tau
// (per unit dt, from k_fas_integrals) is added to them.
// ---------------------------------------------------------------------------

// Instantiated separately for the rows V .. Rbar (GATES = false: collocation
// weights, memory streams only) and the gate rows (exponential coefficients).
// The gate rows form, complete and store one I_i at a time, so only the moments
// stay live across the phi evaluations (46 VGPRs at M = 6, eight waves per
// SIMD); with all I_i formed first they took 128 VGPRs and spilled.
template <int M, class T, bool GATES>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4)))
k_assemble(Grid g0, StagesT<T> st, Colloc co, int slice0, const double *RI, int64_t sRI, int spread,
           Stim stim) {
  const int64_t step0 = *stim.step;
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  // one field per block row: no divergence between field kinds
  const int f = GATES ? GATE0 + (int)blockIdx.y : (int)blockIdx.y;
  const int n = slice0 + blockIdx.z;
  if (p >= slice_grid(g0, n).N) return;
  const int64_t Np = st.Np;
  const T *G = st.G + n * st.sY() + f * Np + p;
  const double *FV = st.FV + n * st.sFV() + p;
  double *RH = st.RH + n * st.sRH() + f * Np + p;
  const double dt = co.dt;
  if constexpr (GATES) {
    // Gate rows: no K V term.  Each I_i is formed, completed and stored in
    // turn, so only the moments stay live across the phi evaluations.  G holds
    // the reaction terms without the anchor part Lambda_n u; that part enters
    // I_i as Lambda_n u c_i phi_1(c_i z), while the Phi term takes the stored
    // G alone: the new stage's node update adds its own reaction term without
    // the anchor part, and the two anchor parts cancel in R_i - R_{i-1}.
    double Gv[M + 1];
    if (spread) {
#pragma unroll
      for (int j = 0; j <= M; ++j) Gv[j] = G[0];
    } else {
#pragma unroll
      for (int j = 0; j <= M; ++j) Gv[j] = G[j * st.sS()];
    }
    const double lam_n = st.L0[n * st.sL() + (f - GATE0) * Np + p];
    const double z = dt * lam_n;
    const double anc = lam_n * st.Y[n * st.sY() + f * Np + p];
    double mom[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < M; ++j) s += co.W[k][j] * Gv[j + 1];
      mom[k] = s;
    }
    double prevI = 0.0;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      double Ii;
      if (z == 0.0) {  // a(0) = Q
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) s += co.Q[i][j] * Gv[j + 1];
        Ii = s;
      } else {
        double ph[M];
        phis<M>(co.c[i] * z, co.invfact, ph);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) s += co.cpow[i][k + 1] * ph[k] * mom[k];
        Ii = s + anc * co.c[i] * ph[0];
      }
      if (RI) Ii += RI[n * sRI + ((int64_t)i * NF + f) * Np + p];
      stream_store<double>(&RH[(int64_t)i * st.sS()],
                           dt * (Ii - prevI) - dt * co.d[i] * (0.0 + phi1(co.d[i] * z) * Gv[i]));
      prevI = Ii;
    }
    return;
  }
  double Gv[M + 1], fv[M + 1], gfull[M], I[M];
  if (spread) {
    const double g0 = G[0];
    const double f0 = (f == 0) ? FV[0] : 0.0;
    const double s0 = (f == 0) ? stim_value(stim, ((double)(step0 + n * stim.tn)) * co.dt, n, p) : 0.0;
    Gv[0] = g0;
    fv[0] = 0.0;
#pragma unroll
    for (int j = 1; j <= M; ++j) {
      double gv = g0;
      if (f == 0) {
        const double sj = stim_value(stim, ((double)(step0 + n * stim.tn) + co.c[j - 1]) * co.dt, n, p);
        if (sj != s0) gv += (sj - s0) / stim.Cm;
      }
      Gv[j] = gv;
      fv[j] = f0;
    }
  } else {
#pragma unroll
    for (int j = 0; j <= M; ++j) Gv[j] = G[j * st.sS()];
#pragma unroll
    for (int j = 0; j <= M; ++j) fv[j] = (f == 0 && j > 0) ? FV[j * Np] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < M; ++j) gfull[j] = Gv[j + 1] + fv[j + 1];
  colloc_weights<M>(co, gfull, I);
  if (RI) {
#pragma unroll
    for (int i = 0; i < M; ++i) I[i] += RI[n * sRI + ((int64_t)i * NF + f) * Np + p];
  }
  double prevI = 0.0;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    // streaming store: read once, by a later kernel
    stream_store<double>(&RH[(int64_t)i * st.sS()],
                         dt * (I[i] - prevI) - dt * co.d[i] * (fv[i + 1] + Gv[i]));
    prevI = I[i];
  }
}

template <class T>
hipError_t launch_assemble(hipStream_t s, const Grid &g, const StagesT<T> &st, const Colloc &co,
                           int slice0, int nslices, const double *RI, int64_t sRI, int spread,
                           const Stim &stim) {
  const dim3 rows(nblocks(g.N), GATE0, nslices), gates(nblocks(g.N), NG, nslices);
  HSDC_DISPATCH_M(co.M, {
    hipLaunchKernelGGL((k_assemble<M, T, false>), rows, dim3(BLOCK), 0, s, g, st, co, slice0, RI,
                       sRI, spread, stim);
    hipLaunchKernelGGL((k_assemble<M, T, true>), gates, dim3(BLOCK), 0, s, g, st, co, slice0, RI,
                       sRI, spread, stim);
  });
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FAS term of tau (Algorithm 1) on the coarse level, per unit dt: rows i >= 1 of
// tau = D_c(S z) - S D_f(z) are dt (S (A G)_f(z) - (A G)_c(S z))_i; the first
// part arrives in RI (fine integrals restricted in time and space), the second
// is computed here from the reaction terms, K V and Lambda of S z.
// ---------------------------------------------------------------------------
template <int M, class T>
__global__ void __launch_bounds__(BLOCK)
k_fas_integrals(Grid g0, StagesT<T> st, Colloc co, int slice0, double *RI, int64_t sRI) {
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int f = blockIdx.y;
  const int n = slice0 + blockIdx.z;
  if (p >= slice_grid(g0, n).N) return;
  const int64_t Np = st.Np;
  const T *G = st.G + n * st.sY() + f * Np + p;
  const double *FV = st.FV + n * st.sFV() + p;
  double gfull[M], I[M];
#pragma unroll
  for (int j = 0; j < M; ++j)
    gfull[j] = (double)G[(j + 1) * st.sS()] + (f == 0 ? FV[(j + 1) * Np] : 0.0);
  // gate rows: Lambda_n and the anchor part (G holds the reaction terms without it)
  const double lam_n = (f >= GATE0) ? (double)st.L0[n * st.sL() + (f - GATE0) * Np + p] : 0.0;
  const double anc = (f >= GATE0) ? lam_n * st.Y[n * st.sY() + f * Np + p] : 0.0;
  colloc_integrals<M>(co, co.dt * lam_n, gfull, I, anc);
  double *R = RI + n * sRI + (int64_t)f * Np + p;
#pragma unroll
  for (int i = 0; i < M; ++i) R[(int64_t)i * NF * Np] -= I[i];
}

template <class T>
hipError_t launch_fas_integrals(hipStream_t s, const Grid &g, const StagesT<T> &st,
                                const Colloc &co, int slice0, int nslices, double *RI,
                                int64_t sRI) {
  dim3 grid(nblocks(g.N), NF, nslices);
  HSDC_DISPATCH_M(co.M, hipLaunchKernelGGL((k_fas_integrals<M, T>), grid, dim3(BLOCK), 0, s, g,
                                           st, co, slice0, RI, sRI));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// node i of the forward substitution with P (eq. def_P): explicit f_E,
// exponential Euler on the gates (phi_1(d_i dt Lambda(u))), and the right-hand
// side of the implicit diffusion solve for V.
// ---------------------------------------------------------------------------

// Log entry of slice n (absolute) of a budgeted solve, written by a whole
// block of NT threads (every thread takes part in the reductions).  When a CG
// launch published convergence its scalars are final; otherwise the residual
// is reduced here from the partial sums of the last writer and compared with
// the tolerance, so a solve needs no launch of its own to be checked.
template <int NT>
__device__ __forceinline__ void cg_log_entry(const Grid &g0, const CgLogArgs &lg, int n,
                                             double *lds) {
  const int q = n - lg.slice0;
  const CgScalars si = lg.sc[2 * q + lg.par];
  const double *part = lg.part + (int64_t)q * 5 * lg.pstride;
  int ng = lg.ngamma;
  if (ng < 0) {  // a CG launch wrote them: its blocks active on this slice's mesh
    const int64_t nb = (slice_grid(g0, n).N + BLOCK - 1) / BLOCK;
    ng = nb < lg.cg_nblk ? (int)nb : lg.cg_nblk;
  }
  double t2[2] = {0.0, 0.0};
  for (int k = threadIdx.x; k < ng; k += NT) t2[0] += part[(2 * lg.par) * lg.pstride + k];
  for (int k = threadIdx.x; k < lg.nbb; k += NT) t2[1] += part[4 * lg.pstride + k];
  block_sums<2, NT>(t2, lds);
  if (threadIdx.x == 0) {
    CgScalars o = si;
    if (!si.done) {
      // bb: published by the first CG launch, or (no launch ran) the node
      // update's partials; a correction solve compares with its start residual
      const double ref = si.bb >= 0.0 ? si.bb : (lg.rel_r0 ? t2[0] : t2[1]);
      o.gamma = t2[0];
      o.bb = ref;
      o.done = (t2[0] <= lg.tol2 * ref || t2[0] == 0.0) ? 1 : 0;
    }
    lg.log[q] = o;
  }
}

__global__ void __launch_bounds__(256) k_cg_log(Grid g0, CgLogArgs lg) {
  __shared__ double lds[2 * (256 / 64)];
  cg_log_entry<256>(g0, lg, lg.slice0 + blockIdx.x, lds);
}

hipError_t launch_cg_log(hipStream_t s, const Grid &g, const CgLogArgs &lg, int nslices) {
  if (!lg.log || nslices <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cg_log, dim3(nslices), dim3(256), 0, s, g, lg);
  return hipGetLastError();
}

// Four waves per SIMD (at most 128 VGPRs): the launch has exactly that many
// waves on the 512 x 512 slab, so a fifth register would halve its occupancy.
// Node-update blocks of NB threads (g.nub; 256 by default): on the 512 x 512
// slab the launch is one round of four waves per SIMD, and blocks of 256
// spread it more evenly than 512 (3% faster); small meshes may fill more
// compute units with smaller blocks.  Other stencil launches keep NUB.
constexpr int NUB = 256;
template <class T, int NB>
__global__ void __launch_bounds__(NB)
__attribute__((amdgpu_waves_per_eu(4)))
k_node_update(Grid g0, StagesT<T> st, Colloc co, Stim stim, double gs0, double gs1, double gs2,
              int slice0, int i, CgBatchT<T> cb, int store_g, int spread, const double *yref,
              CgLogArgs lg) {
  __shared__ double lds[3 * (NB / 64)];
  const int64_t step0 = *stim.step;
  const int64_t qb = stencil_node_block(g0, blockIdx.x, gridDim.x);
  const int64_t p = qb * NB + threadIdx.x;
  const int n = slice0 + blockIdx.z;
  // the previous solve of this slice is checked by one block (its partial sums
  // are the other stage parity's, which this launch does not write)
  if (lg.log && blockIdx.x == 0) cg_log_entry<NB>(g0, lg, n, lds);
  const Grid g = slice_grid(g0, n);
  const int64_t Np = st.Np;
  const double ddt = co.dt * co.d[i - 1];
  double bb = 0.0, rr = 0.0;
  if (p < g.N) {
    const double *Yp = st.Y + n * st.sY() + (int64_t)(i - 1) * st.sS();
    double *Yi = st.Y + n * st.sY() + (int64_t)i * st.sS();
    const double *RH = st.RH + n * st.sRH() + (int64_t)(i - 1) * st.sS();
    const T *Lu = st.L0 + n * st.sL();  // Lambda of the anchor u
    T *Gp = st.G + n * st.sY() + (int64_t)(i - 1) * st.sS();
    // the state accumulates in FP64; the cell model runs in T.  The new stage's
    // rows and reaction terms are stored with a streaming hint (read again only
    // by later kernels)
    double yd[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) yd[f] = Yp[f * Np + p];
    T gV;
    // operands of the V row: right-hand side, warm start x_0 = V^k_i and its
    // cached K x_0 (loaded first on node 1, after the cell model otherwise)
    const double *fvp = st.FV + n * st.sFV() + (int64_t)(spread ? 0 : i) * Np + p;
    double rh0, x0, kx0;
    if (i == 1) {
      // y_{n,0} = u: its reaction term is the stored one (gates without the
      // anchor part, like every gate reaction term)
      rh0 = RH[p];
      x0 = Yi[p];
      kx0 = *fvp;
#pragma unroll
      for (int f = 1; f < GATE0; ++f)
        stream_store<double>(&Yi[f * Np + p],
                             yd[f] + RH[f * Np + p] + ddt * (double)Gp[f * Np + p]);
      // gates, software-pipelined by one gate like the cell-model path below
      T nlu = Lu[p], ngv = Gp[GATE0 * Np + p];
      double nrh = RH[GATE0 * Np + p];
#pragma unroll
      for (int k = 0; k < NG; ++k) {
        const int f = GATE0 + k;
        const T lu = nlu, gv = ngv;
        const double rh = nrh;
        if (k + 1 < NG) {
          nlu = Lu[(k + 1) * Np + p];
          ngv = Gp[(f + 1) * Np + p];
          nrh = RH[(f + 1) * Np + p];
        }
        stream_store<double>(&Yi[f * Np + p],
                             yd[f] + rh + ddt * phi1(ddt * (double)lu) * (double)gv);
      }
      gV = Gp[p];
    } else {
      T yv[NF];
      if constexpr (std::is_same<T, double>::value) {
#pragma unroll
        for (int f = 0; f < NF; ++f) yv[f] = yd[f];
      } else {
        // A cell model in FP32 rounds its inputs, and that rounding jumps: two
        // FP64 states 1e-16 apart can round to neighbouring FP32 values.  With a
        // reference state (the iterate whose terms the right-hand side holds)
        // the model is evaluated at fl(ref) + fl(y - ref), which equals fl(ref)
        // exactly once y has converged to ref, so the FP32 terms of both sides
        // of the sweep cancel bitwise at the fixed point.
        if (yref) {
          const double *yr = yref + n * st.sY() + (int64_t)(i - 1) * st.sS();
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            const double r = yr[f * Np + p];
            yv[f] = T(r) + T(yd[f] - r);
          }
        } else {
#pragma unroll
          for (int f = 0; f < NF; ++f) yv[f] = T(yd[f]);
        }
      }
      const double t = ((double)(step0 + n * stim.tn) + co.c[i - 2]) * co.dt;
      // software-pipelined by one gate: the operands of gate k + 1 (Lambda_n
      // and right-hand side) are loaded when gate k is applied, so they are in
      // flight while the cell model computes gate k + 1.  The reaction term is
      // formed without the anchor part Lambda_n u (the right-hand side holds it)
      T nlu = Lu[p];
      double nrh = RH[GATE0 * Np + p];
      ttp06::gates<T>(yv[0], yv[3], [&](int k, T inf, T rate) {
        const int f = GATE0 + k;
        const T lu = nlu;
        const double rh = nrh;
        if (k + 1 < NG) {
          nlu = Lu[(k + 1) * Np + p];
          nrh = RH[(f + 1) * Np + p];
        }
        const T w = yv[f];
        const T gv = -rate * (w - inf) - lu * w;
        if (store_g) stream_store<T>(&Gp[f * Np + p], gv);
        stream_store<double>(&Yi[f * Np + p],
                             yd[f] + rh + ddt * phi1(ddt * (double)lu) * (double)gv);
      });
      // right-hand sides of the rows after the cell model, in flight during the
      // currents (the V row's operands follow them: registers are the limit)
      double rha[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) rha[k] = RH[(1 + k) * Np + p];
      T I_ion, ha[6];
      ttp06::currents<T>(yv, T(gs0), T(gs1), T(gs2), I_ion, ha);
      gV = (T(stim_value(stim, t, n, p)) - T(stim.Cm) * I_ion) / T(stim.Cm);
      if (store_g) stream_store<T>(&Gp[p], gV);
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        if (store_g) stream_store<T>(&Gp[(1 + k) * Np + p], ha[k]);
        stream_store<double>(&Yi[(1 + k) * Np + p], yd[1 + k] + rha[k] + ddt * (double)ha[k]);
      }
      rh0 = RH[p];
      x0 = Yi[p];
      kx0 = *fvp;
    }
    // right-hand side of (I - dt d_i K) V_i = b and the CG start residual for
    // the warm start x_0 = V^k_i, whose K x_0 is cached from the previous sweep
    const double bv = yd[0] + rh0 + ddt * (double)gV;
    const double r0 = bv - x0 + cb.a * kx0;
    if (cb.direct) {
      cb.bout[(int64_t)(n - slice0) * Np + p] = bv;  // the DCT-II solve takes b
    } else if (cb.xt) {
      // Chebyshev: b and the first iterate x_1 = x_0 + r_0 / theta (and x_0 for
      // the tiled start, which writes x_D over x)
      cb.bout[(int64_t)(n - slice0) * Np + p] = bv;
      cb.xt[(int64_t)(n - slice0) * Np + p] = x0 + r0 * cb.tab[n * cb.tab_stride].inv_theta;
      if (cb.x0_to_p) cb.p[(int64_t)(n - slice0) * Np + p] = x0;
    } else {
      cb.r[0][(int64_t)(n - slice0) * Np + p] = T(r0);
    }
    bb = bv * bv;
    rr = r0 * r0;
  }
  double t2[2] = {bb, rr};
  block_sums<2, NB>(t2, lds);
  if (threadIdx.x == 0) {
    double *part = cb.part + (int64_t)(n - slice0) * 5 * cb.pstride;
    part[4 * cb.pstride + qb] = t2[0];
    part[qb] = t2[1];
  }
}

// Blocks of nb threads over one slice's nodes (XCD-padded unless the slices
// are a ragged batch); the first CG iteration reduces node_blocks(g) partials
// of the node update.
int node_blocks_of(const Grid &g, int nb) {
  const unsigned n = (unsigned)((g.N + nb - 1) / nb);
  return (int)(g.rag ? n : (n + kXcds - 1) / kXcds * kXcds);
}
int node_blocks(const Grid &g) { return node_blocks_of(g, g.nub); }

template <class T>
hipError_t launch_node_update(hipStream_t s, const Grid &g, const StagesT<T> &st,
                              const Colloc &co, const Stim &stim, double gs0, double gs1,
                              double gs2, int slice0, int nslices, int i,
                              const CgBatchT<T> &cb, int store_g, int spread,
                              const double *yref, const CgLogArgs &lg) {
  dim3 grid(node_blocks(g), 1, nslices);
#define HSDC_NU_LAUNCH(NB_)                                                                    \
  hipLaunchKernelGGL((k_node_update<T, NB_>), grid, dim3(NB_), 0, s, g, st, co, stim, gs0, gs1, \
                     gs2, slice0, i, cb, store_g, spread, yref, lg)
  if constexpr (std::is_same<T, float>::value) {  // an FP32 coarse level keeps the default
    if (g.nub != kDefaultNodeBlock) return hipErrorInvalidValue;
    HSDC_NU_LAUNCH(kDefaultNodeBlock);
  } else {
    switch (g.nub) {
      case 64: HSDC_NU_LAUNCH(64); break;
      case 128: HSDC_NU_LAUNCH(128); break;
      case 256: HSDC_NU_LAUNCH(256); break;
      case 512: HSDC_NU_LAUNCH(512); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef HSDC_NU_LAUNCH
  return hipGetLastError();
}

// V of stage 0 to stages 1..M (the CG warm starts of the first sweep of a step).
__global__ void __launch_bounds__(BLOCK) k_copy_V_to_stages(Grid g0, Stages st, int slice0) {
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (p >= slice_grid(g0, slice0 + blockIdx.z).N) return;
  double *Y = st.Y + (slice0 + blockIdx.z) * st.sY();
  const double v = Y[p];
  for (int j = 1; j <= st.M; ++j) Y[(int64_t)j * st.sS() + p] = v;
}

hipError_t launch_copy_V_to_stages(hipStream_t s, const Grid &g, const Stages &st, int slice0,
                                   int nslices) {
  hipLaunchKernelGGL(k_copy_V_to_stages, dim3(nblocks(g.N), 1, nslices), dim3(BLOCK), 0, s, g, st,
                     slice0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// residual r_n = C(y_n) - 1 (x) u_prev (Algorithm 1), per-slice inf norms of r
// and y; optionally the time-restricted integrals RI_i = sum_l R_il I_l.
// ---------------------------------------------------------------------------

// One thread per (node, field) like the assembly, instantiated separately for
// the rows V .. Rbar and the gate rows (held to four waves per SIMD); each
// block writes the maxima of its row, reduced per (slice, field) by k_reduce_max2.
template <int M, bool GATES>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4)))
k_residual(Grid g0, Stages st, Colloc co, int slice0, const double *yblk0, double *part, int nbx,
           const double *Rt, int Mc, double *RI, int64_t sRI, const double *RIadd,
           int64_t sRIadd) {
  __shared__ double lds[BLOCK / 64];
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int f = GATES ? GATE0 + (int)blockIdx.y : (int)blockIdx.y;
  const int n = slice0 + blockIdx.z;
  const Grid g = slice_grid(g0, n);
  const int64_t Np = st.Np;
  double rmax = 0.0, ymax = 0.0;
  if (p < g.N) {
    const double *Y = st.Y + n * st.sY() + f * Np + p;
    const double *G = st.G + n * st.sY() + f * Np + p;
    // u: the block start (slice 0), the previous slice's end, or, for independent
    // slices (yblk0 == NULL: serial steps, tissues of a batch), the own start value
    const double *up = (yblk0 == nullptr) ? st.Y + n * st.sY()
                       : (n == 0)         ? yblk0
                                          : st.Y + (n - 1) * st.sY() + (int64_t)M * st.sS();
    double gfull[M], I[M];
#pragma unroll
    for (int j = 0; j < M; ++j)
      gfull[j] = G[(j + 1) * st.sS()] + (f == 0 ? st.FV[n * st.sFV() + (j + 1) * Np + p] : 0.0);
    const double y0 = Y[0];
    if constexpr (GATES) {
      // G holds the gate reaction terms without the anchor part Lambda_n y_{n,0}
      const double lam_n = st.L0[n * st.sL() + (f - GATE0) * Np + p];
      colloc_integrals<M>(co, co.dt * lam_n, gfull, I, lam_n * y0);
    } else {
      colloc_weights<M>(co, gfull, I);
    }
    const double u = up[f * Np + p];
    rmax = nmax(rmax, fabs(y0 - u));
    ymax = nmax(ymax, fabs(y0));
#pragma unroll
    for (int i = 0; i < M; ++i) {
      const double yi = Y[(i + 1) * st.sS()];
      rmax = nmax(rmax, fabs(yi - co.dt * I[i] - u));
      ymax = nmax(ymax, fabs(yi));
    }
    if (RI) {
      // the integrals, plus the level's own FAS term (a middle level of three),
      // restricted in time to the coarser level's nodes
      if (RIadd) {
#pragma unroll
        for (int l = 0; l < M; ++l) I[l] += RIadd[n * sRIadd + ((int64_t)l * NF + f) * Np + p];
      }
      for (int ic = 0; ic < Mc; ++ic) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < M; ++l) s += Rt[(ic + 1) * (M + 1) + (l + 1)] * I[l];
        RI[n * sRI + ((int64_t)ic * NF + f) * Np + p] = s;
      }
    }
  }
  const double br = block_max(rmax, lds);
  const double by = block_max(ymax, lds);
  if (threadIdx.x == 0) {
    const int64_t k = ((int64_t)blockIdx.z * NF + f) * nbx + blockIdx.x;
    part[2 * k + 0] = br;
    part[2 * k + 1] = by;
  }
}

__global__ void __launch_bounds__(BLOCK) k_reduce_max2(const double *part, int nblk, double *out) {
  __shared__ double lds[BLOCK / 64];
  const int n = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nblk; k += BLOCK) {
    a = nmax(a, part[((int64_t)n * nblk + k) * 2 + 0]);
    b = nmax(b, part[((int64_t)n * nblk + k) * 2 + 1]);
  }
  a = block_max(a, lds);
  b = block_max(b, lds);
  if (threadIdx.x == 0) {
    out[2 * n] = a;
    out[2 * n + 1] = b;
  }
}

// Partials per slice of a residual launch: one per (field, node block).
int residual_blocks(const Grid &g) { return NF * (int)nblocks(g.N); }

hipError_t launch_residual(hipStream_t s, const Grid &g, const Stages &st, const Colloc &co,
                           int slice0, int nslices, const double *y_block0, double *part,
                           int nblk, double *out2, const double *Rt, int Mc, double *RI,
                           int64_t sRI, const double *RIadd, int64_t sRIadd) {
  // nblk = NF node-block rows per slice (residual_blocks)
  const int nbx = (int)nblocks(g.N);
  const dim3 rows(nbx, GATE0, nslices), gates(nbx, NG, nslices);
  HSDC_DISPATCH_M(co.M, {
    hipLaunchKernelGGL((k_residual<M, false>), rows, dim3(BLOCK), 0, s, g, st, co, slice0,
                       y_block0, part, nbx, Rt, Mc, RI, sRI, RIadd, sRIadd);
    hipLaunchKernelGGL((k_residual<M, true>), gates, dim3(BLOCK), 0, s, g, st, co, slice0,
                       y_block0, part, nbx, Rt, Mc, RI, sRI, RIadd, sRIadd);
  });
  // one reduction per (slice, field): the partials of a slice are laid out
  // field by field, nbx per field
  hipLaunchKernelGGL(k_reduce_max2, dim3(nslices * NF), dim3(BLOCK), 0, s, part, nbx, out2);
  return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK)
k_copy_fields(int64_t Np, double *dst, int64_t sdst, const double *src, int64_t ssrc, int nf) {
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (p >= Np) return;
  const int n = blockIdx.z;
  for (int f = 0; f < nf; ++f) dst[n * sdst + f * Np + p] = src[n * ssrc + f * Np + p];
}

hipError_t launch_copy_fields(hipStream_t s, int64_t Np, double *dst, int64_t sdst,
                              const double *src, int64_t ssrc, int nf, int nslices) {
  if (nslices <= 0) return hipSuccess;
  dim3 grid(nblocks(Np), 1, nslices);
  hipLaunchKernelGGL(k_copy_fields, grid, dim3(BLOCK), 0, s, Np, dst, sdst, src, ssrc, nf);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CG on A x = b, A = I - a K, batched over slices, in the single-reduction
// (Chronopoulos-Gear) form:
//   gamma = (r, r), delta = (A r, r), beta = gamma / gamma_prev,
//   alpha = gamma / (delta - beta gamma / alpha_prev),
//   p = r + beta p, s = A r + beta s, x += alpha p, r -= alpha s, w = A r.
// One stencil kernel per iteration: the new r at the stencil neighbours is
// formed on the fly from the previous r, w, s (ping-pong buffers), so one grid
// synchronisation (the kernel boundary) and one reduction suffice.  Converged
// slices return at once; the iteration budget is set by the host.
// Partials per slice: [gamma par0 | delta par0 | gamma par1 | delta par1 | bb].
// ---------------------------------------------------------------------------

// Blocks of the CG kernels: at most cap (<= 2 BLOCK partials per reduction);
// nodes beyond cap * BLOCK are handled by a grid-stride loop.
int cg_blocks(const Grid &g, int cap) {
  const int64_t nb = ((int64_t)g.N + BLOCK - 1) / BLOCK;
  cap = cap < 1 ? 1 : (cap > 2 * BLOCK ? 2 * BLOCK : cap);
  return (int)(nb < cap ? nb : cap);
}

// Blocks of a CG launch that own nodes of a slice with g.N nodes: a small
// tissue of a batch needs fewer than the launch has, and the others exit at
// once; every reduction reads the partials of the active blocks only.
__device__ __forceinline__ int active_blocks(const Grid &g, int nblk) {
  const int64_t nb = (g.N + BLOCK - 1) / BLOCK;
  return nb < nblk ? (int)nb : nblk;
}

// Start residual r_0 = b - A x_0 with the partials of ||r_0||^2 and ||b||^2
// (used when r_0 is not produced by the node update).
template <int DIM, bool PN, class T>
__global__ void __launch_bounds__(BLOCK) k_cg_resid0(Grid g0, CgBatchT<T> cb) {
  __shared__ double lds[3 * (BLOCK / 64)];
  const int n = blockIdx.y;
  const Grid g = slice_grid(g0, cb.slice0 + n);
  if ((int)blockIdx.x >= active_blocks(g, cb.nblk)) return;
  const double *x = cb.x + n * cb.sx;
  const double *b = cb.b + n * cb.sb;
  T *r = cb.r[0] + n * g.Np;
  double rr = 0.0, bb = 0.0;
  const int64_t qb = stencil_node_block(g0, blockIdx.x, cb.nblk);
  for (int64_t p = qb * BLOCK + threadIdx.x; p < g.N; p += (int64_t)cb.nblk * BLOCK) {
    const Ijk c = ijk(g, p);
    const double xc = x[p];
    const double bv = b[p];
    const double rc = bv - (xc - cb.a * applyK<DIM, PN>(g, p, c, xc, [&](int64_t k) { return x[k]; }));
    r[p] = rc;
    rr += rc * rc;
    bb += bv * bv;
  }
  double *part = cb.part + (int64_t)n * 5 * cb.pstride;
  double t2[2] = {rr, bb};
  block_sums<2>(t2, lds);
  if (threadIdx.x == 0) {
    part[qb] = t2[0];
    part[4 * cb.pstride + qb] = t2[1];
  }
}

// w_0 = A r_0 and the partials of delta_0 = (w_0, r_0); resets the scalars.
template <int DIM, bool PN, class T>
__global__ void __launch_bounds__(BLOCK) k_cg_init(Grid g0, CgBatchT<T> cb) {
  __shared__ double lds[BLOCK / 64];
  const int n = blockIdx.y;
  const Grid g = slice_grid(g0, cb.slice0 + n);
  if ((int)blockIdx.x >= active_blocks(g, cb.nblk)) return;
  const T *r = cb.r[0] + n * g.Np;
  T *w = cb.w[0] + n * g.Np;
  double del = 0.0;
  const int64_t qb = stencil_node_block(g0, blockIdx.x, cb.nblk);
  for (int64_t p = qb * BLOCK + threadIdx.x; p < g.N; p += (int64_t)cb.nblk * BLOCK) {
    const Ijk c = ijk(g, p);
    const double rc = r[p];
    const double wv = rc - cb.a * applyK<DIM, PN>(g, p, c, rc, [&](int64_t k) { return (double)r[k]; });
    w[p] = wv;
    del += wv * rc;
  }
  double *part = cb.part + (int64_t)n * 5 * cb.pstride;
  const double td = block_sum(del, lds);
  if (threadIdx.x == 0) {
    part[cb.pstride + qb] = td;
    if (blockIdx.x == 0) {
      CgScalars o;
      o.bb = -1.0;  // reduced by the first iteration kernel
      o.gamma = 1.0;
      o.alpha = 1.0;
      o.it = 0;
      o.done = 0;
      cb.sc[2 * n] = o;
    }
  }
}

template <int DIM, bool PN, class T>
__global__ void __launch_bounds__(BLOCK) k_cg_iter(Grid g0, CgBatchT<T> cb, int k) {
  __shared__ double lds[3 * (BLOCK / 64)];
  const int n = blockIdx.y;
  const Grid g = slice_grid(g0, cb.slice0 + n);
  // a ragged batch skips the CG blocks past a small tissue; every block of the
  // launch that produced r_0 wrote partials (zeros past a small tissue or the
  // node count), whatever that launch's block size
  const int nba = active_blocks(g, cb.nblk);
  const int nba0 = cb.nblk0;
  if ((int)blockIdx.x >= nba) return;
  const int in = k & 1, out = in ^ 1;
  CgScalars si = cb.sc[2 * n + in];
  CgScalars *so = cb.sc + 2 * n + out;
  const bool publish = blockIdx.x == 0 && threadIdx.x == 0;
  const bool logit = publish && cb.log && k == cb.last_k;
  if (si.done) {
    if (publish) *so = si;
    if (logit) cb.log[n] = si;
    return;
  }
  double *part = cb.part + (int64_t)n * 5 * cb.pstride;
  const T *r = cb.r[in] + n * g.Np;
  const T *w = cb.w[in] + n * g.Np;
  const T *s = cb.s[in] + n * g.Np;
  double gamma, delta;
  // first owned node: its stencil loads are issued before the partial sums
  // are combined, so the reduction latency overlaps the memory traffic
  const int64_t qb = stencil_node_block(g0, blockIdx.x, cb.nblk);
  const int64_t p0 = qb * BLOCK + threadIdx.x;
  double r_c = 0.0, w_c = 0.0, s_c = 0.0, rn_[2 * DIM], wn_[2 * DIM], sn_[2 * DIM];
  Ijk c0{0, 0, 0};
  if (si.it == 0) {
    double t3[3] = {0.0, 0.0, 0.0};
    if (cb.cstart) {
      // gamma and delta of the Chebyshev start (this parity, over the start's
      // blocks) and ||b||^2 (over the node update's)
      const double *pg = part + (2 * in) * cb.pstride, *pd = part + (2 * in + 1) * cb.pstride;
      for (int k = threadIdx.x; k < cb.nblk_s; k += BLOCK) {
        t3[0] += pg[k];
        t3[2] += pd[k];
      }
      for (int k = threadIdx.x; k < nba0; k += BLOCK) t3[1] += part[4 * cb.pstride + k];
    } else {
      for (int k = threadIdx.x; k < nba0; k += BLOCK) {
        t3[0] += part[k];
        t3[1] += part[4 * cb.pstride + k];
      }
      for (int k = threadIdx.x; k < nba; k += BLOCK) t3[2] += part[cb.pstride + k];
    }
    block_sums<3>(t3, lds);
    gamma = t3[0];
    // stop relative to ||b|| or, for a correction solve, to ||r_0||
    si.bb = cb.rel_r0 ? gamma : t3[1];
    delta = t3[2];
  } else {
    const double *pg = part + (2 * in) * cb.pstride, *pd = part + (2 * in + 1) * cb.pstride;
    const int t = threadIdx.x;
    const double g0 = t < nba ? pg[t] : 0.0, g1 = t + BLOCK < nba ? pg[t + BLOCK] : 0.0;
    const double d0 = t < nba ? pd[t] : 0.0, d1 = t + BLOCK < nba ? pd[t + BLOCK] : 0.0;
    if (!PN && p0 < g.N) {
      c0 = ijk(g, p0);
      r_c = r[p0];
      w_c = w[p0];
      s_c = s[p0];
      const int64_t off[6] = {-1, 1, -(int64_t)g.nx, (int64_t)g.nx, -(int64_t)g.nx * g.ny,
                              (int64_t)g.nx * g.ny};
      const bool ok[6] = {c0.ix > 0, c0.ix < g.nx - 1, c0.iy > 0, c0.iy < g.ny - 1, c0.iz > 0,
                          c0.iz < g.nz - 1};
#pragma unroll
      for (int q = 0; q < 2 * DIM; ++q) {
        const int64_t idx = ok[q] ? p0 + off[q] : p0;
        rn_[q] = r[idx];
        wn_[q] = w[idx];
        sn_[q] = s[idx];
      }
    }
    double t2[2] = {g0 + g1, d0 + d1};
    block_sums<2>(t2, lds);
    gamma = t2[0];
    delta = t2[1];
  }
  // a NaN or Inf residual or right-hand side (a non-finite state) ends the
  // solve at once: no iteration can recover, and the host reports it
  const bool nonfinite = !(gamma - gamma == 0.0) || !(si.bb - si.bb == 0.0);
  if (gamma <= cb.tol2 * si.bb || gamma == 0.0 || si.it >= cb.maxit || nonfinite) {
    if (publish) {
      CgScalars o = si;
      o.gamma = gamma;
      o.done = 1;
      *so = o;
      if (logit) cb.log[n] = o;
    }
    return;
  }
  const bool first = si.it == 0;
  const double beta = first ? 0.0 : gamma / si.gamma;
  const double alpha = first ? gamma / delta : gamma / (delta - beta * gamma / si.alpha);
  T *ro = cb.r[out] + n * g.Np;
  T *wo = cb.w[out] + n * g.Np;
  T *sout = cb.s[out] + n * g.Np;
  T *pp = cb.p + n * g.Np;
  double *x = cb.x + n * cb.sx;
  double gam = 0.0, del = 0.0;
  // iteration 0 takes p = r, s = w (p and s hold nothing yet)
  auto update = [&](int64_t p, const Ijk &c, double rc0, double wc0, double sc0, auto &&rn) {
    const double pn = first ? rc0 : rc0 + beta * pp[p];
    const double sn = first ? wc0 : wc0 + beta * sc0;
    const double rc = rc0 - alpha * sn;
    x[p] += alpha * pn;
    const double wn = rc - cb.a * applyK<DIM, PN>(g, p, c, rc, rn);
    pp[p] = pn;
    sout[p] = sn;
    ro[p] = rc;
    wo[p] = wn;
    gam += rc * rc;
    del += wn * rc;
  };
  // r of this iteration at a stencil neighbour, formed from the previous r, w, s
  auto rfull = [&](int64_t qq) {
    return first ? r[qq] - alpha * w[qq] : r[qq] - alpha * (w[qq] + beta * s[qq]);
  };
  int64_t p = p0;
  if (!PN && !first && p0 < g.N) {
    // first owned node from the prefetched registers; the neighbour order
    // -x, +x, -y, +y, -z, +z and the per-axis grouping follow applyK
    const bool ok[6] = {c0.ix > 0, c0.ix < g.nx - 1, c0.iy > 0, c0.iy < g.ny - 1, c0.iz > 0,
                        c0.iz < g.nz - 1};
    const double pn = r_c + beta * pp[p0];
    const double sn = w_c + beta * s_c;
    const double rc = r_c - alpha * sn;
    x[p0] += alpha * pn;
    double ax[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int qq = 0; qq < 2 * DIM; ++qq)
      if (ok[qq]) ax[qq >> 1] += (rn_[qq] - alpha * (wn_[qq] + beta * sn_[qq])) - rc;
    double acc = g.cx * ax[0];
    if (DIM >= 2) acc += g.cy * ax[1];
    if (DIM >= 3) acc += g.cz * ax[2];
    const double wn = rc - cb.a * acc;
    pp[p0] = pn;
    sout[p0] = sn;
    ro[p0] = rc;
    wo[p0] = wn;
    gam += rc * rc;
    del += wn * rc;
    p += (int64_t)cb.nblk * BLOCK;
  }
  for (; p < g.N; p += (int64_t)cb.nblk * BLOCK) {
    const Ijk c = ijk(g, p);
    update(p, c, r[p], w[p], s[p], rfull);
  }
  double t2[2] = {gam, del};
  block_sums<2>(t2, lds);
  if (threadIdx.x == 0) {
    part[(2 * out) * cb.pstride + qb] = t2[0];
    part[(2 * out + 1) * cb.pstride + qb] = t2[1];
  }
  if (publish) {
    CgScalars o = si;
    o.gamma = gamma;
    o.alpha = alpha;
    o.it = si.it + 1;
    o.done = 0;
    *so = o;
    if (logit) cb.log[n] = o;
  }
}

template <class T>
hipError_t launch_cg_init(hipStream_t s, const Grid &g, const CgBatchT<T> &cb) {
  dim3 grid(cb.nblk, cb.nslices);
  HSDC_DISPATCH_OP(g, hipLaunchKernelGGL((k_cg_init<DIM, PN, T>), grid, dim3(BLOCK), 0, s, g, cb));
  return hipGetLastError();
}

template <class T>
hipError_t launch_cg_resid0(hipStream_t s, const Grid &g, const CgBatchT<T> &cb) {
  dim3 grid(cb.nblk, cb.nslices);
  HSDC_DISPATCH_OP(g,
                   hipLaunchKernelGGL((k_cg_resid0<DIM, PN, T>), grid, dim3(BLOCK), 0, s, g, cb));
  return hipGetLastError();
}

template <class T>
hipError_t launch_cg_iter(hipStream_t s, const Grid &g, const CgBatchT<T> &cb, int k) {
  dim3 grid(cb.nblk, cb.nslices);
  HSDC_DISPATCH_OP(
      g, hipLaunchKernelGGL((k_cg_iter<DIM, PN, T>), grid, dim3(BLOCK), 0, s, g, cb, k));
  return hipGetLastError();
}

// CG start from the Chebyshev iterate x_D, D = cb.cstart (in x for D even, in
// xt for D odd, then copied to x): r_D = b - A x_D and w_D = A r_D, with r_D at
// the stencil neighbours formed from x_D at radius 2.  One node per thread in
// node-update blocks, so the partials of (r_D, r_D) and (w_D, r_D) (parity-1
// slots) line up with the node update's partials of ||b||^2; the parity-1
// scalars are reset for the CG launch k = 1.
// Uniform coefficients: every stencil read goes through clamped coordinates,
// so a neighbour missing at the boundary reads the node itself and its term
// v_q - v_p is exactly 0, as applyK's omitted term; the loads carry no
// branches.
template <int DIM, bool PN>
__global__ void __launch_bounds__(NUB) k_cg_start(Grid g0, CgBatch cb) {
  __shared__ double lds[2 * (NUB / 64)];
  const int n = blockIdx.y;
  const Grid g = slice_grid(g0, cb.slice0 + n);
  const int64_t qb = stencil_node_block(g0, blockIdx.x, gridDim.x);
  const int64_t p = qb * NUB + threadIdx.x;
  const bool odd = cb.cstart & 1;
  const double *x = odd ? cb.xt + (int64_t)n * g0.Np : cb.x + n * cb.sx;
  const double *b = cb.b + n * cb.sb;
  double gam = 0.0, del = 0.0;
  if (p < g.N) {
    const Ijk c = ijk(g, p);
    if (odd) cb.x[n * cb.sx + p] = x[p];
    double rc, wv;
    if constexpr (!PN) {
      const int nx = g.nx, ny = g.ny, nz = g.nz;
      auto cl = [](int v, int m) { return v < 0 ? 0 : (v > m - 1 ? m - 1 : v); };
      auto at = [&](int ix, int iy, int iz) {
        return (int64_t)ix + (int64_t)nx * ((int64_t)iy + (int64_t)ny * iz);
      };
      // b - A x at the node (ix, iy, iz), the sums grouped per axis as applyK
      auto resid = [&](int ix, int iy, int iz) {
        const double xq = x[at(ix, iy, iz)];
        const double ax = (x[at(cl(ix - 1, nx), iy, iz)] - xq) + (x[at(cl(ix + 1, nx), iy, iz)] - xq);
        double acc = g.cx * ax;
        if (DIM >= 2)
          acc += g.cy * ((x[at(ix, cl(iy - 1, ny), iz)] - xq) + (x[at(ix, cl(iy + 1, ny), iz)] - xq));
        if (DIM >= 3)
          acc += g.cz * ((x[at(ix, iy, cl(iz - 1, nz))] - xq) + (x[at(ix, iy, cl(iz + 1, nz))] - xq));
        return b[at(ix, iy, iz)] - (xq - cb.a * acc);
      };
      rc = resid(c.ix, c.iy, c.iz);
      const double ax = (resid(cl(c.ix - 1, nx), c.iy, c.iz) - rc) +
                        (resid(cl(c.ix + 1, nx), c.iy, c.iz) - rc);
      double acc = g.cx * ax;
      if (DIM >= 2)
        acc += g.cy * ((resid(c.ix, cl(c.iy - 1, ny), c.iz) - rc) +
                       (resid(c.ix, cl(c.iy + 1, ny), c.iz) - rc));
      if (DIM >= 3)
        acc += g.cz * ((resid(c.ix, c.iy, cl(c.iz - 1, nz)) - rc) +
                       (resid(c.ix, c.iy, cl(c.iz + 1, nz)) - rc));
      wv = rc - cb.a * acc;
    } else {
      auto resid = [&](int64_t q, const Ijk &cq) {
        const double xq = x[q];
        return b[q] - (xq - cb.a * applyK<DIM, PN>(g, q, cq, xq, [&](int64_t k) { return x[k]; }));
      };
      rc = resid(p, c);
      wv = rc - cb.a * applyK_nb<DIM, PN>(g, p, c, rc, resid);
    }
    cb.r[1][n * g.Np + p] = rc;
    cb.w[1][n * g.Np + p] = wv;
    gam = rc * rc;
    del = wv * rc;
  }
  double *part = cb.part + (int64_t)n * 5 * cb.pstride;
  double t2[2] = {gam, del};
  block_sums<2, NUB>(t2, lds);
  if (threadIdx.x == 0) {
    part[2 * cb.pstride + qb] = t2[0];
    part[3 * cb.pstride + qb] = t2[1];
    if (blockIdx.x == 0) {
      CgScalars o;
      o.bb = -1.0;  // reduced by the first iteration kernel
      o.gamma = 1.0;
      o.alpha = 1.0;
      o.it = 0;
      o.done = 0;
      cb.sc[2 * n + 1] = o;
    }
  }
}

hipError_t launch_cg_start(hipStream_t s, const Grid &g, const CgBatch &cb) {
  // the node update's block count (every block writes its partials)
  dim3 grid(node_blocks_of(g, NUB), cb.nslices);
  HSDC_DISPATCH_OP(g, hipLaunchKernelGGL((k_cg_start<DIM, PN>), grid, dim3(NUB), 0, s, g, cb));
  return hipGetLastError();
}

// out = K v, one node per thread in XCD block order (a neighbour row is then
// read by a block of the same XCD, from its L2), as k_spmv_stages.
template <int DIM, bool PN>
__global__ void __launch_bounds__(BLOCK) k_apply_K(Grid g, const double *v, double *out) {
  const int64_t p = stencil_node_block(g, blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (p >= g.N) return;
  const Ijk c = ijk(g, p);
  out[p] = applyK<DIM, PN>(g, p, c, v[p], [&](int64_t k) { return v[k]; });
}

// out = K v on a 2D mesh with uniform sigma, streamed along y: a thread owns
// two neighbouring nodes of a row (16-byte loads and stores) and walks SY
// rows, keeping the rows below and above its own in registers, so v is read
// from memory about once (plus one row per SY); the x neighbours come from
// the adjacent lanes by shuffles, the wave's edge lanes read them from memory.
// A neighbour missing at the wall is the node itself (its term is exactly 0),
// and the sums are grouped as applyK groups them, so the result is the same.
// Lanes past the mesh (nx not a multiple of the block's width) load the last
// pair and store nothing.  nx must be even and v, out 16-byte aligned.
typedef double d2v __attribute__((ext_vector_type(2)));
constexpr int SPX = 256, SY = 16;
__global__ void __launch_bounds__(SPX) k_apply_K2d(Grid g, const double *v, double *out) {
  const int nx = g.nx, ny = g.ny;
  const int ix = 2 * (blockIdx.x * SPX + threadIdx.x);
  const bool own = ix < nx;
  const int ixc = own ? ix : nx - 2;
  const int lane = threadIdx.x & 63;
  const int y0 = blockIdx.y * SY;
  const d2v *v2 = (const d2v *)v;
  d2v *o2 = (d2v *)out;
  const int64_t hr = nx / 2;  // a row in pairs
  int64_t q = ((int64_t)y0 * nx + ixc) >> 1;
  d2v cur = v2[q];
  d2v below = y0 > 0 ? v2[q - hr] : cur;
  for (int k = 0; k < SY; ++k, q += hr) {
    const int iy = y0 + k;
    if (iy >= ny) break;  // uniform over the block
    const d2v above = iy < ny - 1 ? v2[q + hr] : cur;
    double l = __shfl_up(cur.y, 1), r = __shfl_down(cur.x, 1);
    if (lane == 0) l = ixc > 0 ? v[2 * q - 1] : cur.x;
    if (lane == 63 || ixc + 2 >= nx) r = ixc + 2 < nx ? v[2 * q + 2] : cur.y;
    if (ixc == 0) l = cur.x;
    double acc0 = g.cx * ((l - cur.x) + (cur.y - cur.x));
    double acc1 = g.cx * ((cur.x - cur.y) + (r - cur.y));
    acc0 += g.cy * ((below.x - cur.x) + (above.x - cur.x));
    acc1 += g.cy * ((below.y - cur.y) + (above.y - cur.y));
    if (own) __builtin_nontemporal_store(d2v{acc0, acc1}, &o2[q]);
    below = cur;
    cur = above;
  }
}

hipError_t launch_apply_K(hipStream_t s, const Grid &g, const double *v, double *out) {
  if (g.order == 4) return launch_apply_K4(s, g, v, out);
  const bool aligned = (((uintptr_t)v | (uintptr_t)out) & 15) == 0;  // 16-byte accesses
  if (g.dim == 2 && g.kx == nullptr && g.nx % 2 == 0 && g.nx >= 2 && aligned) {
    const dim3 grid((g.nx / 2 + SPX - 1) / SPX, (g.ny + SY - 1) / SY);
    hipLaunchKernelGGL(k_apply_K2d, grid, dim3(SPX), 0, s, g, v, out);
    return hipGetLastError();
  }
  HSDC_DISPATCH_OP(g, hipLaunchKernelGGL((k_apply_K<DIM, PN>), dim3(nblocks_xcd(g.N)), dim3(BLOCK),
                                         0, s, g, v, out));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Chebyshev iteration on A x = b, A = I - a K.  The spectrum of A lies in
// [1, 1 + a lam] (lam: Gershgorin bound on the spectrum of -K); theta and delta
// are the centre and half-width of that interval and sigma = theta / delta.
// After m steps the residual is r_m = T_m((theta - A) / delta) r_0 / T_m(sigma),
// so ||r_m|| <= ||r_0|| / T_m(sigma) for symmetric A: the iteration needs no
// inner products, and the count follows from ||r_0|| and ||b|| alone.  Three-
// term form: x_1 = x_0 + r_0 / theta,
//   x_{k+1} = x_{k-1} + omega_{k+1} (x_k - x_{k-1} + (b - A x_k) / theta),
//   omega_{k+1} = 2 sigma T_k(sigma) / T_{k+1}(sigma).
// ---------------------------------------------------------------------------

// omega_{k+1}, k >= 1, from the table or, past it, with T_k(sigma) = cosh(k s):
// cosh(k s) / cosh((k+1) s) = e^{-s} (1 + e^{-2ks}) / (1 + e^{-2(k+1)s}).
__device__ __forceinline__ double cheb_omega(const ChebTab &t, int k) {
  if (k <= CHEB_KT) return t.omega[k - 1];
  if (t.s == 0.0) return 1.0;
  return 2.0 * t.sigma * exp(-t.s) * (1.0 + exp(-2.0 * k * t.s)) / (1.0 + exp(-2.0 * (k + 1) * t.s));
}

// Iteration count: the smallest even m >= 2 with T_m(sigma) >= 2 ||r_0|| / (rtol
// ref) (ref = ||b||, or ||r_0|| for a solve relative to the warm start; the
// factor 2 covers rounding), capped at maxit.  *bound receives the bound
// ||r_0||^2 / T_m(sigma)^2 on ||r_m||^2 (NaN inputs give NaN).  The first
// launch forms x_2 whatever the count, so m is at least 2 (x_2 only improves
// on x_0).
__device__ __forceinline__ int cheb_count(const ChebTab &t, double rr0, double ref2, double tol2,
                                          int maxit, double *bound) {
  int m = 2;
  if (rr0 == rr0 && ref2 == ref2 && t.s > 0.0 && rr0 > tol2 * ref2) {
    const double ratio = 2.0 * sqrt(rr0 / (tol2 * ref2));  // > 2, also for ref2 = 0 (inf)
    const double mr = acosh(ratio) / t.s;
    m = mr < (double)maxit ? (int)ceil(mr) : maxit;
    m = (m + 1) & ~1;
    if (m > maxit) m = maxit & ~1;
    if (m < 2) m = 2;
  }
  const double tm = t.s == 0.0 ? INFINITY : cosh(m * t.s);
  *bound = (rr0 == rr0 && ref2 == ref2) ? rr0 / (tm * tm) : rr0 + ref2;
  return m;
}

// Launch k >= 1 forms x_{k+1} over x_{k-1}.  Blocks [0, nbx) own nodes; launch 1
// has one more block per slice that reduces the node update's partials of
// ||r_0||^2 and ||b||^2 and publishes the count while the others iterate.
template <int DIM, bool PN>
__global__ void __launch_bounds__(BLOCK) k_cheb_iter(Grid g0, CgBatch cb, int k, int nbx,
                                                     int step_only) {
  __shared__ double lds[3 * (BLOCK / 64)];
  const int n = blockIdx.y;
  const ChebTab &t = cb.tab[(cb.slice0 + n) * cb.tab_stride];
  CgScalars *sc = cb.sc + 2 * n;
  if ((int)blockIdx.x >= nbx) {
    const double *part = cb.part + (int64_t)n * 5 * cb.pstride;
    double t2[2] = {0.0, 0.0};
    for (int k = threadIdx.x; k < cb.nblk0; k += BLOCK) {
      t2[0] += part[k];
      t2[1] += part[4 * cb.pstride + k];
    }
    block_sums<2>(t2, lds);
    const double rr0 = t2[0];
    const double ref2 = cb.rel_r0 ? rr0 : t2[1];
    if (threadIdx.x == 0) {
      double bound;
      CgScalars o;
      o.it = cheb_count(t, rr0, ref2, cb.tol2, cb.maxit, &bound);
      o.bb = ref2;
      o.gamma = bound;
      o.alpha = 0.0;
      o.done = o.it <= 2;  // x_2, written by this launch, is in x
      sc[0] = o;
      if (cb.log && k == cb.last_k) cb.log[n] = o;
    }
    return;
  }
  if (k > 1 && !step_only) {
    const int m = sc[0].it;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc[0].done = k + 1 >= m;
      if (cb.log && k == cb.last_k) cb.log[n] = sc[0];
    }
    if (k >= m) return;
  }
  const Grid g = slice_grid(g0, cb.slice0 + n);
  const int64_t p = stencil_node_block(g0, blockIdx.x, nbx) * BLOCK + threadIdx.x;
  if (p >= g.N) return;
  const int64_t Np = g0.Np;
  const double *xk = (k & 1) ? cb.xt + (int64_t)n * Np : cb.x + n * cb.sx;
  double *xm = (k & 1) ? cb.x + n * cb.sx : cb.xt + (int64_t)n * Np;
  const double *b = cb.b + n * cb.sb;
  const double om = cheb_omega(t, k);
  const Ijk c = ijk(g, p);
  const double xc = xk[p];
  const double r = b[p] - (xc - cb.a * applyK<DIM, PN>(g, p, c, xc, [&](int64_t q) { return xk[q]; }));
  const double xo = xm[p];
  xm[p] = xo + om * (xc - xo + t.inv_theta * r);
}

hipError_t launch_cheb_iter(hipStream_t s, const Grid &g, const CgBatch &cb, int k) {
  if (cb.nslices <= 0) return hipSuccess;
  const int nbx = (int)(g.rag ? nblocks(g.N) : nblocks_xcd(g.N));
  dim3 grid(nbx + (k == 1 ? 1 : 0), cb.nslices);
  HSDC_DISPATCH_OP(g, hipLaunchKernelGGL((k_cheb_iter<DIM, PN>), grid, dim3(BLOCK), 0, s, g, cb,
                                         k, nbx, 0));
  return hipGetLastError();
}

hipError_t launch_cheb_steps(hipStream_t s, const Grid &g, const CgBatch &cb, int kmax) {
  if (cb.nslices <= 0) return hipSuccess;
  const int nbx = (int)(g.rag ? nblocks(g.N) : nblocks_xcd(g.N));
  dim3 grid(nbx, cb.nslices);
  for (int k = 1; k <= kmax; ++k)
    HSDC_DISPATCH_OP(g, hipLaunchKernelGGL((k_cheb_iter<DIM, PN>), grid, dim3(BLOCK), 0, s, g,
                                           cb, k, nbx, 1));
  return hipGetLastError();
}

// The CG start of degree D in one launch on 2D meshes: a block holds a 64 x 16
// tile of nodes with a halo of D + 1 in LDS and runs the Chebyshev steps x_2
// .. x_D there (x_k on the tile's radius D + 1 - k), then r_D = b - A x_D
// (radius 1) and w_D = A r_D (tile), from x_1 (xt), x_0 (x) and b, in the
// arithmetic of the Chebyshev and start kernels (a neighbour missing at the
// boundary reads the node itself, so its term is exactly 0; with per-node
// sigma the face coefficients come along in LDS and a missing face adds 0).
// x_{k+1} overwrites x_{k-1} cell by cell, so two LDS vectors and b suffice.
// x_0 comes from p (the node update stores it there) and x_D goes to x, so no
// tile overwrites what a neighbouring tile still reads.  Partials of (r_D,
// r_D) and (w_D, r_D) per tile, numbered within each tissue (tile t at (t %
// tiles_x, t / tiles_x) of the tissue's own tiles_x), so that a tissue of a
// ragged batch and its own context reduce the same partials in the same order;
// blocks past a smaller tissue's tiles write zeros.
int cg_start_tiles_of(int nx, int ny, int tile) {
  const TileShape &ts = kCgTiles[tile];
  return ((nx + ts.tx - 1) / ts.tx) * ((ny + ts.ty - 1) / ts.ty);
}

int cg_start_tiles(const Grid &g, int degree) {
  if (degree != 7 || g.dim != 2 || g.rag != nullptr) return 0;
  return cg_start_tiles_of(g.nx, g.ny, g.ctile);
}

template <int D, bool PN, int CTX, int CTY, int CT_THREADS>
__global__ void __launch_bounds__(CT_THREADS) k_cg_start_tiled(Grid g0, CgBatch cb) {
  constexpr int H = D + 1, W = CTX + 2 * H, HH = CTY + 2 * H;
  constexpr int WK = PN ? W : 1, HK = PN ? HH : 1;
  __shared__ double sa[HH][W], sk[HH][W], sb[HH][W];
  __shared__ double skx[HK][WK], sky[HK][WK];
  __shared__ double lds[2 * (CT_THREADS / 64)];
  const int n = blockIdx.y;
  const Grid g = slice_grid(g0, cb.slice0 + n);
  const int nx = g.nx, ny = g.ny;
  const int tiles_x = (nx + CTX - 1) / CTX;
  const int t = (int)blockIdx.x;
  double *part = cb.part + (int64_t)n * 5 * cb.pstride;
  if (t >= tiles_x * ((ny + CTY - 1) / CTY)) {
    // past this tissue's tiles (a smaller tissue of a ragged batch)
    if (threadIdx.x == 0) {
      part[2 * cb.pstride + t] = 0.0;
      part[3 * cb.pstride + t] = 0.0;
    }
    return;
  }
  const int X0 = (t % tiles_x) * CTX - H, Y0 = (t / tiles_x) * CTY - H;
  const double *x1g = cb.xt + (int64_t)n * g.Np;
  const double *x0g = cb.p + (int64_t)n * g.Np;  // x_0, stored there by the node update
  const double *bg = cb.b + n * cb.sb;
  const ChebTab &tb = cb.tab[(cb.slice0 + n) * cb.tab_stride];
  const double ith = tb.inv_theta, a = cb.a;
  // sa: x_{k-1}, sk: x_k (x_0 and x_1 to start with)
  double (*xm)[W] = sa, (*xk)[W] = sk;
  for (int q = threadIdx.x; q < W * HH; q += CT_THREADS) {
    const int u = q % W, v = q / W, gx = X0 + u, gy = Y0 + v;
    double v1 = 0.0, v0 = 0.0, vb = 0.0, fx = 0.0, fy = 0.0;
    if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
      const int64_t p = gx + (int64_t)nx * gy;
      v1 = x1g[p];
      v0 = x0g[p];
      vb = bg[p];
      if (PN) {
        fx = g.kx[p];
        fy = g.ky[p];
      }
    }
    sk[v][u] = v1;
    sa[v][u] = v0;
    sb[v][u] = vb;
    if (PN) {
      skx[v % HK][u % WK] = fx;
      sky[v % HK][u % WK] = fy;
    }
  }
  __syncthreads();
  // K S at cell (u, v), in applyK's order
  auto Kat = [&](double (*S)[W], int u, int v) {
    const int gx = X0 + u, gy = Y0 + v;
    const double c = S[v][u];
    if (PN) {
      double acc = 0.0;
      if (gx > 0) acc += skx[v % HK][(u - 1) % WK] * (S[v][u - 1] - c);
      if (gx < nx - 1) acc += skx[v % HK][u % WK] * (S[v][u + 1] - c);
      if (gy > 0) acc += sky[(v - 1) % HK][u % WK] * (S[v - 1][u] - c);
      if (gy < ny - 1) acc += sky[v % HK][u % WK] * (S[v + 1][u] - c);
      return acc;
    }
    const double l = gx > 0 ? S[v][u - 1] : c, r = gx < nx - 1 ? S[v][u + 1] : c;
    const double d = gy > 0 ? S[v - 1][u] : c, up = gy < ny - 1 ? S[v + 1][u] : c;
    double acc = g.cx * ((l - c) + (r - c));
    acc += g.cy * ((d - c) + (up - c));
    return acc;
  };
  auto inside = [&](int u, int v) {
    const int gx = X0 + u, gy = Y0 + v;
    return gx >= 0 && gx < nx && gy >= 0 && gy < ny;
  };
  // x_{k+1} = x_{k-1} + omega_{k+1} (x_k - x_{k-1} + (b - A x_k) / theta) on
  // radius D - k, written over x_{k-1}
#pragma unroll
  for (int k = 1; k < D; ++k) {
    const double om = cheb_omega(tb, k);
    const int m = k, w = W - 2 * m, h = HH - 2 * m;
    for (int q = threadIdx.x; q < w * h; q += CT_THREADS) {
      const int u = m + q % w, v = m + q / w;
      if (!inside(u, v)) continue;
      const double xc = xk[v][u], xo = xm[v][u];
      const double r = sb[v][u] - (xc - a * Kat(xk, u, v));
      xm[v][u] = xo + om * (xc - xo + ith * r);
    }
    __syncthreads();
    double (*tmp)[W] = xm;
    xm = xk;
    xk = tmp;
  }
  // r_D = b - A x_D on radius 1, over x_{D-1}
  {
    const int m = D, w = W - 2 * m, h = HH - 2 * m;
    for (int q = threadIdx.x; q < w * h; q += CT_THREADS) {
      const int u = m + q % w, v = m + q / w;
      if (!inside(u, v)) continue;
      const double xq = xk[v][u];
      xm[v][u] = sb[v][u] - (xq - a * Kat(xk, u, v));
    }
  }
  __syncthreads();
  // w_D = A r_D on the tile; x_D to x, r_D and w_D to the parity-1 vectors
  double gam = 0.0, del = 0.0;
  for (int q = threadIdx.x; q < CTX * CTY; q += CT_THREADS) {
    const int u = H + q % CTX, v = H + q / CTX;
    if (!inside(u, v)) continue;
    const double rc = xm[v][u];
    const double wv = rc - a * Kat(xm, u, v);
    const int64_t p = (X0 + u) + (int64_t)nx * (Y0 + v);
    cb.x[n * cb.sx + p] = xk[v][u];
    cb.r[1][n * g.Np + p] = rc;
    cb.w[1][n * g.Np + p] = wv;
    gam += rc * rc;
    del += wv * rc;
  }
  double t2[2] = {gam, del};
  block_sums<2, CT_THREADS>(t2, lds);
  if (threadIdx.x == 0) {
    part[2 * cb.pstride + t] = t2[0];
    part[3 * cb.pstride + t] = t2[1];
    if (blockIdx.x == 0) {
      CgScalars o;
      o.bb = -1.0;  // reduced by the first iteration kernel
      o.gamma = 1.0;
      o.alpha = 1.0;
      o.it = 0;
      o.done = 0;
      cb.sc[2 * n + 1] = o;
    }
  }
}

// The same CG start with the iterates in registers.  A block covers 64
// columns of the mesh (one per lane) by NW RW rows (RW consecutive rows per
// wave); its tile is the interior 48 x (NW RW - 2 H), H = D + 1 cells in from
// every edge.  A lane takes its left and right neighbours from the adjacent
// lanes (DPP shifts across the wave), the rows above and below from its own
// registers, and only the first and last row of each wave go through LDS
// (two buffers by step parity, one barrier a step, the rows inside a strip
// updated while the waves meet there).  Every cell of the block
// is updated in every step: after s applications of K a cell closer than s
// to the block's edge holds a wrong value (a neighbour beyond the block reads
// zero or the cell itself), which never reaches the tile, H applications
// away.  Cells outside the mesh hold zeros and are read by none inside (a
// boundary node reads itself for its missing neighbour, as in the LDS-tiled
// kernel, whose arithmetic this one repeats expression by expression).

// The value of lane - 1 (lane 0: 0) and of lane + 1 (lane 63: 0).
__device__ __forceinline__ double lane_from_left(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_from_right(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

template <int D, bool PN, int RW, int NW>
__global__ void __launch_bounds__(64 * NW) k_cg_start_strip(Grid g0, CgBatch cb) {
  constexpr int H = D + 1, TX = 64 - 2 * H, TY = NW * RW - 2 * H;
  static_assert(TX > 0 && TY > 0, "the block must hold the tile and its halo");
  static_assert(RW >= 2, "a strip's first and last row are distinct");
  __shared__ double s_first[2][NW][64], s_last[2][NW][64];
  __shared__ double lds[2 * NW];
  const int n = blockIdx.y;
  const Grid g = slice_grid(g0, cb.slice0 + n);
  const int nx = g.nx, ny = g.ny;
  const int tiles_x = (nx + TX - 1) / TX;
  const int t = (int)blockIdx.x;
  double *part = cb.part + (int64_t)n * 5 * cb.pstride;
  if (t >= tiles_x * ((ny + TY - 1) / TY)) {
    // past this tissue's tiles (a smaller tissue of a ragged batch)
    if (threadIdx.x == 0) {
      part[2 * cb.pstride + t] = 0.0;
      part[3 * cb.pstride + t] = 0.0;
    }
    return;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // the block's first column and row on the mesh, and this lane's
  const int X0 = (t % tiles_x) * TX - H, Y0 = (t / tiles_x) * TY - H;
  const int gx = X0 + lane, gy0 = Y0 + w * RW;
  const bool colin = gx >= 0 && gx < nx;
  const double *x1g = cb.xt + (int64_t)n * g.Np;
  const double *x0g = cb.p + (int64_t)n * g.Np;  // x_0, stored there by the node update
  const double *bg = cb.b + n * cb.sb;
  const ChebTab &tb = cb.tab[(cb.slice0 + n) * cb.tab_stride];
  const double ith = tb.inv_theta, a = cb.a;
  // xm: x_{k-1}, xk: x_k (x_0 and x_1 to start with); kl, kr, kd, ku: the
  // face coefficients left, right, below and above (per-node sigma)
  double xm[RW], xk[RW], bv[RW];
  double kl[PN ? RW : 1], kr[PN ? RW : 1], kd[PN ? RW : 1], ku[PN ? RW : 1];
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    const int gy = gy0 + j;
    const bool in = colin && gy >= 0 && gy < ny;
    const int64_t p = gx + (int64_t)nx * gy;
    xk[j] = in ? x1g[p] : 0.0;
    xm[j] = in ? x0g[p] : 0.0;
    bv[j] = in ? bg[p] : 0.0;
    if (PN) {
      kr[j] = in ? g.kx[p] : 0.0;
      kl[j] = in && gx > 0 ? g.kx[p - 1] : 0.0;
      ku[j] = in ? g.ky[p] : 0.0;
      kd[j] = in && gy > 0 ? g.ky[p - nx] : 0.0;
    }
  }
  // Blocks with no cell on the mesh's boundary take every neighbour as it
  // is; the others select the cell itself for a missing one.
  const bool edge = !(X0 > 0 && X0 + 63 < nx - 1 && Y0 > 0 && Y0 + NW * RW - 1 < ny - 1);
  const bool hl = gx > 0, hr = gx < nx - 1;
  double gam = 0.0, del = 0.0;
  auto body = [&](auto edge_c) {
    constexpr bool E = decltype(edge_c)::value;
    // K at row j from the cell c and its neighbours, in the LDS-tiled kernel's order
    auto Kat = [&](int j, double c, double l, double r, double d, double up) {
      const int gy = gy0 + j;
      const bool hd = !E || gy > 0, hu = !E || gy < ny - 1;
      const bool el = !E || hl, er = !E || hr;
      if (PN) {
        double acc = 0.0;
        if (el) acc += kl[PN ? j : 0] * (l - c);
        if (er) acc += kr[PN ? j : 0] * (r - c);
        if (hd) acc += kd[PN ? j : 0] * (d - c);
        if (hu) acc += ku[PN ? j : 0] * (up - c);
        return acc;
      }
      l = el ? l : c;
      r = er ? r : c;
      d = hd ? d : c;
      up = hu ? up : c;
      double acc = g.cx * ((l - c) + (r - c));
      acc += g.cy * ((d - c) + (up - c));
      return acc;
    };
    // One application of K over the block: the wave publishes its strip's
    // first and last row, updates the rows inside the strip (their
    // neighbours above and below are its own) while the other waves catch
    // up, then takes the previous wave's last row and the next wave's first
    // (the block's edge rows take the strip's own) and updates its first and
    // last row.  row(j, below, above) updates row j.
    auto phase = [&](const double (&x)[RW], int k, auto &&row) {
      s_first[k & 1][w][lane] = x[0];
      s_last[k & 1][w][lane] = x[RW - 1];
#pragma unroll
      for (int j = 1; j < RW - 1; ++j) row(j, x[j - 1], x[j + 1]);
      __syncthreads();
      const double below = w > 0 ? s_last[k & 1][w - 1][lane] : x[0];
      const double above = w < NW - 1 ? s_first[k & 1][w + 1][lane] : x[RW - 1];
      row(0, below, x[1]);
      row(RW - 1, x[RW - 2], above);
    };
    // x_{k+1} = x_{k-1} + omega_{k+1} (x_k - x_{k-1} + (b - A x_k) / theta)
#pragma unroll
    for (int k = 1; k < D; ++k) {
      const double om = cheb_omega(tb, k);
      phase(xk, k, [&](int j, double d, double up) {
        const double xc = xk[j], xo = xm[j];
        const double l = lane_from_left(xc), r = lane_from_right(xc);
        const double rr = bv[j] - (xc - a * Kat(j, xc, l, r, d, up));
        xm[j] = xo + om * (xc - xo + ith * rr);
      });
#pragma unroll
      for (int j = 0; j < RW; ++j) {
        const double tmp = xm[j];
        xm[j] = xk[j];
        xk[j] = tmp;
      }
    }
    // r_D = b - A x_D, over x_{D-1}
    phase(xk, D, [&](int j, double d, double up) {
      const double xq = xk[j];
      const double l = lane_from_left(xq), r = lane_from_right(xq);
      xm[j] = bv[j] - (xq - a * Kat(j, xq, l, r, d, up));
    });
    // w_D = A r_D on the tile; x_D to x, r_D and w_D to the parity-1 vectors
    const bool tcol = lane >= H && lane < H + TX && colin;
    phase(xm, D + 1, [&](int j, double d, double up) {
      const double rc = xm[j];
      const double l = lane_from_left(rc), r = lane_from_right(rc);
      const double wv = rc - a * Kat(j, rc, l, r, d, up);
      const int v = w * RW + j, gy = gy0 + j;
      if (tcol && v >= H && v < H + TY && gy < ny) {
        const int64_t p = gx + (int64_t)nx * gy;
        cb.x[n * cb.sx + p] = xk[j];
        cb.r[1][n * g.Np + p] = rc;
        cb.w[1][n * g.Np + p] = wv;
        gam += rc * rc;
        del += wv * rc;
      }
    });
  };
  if (edge)
    body(std::true_type{});
  else
    body(std::false_type{});
  double t2[2] = {gam, del};
  block_sums<2, 64 * NW>(t2, lds);
  if (threadIdx.x == 0) {
    part[2 * cb.pstride + t] = t2[0];
    part[3 * cb.pstride + t] = t2[1];
    if (blockIdx.x == 0) {
      CgScalars o;
      o.bb = -1.0;  // reduced by the first iteration kernel
      o.gamma = 1.0;
      o.alpha = 1.0;
      o.it = 0;
      o.done = 0;
      cb.sc[2 * n + 1] = o;
    }
  }
}

hipError_t launch_cg_start_tiled(hipStream_t s, const Grid &g, const CgBatch &cb, int ntiles) {
  if (ntiles <= 0 || cb.nslices <= 0 || g.dim != 2 || cb.cstart != 7) return hipErrorInvalidValue;
  const dim3 grid(ntiles, cb.nslices);
  const bool pn = g.kx != nullptr;
#define HSDC_CT_LAUNCH(X_, Y_, NT_)                                                            \
  do {                                                                                        \
    if (pn)                                                                                   \
      hipLaunchKernelGGL((k_cg_start_tiled<7, true, X_, Y_, NT_>), grid, dim3(NT_), 0, s, g, cb); \
    else                                                                                      \
      hipLaunchKernelGGL((k_cg_start_tiled<7, false, X_, Y_, NT_>), grid, dim3(NT_), 0, s, g,   \
                         cb);                                                                 \
  } while (0)
#define HSDC_CS_LAUNCH(RW_, NW_)                                                               \
  do {                                                                                        \
    if (pn)                                                                                   \
      hipLaunchKernelGGL((k_cg_start_strip<7, true, RW_, NW_>), grid, dim3(64 * NW_), 0, s, g, cb); \
    else                                                                                      \
      hipLaunchKernelGGL((k_cg_start_strip<7, false, RW_, NW_>), grid, dim3(64 * NW_), 0, s, g,   \
                         cb);                                                                 \
  } while (0)
  static_assert(kNumCgTiles == 9, "one launch per tile of kCgTiles");
  switch (g.ctile) {
    case 0: HSDC_CT_LAUNCH(64, 16, 1024); break;
    case 1: HSDC_CT_LAUNCH(32, 32, 1024); break;
    case 2: HSDC_CT_LAUNCH(32, 16, 512); break;
    case 3: HSDC_CT_LAUNCH(32, 8, 256); break;
    case 4: HSDC_CT_LAUNCH(16, 16, 256); break;
    case 5: HSDC_CS_LAUNCH(4, 8); break;  // 48 x 16 nodes, 512 threads
    case 6: HSDC_CS_LAUNCH(3, 8); break;  // 48 x 8
    case 7: HSDC_CS_LAUNCH(5, 8); break;  // 48 x 24
    case 8: HSDC_CS_LAUNCH(6, 8); break;  // 48 x 32
    default: return hipErrorInvalidValue;
  }
#undef HSDC_CS_LAUNCH
#undef HSDC_CT_LAUNCH
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// transfers between levels: time (R, T) composed with space (average of the
// 2^d children / cell-centred multilinear interpolation), or time only.
// ---------------------------------------------------------------------------

// Mean of val(q) over the fine children q of coarse node pc (2 per coarsened
// axis, or pc itself without space coarsening); indices are formed in
// registers with the child loops unrolled.
template <class Val>
__device__ __forceinline__ double child_mean(const Grid &gf, const Grid &gc, int64_t pc, int scf,
                                             Val &&val) {
  if (scf == 1) return val(pc);
  const Ijk c = ijk(gc, pc);
  const int ax = gf.nx > 1 ? 2 : 1, ay = gf.ny > 1 ? 2 : 1, az = gf.nz > 1 ? 2 : 1;
  const int64_t sy = gf.nx, sz = (int64_t)gf.nx * gf.ny;
  const int64_t base = (int64_t)c.ix * ax + sy * ((int64_t)c.iy * ay) + sz * ((int64_t)c.iz * az);
  double s = 0.0;
#pragma unroll
  for (int c2 = 0; c2 < 2; ++c2) {
    if (c2 < az) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (b < ay) {
#pragma unroll
          for (int a = 0; a < 2; ++a)
            if (a < ax) s += val(base + a + sy * b + sz * c2);
        }
      }
    }
  }
  return s * (1.0 / (ax * ay * az));
}

// One thread per (node, field): the field is the grid's y index.  Stage loops
// run to the compile-time maximum with predication, so the per-node stage
// values stay in registers.
__global__ void __launch_bounds__(BLOCK)
k_restrict_stages(Grid gf, Grid gc, int scf, const double *Yf, int64_t sYf, int Mf,
                  const double *Rt, int Mc, double *Yc, int64_t sYc, double *Yc2) {
  const int64_t pc = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (pc >= gc.N) return;
  const int n = blockIdx.z;
  const int f = blockIdx.y;
  {
    double av[MAXM + 1];
#pragma unroll
    for (int l = 0; l <= MAXM; ++l) {
      const double *y = Yf + n * sYf + ((int64_t)l * NF + f) * gf.Np;
      av[l] = (l <= Mf) ? child_mean(gf, gc, pc, scf, [&](int64_t q) { return y[q]; }) : 0.0;
    }
#pragma unroll
    for (int i = 0; i <= MAXM; ++i) {
      if (i <= Mc) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l <= MAXM; ++l)
          if (l <= Mf) s += Rt[i * (Mf + 1) + l] * av[l];
        const int64_t o = n * sYc + ((int64_t)i * NF + f) * gc.Np + pc;
        Yc[o] = s;
        if (Yc2) Yc2[o] = s;
      }
    }
  }
}

hipError_t launch_restrict_stages(hipStream_t s, const Grid &gf, const Grid &gc, int sc_factor,
                                  const double *Yf, int64_t sYf, int Mf, const double *Rt,
                                  int Mc, double *Yc, int64_t sYc, double *Yc_copy, int nslices) {
  dim3 grid(nblocks(gc.N), NF, nslices);
  hipLaunchKernelGGL(k_restrict_stages, grid, dim3(BLOCK), 0, s, gf, gc, sc_factor, Yf, sYf,
                     Mf, Rt, Mc, Yc, sYc, Yc_copy);
  return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK)
k_restrict_fields(Grid gf, Grid gc, int scf, const double *src, int64_t ssrc, double *dst,
                  int64_t sdst, int nrows) {
  const int64_t pc = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (pc >= gc.N) return;
  const int n = blockIdx.z;
  const int r = blockIdx.y;  // one row per grid row
  const double *x = src + n * ssrc + (int64_t)r * gf.Np;
  dst[n * sdst + (int64_t)r * gc.Np + pc] = child_mean(gf, gc, pc, scf, [&](int64_t q) { return x[q]; });
}

hipError_t launch_restrict_fields(hipStream_t s, const Grid &gf, const Grid &gc, int sc_factor,
                                  const double *src, int64_t ssrc, double *dst, int64_t sdst,
                                  int nrows, int nslices) {
  if (nrows <= 0 || nslices <= 0) return hipSuccess;
  dim3 grid(nblocks(gc.N), nrows, nslices);
  hipLaunchKernelGGL(k_restrict_fields, grid, dim3(BLOCK), 0, s, gf, gc, sc_factor, src,
                     ssrc, dst, sdst, nrows);
  return hipGetLastError();
}

// y_f += T P(z_c - S z) at fine stages i0..Mf: the coarse difference Dc is read
// at the (up to 8) coarse cells that interpolate onto fine node p.  Per axis
// the two cells and weights are kept in registers and the 2 x 2 x 2 taps are
// unrolled (an axis of one node has weight 0 on its second cell and is
// skipped).  Fine node blocks sharing coarse cells run on one XCD
// (xcd_node_block).
__global__ void __launch_bounds__(BLOCK)
k_prolong_correct(Grid gf, Grid gc, int scf, const double *Dc, int64_t sYc, int Mc,
                  const double *Tt, int Mf, int i0, double *Yf, int64_t sYf) {
  const int64_t p = xcd_node_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (p >= gf.N) return;
  const int n = blockIdx.z;
  const int f = blockIdx.y;
  int64_t ax0[3], ax1[3];  // coarse index offsets per axis (cell I and neighbour J)
  double w0[3], w1[3];
  if (scf == 1) {
    ax0[0] = p;
    ax1[0] = p;
    w0[0] = 1.0;
    w1[0] = 0.0;
    ax0[1] = ax1[1] = ax0[2] = ax1[2] = 0;
    w0[1] = w0[2] = 1.0;
    w1[1] = w1[2] = 0.0;
  } else {
    const Ijk c = ijk(gf, p);
    const int fi[3] = {c.ix, c.iy, c.iz};
    const int nf_[3] = {gf.nx, gf.ny, gf.nz};
    const int nc_[3] = {gc.nx, gc.ny, gc.nz};
    const int64_t st[3] = {1, gc.nx, (int64_t)gc.nx * gc.ny};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (nf_[a] > 1) {
        const int I = fi[a] >> 1;
        int J = (fi[a] & 1) ? I + 1 : I - 1;
        J = J < 0 ? 0 : (J > nc_[a] - 1 ? nc_[a] - 1 : J);
        ax0[a] = I * st[a];
        ax1[a] = J * st[a];
        w0[a] = 0.75;
        w1[a] = 0.25;
      } else {
        ax0[a] = ax1[a] = 0;
        w0[a] = 1.0;
        w1[a] = 0.0;
      }
    }
  }
  // the fine values first: every load of the thread is issued before its first
  // store (a store would order the later loads behind it)
  double yv[MAXM + 1];
  double *yf0 = Yf + n * sYf + (int64_t)f * gf.Np + p;
#pragma unroll
  for (int i = 0; i <= MAXM; ++i)
    yv[i] = (i >= i0 && i <= Mf) ? yf0[(int64_t)i * NF * gf.Np] : 0.0;
  double dc[MAXM + 1];
#pragma unroll
  for (int j = 0; j <= MAXM; ++j) {
    double s = 0.0;
    if (j <= Mc) {
      const double *dc_ = Dc + n * sYc + ((int64_t)j * NF + f) * gc.Np;
#pragma unroll
      for (int cz = 0; cz < 2; ++cz) {
        const double wz = cz ? w1[2] : w0[2];
        if (wz == 0.0) continue;
        const int64_t oz = cz ? ax1[2] : ax0[2];
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
          const double wy = cy ? w1[1] : w0[1];
          if (wy == 0.0) continue;
          const int64_t oy = oz + (cy ? ax1[1] : ax0[1]);
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) {
            const double wx = cx ? w1[0] : w0[0];
            if (wx == 0.0) continue;
            const int64_t q = oy + (cx ? ax1[0] : ax0[0]);
            s += (wx * wy * wz) * dc_[q];
          }
        }
      }
    }
    dc[j] = s;
  }
#pragma unroll
  for (int i = 0; i <= MAXM; ++i) {
    if (i >= i0 && i <= Mf) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j <= MAXM; ++j)
        if (j <= Mc) s += Tt[i * (Mc + 1) + j] * dc[j];
      // streaming store: the fine stages are read next by a later kernel
      stream_store<double>(yf0 + (int64_t)i * NF * gf.Np, yv[i] + s);
    }
  }
}

// d = y - d over n values (the coarse correction z_c - S z, formed once per
// coarse value rather than at each of the 2^d fine taps that read it)
__global__ void __launch_bounds__(BLOCK) k_sub_from(double *d, const double *y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) d[i] = y[i] - d[i];
}

// The same correction for a mesh coarsened 2x, by tiles: a block takes a tile
// of TX x TY x TZ fine nodes of one field and slice, stages the coarse values
// its taps read (the tile's coarse cells and one more on each side, clamped at
// the mesh edge as the taps are) in LDS, and forms each fine node's taps from
// there, in the order and arithmetic of k_prolong_correct.  Every coarse value
// is read from memory about once per tile instead of once per tap.  An axis
// of the mesh with more than one node needs a tile extent above one.
template <int TX, int TY, int TZ>
__global__ void __launch_bounds__(TX * TY * TZ)
k_prolong_tiled(Grid gf, Grid gc, const double *Dc, int64_t sYc, int Mc, const double *Tt, int Mf,
                int i0, double *Yf, int64_t sYf) {
  constexpr int CW = TX > 1 ? TX / 2 + 2 : 1, CH = TY > 1 ? TY / 2 + 2 : 1,
                CD = TZ > 1 ? TZ / 2 + 2 : 1;
  __shared__ double lc[MAXM + 1][CD][CH][CW];
  const int n = blockIdx.z;
  const int f = blockIdx.y;
  const int ntx = (gf.nx + TX - 1) / TX, nty = (gf.ny + TY - 1) / TY;
  // tiles in XCD order: neighbouring tiles, which stage overlapping coarse
  // blocks, run on one XCD and find each other's coarse values in its L2
  const int t = gridDim.x % kXcds == 0 ? (int)xcd_node_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const int fx0 = (t % ntx) * TX, fy0 = ((t / ntx) % nty) * TY, fz0 = (t / (ntx * nty)) * TZ;
  // coarse origin of the staged block (one cell before the tile's first)
  const int cx0 = TX > 1 ? (fx0 >> 1) - 1 : 0, cy0 = TY > 1 ? (fy0 >> 1) - 1 : 0,
            cz0 = TZ > 1 ? (fz0 >> 1) - 1 : 0;
  const int tid = threadIdx.x;
  const int fx = fx0 + tid % TX, fy = fy0 + (tid / TX) % TY, fz = fz0 + tid / (TX * TY);
  const bool in = fx < gf.nx && fy < gf.ny && fz < gf.nz;
  const int64_t p = fx + (int64_t)gf.nx * (fy + (int64_t)gf.ny * fz);
  // the fine values first, in flight while the coarse block is staged
  double yv[MAXM + 1];
  double *yf0 = Yf + n * sYf + (int64_t)f * gf.Np + p;
#pragma unroll
  for (int i = 0; i <= MAXM; ++i)
    yv[i] = (in && i >= i0 && i <= Mf) ? yf0[(int64_t)i * NF * gf.Np] : 0.0;
  const int per = CD * CH * CW;
  for (int q = tid; q < (Mc + 1) * per; q += TX * TY * TZ) {
    const int j = q / per, r = q % per;
    const int a = r % CW, b = (r / CW) % CH, c = r / (CW * CH);
    const int gx = min(max(cx0 + a, 0), gc.nx - 1), gy = min(max(cy0 + b, 0), gc.ny - 1),
              gz = min(max(cz0 + c, 0), gc.nz - 1);
    lc[j][c][b][a] = Dc[n * sYc + ((int64_t)j * NF + f) * gc.Np + gx +
                        (int64_t)gc.nx * (gy + (int64_t)gc.ny * gz)];
  }
  __syncthreads();
  if (!in) return;
  // per axis: the cell I and its neighbour J (clamped), as block-local indices
  int aI[3], aJ[3];
  double w0[3], w1[3];
  {
    const int fi[3] = {fx, fy, fz}, nf_[3] = {gf.nx, gf.ny, gf.nz}, nc_[3] = {gc.nx, gc.ny, gc.nz};
    const int c0[3] = {cx0, cy0, cz0};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      if (nf_[ax] > 1) {
        const int I = fi[ax] >> 1;
        int J = (fi[ax] & 1) ? I + 1 : I - 1;
        J = J < 0 ? 0 : (J > nc_[ax] - 1 ? nc_[ax] - 1 : J);
        aI[ax] = I - c0[ax];
        aJ[ax] = J - c0[ax];
        w0[ax] = 0.75;
        w1[ax] = 0.25;
      } else {
        aI[ax] = aJ[ax] = 0;
        w0[ax] = 1.0;
        w1[ax] = 0.0;
      }
    }
  }
  double dc[MAXM + 1];
#pragma unroll
  for (int j = 0; j <= MAXM; ++j) {
    double sum = 0.0;
    if (j <= Mc) {
#pragma unroll
      for (int cz = 0; cz < 2; ++cz) {
        const double wz = cz ? w1[2] : w0[2];
        if (wz == 0.0) continue;
        const int oz = cz ? aJ[2] : aI[2];
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
          const double wy = cy ? w1[1] : w0[1];
          if (wy == 0.0) continue;
          const int oy = cy ? aJ[1] : aI[1];
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) {
            const double wx = cx ? w1[0] : w0[0];
            if (wx == 0.0) continue;
            sum += (wx * wy * wz) * lc[j][oz][oy][cx ? aJ[0] : aI[0]];
          }
        }
      }
    }
    dc[j] = sum;
  }
#pragma unroll
  for (int i = 0; i <= MAXM; ++i) {
    if (i >= i0 && i <= Mf) {
      double sum = 0.0;
#pragma unroll
      for (int j = 0; j <= MAXM; ++j)
        if (j <= Mc) sum += Tt[i * (Mc + 1) + j] * dc[j];
      stream_store<double>(yf0 + (int64_t)i * NF * gf.Np, yv[i] + sum);
    }
  }
}

hipError_t launch_prolong_correct(hipStream_t s, const Grid &gf, const Grid &gc, int sc_factor,
                                  const double *Yc, double *Sz, int64_t sYc, int Mc,
                                  const double *Tt, int Mf, int i0, double *Yf, int64_t sYf,
                                  int nslices) {
  const int64_t nc = (int64_t)nslices * sYc;
  hipLaunchKernelGGL(k_sub_from, dim3(nblocks(nc)), dim3(BLOCK), 0, s, Sz, Yc, nc);
  if (sc_factor == 2 && gf.rag == nullptr) {
    // tiles of 256 fine nodes (kProlongTiles3D / 2D[gf.ptile]); every active
    // axis of a tile spans an even number of nodes (two per coarse cell)
#define HSDC_PT_LAUNCH(X_, Y_, Z_)                                                              \
  do {                                                                                         \
    const unsigned nt = ((gf.nx + X_ - 1) / X_) * ((gf.ny + Y_ - 1) / Y_) * ((gf.nz + Z_ - 1) / Z_); \
    hipLaunchKernelGGL((k_prolong_tiled<X_, Y_, Z_>), dim3(nt, NF, nslices), dim3(256), 0, s, gf, \
                       gc, Sz, sYc, Mc, Tt, Mf, i0, Yf, sYf);                                  \
  } while (0)
    static_assert(kNumProlongTiles == 4, "one launch per tile of kProlongTiles2D / 3D");
    if (gf.nz > 1) {
      switch (gf.ptile) {
        case 0: HSDC_PT_LAUNCH(32, 4, 2); break;
        case 1: HSDC_PT_LAUNCH(64, 2, 2); break;
        case 2: HSDC_PT_LAUNCH(16, 8, 2); break;
        case 3: HSDC_PT_LAUNCH(16, 4, 4); break;
        default: return hipErrorInvalidValue;
      }
    } else if (gf.ny > 1) {
      switch (gf.ptile) {
        case 0: HSDC_PT_LAUNCH(32, 8, 1); break;
        case 1: HSDC_PT_LAUNCH(64, 4, 1); break;
        case 2: HSDC_PT_LAUNCH(16, 16, 1); break;
        case 3: HSDC_PT_LAUNCH(128, 2, 1); break;
        default: return hipErrorInvalidValue;
      }
#undef HSDC_PT_LAUNCH
    } else {
      const unsigned nt = (gf.nx + 255) / 256;
      hipLaunchKernelGGL((k_prolong_tiled<256, 1, 1>), dim3(nt, NF, nslices), dim3(256), 0, s, gf,
                         gc, Sz, sYc, Mc, Tt, Mf, i0, Yf, sYf);
    }
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_prolong_correct, dim3(nblocks_xcd(gf.N), NF, nslices), dim3(BLOCK), 0, s,
                     gf, gc, sc_factor, Sz, sYc, Mc, Tt, Mf, i0, Yf, sYf);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exported building blocks
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(BLOCK)
k_ionic_test(int64_t n, const double *y, double gs0, double gs1, double gs2, double *I_ion,
             double *ha, double *lam, double *winf) {
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (p >= n) return;
  double yv[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) yv[f] = y[f * n + p];
  ttp06::gates(yv[0], yv[3], [&](int k, double inf, double rate) {
    lam[k * n + p] = -rate;
    winf[k * n + p] = inf;
  });
  double I, h[6];
  ttp06::currents(yv, gs0, gs1, gs2, I, h);
  I_ion[p] = I;
#pragma unroll
  for (int k = 0; k < 6; ++k) ha[k * n + p] = h[k];
}

hipError_t launch_ionic_test(hipStream_t s, int64_t n, const double *y, double gs0, double gs1,
                             double gs2, double *I_ion, double *ha, double *lam, double *winf) {
  hipLaunchKernelGGL(k_ionic_test, dim3(nblocks(n)), dim3(BLOCK), 0, s, n, y, gs0, gs1, gs2, I_ion,
                     ha, lam, winf);
  return hipGetLastError();
}

template <int K>
__global__ void __launch_bounds__(BLOCK) k_phi_test(int64_t n, const double *x, double *out) {
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (p >= n) return;
  double invf[MAXM + 10];
  invf[0] = 1.0;
  for (int k = 1; k < MAXM + 10; ++k) invf[k] = invf[k - 1] / (double)k;
  double ph[K];
  phis<K>(x[p], invf, ph);
#pragma unroll
  for (int k = 0; k < K; ++k) out[k * n + p] = ph[k];
}

hipError_t launch_phi_test(hipStream_t s, int64_t n, const double *x, int kmax, double *out) {
  HSDC_DISPATCH_M(kmax, hipLaunchKernelGGL((k_phi_test<M>), dim3(nblocks(n)), dim3(BLOCK), 0, s, n,
                                           x, out));
  return hipGetLastError();
}

// a_ij(z) through colloc_integrals applied to the unit vectors e_j.
template <int M>
__global__ void __launch_bounds__(BLOCK)
k_aij_test(int64_t n, const double *z, Colloc co, double *out) {
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (p >= n) return;
  for (int j = 0; j < M; ++j) {
    double e[M], I[M];
#pragma unroll
    for (int k = 0; k < M; ++k) e[k] = (k == j) ? 1.0 : 0.0;
    colloc_integrals<M>(co, z[p], e, I);
    for (int i = 0; i < M; ++i) out[(p * M + i) * M + j] = I[i];
  }
}

hipError_t launch_aij_test(hipStream_t s, int64_t n, const double *z, const Colloc &co,
                           double *out) {
  HSDC_DISPATCH_M(co.M, hipLaunchKernelGGL((k_aij_test<M>), dim3(nblocks(n)), dim3(BLOCK), 0, s, n,
                                           z, co, out));
  return hipGetLastError();
}

// Face coefficients of a per-node conductivity field: the face p -> p + e_axis
// takes the harmonic mean of the two node values times sc = 1/(dx^2 chi Cm),
// 0 on the last layer of the axis (the same expression as the host's).
__global__ void __launch_bounds__(BLOCK)
k_faces(Grid g, const double *sig, double sc, double *kx, double *ky, double *kz) {
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (p >= g.N) return;
  const Ijk c = ijk(g, p);
  const double sp = sig[p];
  auto face = [&](bool last, int64_t q) {
    if (last) return 0.0;
    const double sq = sig[q];
    return (sp + sq > 0) ? 2.0 * sp * sq / (sp + sq) * sc : 0.0;
  };
  kx[p] = face(c.ix == g.nx - 1, p + 1);
  if (g.dim >= 2) ky[p] = face(c.iy == g.ny - 1, p + g.nx);
  if (g.dim >= 3) kz[p] = face(c.iz == g.nz - 1, p + (int64_t)g.nx * g.ny);
}

hipError_t launch_faces(hipStream_t s, const Grid &g, const double *sigma_node, double sc,
                        double *kx, double *ky, double *kz) {
  hipLaunchKernelGGL(k_faces, dim3(nblocks(g.N)), dim3(BLOCK), 0, s, g, sigma_node, sc, kx, ky, kz);
  return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK) k_fill_rest(int64_t N, int64_t Np, double *y) {
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (p >= N) return;
#pragma unroll
  for (int f = 0; f < NF; ++f) y[f * Np + p] = ttp06::kRest[f];
}

hipError_t launch_fill_rest(hipStream_t s, int64_t N, int64_t Np, double *y) {
  hipLaunchKernelGGL(k_fill_rest, dim3(nblocks(N)), dim3(BLOCK), 0, s, N, Np, y);
  return hipGetLastError();
}

// The device step counter read by the time-dependent kernels (a captured
// step advances it inside the graph).
__global__ void k_step_set(int64_t *step, int64_t value, int64_t add) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *step = (add != 0) ? *step + add : value;
}

hipError_t launch_step_set(hipStream_t s, int64_t *step, int64_t value) {
  hipLaunchKernelGGL(k_step_set, dim3(1), dim3(64), 0, s, step, value, (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_step_add(hipStream_t s, int64_t *step, int64_t add) {
  hipLaunchKernelGGL(k_step_set, dim3(1), dim3(64), 0, s, step, (int64_t)0, add);
  return hipGetLastError();
}

// ---- instantiations for the two storage types -------------------------------
#define HSDC_INSTANTIATE(T)                                                                   \
  template hipError_t launch_eval_stages<T>(hipStream_t, const Grid &, const StagesT<T> &,    \
                                            const Colloc &, const Stim &, double, double,    \
                                            double, int, int, int, int, T *, const T *);     \
  template hipError_t launch_spmv_stages<T>(hipStream_t, const Grid &, const StagesT<T> &,    \
                                            int, int, int, int);                             \
  template hipError_t launch_assemble<T>(hipStream_t, const Grid &, const StagesT<T> &,       \
                                         const Colloc &, int, int, const double *, int64_t,  \
                                         int, const Stim &);                                 \
  template hipError_t launch_fas_integrals<T>(hipStream_t, const Grid &, const StagesT<T> &,  \
                                              const Colloc &, int, int, double *, int64_t);  \
  template hipError_t launch_node_update<T>(hipStream_t, const Grid &, const StagesT<T> &,    \
                                            const Colloc &, const Stim &, double, double,    \
                                            double, int, int, int, const CgBatchT<T> &, int, \
                                            int, const double *, const CgLogArgs &);         \
  template hipError_t launch_cg_init<T>(hipStream_t, const Grid &, const CgBatchT<T> &);      \
  template hipError_t launch_cg_resid0<T>(hipStream_t, const Grid &, const CgBatchT<T> &);    \
  template hipError_t launch_cg_iter<T>(hipStream_t, const Grid &, const CgBatchT<T> &, int);
HSDC_INSTANTIATE(double)
HSDC_INSTANTIATE(float)
#undef HSDC_INSTANTIATE
}  // namespace hsdc
