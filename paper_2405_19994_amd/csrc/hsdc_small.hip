// hsdc_small.hip -- serial hybrid SDC steps of a 1D mesh that fits one
// workgroup (at most 256 nodes), all steps of an advance in one launch.
//
// On such a mesh every kernel of a step is a few microseconds of launch
// latency around a few hundred nanoseconds of work (a step of the 128-node
// cable is about a hundred launches).  Here one workgroup runs the whole
// step sequence: thread p owns node p and keeps its stage vectors and
// reaction terms in the level's arrays (a mesh of at most 128 nodes gives the
// gate rows of each node to a second thread), the right-hand sides of the
// (field, node) pairs are shared among all 256 threads, and the nodes meet
// in the stencil products and the diffusion solves, which go through LDS.  The arithmetic is that of the
// per-phase kernels (hsdc_kernels.hip): the same sweep (eq. prec_picard with
// the preconditioner of eq. def_P, the integrals of eq. def_C), except that
// (I - dt d_i K) V = b is solved directly: parallel cyclic reduction of the
// tridiagonal system in LDS (exact up to rounding; the system is diagonally
// dominant), where the per-phase path runs CG to cg_rtol.
#include <hip/hip_runtime.h>

#include "hsdc_device.h"
#include "hsdc_internal.h"
#include "ttp06_device.h"

namespace hsdc {

constexpr int kSmallMaxNodes = 256;  // one wave per SIMD of one CU: registers for the cell model

struct SmallArgs {
  Grid g;        // 1D, N <= kSmallMaxNodes
  Stages st;     // the level's stage vectors (one slice)
  Colloc co;
  Stim stim;
  double gs0, gs1, gs2;
  int K;         // sweeps per step
  int nsteps;
  int *flag;     // device: steps done, or -(steps done) when the last one turned a state non-finite
};

// The stimulus of node p at time t (slice 0): amp w_p while t is in
// (t0, t0 + dur], both ends shifted by eps, as in the per-phase kernels.
__device__ __forceinline__ double stim_value(const Stim &st, double t, int n, int64_t p) {
  if (st.w == nullptr) return 0.0;
  const bool on = (t > st.t0 + st.eps) && (t <= st.t0 + st.dur + st.eps);
  return on ? st.amp * st.w[n * st.sw + p] : 0.0;
}

// (K v)_p on the 1D mesh with v in LDS (no-flux ends; per-face coefficients
// or the uniform one), as applyK forms it.
__device__ __forceinline__ double small_K(const Grid &g, int p, const double *v) {
  const double vc = v[p];
  if (g.kx) {
    double acc = 0.0;
    if (p > 0) acc += g.kx[p - 1] * (v[p - 1] - vc);
    if (p < g.nx - 1) acc += g.kx[p] * (v[p + 1] - vc);
    return acc;
  }
  double ax = 0.0;
  if (p > 0) ax += v[p - 1] - vc;
  if (p < g.nx - 1) ax += v[p + 1] - vc;
  return g.cx * ax;
}

// x = (I - a K)^{-1} b by parallel cyclic reduction: every thread keeps the
// row (l, m, u | r) of its node, x_{p-s} l + x_p m + x_{p+s} u = r, and each
// level eliminates the couplings at distance s with the neighbours' rows.
// All threads of the block call it; b is the caller's value for its node.
__device__ double small_solve(const Grid &g, double a, bool live, int p, double b,
                              double *sl, double *sm, double *su, double *sr) {
  const int n = g.nx;
  double l = 0.0, m = 1.0, u = 0.0, r = 0.0;
  if (live) {
    const double kl = p > 0 ? (g.kx ? g.kx[p - 1] : g.cx) : 0.0;
    const double ku = p < n - 1 ? (g.kx ? g.kx[p] : g.cx) : 0.0;
    l = -a * kl;
    u = -a * ku;
    m = 1.0 + a * (kl + ku);
    r = b;
  }
#pragma unroll 1
  for (int s = 1; s < n; s <<= 1) {
    if (live) {
      sl[p] = l;
      sm[p] = m;
      su[p] = u;
      sr[p] = r;
    }
    __syncthreads();
    if (live) {
      double nl = 0.0, nm = m, nu = 0.0, nr = r;
      if (p - s >= 0) {
        const double k1 = l / sm[p - s];
        nl = -sl[p - s] * k1;
        nm -= su[p - s] * k1;
        nr -= sr[p - s] * k1;
      }
      if (p + s < n) {
        const double k2 = u / sm[p + s];
        nu = -su[p + s] * k2;
        nm -= sl[p + s] * k2;
        nr -= sr[p + s] * k2;
      }
      l = nl;
      m = nm;
      u = nu;
      r = nr;
    }
    __syncthreads();
  }
  return r / m;
}

template <int M>
__global__ void __launch_bounds__(kSmallMaxNodes) k_small_steps(SmallArgs a) {
  __shared__ double sv[kSmallMaxNodes], sl[kSmallMaxNodes], sm[kSmallMaxNodes],
      su[kSmallMaxNodes], sr[kSmallMaxNodes];
  __shared__ int bad;
  const Grid &g = a.g;
  const Colloc &co = a.co;
  // Meshes of at most 128 nodes give each node two threads, one wave apart:
  // one forms the gate rows, the other (the owner) the V and auxiliary rows,
  // the currents, the solve's row and the copies; larger meshes do both in
  // one thread.
  constexpr int H = kSmallMaxNodes / 2;
  const int t = threadIdx.x;
  const bool split = g.nx <= H;
  const int p = split ? t % H : t;
  const bool own = p < g.nx && (!split || t >= H);
  const bool gat = p < g.nx && (!split || t < H);
  const int64_t Np = a.st.Np, sS = a.st.sS();
  double *Y = a.st.Y + p, *G = a.st.G + p, *FV = a.st.FV + p, *RH = a.st.RH + p;
  double *L0 = a.st.L0 + p;
  const double dt = co.dt;
  const double Cm = a.stim.Cm;
  const int64_t step00 = *a.stim.step;
  if (t == 0) bad = 0;
#pragma unroll 1
  for (int step = 0; step < a.nsteps; ++step) {
    const int64_t step0 = step00 + step;
    // ---- stage 0 = y_n: its reaction terms, Lambda_n, K V; spread to 1..M
    if (own || gat) {
      double y[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) y[f] = Y[f * Np];
      if (gat)
        ttp06::gates<double>(y[0], y[3], [&](int k, double inf, double rate) {
          const double lam = -rate;
          const double w = y[GATE0 + k];
          G[(GATE0 + k) * Np] = lam * (w - inf) - lam * w;
          L0[k * Np] = lam;
        });
      if (own) {
        double I_ion, ha[6];
        ttp06::currents<double>(y, a.gs0, a.gs1, a.gs2, I_ion, ha);
        const double s0 = stim_value(a.stim, (double)step0 * dt, 0, p);
        G[0] = (s0 - Cm * I_ion) / Cm;
#pragma unroll
        for (int k = 0; k < 6; ++k) G[(1 + k) * Np] = ha[k];
        sv[p] = y[0];
      }
    }
    __syncthreads();
    if (own) {
      const double fv0 = small_K(g, p, sv);
      FV[0] = fv0;
      const double s0 = stim_value(a.stim, (double)step0 * dt, 0, p);
#pragma unroll 1
      for (int j = 1; j <= M; ++j) {
        const double sj = stim_value(a.stim, ((double)step0 + co.c[j - 1]) * dt, 0, p);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          double gv = G[f * Np];
          if (f == 0 && sj != s0) gv += (sj - s0) / Cm;
          G[j * sS + f * Np] = gv;
          Y[j * sS + f * Np] = Y[f * Np];
        }
        FV[j * Np] = fv0;
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int k = 0; k < a.K; ++k) {
      const bool last = k == a.K - 1;
      // ---- right-hand sides RH_i = R_i - R_{i-1} of every row: the (field,
      // node) pairs are shared among all threads of the block (a node's rows
      // are independent)
#pragma unroll 1
      for (int q = t; q < NF * g.nx; q += blockDim.x) {
        const int f = q / g.nx, nd = q - f * g.nx;
        const double *Gq = a.st.G + nd + f * Np;
        double Gv[M + 1], gfull[M], I[M];
#pragma unroll
        for (int j = 0; j <= M; ++j) Gv[j] = Gq[j * sS];
        double fvn[M + 1];  // K V of the V row (0 elsewhere)
#pragma unroll
        for (int j = 0; j <= M; ++j) fvn[j] = (f == 0 && j > 0) ? a.st.FV[nd + j * Np] : 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) gfull[j] = Gv[j + 1] + fvn[j + 1];
        double pz = 0.0;  // dt Lambda_n of a gate row (the Phi term's phi_1(d_i pz))
        if (f >= GATE0) {
          const double lam_n = a.st.L0[nd + (f - GATE0) * Np];
          colloc_integrals<M>(co, dt * lam_n, gfull, I, lam_n * a.st.Y[nd + f * Np]);
          pz = dt * lam_n;
        } else {
          colloc_weights<M>(co, gfull, I);
        }
        double prevI = 0.0;
        double *Rq = a.st.RH + nd + f * Np;
#pragma unroll
        for (int i = 0; i < M; ++i) {
          const double phi = f >= GATE0 ? phi1(co.d[i] * pz) * Gv[i] : fvn[i + 1] + Gv[i];
          Rq[(int64_t)i * sS] = dt * (I[i] - prevI) - dt * co.d[i] * phi;
          prevI = I[i];
        }
      }
      __syncthreads();  // a node's right-hand sides come from other threads
      // ---- node to node: stage i from stage i - 1, then V_i by the solve
#pragma unroll 1
      for (int i = 1; i <= M; ++i) {
        const double ddt = dt * co.d[i - 1];
        double bv = 0.0;
        if (own || gat) {
          const double *Yp = Y + (int64_t)(i - 1) * sS;
          double *Yi = Y + (int64_t)i * sS;
          const double *R = RH + (int64_t)(i - 1) * sS;
          double *Gp = G + (int64_t)(i - 1) * sS;
          double yd[NF];
#pragma unroll
          for (int f = 0; f < NF; ++f) yd[f] = Yp[f * Np];
          double gV = 0.0;
          if (i == 1) {
            // y_{n,0}: its stored reaction terms
            if (own) {
#pragma unroll
              for (int f = 1; f < GATE0; ++f) Yi[f * Np] = yd[f] + R[f * Np] + ddt * Gp[f * Np];
              gV = Gp[0];
            }
            if (gat) {
#pragma unroll
              for (int kk = 0; kk < NG; ++kk) {
                const int f = GATE0 + kk;
                Yi[f * Np] = yd[f] + R[f * Np] + ddt * phi1(ddt * L0[kk * Np]) * Gp[f * Np];
              }
            }
          } else {
            if (gat)
              ttp06::gates<double>(yd[0], yd[3], [&](int kk, double inf, double rate) {
                const int f = GATE0 + kk;
                const double lu = L0[kk * Np];
                const double w = yd[f];
                const double gv = -rate * (w - inf) - lu * w;
                if (!last) Gp[f * Np] = gv;
                Yi[f * Np] = yd[f] + R[f * Np] + ddt * phi1(ddt * lu) * gv;
              });
            if (own) {
              const double tt = ((double)step0 + co.c[i - 2]) * dt;
              double I_ion, ha[6];
              ttp06::currents<double>(yd, a.gs0, a.gs1, a.gs2, I_ion, ha);
              gV = (stim_value(a.stim, tt, 0, p) - Cm * I_ion) / Cm;
              if (!last) Gp[0] = gV;
#pragma unroll
              for (int kk = 0; kk < 6; ++kk) {
                if (!last) Gp[(1 + kk) * Np] = ha[kk];
                Yi[(1 + kk) * Np] = yd[1 + kk] + R[(1 + kk) * Np] + ddt * ha[kk];
              }
            }
          }
          if (own) bv = yd[0] + R[0] + ddt * gV;
        }
        const double v = small_solve(g, ddt, own, p, bv, sl, sm, su, sr);
        if (own) Y[(int64_t)i * sS] = v;
        __syncthreads();  // stage i whole (its rows come from two threads) before node i + 1
      }
      if (!last) {
        // reaction terms of stage M and K V of stages 1..M for the next sweep
        if (own || gat) {
          const double *Ym = Y + (int64_t)M * sS;
          double *Gm = G + (int64_t)M * sS;
          double y[NF];
#pragma unroll
          for (int f = 0; f < NF; ++f) y[f] = Ym[f * Np];
          if (gat)
            ttp06::gates<double>(y[0], y[3], [&](int kk, double inf, double rate) {
              const double w = y[GATE0 + kk];
              Gm[(GATE0 + kk) * Np] = -rate * (w - inf) - L0[kk * Np] * w;
            });
          if (own) {
            double I_ion, ha[6];
            ttp06::currents<double>(y, a.gs0, a.gs1, a.gs2, I_ion, ha);
            const double tt = ((double)step0 + co.c[M - 1]) * dt;
            Gm[0] = (stim_value(a.stim, tt, 0, p) - Cm * I_ion) / Cm;
#pragma unroll
            for (int kk = 0; kk < 6; ++kk) Gm[(1 + kk) * Np] = ha[kk];
          }
        }
#pragma unroll 1
        for (int j = 1; j <= M; ++j) {
          if (own) sv[p] = Y[(int64_t)j * sS];
          __syncthreads();
          if (own) FV[j * Np] = small_K(g, p, sv);
          __syncthreads();
        }
      }
    }
    // ---- y_{n+1} = y_{n,M}; stop after a step whose state is not finite
    bool nf = false;
    if (own) {
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double v = Y[(int64_t)M * sS + f * Np];
        nf = nf || !isfinite(v);
        Y[f * Np] = v;
      }
    }
    if (nf) bad = 1;
    __syncthreads();
    if (bad) {
      if (t == 0) *a.flag = -(step + 1);
      return;
    }
  }
  if (t == 0) *a.flag = a.nsteps;
}

hipError_t launch_small_steps(hipStream_t s, const Grid &g, const Stages &st, const Colloc &co,
                              const Stim &stim, double gs0, double gs1, double gs2, int K,
                              int nsteps, int *flag) {
  // one thread per node, one workgroup
  if (g.dim != 1 || g.nx < 1 || g.nx > kSmallMaxNodes || g.rag || nsteps < 0 || K < 1)
    return hipErrorInvalidValue;
  if (nsteps == 0) return hipSuccess;
  SmallArgs a{g, st, co, stim, gs0, gs1, gs2, K, nsteps, flag};
  const dim3 block(kSmallMaxNodes);
  HSDC_DISPATCH_M(co.M, hipLaunchKernelGGL(k_small_steps<M>, dim3(1), block, 0, s, a));
  return hipGetLastError();
}

}  // namespace hsdc
