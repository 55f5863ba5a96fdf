// hsdc_adjoint.hip -- kernels of the discrete adjoint of a serial hybrid SDC
// step (the transposed sweep of eqs. prec_picard, def_P and def_C), for the
// gradient of a probe-voltage misfit with respect to the per-node
// conductivity field and the G_Na, G_CaL, G_Kr scalings.
//
// One step of the forward map, in the node-to-node form the library computes
// (anchor u = y_n, Lambda_n = Lambda(u), z = dt Lambda_n, the previous
// iterate X = (u, X_1..X_M), the new one Z = (u, Z_1..Z_M)):
//   g_j   = G(X_j) + e_V K X_j^V,            G the reaction terms (anchor u)
//   p_i   = dt d_i (e_V K X_i^V + Gh_i(X_{i-1})),  Gh_i = G with its gate rows
//           times phi_1(d_i z)
//   RH_i  = dt sum_j (a_ij - a_{i-1,j}) g_j - p_i    (a = Q on rows V .. Rbar,
//           a(z) on the gate rows)
//   b_i   = Z_{i-1} + RH_i + dt d_i Gh_i(Z_{i-1}),  Z_i = b_i but
//           Z_i^V = (I - dt d_i K)^-1 b_i^V.
// The adjoint runs these backwards: the node-local parts here (the cell
// model's Jacobian applied transposed, by forward-mode dual numbers), the
// symmetric solves and stencil products with the library's operator, and the
// derivative of a_ij(z) and phi_1 through phi_k' = phi_k - k phi_{k+1}.
#include <hip/hip_runtime.h>

#include "hsdc_device.h"
#include "hsdc_internal.h"
#include "ttp06_device.h"
#include "ttp06_vjp.h"

namespace hsdc {
namespace ad {

// Forward-mode dual number: a value and one directional derivative.
struct D {
  double v, d;
  __device__ D() : v(0.0), d(0.0) {}
  __device__ D(double x) : v(x), d(0.0) {}
  __device__ D(double x, double dx) : v(x), d(dx) {}
};
__device__ __forceinline__ D operator+(D a, D b) { return D(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ D operator-(D a, D b) { return D(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ D operator-(D a) { return D(-a.v, -a.d); }
__device__ __forceinline__ D operator*(D a, D b) { return D(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ D operator/(D a, D b) {
  const double q = a.v / b.v;
  return D(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ bool operator<(D a, D b) { return a.v < b.v; }
__device__ __forceinline__ bool operator==(D a, D b) { return a.v == b.v; }
__device__ __forceinline__ D exp(D a) {
  const double e = ::exp(a.v);
  return D(e, e * a.d);
}
__device__ __forceinline__ D expm1(D a) { return D(::expm1(a.v), ::exp(a.v) * a.d); }
__device__ __forceinline__ D log(D a) { return D(::log(a.v), a.d / a.v); }
__device__ __forceinline__ D sqrt(D a) {
  const double r = ::sqrt(a.v);
  return D(r, 0.5 * a.d / r);
}

}  // namespace ad

// Transposed Jacobian of the reaction terms at one node state x, anchor values
// ug and rates lam_n of the gates (eqs. def_f_IE, def_Lambda; the gates'
// anchor part Lambda_n (u - x)):
//   G_V = (I_stim - Cm I_ion(x)) / Cm,  G_aux = h_a(x),
//   G_g = Lambda_g(x) (x_g - w_inf,g(x)) + Lambda_n,g (u_g - x_g).
// vx += (dG/dx)^T cot and vgs += (dG/dgs)^T cot (u and Lambda_n held fixed);
// Gg receives the gate terms G_g(x).  The currents are taken back in one
// reverse pass (currents_vjp), the gates by one dual pass in V (their rates
// and steady states depend on V, except fCass, which depends on Ca_ss alone).
__device__ __forceinline__ void reaction_vjp(const double *x, const double *gs,
                                                      const double *lam_n, const double *ug,
                                                      const double *cot, double *vx, double *vgs,
                                                      double *Gg) {
  // pass 1, dual in V: the gate terms, their V derivatives and the diagonal
  ttp06::gates<ad::D>(ad::D(x[0], 1.0), ad::D(x[3], 0.0), [&](int k, ad::D in, ad::D rate) {
    const double w = x[GATE0 + k], c = cot[GATE0 + k], lam = -rate.v;
    Gg[k] = lam * (w - in.v) + lam_n[k] * (ug[k] - w);
    vx[0] += c * (-rate.d * (w - in.v) - lam * in.d);
    vx[GATE0 + k] += c * (lam - lam_n[k]);
  });
  // Ca_ss derivatives: fCass is the only gate that depends on Ca_ss
  {
    ad::D in, rate;
    ttp06::fcass_gate<ad::D>(ad::D(x[3], 1.0), in, rate);
    const double w = x[GATE0 + NG - 1], c = cot[GATE0 + NG - 1];
    vx[3] += c * (-rate.d * (w - in.v) + rate.v * in.d);
  }
  // d G_V = -d I_ion; the auxiliary rows take h_a directly
  ttp06::currents_vjp<double>(x, gs[0], gs[1], gs[2], -cot[0], cot + 1, vx, vgs);
}

// phi_1(x) and phi_1'(x) = phi_1(x) - phi_2(x).
__device__ __forceinline__ void phi1_d(double x, const double *invfact, double &p1, double &dp1) {
  double ph[2];
  phis<2>(x, invfact, ph);
  p1 = ph[0];
  dp1 = ph[0] - ph[1];
}

// Sums of the conductance-scaling gradient over a block, one row of partials
// per block (reduced by k_adj_gs_reduce).
template <int NT>
__device__ __forceinline__ void block_gs(double (&vgs)[3], double *lds, double *part) {
  block_sums<3, NT>(vgs, lds);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = vgs[0];
    part[3 * blockIdx.x + 1] = vgs[1];
    part[3 * blockIdx.x + 2] = vgs[2];
  }
}

constexpr int ADB = kAdjBlock;

// Node i of the forward substitution, backwards.  beta_i (the adjoint of b_i)
// is MU_i with its V row replaced by the adjoint solve's result (in RHO_i);
// RHO_i receives all of beta_i.  With s = Z_{i-1} and the cotangent c =
// dt d_i beta (gate rows times phi_1(d_i z)):
//   MU_{i-1} (or DYN for i = 1, Z_0 = u) += beta + (dG/dx)^T c,
//   DLAM_g += c_g (u_g - s_g), DYN_g += c_g Lambda_n,g (the anchor part),
//   DZ_g += dt d_i beta_g G_g(s) d_i phi_1'(d_i z_g).
__global__ void __launch_bounds__(ADB)
k_adj_backsub(AdjArgs a, int i) {
  __shared__ double lds[3 * (ADB / 64)];
  const int64_t p = (int64_t)blockIdx.x * ADB + threadIdx.x;
  double vgs[3] = {0.0, 0.0, 0.0};
  if (p < a.N) {
    const int64_t Np = a.Np, sS = (int64_t)NF * Np;
    const double *Zs = a.Z + (int64_t)(i - 1) * sS + p;
    const double *U = a.Z + p;  // stage 0 = u
    double *mu_i = a.MU + (int64_t)i * sS + p;
    double *rho_i = a.RHO + (int64_t)i * sS + p;
    double *tgt = (i == 1) ? a.DYN + p : a.MU + (int64_t)(i - 1) * sS + p;
    const double ddt = a.co.dt * a.co.d[i - 1];
    double x[NF], beta[NF], cot[NF], vx[NF], lam_n[NG], ug[NG], Gg[NG], p1[NG], dp1[NG];
    for (int f = 0; f < NF; ++f) {
      x[f] = Zs[f * Np];
      beta[f] = (f == 0) ? rho_i[0] : mu_i[f * Np];
      if (f > 0) rho_i[f * Np] = beta[f];
      vx[f] = 0.0;
    }
    for (int k = 0; k < NG; ++k) {
      lam_n[k] = a.L0[k * Np + p];
      ug[k] = U[(GATE0 + k) * Np];
      phi1_d(a.co.d[i - 1] * a.co.dt * lam_n[k], a.co.invfact, p1[k], dp1[k]);
    }
    for (int f = 0; f < NF; ++f)
      cot[f] = ddt * beta[f] * (f >= GATE0 ? p1[f - GATE0] : 1.0);
    const double gs[3] = {a.gs[0], a.gs[1], a.gs[2]};
    reaction_vjp(x, gs, lam_n, ug, cot, vx, vgs, Gg);
    for (int f = 0; f < NF; ++f) tgt[f * Np] += beta[f] + vx[f];
    for (int k = 0; k < NG; ++k) {
      const double c = cot[GATE0 + k];
      a.DLAM[k * Np + p] += c * (ug[k] - x[GATE0 + k]);
      a.DYN[(GATE0 + k) * Np + p] += c * lam_n[k];
      a.DZ[k * Np + p] += ddt * beta[GATE0 + k] * Gg[k] * a.co.d[i - 1] * dp1[k];
    }
  }
  block_gs<ADB>(vgs, lds, a.gs_part);
}

// The collocation integrals and the P terms built from the previous iterate,
// backwards, for every stage j = 0..M of X (X_0 = u):
//   gamma_j = dt sum_i (a_ij - a_{i-1,j}) rho_i          (j >= 1; a_0j = 0)
//   cot_j   = gamma_j - dt d_{j+1} rho_{j+1} (gate rows times phi_1(d_{j+1} z))
//   MUX_j (or DYN for j = 0) += (dG/dx)^T cot_j at X_j, the anchor parts as
//   in k_adj_backsub, and
//   DZ_g += dt sum_i rho_i,g sum_j (a'_ij - a'_{i-1,j}) G_g(X_j)
//           - rho_{j+1,g} dt d_{j+1} G_g(X_j) d_{j+1} phi_1'(d_{j+1} z),
//   a'_ij(z) = sum_k c_i^{k+1} w_j^{k-1} phi_k'(c_i z).
// W_j = gamma_j^V - dt d_j rho_j^V is the adjoint the stencil products K X_j^V
// receive (applied by the host with the operator, j = 1..M).
// The stages are independent given rho, so each (node, stage) pair has a
// thread of its own (blockIdx.y = j): M + 1 times the waves of one thread per
// node, which the transposed cell model needs to hide its latencies.  What
// every stage adds to one node (cot_g lambda_n,g to the gate rows of DYN,
// cot_g (u_g - x_g) to DLAM, the DZ terms) goes to PS[j] and is summed in
// stage order by k_adj_assemble_sum.
template <int M>
__global__ void __launch_bounds__(ADB)
k_adj_assemble(AdjArgs a) {
  __shared__ double lds[3 * (ADB / 64)];
  const int64_t p = (int64_t)blockIdx.x * ADB + threadIdx.x;
  const int j = blockIdx.y;
  double vgs[3] = {0.0, 0.0, 0.0};
  if (p < a.N) {
    const int64_t Np = a.Np, sS = (int64_t)NF * Np;
    const Colloc &co = a.co;
    const double dt = co.dt;
    const double *X = a.X + p;
    const double *rho = a.RHO + p;
    const bool nxt = j + 1 <= M;
    const double ddn = nxt ? dt * co.d[j] : 0.0;  // dt d_{j+1}
    double lam_n[NG], ug[NG], x[NF], cot[NF], vx[NF], ck[NG], Gg[NG];
    for (int k = 0; k < NG; ++k) {
      lam_n[k] = a.L0[k * Np + p];
      ug[k] = X[(GATE0 + k) * Np];
    }
    for (int f = 0; f < NF; ++f) {
      x[f] = X[(int64_t)j * sS + f * Np];
      vx[f] = 0.0;
    }
    // rows V .. Rbar: collocation weights Q
    double gam0 = 0.0;
    for (int f = 0; f < GATE0; ++f) {
      double c = 0.0;
      if (j >= 1)
        for (int i = 1; i <= M; ++i)
          c += dt * (co.Q[i - 1][j - 1] - (i > 1 ? co.Q[i - 2][j - 1] : 0.0)) *
               rho[(int64_t)i * sS + f * Np];
      if (f == 0) gam0 = c;
      if (nxt) c -= ddn * rho[(int64_t)(j + 1) * sS + f * Np];
      cot[f] = c;
    }
    // gate rows: column j of a_ij(z) and of its derivative in z; ck collects
    // the factor of G_g(X_j) in the DZ terms
    for (int k = 0; k < NG; ++k) {
      const int f = GATE0 + k;
      const double z = dt * lam_n[k];
      double c = 0.0, s = 0.0;
      if (j >= 1) {
        double Ap = 0.0, Dp = 0.0;  // row i - 1 (row 0: zero)
        for (int i = 1; i <= M; ++i) {
          double ph[M + 1], Aij = 0.0, Dij = 0.0;
          if (z == 0.0) {
            Aij = co.Q[i - 1][j - 1];
            for (int q = 0; q <= M; ++q) ph[q] = co.invfact[q + 1];  // phi_k(0) = 1/k!
          } else {
            phis<M + 1>(co.c[i - 1] * z, co.invfact, ph);
            for (int q = 0; q < M; ++q) Aij += co.cpow[i - 1][q + 1] * co.W[q][j - 1] * ph[q];
          }
          for (int q = 0; q < M; ++q)
            Dij += co.cpow[i - 1][q + 1] * co.c[i - 1] * co.W[q][j - 1] *
                   (ph[q] - (q + 1) * ph[q + 1]);
          const double r = rho[(int64_t)i * sS + f * Np];
          c += dt * (Aij - Ap) * r;
          s += dt * r * (Dij - Dp);
          Ap = Aij;
          Dp = Dij;
        }
      }
      if (nxt) {
        double p1, dp1;
        phi1_d(co.d[j] * dt * lam_n[k], co.invfact, p1, dp1);
        const double r = rho[(int64_t)(j + 1) * sS + f * Np];
        c -= ddn * p1 * r;
        s -= r * ddn * co.d[j] * dp1;
      }
      cot[f] = c;
      ck[k] = s;
    }
    const double gs[3] = {a.gs[0], a.gs[1], a.gs[2]};
    reaction_vjp(x, gs, lam_n, ug, cot, vx, vgs, Gg);
    double *tgt = (j == 0) ? a.DYN + p : a.MUX + (int64_t)j * sS + p;
    for (int f = 0; f < NF; ++f) tgt[f * Np] += vx[f];
    double *ps = a.PS + (int64_t)j * (3 * NG) * Np + p;
    for (int k = 0; k < NG; ++k) {
      const double c = cot[GATE0 + k];
      ps[k * Np] = c;
      ps[(NG + k) * Np] = c * (ug[k] - x[GATE0 + k]);
      ps[(2 * NG + k) * Np] = ck[k] * Gg[k];
    }
    if (j >= 1) a.W[(int64_t)j * Np + p] = gam0 - dt * co.d[j - 1] * rho[(int64_t)j * sS];
  }
  block_sums<3, ADB>(vgs, lds);
  if (threadIdx.x == 0) {
    double *part = a.gs_part + 3 * ((int64_t)blockIdx.y * gridDim.x + blockIdx.x);
    part[0] = vgs[0];
    part[1] = vgs[1];
    part[2] = vgs[2];
  }
}

// The stage contributions of k_adj_assemble, summed in stage order.
__global__ void __launch_bounds__(ADB) k_adj_assemble_sum(AdjArgs a, int nstages) {
  const int64_t p = (int64_t)blockIdx.x * ADB + threadIdx.x;
  if (p >= a.N) return;
  const int64_t Np = a.Np;
  for (int k = 0; k < NG; ++k) {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int j = 0; j < nstages; ++j) {
      const double *ps = a.PS + (int64_t)j * (3 * NG) * Np + p;
      s1 += ps[k * Np];
      s2 += ps[(NG + k) * Np];
      s3 += ps[(2 * NG + k) * Np];
    }
    a.DYN[(GATE0 + k) * Np + p] += s1 * a.L0[k * Np + p];
    a.DLAM[k * Np + p] += s2;
    a.DZ[k * Np + p] += s3;
  }
}

// Lambda_n = Lambda(u) backwards: DYN at V and Ca_ss += (dLambda/du)^T (dt DZ + DLAM).
__global__ void __launch_bounds__(ADB) k_adj_anchor(AdjArgs a) {
  const int64_t p = (int64_t)blockIdx.x * ADB + threadIdx.x;
  if (p >= a.N) return;
  const int64_t Np = a.Np;
  const double V = a.Z[p], C = a.Z[3 * Np + p];
  double sv = 0.0, sc = 0.0;
  ttp06::gates<ad::D>(ad::D(V, 1.0), ad::D(C, 0.0), [&](int k, ad::D, ad::D rate) {
    sv += (a.co.dt * a.DZ[k * Np + p] + a.DLAM[k * Np + p]) * (-rate.d);
  });
  {  // Ca_ss enters the rate of fCass only
    constexpr int k = NG - 1;
    ad::D in, rate;
    ttp06::fcass_gate<ad::D>(ad::D(C, 1.0), in, rate);
    sc = (a.co.dt * a.DZ[k * Np + p] + a.DLAM[k * Np + p]) * (-rate.d);
  }
  a.DYN[p] += sv;
  a.DYN[3 * Np + p] += sc;
}

// Gradient of u^T K v with respect to the face coefficients, scaled:
// dk_face(p, p + e_a) += s (-(u_q - u_p)(v_q - v_p)).
__global__ void __launch_bounds__(ADB)
k_adj_faces(Grid g, const double *u, const double *v, double s, double *dkx, double *dky,
            double *dkz) {
  const int64_t p = (int64_t)blockIdx.x * ADB + threadIdx.x;
  if (p >= g.N) return;
  const Ijk c = ijk(g, p);
  const double up = u[p], vp = v[p];
  auto face = [&](int64_t q) { return -s * (u[q] - up) * (v[q] - vp); };
  if (c.ix < g.nx - 1) dkx[p] += face(p + 1);
  if (g.dim >= 2 && c.iy < g.ny - 1) dky[p] += face(p + g.nx);
  if (g.dim >= 3 && c.iz < g.nz - 1) dkz[p] += face(p + (int64_t)g.nx * g.ny);
}

// out += s K v (the library's operator, per-node faces or uniform).
template <int DIM, bool PN>
__global__ void __launch_bounds__(ADB) k_adj_spmv_add(Grid g, const double *v, double s, double *out) {
  const int64_t p = (int64_t)blockIdx.x * ADB + threadIdx.x;
  if (p >= g.N) return;
  const Ijk c = ijk(g, p);
  out[p] += s * applyK<DIM, PN>(g, p, c, v[p], [&](int64_t k) { return v[k]; });
}

// The first Chebyshev step of an adjoint solve, x_1 = x_0 + (b - A x_0) / theta
// with A = I - a K (as the node update forms it for the forward solves); with
// bpart, also the block partials of ||b||^2 (the reference of CG's stop test).
template <int DIM, bool PN>
__global__ void __launch_bounds__(ADB)
k_adj_cheb_x1(Grid g, const double *x0, const double *b, double a, const ChebTab *tab,
              double *x1, double *bpart) {
  __shared__ double lds[ADB / 64];
  const int64_t p = (int64_t)blockIdx.x * ADB + threadIdx.x;
  double bb = 0.0;
  if (p < g.N) {
    const Ijk c = ijk(g, p);
    const double xc = x0[p], bp = b[p];
    const double r = bp - (xc - a * applyK<DIM, PN>(g, p, c, xc, [&](int64_t q) { return x0[q]; }));
    x1[p] = xc + r * tab->inv_theta;
    bb = bp * bp;
  }
  if (bpart == nullptr) return;  // the same for every thread of the launch
  double t1[1] = {bb};
  block_sums<1, ADB>(t1, lds);
  if (threadIdx.x == 0) bpart[blockIdx.x] = t1[0];
}

// dsigma_p from the face gradients: a face coefficient is sc 2 s_p s_q / (s_p + s_q).
__global__ void __launch_bounds__(ADB)
k_adj_sigma(Grid g, const double *sig, double sc, const double *dkx, const double *dky,
            const double *dkz, double *dsig) {
  const int64_t p = (int64_t)blockIdx.x * ADB + threadIdx.x;
  if (p >= g.N) return;
  const Ijk c = ijk(g, p);
  const double sp = sig[p];
  double acc = 0.0;
  // face (p, q): d k / d s_p = sc 2 s_q^2 / (s_p + s_q)^2
  auto add = [&](const double *dk, int64_t face, int64_t other) {
    const double so = sig[other], t = sp + so;
    if (t > 0.0) acc += dk[face] * sc * 2.0 * so * so / (t * t);
  };
  const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
  if (c.ix < g.nx - 1) add(dkx, p, p + 1);
  if (c.ix > 0) add(dkx, p - 1, p - 1);
  if (g.dim >= 2) {
    if (c.iy < g.ny - 1) add(dky, p, p + sy);
    if (c.iy > 0) add(dky, p - sy, p - sy);
  }
  if (g.dim >= 3) {
    if (c.iz < g.nz - 1) add(dkz, p, p + sz);
    if (c.iz > 0) add(dkz, p - sz, p - sz);
  }
  dsig[p] = acc;
}

// Misfit at the probes: r_q = V(probe_q) - target_q; out_sq[q] = r_q^2, and
// (seed) lambda[V][probe_q] += 2 r_q.
__global__ void k_adj_probes(const double *y, const int64_t *probes, const double *target, int np,
                             double *out_sq, double *lambda) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= np) return;
  const double r = y[probes[q]] - target[q];
  if (out_sq) out_sq[q] = r * r;
  if (lambda) lambda[probes[q]] += 2.0 * r;  // probes are distinct
}

// Sums block partials of the scaling gradient into acc[3] (one block, fixed order).
__global__ void __launch_bounds__(ADB) k_adj_gs_reduce(const double *part, int nb, double *acc) {
  __shared__ double lds[3 * (ADB / 64)];
  double v[3] = {0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < nb; k += ADB)
    for (int q = 0; q < 3; ++q) v[q] += part[3 * k + q];
  block_sums<3, ADB>(v, lds);
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) acc[q] += v[q];
}

// y += x over n values.
__global__ void __launch_bounds__(ADB) k_adj_axpy(double *y, const double *x, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * ADB + threadIdx.x;
  if (p < n) y[p] += x[p];
}

static unsigned adj_blocks(int64_t n) { return (unsigned)((n + ADB - 1) / ADB); }

hipError_t launch_adj_backsub(hipStream_t s, const AdjArgs &a, int i) {
  hipLaunchKernelGGL(k_adj_backsub, dim3(adj_blocks(a.N)), dim3(ADB), 0, s, a, i);
  hipLaunchKernelGGL(k_adj_gs_reduce, dim3(1), dim3(ADB), 0, s, a.gs_part, (int)adj_blocks(a.N),
                     a.gs_acc);
  return hipGetLastError();
}

hipError_t launch_adj_assemble(hipStream_t s, const AdjArgs &a) {
  const dim3 grid(adj_blocks(a.N), a.co.M + 1);
  switch (a.co.M) {
    case 1: hipLaunchKernelGGL(k_adj_assemble<1>, grid, dim3(ADB), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_adj_assemble<2>, grid, dim3(ADB), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_adj_assemble<3>, grid, dim3(ADB), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_adj_assemble<4>, grid, dim3(ADB), 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_adj_assemble<5>, grid, dim3(ADB), 0, s, a); break;
    case 6: hipLaunchKernelGGL(k_adj_assemble<6>, grid, dim3(ADB), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_adj_assemble_sum, dim3(adj_blocks(a.N)), dim3(ADB), 0, s, a, a.co.M + 1);
  hipLaunchKernelGGL(k_adj_gs_reduce, dim3(1), dim3(ADB), 0, s, a.gs_part,
                     (int)(adj_blocks(a.N) * (a.co.M + 1)), a.gs_acc);
  return hipGetLastError();
}

hipError_t launch_adj_anchor(hipStream_t s, const AdjArgs &a) {
  hipLaunchKernelGGL(k_adj_anchor, dim3(adj_blocks(a.N)), dim3(ADB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adj_faces(hipStream_t s, const Grid &g, const double *u, const double *v,
                            double scale, double *dkx, double *dky, double *dkz) {
  hipLaunchKernelGGL(k_adj_faces, dim3(adj_blocks(g.N)), dim3(ADB), 0, s, g, u, v, scale, dkx,
                     dky, dkz);
  return hipGetLastError();
}

hipError_t launch_adj_spmv_add(hipStream_t s, const Grid &g, const double *v, double scale,
                               double *out) {
  HSDC_DISPATCH_OP(g, hipLaunchKernelGGL((k_adj_spmv_add<DIM, PN>), dim3(adj_blocks(g.N)),
                                         dim3(ADB), 0, s, g, v, scale, out));
  return hipGetLastError();
}

hipError_t launch_adj_cheb_x1(hipStream_t s, const Grid &g, const double *x0, const double *b,
                              double a, const ChebTab *tab, double *x1, double *bpart) {
  HSDC_DISPATCH_OP(g, hipLaunchKernelGGL((k_adj_cheb_x1<DIM, PN>), dim3(adj_blocks(g.N)),
                                         dim3(ADB), 0, s, g, x0, b, a, tab, x1, bpart));
  return hipGetLastError();
}

hipError_t launch_adj_sigma(hipStream_t s, const Grid &g, const double *sig, double sc,
                            const double *dkx, const double *dky, const double *dkz, double *dsig) {
  hipLaunchKernelGGL(k_adj_sigma, dim3(adj_blocks(g.N)), dim3(ADB), 0, s, g, sig, sc, dkx, dky,
                     dkz, dsig);
  return hipGetLastError();
}

hipError_t launch_adj_probes(hipStream_t s, const double *y, const int64_t *probes,
                             const double *target, int np, double *out_sq, double *lambda) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_probes, dim3((np + 255) / 256), dim3(256), 0, s, y, probes, target, np,
                     out_sq, lambda);
  return hipGetLastError();
}

hipError_t launch_adj_axpy(hipStream_t s, double *y, const double *x, int64_t n) {
  hipLaunchKernelGGL(k_adj_axpy, dim3(adj_blocks(n)), dim3(ADB), 0, s, y, x, n);
  return hipGetLastError();
}

}  // namespace hsdc
