// hsdc_device.h -- device helpers shared by the kernels of libhsdc: phi
// functions and collocation integrals (Appendix A), wave and block reductions,
// mesh coordinates, and the cell-centred no-flux diffusion stencil.
#pragma once

#include <hip/hip_runtime.h>

#include "hsdc_internal.h"

namespace hsdc {

// Store with a streaming (non-temporal) hint: for values that only a later
// kernel reads.
template <class V>
__device__ __forceinline__ void stream_store(V *dst, V v) {
  __builtin_nontemporal_store(v, dst);
}

// ---------------------------------------------------------------------------
// phi functions (Appendix A, eq. def_phik)
// ---------------------------------------------------------------------------

// Polynomial sum_{m=0..N} c_m x^m as a sum of powers, each coefficient after
// c_0 a multiplier: an FP64 constant cannot be an immediate operand, and
// Horner's form, which adds the constants, spends two VALU moves per term on
// them, while a multiplying constant is held in scalar registers.  The terms
// decrease in size here, so the rounding stays at a few ulp.
template <int N, class C>
__device__ __forceinline__ double power_sum(double x, C &&c) {
  double acc = c(0), xp = x;
#pragma unroll
  for (int m = 1; m <= N; ++m) {
    acc = fma(c(m), xp, acc);
    if (m < N) xp *= x;
  }
  return acc;
}

// phi_1(x) = (e^x - 1)/x.  For |x| < 1/8 the Taylor series sum_{m<=9} x^m/(m+1)!
// (truncation below 2e-17 relative) replaces expm1 and the division.
__device__ __forceinline__ double phi1(double x) {
  if (fabs(x) < 0.125) {
    constexpr double c[10] = {1.0,           1.0 / 2.0,      1.0 / 6.0,      1.0 / 24.0,
                              1.0 / 120.0,   1.0 / 720.0,    1.0 / 5040.0,   1.0 / 40320.0,
                              1.0 / 362880.0, 1.0 / 3628800.0};
    return power_sum<9>(x, [&](int m) { return c[m]; });
  }
  return expm1(x) / x;
}

// Coefficients 1/(M+m)!, m = 0..N, of the Taylor series of phi_M, formed at
// compile time.
template <int M, int N>
struct PhiSeries {
  double c[N + 1];
  constexpr PhiSeries() : c() {
    double f = 1.0;
    for (int k = 2; k <= M; ++k) f *= k;
    c[0] = 1.0 / f;
    for (int m = 1; m <= N; ++m) c[m] = c[m - 1] / (M + m);
  }
};

// phi_1(x) .. phi_M(x) into out[0..M-1], by one of three branches.
//   |x| < 1/8: phi_M from its Taylor series sum_m x^m/(m+M)!, m <= 9 (truncation
//     below 2e-17 relative), then the backward recurrence
//     phi_k = 1/k! + x phi_{k+1}, which damps errors for k + 1 > |x|.
//   |x| >= F (F = M/2, or 1/8 for M = 1): the forward recurrence
//     phi_{k+1} = (phi_k - 1/k!)/x from phi_1 = expm1(x)/x.  It multiplies the
//     relative error by about (k+1)/|x| per step where k + 1 > |x|, at most
//     prod_{k >= F} (k+1)/F over the whole range (4.4 for M = 6, 6.6 for M = 8).
//   otherwise: phi_M from its Taylor series with N = 18 + M terms (below 1e-18
//     relative for |x| < M/2), as a sum of powers with compile-time
//     coefficients (power_sum), then the backward recurrence.
// Relative error below 6e-15 for M <= 8 over x in [-4000, 12] (checked against a
// 60-digit evaluation).
template <int M>
__device__ __forceinline__ void phis(double x, const double *invfact, double *out) {
  const double ax = fabs(x);
  constexpr double F = M == 1 ? 0.125 : 0.5 * M;
  if (ax >= F) {
    const double xi = 1.0 / x;
    double p = expm1(x) * xi;
    out[0] = p;
#pragma unroll
    for (int k = 1; k < M; ++k) {
      p = (p - invfact[k]) * xi;
      out[k] = p;
    }
    return;
  }
  double acc;
  if (ax < 0.125) {
    acc = invfact[M + 9];
#pragma unroll
    for (int m = 8; m >= 0; --m) acc = fma(acc, x, invfact[M + m]);
  } else {
    constexpr int N = 18 + M;
    constexpr PhiSeries<M, N> S{};
    acc = power_sum<N>(x, [&](int m) { return S.c[m]; });
  }
  out[M - 1] = acc;
#pragma unroll
  for (int k = M - 1; k >= 1; --k) {
    acc = invfact[k] + x * acc;
    out[k - 1] = acc;
  }
}

// I_i = sum_j a_ij(z) g_j, i, j = 1..M, with a_ij(z) = sum_k c_i^k w_j^{k-1} phi_k(c_i z)
// (eq. def_aij_computable) evaluated through the moments m_k = sum_j w_j^{k-1} g_j;
// z = 0 uses the collocation weights a(0) = Q.
template <int M>
__device__ __forceinline__ void colloc_weights(const Colloc &co, const double *g, double *I) {
#pragma unroll
  for (int i = 0; i < M; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) s += co.Q[i][j] * g[j];
    I[i] = s;
  }
}

// Gate rows store their reaction terms without the anchor part: G_j holds
// f_e(y_j) - Lambda_n y_j, and g_j = G_j + Lambda_n u (plus f_I, f_E) with u =
// y_{n,0}.  The anchor part is the same at every stage, and sum_j a_ij(z) =
// c_i phi_1(c_i z) (the integral of e^{(c_i - s) z} over [0, c_i]), so it adds
// anc c_i phi_1(c_i z), anc = Lambda_n u, to I_i; phi_1(c_i z) is the first of
// the phi values formed for row i anyway.  A node update then needs neither u
// nor Lambda_n u: in the node-to-node form the anchor parts of R_i - R_{i-1}
// and of the new reaction term cancel.
template <int M>
__device__ __forceinline__ void colloc_integrals(const Colloc &co, double z, const double *g,
                                                 double *I, double anc = 0.0) {
  if (z == 0.0) {  // Lambda_n = 0: no anchor part
    colloc_weights<M>(co, g, I);
    return;
  }
  double mom[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) s += co.W[k][j] * g[j];
    mom[k] = s;
  }
#pragma unroll
  for (int i = 0; i < M; ++i) {
    double ph[M];
    phis<M>(co.c[i] * z, co.invfact, ph);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) s += co.cpow[i][k + 1] * ph[k] * mom[k];
    I[i] = s + anc * co.c[i] * ph[0];
  }
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

// DPP copy of a double between lanes of a wave (two 32-bit moves); a lane
// whose source lies outside its row, or whose row the mask leaves out, reads
// `fill`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double v, double fill) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned long long f = (unsigned long long)__double_as_longlong(fill);
  const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)f, (int)(unsigned)b, CTRL, ROW_MASK,
                                             0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(f >> 32), (int)(unsigned)(b >> 32),
                                             CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(
      (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo));
}

// Wave reduction in registers (DPP, no LDS), in a fixed order, result in lane
// 63: windows of 2, 4, 8 and 16 lanes within each row of 16 (row_shr 1, 2, 4,
// 8), then row 0's total into row 1 and row 2's into row 3 (row_bcast 15), then
// rows 0-1 into row 3 (row_bcast 31).
template <class Op>
__device__ __forceinline__ double wave_reduce(double v, double id, Op op) {
  v = op(v, dpp_d<0x111, 0xf>(v, id));
  v = op(v, dpp_d<0x112, 0xf>(v, id));
  v = op(v, dpp_d<0x114, 0xf>(v, id));
  v = op(v, dpp_d<0x118, 0xf>(v, id));
  v = op(v, dpp_d<0x142, 0xa>(v, id));
  v = op(v, dpp_d<0x143, 0xc>(v, id));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
  return wave_reduce(v, 0.0, [](double a, double b) { return a + b; });
}

// NaN-propagating maximum
__device__ __forceinline__ double nmax(double a, double b) { return (b != b || b > a) ? b : a; }

__device__ __forceinline__ double wave_max(double v) {
  return wave_reduce(v, -INFINITY, nmax);
}

// Sum over the block (BLOCK threads); the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 63) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < BLOCK / 64; ++k) t += lds[k];
  }
  __syncthreads();
  return t;
}

__device__ __forceinline__ double block_max(double v, double *lds) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 63) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    t = lds[0];
#pragma unroll
    for (int k = 1; k < BLOCK / 64; ++k) t = nmax(t, lds[k]);
  }
  __syncthreads();
  return t;
}

// N sums over the block at once, every thread receiving all of them (the wave
// reductions interleave; one exchange through lds, which holds N * BLOCK/64
// doubles; the waves' totals are added in wave order, as block_sum does).
// Partial sums over blocks are combined the same way: each block of a kernel
// writes its partials, and every block of the next kernel adds them in the same
// fixed order and obtains the same value, so reductions need no atomics and no
// cross-block fences.
template <int N, int NT = BLOCK>
__device__ __forceinline__ void block_sums(double (&v)[N], double *lds) {
  constexpr int NW = NT / 64;
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = wave_sum(v[q]);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) {
#pragma unroll
    for (int q = 0; q < N; ++q) lds[q * NW + w] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) t += lds[q * NW + k];
    v[q] = t;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// diffusion operator K = (chi Cm)^-1 A, cell-centred, no-flux
// ---------------------------------------------------------------------------

struct Ijk {
  int ix, iy, iz;
};
__device__ __forceinline__ Ijk ijk(const Grid &g, int64_t p) {
  Ijk r;
  const uint32_t pu = (uint32_t)p;  // node indices are below 2^31
  const uint32_t q = fastdiv(pu, g.fx);
  r.ix = (int)(pu - q * (uint32_t)g.nx);
  const uint32_t q2 = fastdiv(q, g.fy);
  r.iy = (int)(q - q2 * (uint32_t)g.ny);
  r.iz = (int)q2;
  return r;
}

// Mesh of slice n: the launch's grid, or the tissue's own for a ragged batch.
__device__ __forceinline__ Grid slice_grid(const Grid &g, int n) {
  if (g.rag == nullptr) return g;
  Grid r = g;
  const int32_t *d = g.rag + RAG * n;
  r.nx = d[0];
  r.ny = d[1];
  r.nz = d[2];
  r.fx = FastDiv{(uint32_t)d[3], d[4], d[5]};
  r.fy = FastDiv{(uint32_t)d[6], d[7], d[8]};
  r.N = (int64_t)r.nx * r.ny * r.nz;
  if (g.kx) r.kx = g.kx + n * g.Np;
  if (g.ky) r.ky = g.ky + n * g.Np;
  if (g.kz) r.kz = g.kz + n * g.Np;
  return r;
}

// (K v)_p with v given through val(k, c_k), c_k the grid coordinates of
// neighbour k (so callers can form v on the fly, also from its own stencil).
template <int DIM, bool PN, class Val>
__device__ __forceinline__ double applyK_nb(const Grid &g, int64_t p, const Ijk &c, double vc,
                                            Val &&val) {
  const Ijk xm{c.ix - 1, c.iy, c.iz}, xp{c.ix + 1, c.iy, c.iz};
  const Ijk ym{c.ix, c.iy - 1, c.iz}, yp{c.ix, c.iy + 1, c.iz};
  const Ijk zm{c.ix, c.iy, c.iz - 1}, zp{c.ix, c.iy, c.iz + 1};
  if (PN) {
    double acc = 0.0;
    if (c.ix > 0) acc += g.kx[p - 1] * (val(p - 1, xm) - vc);
    if (c.ix < g.nx - 1) acc += g.kx[p] * (val(p + 1, xp) - vc);
    if (DIM >= 2) {
      if (c.iy > 0) acc += g.ky[p - g.nx] * (val(p - g.nx, ym) - vc);
      if (c.iy < g.ny - 1) acc += g.ky[p] * (val(p + g.nx, yp) - vc);
    }
    if (DIM >= 3) {
      const int64_t pl = (int64_t)g.nx * g.ny;
      if (c.iz > 0) acc += g.kz[p - pl] * (val(p - pl, zm) - vc);
      if (c.iz < g.nz - 1) acc += g.kz[p] * (val(p + pl, zp) - vc);
    }
    return acc;
  }
  double ax = 0.0;
  if (c.ix > 0) ax += val(p - 1, xm) - vc;
  if (c.ix < g.nx - 1) ax += val(p + 1, xp) - vc;
  double acc = g.cx * ax;
  if (DIM >= 2) {
    double ay = 0.0;
    if (c.iy > 0) ay += val(p - g.nx, ym) - vc;
    if (c.iy < g.ny - 1) ay += val(p + g.nx, yp) - vc;
    acc += g.cy * ay;
  }
  if (DIM >= 3) {
    const int64_t pl = (int64_t)g.nx * g.ny;
    double az = 0.0;
    if (c.iz > 0) az += val(p - pl, zm) - vc;
    if (c.iz < g.nz - 1) az += val(p + pl, zp) - vc;
    acc += g.cz * az;
  }
  return acc;
}

// (K v)_p with v given through val(k) (so callers can form v on the fly).
template <int DIM, bool PN, class Val>
__device__ __forceinline__ double applyK(const Grid &g, int64_t p, const Ijk &c, double vc,
                                         Val &&val) {
  return applyK_nb<DIM, PN>(g, p, c, vc, [&](int64_t k, const Ijk &) { return val(k); });
}

#define HSDC_DISPATCH_OP(g, ...)                                    \
  do {                                                              \
    const bool pn_ = (g).kx != nullptr;                             \
    if ((g).dim == 1) {                                             \
      if (pn_) { constexpr int DIM = 1; constexpr bool PN = true; __VA_ARGS__; }  \
      else { constexpr int DIM = 1; constexpr bool PN = false; __VA_ARGS__; }     \
    } else if ((g).dim == 2) {                                      \
      if (pn_) { constexpr int DIM = 2; constexpr bool PN = true; __VA_ARGS__; }  \
      else { constexpr int DIM = 2; constexpr bool PN = false; __VA_ARGS__; }     \
    } else {                                                        \
      if (pn_) { constexpr int DIM = 3; constexpr bool PN = true; __VA_ARGS__; }  \
      else { constexpr int DIM = 3; constexpr bool PN = false; __VA_ARGS__; }     \
    }                                                               \
  } while (0)

#define HSDC_DISPATCH_M(M_, ...)                               \
  do {                                                         \
    switch (M_) {                                              \
      case 1: { constexpr int M = 1; __VA_ARGS__; } break;     \
      case 2: { constexpr int M = 2; __VA_ARGS__; } break;     \
      case 3: { constexpr int M = 3; __VA_ARGS__; } break;     \
      case 4: { constexpr int M = 4; __VA_ARGS__; } break;     \
      case 5: { constexpr int M = 5; __VA_ARGS__; } break;     \
      case 6: { constexpr int M = 6; __VA_ARGS__; } break;     \
      case 7: { constexpr int M = 7; __VA_ARGS__; } break;     \
      case 8: { constexpr int M = 8; __VA_ARGS__; } break;     \
      default: return hipErrorInvalidValue;                    \
    }                                                          \
  } while (0)

static inline unsigned nblocks(int64_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

// Workgroups are dealt to the 8 XCDs round-robin in launch order, and each XCD
// has its own L2.  For a grid whose x extent nbx is a multiple of 8, block x
// runs on XCD x % 8; mapping it to node block (x % 8) nbx/8 + x / 8 gives every
// XCD one contiguous range of nodes, so data shared by neighbouring node blocks
// stays in one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_node_block(int64_t bx, int64_t nbx) {
  return (bx % kXcds) * (nbx / kXcds) + bx / kXcds;
}
static inline unsigned nblocks_xcd(int64_t n) {
  const unsigned nb = nblocks(n);
  return (nb + kXcds - 1) / kXcds * kXcds;
}

// Node block of a kernel's block: XCD-ordered (a stencil's neighbour rows are
// read by adjacent node blocks, and the node update, the CG start and the CG
// iterations then place each node block on the same XCD) unless the grid's x
// extent is not a multiple of 8 or the slices are a ragged batch (whose partial
// sums are read in launch order by active block).  A block stores its partial
// sums at its node block's index, so every reduction adds the same partials in
// the same order whatever the placement (a batch's tissue and its own single
// context agree bitwise).
__device__ __forceinline__ int64_t stencil_node_block(const Grid &g0, int64_t bx, int64_t nbx) {
  return (g0.rag == nullptr && nbx % kXcds == 0) ? xcd_node_block(bx, nbx) : bx;
}


}  // namespace hsdc
