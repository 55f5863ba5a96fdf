// hsdc_dct.hip -- the fourth-order diffusion stencil and the direct solve of
// (I - a K) x = b in the DCT-II eigenbasis, for meshes with a uniform
// conductivity tensor (Sec. 2.2: fourth-order finite differences; Sec. 5,
// computational setup: Laplacian solves by DCT-II).
//
// Both stencils (second and fourth order) take the even mirror at the no-flux
// walls of the cell-centred mesh (V_{-1} = V_0, V_{-2} = V_1), so K is
// diagonal in the orthonormal DCT-II basis of every axis: with C[k][p] =
// s_k cos(pi k (p + 1/2) / n) (s_0 = 1/sqrt(n), s_k = sqrt(2/n)),
//   x = (C_z C_y C_x)^T diag(1 / (1 - a (l_x + l_y + l_z))) (C_z C_y C_x) b,
// l_axis the eigenvalue of the axis mode (the stencil's symbol at theta =
// pi k / n times sigma_axis / (dx^2 chi Cm)).  Meshes whose transformed axes
// all have power-of-two lengths take fast transforms (an FFT per pair of mesh
// lines in LDS, the last axis's forward transform, scaling and inverse in one
// launch); other lengths take dense products of the n x n matrix with the
// mesh lines along each axis, run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64): 32 x 32 output tiles per block of sixteen waves,
// the contraction split over the waves (four waves per SIMD hide each other's
// operand loads) and summed in LDS.
#include <hip/hip_runtime.h>

#include "hsdc_device.h"
#include "hsdc_internal.h"

namespace hsdc {

// ---------------------------------------------------------------------------
// fourth-order stencil, uniform sigma
// ---------------------------------------------------------------------------

// Mirror of index q into [0, n) about the walls at -1/2 and n - 1/2 (n >= 2).
__device__ __forceinline__ int mirror(int q, int n) {
  return q < 0 ? -1 - q : (q >= n ? 2 * n - 1 - q : q);
}

// (K v)_p: per active axis c_axis (16 ((v_-1 - v_0) + (v_+1 - v_0))
// - ((v_-2 - v_0) + (v_+2 - v_0))) / 12 over the mirrored neighbours.
template <int DIM>
__device__ __forceinline__ double applyK4(const Grid &g, int64_t p, const Ijk &c, const double *v) {
  const double vc = v[p];
  double acc = 0.0;
  const int nn[3] = {g.nx, g.ny, g.nz}, ci[3] = {c.ix, c.iy, c.iz};
  const int64_t st[3] = {1, (int64_t)g.nx, (int64_t)g.nx * g.ny};
  const double ca[3] = {g.cx, g.cy, g.cz};
#pragma unroll
  for (int ax = 0; ax < DIM; ++ax) {
    const int n = nn[ax];
    if (n < 2) continue;
    const int i = ci[ax];
    const int64_t base = p - (int64_t)i * st[ax];
    const double m1 = v[base + mirror(i - 1, n) * st[ax]] - vc;
    const double p1 = v[base + mirror(i + 1, n) * st[ax]] - vc;
    const double m2 = v[base + mirror(mirror(i - 2, n), n) * st[ax]] - vc;
    const double p2 = v[base + mirror(mirror(i + 2, n), n) * st[ax]] - vc;
    acc += ca[ax] * ((16.0 * (m1 + p1) - (m2 + p2)) * (1.0 / 12.0));
  }
  return acc;
}

template <int DIM>
__global__ void __launch_bounds__(BLOCK) k_spmv4_stages(Grid g, const double *Y, int64_t sY,
                                                        int64_t sS, double *FV, int64_t sFV,
                                                        int slice0, int stage0) {
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (p >= g.N) return;
  const int n = slice0 + blockIdx.z, j = stage0 + blockIdx.y;
  const double *v = Y + n * sY + j * sS;
  FV[n * sFV + j * g.Np + p] = applyK4<DIM>(g, p, ijk(g, p), v);
}

hipError_t launch_spmv4_stages(hipStream_t s, const Grid &g, const double *Y, int64_t sY,
                               int64_t sS, double *FV, int64_t sFV, int slice0, int nslices,
                               int stage0, int nstages) {
  if (nslices <= 0 || nstages <= 0) return hipSuccess;
  if (g.kx != nullptr || g.rag != nullptr) return hipErrorInvalidValue;
  const dim3 grid(nblocks(g.N), nstages, nslices);
  if (g.dim == 1)
    hipLaunchKernelGGL(k_spmv4_stages<1>, grid, dim3(BLOCK), 0, s, g, Y, sY, sS, FV, sFV, slice0,
                       stage0);
  else if (g.dim == 2)
    hipLaunchKernelGGL(k_spmv4_stages<2>, grid, dim3(BLOCK), 0, s, g, Y, sY, sS, FV, sFV, slice0,
                       stage0);
  else
    hipLaunchKernelGGL(k_spmv4_stages<3>, grid, dim3(BLOCK), 0, s, g, Y, sY, sS, FV, sFV, slice0,
                       stage0);
  return hipGetLastError();
}

hipError_t launch_apply_K4(hipStream_t s, const Grid &g, const double *v, double *out) {
  return launch_spmv4_stages(s, g, v, 0, 0, out, 0, 0, 1, 0, 1);
}

// ---------------------------------------------------------------------------
// axis transforms on the FP64 matrix cores
// ---------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));

// out = T applied along one axis of n nodes, T given as its transpose TT
// (row-major n x n: TT[p][k] = T[k][p]), so that the lanes of a matrix-core
// fragment read consecutive addresses.
//   ROWS (the x axis, lines contiguous): D[r][k] = sum_p In[r][p] T[k][p] over
//     the rows r of a slice (outer of them);
//   COLS (a slower axis with stride inner): D_o[k][i] = sum_p T[k][p] In_o[p][i]
//     for each of the outer groups o of n x inner values.
// With scale, the result at spectral index (ix, iy, iz) is divided by
// 1 - a (lam_x[ix] + lam_y[iy] + lam_z[iz]).
struct Xform {
  const double *in;
  int64_t sin;  // slice stride of in
  double *out;
  int64_t sout;  // slice stride of out
  const double *TT;
  int n;
  int64_t inner, outer;
  const double *lam[3];
  int nx, ny;
  double a;
  int scale;
};

constexpr int XT = 32;  // output tile edge
constexpr int XW = 16;  // waves per block, each a share of the contraction
constexpr int KU = 4;   // steps of 4 per group of loads

template <bool ROWS>
__global__ void __launch_bounds__(64 * XW) k_xform(Xform f) {
  __shared__ double red[XW][XT * XT];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t M = ROWS ? f.outer : f.n;
  const int64_t Nn = ROWS ? (int64_t)f.n : f.inner;
  const int K = f.n;
  const int64_t tiles_n = (Nn + XT - 1) / XT;
  const int64_t m0 = (int64_t)(blockIdx.x / tiles_n) * XT, n0 = (int64_t)(blockIdx.x % tiles_n) * XT;
  const int64_t slice = ROWS ? blockIdx.y : blockIdx.y / f.outer;
  const int64_t grp = ROWS ? 0 : (blockIdx.y % f.outer) * (int64_t)f.n * f.inner;
  const double *in = f.in + slice * f.sin + grp;
  double *out = f.out + slice * f.sout + grp;
  // the contraction split over the waves, in steps of 4
  const int kq = (K + 4 * XW - 1) / (4 * XW) * 4;
  const int kb = w * kq, ke = min(K, kb + kq);
  const int lr = l & 15, lk = l >> 4;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  // the operands of KU steps of 4 are loaded one group ahead of the matrix-core
  // work on the current group, so a wave keeps 4 KU loads in flight
  auto load = [&](int k0, double (&av)[KU][2], double (&bv)[KU][2]) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int k = k0 + 4 * u + lk;
      const bool kin = k < ke;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int64_t m = m0 + t * 16 + lr, nn = n0 + t * 16 + lr;
        if (ROWS) {
          av[u][t] = (kin && m < M) ? in[m * f.n + k] : 0.0;                // In[r][p]
          bv[u][t] = (kin && nn < Nn) ? f.TT[(int64_t)k * f.n + nn] : 0.0;  // T[k][p] as TT[p][k]
        } else {
          av[u][t] = (kin && m < M) ? f.TT[(int64_t)k * f.n + m] : 0.0;     // T[k][p] as TT[p][k]
          bv[u][t] = (kin && nn < Nn) ? in[(int64_t)k * f.inner + nn] : 0.0;  // In_o[p][i]
        }
      }
    }
  };
  double an[KU][2], bn[KU][2];
  if (kb < ke) load(kb, an, bn);
  for (int k0 = kb; k0 < ke; k0 += 4 * KU) {
    double ac[KU][2], bc[KU][2];
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        ac[u][t] = an[u][t];
        bc[u][t] = bn[u][t];
      }
    if (k0 + 4 * KU < ke) load(k0 + 4 * KU, an, bn);
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[u][i], bc[u][j], acc[i][j], 0, 0, 0);
  }
  // D[m][n] of a 16 x 16 tile: lane n + 16 (m % 4), register m / 4 (operands:
  // A[m][k] in lane m + 16 k, B[k][n] in lane n + 16 k)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        red[w][(i * 16 + 4 * r + lk) * XT + j * 16 + lr] = acc[i][j][r];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < XT * XT / (64 * XW); ++q) {
    const int e = threadIdx.x + 64 * XW * q;
    const int64_t m = m0 + e / XT, nn = n0 + e % XT;
    if (m >= M || nn >= Nn) continue;
    double v = red[0][e];
#pragma unroll
    for (int u = 1; u < XW; ++u) v += red[u][e];
    const int64_t lin = ROWS ? m * f.n + nn : grp + m * f.inner + nn;
    if (f.scale) {
      const int64_t q1 = lin / f.nx;
      const int ix = (int)(lin - q1 * f.nx);
      const int64_t q2 = q1 / f.ny;
      const int iy = (int)(q1 - q2 * f.ny), iz = (int)q2;
      v = v / (1.0 - f.a * ((f.lam[0][ix] + f.lam[1][iy]) + f.lam[2][iz]));
    }
    out[ROWS ? m * f.n + nn : m * f.inner + nn] = v;
  }
}

static hipError_t launch_xform(hipStream_t s, const Xform &f, bool rows, int nslices) {
  const int64_t M = rows ? f.outer : f.n, Nn = rows ? (int64_t)f.n : f.inner;
  const int64_t tiles = ((M + XT - 1) / XT) * ((Nn + XT - 1) / XT);
  const int64_t batch = rows ? nslices : (int64_t)nslices * f.outer;
  if (tiles > 0x7fffffff || batch > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tiles, (unsigned)batch);
  if (rows)
    hipLaunchKernelGGL(k_xform<true>, grid, dim3(64 * XW), 0, s, f);
  else
    hipLaunchKernelGGL(k_xform<false>, grid, dim3(64 * XW), 0, s, f);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fast transforms for lines of a power-of-two length n <= 2048 (Makhoul's
// reordering: the DCT-II of x is Re(e^{-i pi k / 2n} V_k) with V the DFT of
// v = (x_0, x_2, x_4, ..., x_5, x_3, x_1), so one n-point FFT per line)
//
// A block takes two lines a and b (n / 2 threads) and transforms them as one
// complex sequence v_a + i v_b by an in-place radix-2 FFT in LDS; the two
// spectra are separated by conjugate symmetry, A_k = (Z_k + conj Z_{n-k}) / 2,
// B_k = (Z_k - conj Z_{n-k}) / 2i.  The inverse (the orthonormal DCT-III)
// rebuilds V_k = e^{i pi k / 2n} (c_k - i c_{n-k}) from c_k = X_k / s_k
// (c_n = 0), again two lines per complex inverse FFT, and undoes the
// reordering.  Twiddles come from tables formed on the host in long double:
// W_k = e^{-2 pi i k / n} (k < n/2), E_k = e^{-i pi k / 2n}, s_k and 1 / s_k (k < n).
// ---------------------------------------------------------------------------

enum FdctMode { FDCT_FWD = 0, FDCT_INV = 1, FDCT_SOLVE = 2 };

struct Fdct {
  const double *in;
  int64_t sin;  // slice stride of in
  double *out;
  int64_t sout;
  const double *tab;  // W (n/2 complex), E (n complex), s (n), 1/s (n)
  int n, logn;
  int64_t inner, lines;  // element stride of a line; lines per slice
  // FDCT_SOLVE (the last transformed axis ax): 1 / (1 - a (lam_x + lam_y +
  // lam_z)) per mode
  const double *lam[3];
  int nx, ax;
  double a;
};

__device__ __forceinline__ double2 cmul(double2 u, double2 v) {
  return make_double2(u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x);
}

// In-place radix-2 decimation in time over z (bit-reversed input), T = n / 2
// threads, one butterfly each per stage; CONJ: the inverse (conjugate
// twiddles, no 1/n).  W holds W_k = e^{-2 pi i k / n}, k < n / 2.  (Radix-4
// steps with n / 4 threads, half the stages and barriers, measured slower:
// the launches are bound by their memory latency, which more waves hide.)
template <bool CONJ>
__device__ __forceinline__ void fft_lds(double2 *z, const double2 *W, int n, int logn) {
  const int t = threadIdx.x;
  for (int s = 0; s < logn; ++s) {
    const int half = 1 << s;
    const int pos = t & (half - 1);
    const int i0 = ((t - pos) << 1) + pos, i1 = i0 + half;
    const double2 wt = W[pos << (logn - 1 - s)];
    const double2 w = make_double2(wt.x, CONJ ? -wt.y : wt.y);
    const double2 x0 = z[i0], x1 = cmul(w, z[i1]);
    z[i0] = make_double2(x0.x + x1.x, x0.y + x1.y);
    z[i1] = make_double2(x0.x - x1.x, x0.y - x1.y);
    // Up to a span of 64 the butterflies of wave w stay in z[128 w, 128 w +
    // 128), so where the next stage's span is 64 or less the wave's own
    // LDS order suffices; wider stages and the last one wait for the block.
    if (half <= 32 && s + 1 < logn) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  }
}

// position of x_j in Makhoul's reordering
__device__ __forceinline__ int mk_pos(int j, int n) { return (j & 1) ? n - 1 - (j >> 1) : j >> 1; }

constexpr int FR = 2;  // indices per thread (n / T)

template <int MODE>
__global__ void __launch_bounds__(1024) k_fdct(Fdct f) {
  extern __shared__ double2 sm2[];  // n complex z, n / 2 twiddles W, then n + n reals
  const int n = f.n, T = n >> 1, t = threadIdx.x;
  double2 *z = sm2, *W = sm2 + n;
  double *xa = reinterpret_cast<double *>(sm2 + n + (n >> 1)), *xb = xa + n;
  // tables: W (n/2 complex), E (n complex), s (n), 1/s (n)
  for (int q = t; q < (n >> 1); q += T) W[q] = make_double2(f.tab[2 * q], f.tab[2 * q + 1]);
  double2 Ek[FR];
  double Sk[FR], ISk[FR], ISr[FR];
#pragma unroll
  for (int i = 0; i < FR; ++i) {
    const int k = t + i * T;
    if (k < n) {
      Ek[i] = make_double2(f.tab[n + 2 * k], f.tab[n + 2 * k + 1]);
      Sk[i] = f.tab[3 * n + k];
      ISk[i] = f.tab[4 * n + k];
      ISr[i] = k ? f.tab[4 * n + n - k] : 0.0;
    }
  }
  const int64_t la = 2 * (int64_t)blockIdx.x, lb = la + 1;
  const bool hb = lb < f.lines;
  const double *in = f.in + blockIdx.z * f.sin;
  double *out = f.out + blockIdx.z * f.sout;
  const int64_t oa = la / f.inner, ob = lb / f.inner;
  const int64_t ra = la - oa * f.inner, rb = lb - ob * f.inner;
  const int64_t ba = oa * n * f.inner + ra;
  const int64_t bb = hb ? ob * n * f.inner + rb : ba;
  const unsigned sh = 32u - (unsigned)f.logn;
  if (MODE != FDCT_INV) {
#pragma unroll
    for (int i = 0; i < FR; ++i) {
      const int j = t + i * T;
      if (j < n) {
        const double va = in[ba + j * f.inner], vb = hb ? in[bb + j * f.inner] : 0.0;
        z[__brev((unsigned)mk_pos(j, n)) >> sh] = make_double2(va, vb);
      }
    }
    __syncthreads();
    fft_lds<false>(z, W, n, f.logn);
    // the last axis: the other axes' modes are the line's position r (x, then
    // y, of the slower axes' lines)
    double lo_a = 0.0, lo_b = 0.0;
    if (MODE == FDCT_SOLVE && f.ax == 1) {
      lo_a = f.lam[0][ra];
      lo_b = f.lam[0][rb];
    } else if (MODE == FDCT_SOLVE && f.ax == 2) {
      lo_a = f.lam[0][ra % f.nx] + f.lam[1][ra / f.nx];
      lo_b = f.lam[0][rb % f.nx] + f.lam[1][rb / f.nx];
    }
#pragma unroll
    for (int i = 0; i < FR; ++i) {
      const int k = t + i * T;
      if (k >= n) continue;
      const double2 Zk = z[k], Zr = z[(n - k) & (n - 1)];
      // A = (Zk + conj Zr) / 2, B = (Zk - conj Zr) / 2i; X = s Re(E A), s Re(E B)
      const double2 A = make_double2(0.5 * (Zk.x + Zr.x), 0.5 * (Zk.y - Zr.y));
      const double2 B = make_double2(0.5 * (Zk.y + Zr.y), -0.5 * (Zk.x - Zr.x));
      const double Xa = Sk[i] * (Ek[i].x * A.x - Ek[i].y * A.y);
      const double Xb = Sk[i] * (Ek[i].x * B.x - Ek[i].y * B.y);
      if (MODE == FDCT_FWD) {
        out[ba + k * f.inner] = Xa;
        if (hb) out[bb + k * f.inner] = Xb;
      } else {
        const double lk = f.lam[f.ax][k];
        xa[k] = Xa / (1.0 - f.a * (lo_a + lk));
        xb[k] = Xb / (1.0 - f.a * (lo_b + lk));
      }
    }
    if (MODE == FDCT_FWD) return;
  } else {
#pragma unroll
    for (int i = 0; i < FR; ++i) {
      const int k = t + i * T;
      if (k < n) {
        xa[k] = in[ba + k * f.inner];
        xb[k] = hb ? in[bb + k * f.inner] : 0.0;
      }
    }
  }
  __syncthreads();
  // V_k = e^{i pi k / 2n} (c_k - i c_{n-k}), c = X / s (c_n = 0); two lines packed
#pragma unroll
  for (int i = 0; i < FR; ++i) {
    const int k = t + i * T;
    if (k >= n) continue;
    const double ca = xa[k] * ISk[i], cb = xb[k] * ISk[i];
    const double da = k ? xa[n - k] * ISr[i] : 0.0, db = k ? xb[n - k] * ISr[i] : 0.0;
    const double2 e = make_double2(Ek[i].x, -Ek[i].y);
    const double2 Ua = cmul(e, make_double2(ca, -da)), Ub = cmul(e, make_double2(cb, -db));
    z[__brev((unsigned)k) >> sh] = make_double2(Ua.x - Ub.y, Ua.y + Ub.x);
  }
  __syncthreads();
  fft_lds<true>(z, W, n, f.logn);
  const double inv_n = 1.0 / n;
#pragma unroll
  for (int i = 0; i < FR; ++i) {
    const int j = t + i * T;
    if (j >= n) continue;
    const double2 q = z[mk_pos(j, n)];
    out[ba + j * f.inner] = q.x * inv_n;
    if (hb) out[bb + j * f.inner] = q.y * inv_n;
  }
}

// Lines longer than 1024 need more than the default 64 KB of dynamic LDS.
hipError_t fdct_setup(int nmax) {
  const int bytes = nmax * 5 * (int)sizeof(double);
  if (bytes <= 65536) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void *)k_fdct<FDCT_FWD>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_fdct<FDCT_INV>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_fdct<FDCT_SOLVE>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return e;
}

static hipError_t launch_fdct(hipStream_t s, const Fdct &f, int mode, int nslices) {
  const int64_t blocks = (f.lines + 1) / 2;
  if (blocks > 0x7fffffff || nslices > 65535 || f.n < 2 || f.n > 2048) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks, 1, (unsigned)nslices), block(f.n / 2);
  const size_t lds = (size_t)f.n * 5 * sizeof(double);  // z, W, two real lines
  switch (mode) {
    case FDCT_FWD: hipLaunchKernelGGL(k_fdct<FDCT_FWD>, grid, block, lds, s, f); break;
    case FDCT_INV: hipLaunchKernelGGL(k_fdct<FDCT_INV>, grid, block, lds, s, f); break;
    default: hipLaunchKernelGGL(k_fdct<FDCT_SOLVE>, grid, block, lds, s, f); break;
  }
  return hipGetLastError();
}

hipError_t launch_dct_solve(hipStream_t s, const Grid &g, const DctPlan &d, double a,
                            const double *b, int64_t sb, double *x, int64_t sx, double *t1,
                            double *t2, int64_t st, int nslices) {
  if (nslices <= 0) return hipSuccess;
  if (g.kx != nullptr || g.rag != nullptr) return hipErrorInvalidValue;
  const int nn[3] = {g.nx, g.ny, g.nz};
  // axes transformed: x always, y and z when they have more than one node
  int axes[3], na = 0;
  for (int ax = 0; ax < 3; ++ax)
    if (ax == 0 || nn[ax] > 1) axes[na++] = ax;
  const int64_t N = g.N;
  if (d.fast) {
    // forward along all axes but the last, the last one forward, scaled and
    // back in one kernel, then back along the others in reverse order
    auto mk = [&](int ax, const double *in, int64_t sin, double *out, int64_t sout) {
      Fdct f{};
      f.in = in;
      f.sin = sin;
      f.out = out;
      f.sout = sout;
      f.tab = d.ft[ax];
      f.n = nn[ax];
      f.logn = 31 - __builtin_clz((unsigned)nn[ax]);
      f.inner = ax == 0 ? 1 : (ax == 1 ? (int64_t)g.nx : (int64_t)g.nx * g.ny);
      f.lines = N / nn[ax];
      for (int q = 0; q < 3; ++q) f.lam[q] = d.lam[q];
      f.nx = g.nx;
      f.ax = ax;
      f.a = a;
      return f;
    };
    const double *cur = b;
    int64_t scur = sb;
    double *bufs[2] = {t1, t2};
    int nb = 0;
    for (int q = 0; q < na - 1; ++q) {
      double *o = bufs[nb];
      nb ^= 1;
      hipError_t e = launch_fdct(s, mk(axes[q], cur, scur, o, st), FDCT_FWD, nslices);
      if (e != hipSuccess) return e;
      cur = o;
      scur = st;
    }
    for (int q = na - 1; q >= 0; --q) {
      double *o = q == 0 ? x : bufs[nb];
      const int64_t so = q == 0 ? sx : st;
      nb ^= 1;
      hipError_t e = launch_fdct(s, mk(axes[q], cur, scur, o, so),
                                 q == na - 1 ? FDCT_SOLVE : FDCT_INV, nslices);
      if (e != hipSuccess) return e;
      cur = o;
      scur = so;
    }
    return hipSuccess;
  }
  auto make = [&](int ax, bool forward, const double *in, int64_t sin, double *out, int64_t sout,
                  bool scale) {
    Xform f{};
    f.in = in;
    f.sin = sin;
    f.out = out;
    f.sout = sout;
    // forward: T = C, given as TT = C^T; inverse: T = C^T, given as TT = C
    f.TT = forward ? d.CT[ax] : d.C[ax];
    f.n = nn[ax];
    f.inner = ax == 0 ? 1 : (ax == 1 ? (int64_t)g.nx : (int64_t)g.nx * g.ny);
    f.outer = ax == 0 ? N / g.nx : N / ((int64_t)nn[ax] * f.inner);
    for (int q = 0; q < 3; ++q) f.lam[q] = d.lam[q];
    f.nx = g.nx;
    f.ny = g.ny;
    f.a = a;
    f.scale = scale ? 1 : 0;
    return f;
  };
  // forward over the axes, the last one scaling; then back in reverse order
  const double *cur = b;
  int64_t scur = sb;
  double *bufs[2] = {t1, t2};
  int nb = 0;
  for (int q = 0; q < na; ++q) {
    double *o = bufs[nb];
    nb ^= 1;
    hipError_t e = launch_xform(s, make(axes[q], true, cur, scur, o, st, q == na - 1),
                                axes[q] == 0, nslices);
    if (e != hipSuccess) return e;
    cur = o;
    scur = st;
  }
  for (int q = na - 1; q >= 0; --q) {
    double *o = q == 0 ? x : bufs[nb];
    const int64_t so = q == 0 ? sx : st;
    nb ^= 1;
    hipError_t e = launch_xform(s, make(axes[q], false, cur, scur, o, so, false), axes[q] == 0,
                                nslices);
    if (e != hipSuccess) return e;
    cur = o;
    scur = so;
  }
  return hipSuccess;
}

}  // namespace hsdc
