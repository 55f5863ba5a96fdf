// ttp06_device.h -- ten Tusscher-Panfilov 2006 epicardial cell model as
// device functions, one mesh node per lane, FP64.
//
// The paper integrates this model (m1 = 6 auxiliary, m2 = 12 gating variables,
// Sec. 5 model setup) without printing it; the equations follow the model's
// original publication (ten Tusscher & Panfilov, Am. J. Physiol. Heart Circ.
// Physiol. 291:H1088, 2006), epicardial cell, rapid-buffering form of Ca_i,
// Ca_SR and Ca_ss.  Gates are delivered in relaxation form
// dw/dt = Lambda (w - w_inf), Lambda = -1/tau (eq. monodomain_g_lambda).
//
// State order: V, Ca_i, Ca_SR, Ca_ss, Na_i, K_i, Rbar, m, h, j, xr1, xr2, xs,
// r, s, d, f, f2, fCass.  Currents in pA/pF, time in ms.
#pragma once

#include <hip/hip_runtime.h>

namespace ttp06 {

constexpr double kR = 8314.472;       // mJ/(K mol)
constexpr double kT = 310.0;          // K
constexpr double kF = 96485.3415;     // C/mol
constexpr double kRTF = kR * kT / kF; // mV
constexpr double kCap = 0.185;        // uF
constexpr double kVc = 0.016404;      // uL
constexpr double kVsr = 0.001094;
constexpr double kVss = 0.00005468;
constexpr double kKo = 5.4, kNao = 140.0, kCao = 2.0;
constexpr double kGNa = 14.838, kGK1 = 5.405, kGto = 0.294, kGKr = 0.153, kGKs = 0.392;
constexpr double kPKNa = 0.03, kGCaL = 3.980e-5;
constexpr double kNaCa = 1000.0, kGammaNaCa = 0.35, kKmCa = 1.38, kKmNai = 87.5;
constexpr double kKsat = 0.1, kAlphaNaCa = 2.5;
constexpr double kPNaK = 2.724, kKmK = 1.0, kKmNa = 40.0;
constexpr double kGpK = 0.0146, kGpCa = 0.1238, kKpCa = 0.0005;
constexpr double kGbNa = 0.00029, kGbCa = 0.000592;
constexpr double kVmaxUp = 0.006375, kKup = 0.00025, kVrel = 0.102;
constexpr double kK1p = 0.15, kK2p = 0.045, kK3 = 0.060, kK4 = 0.005;
constexpr double kEC = 1.5, kMaxSR = 2.5, kMinSR = 1.0;
constexpr double kVleak = 0.00036, kVxfer = 0.0038;
constexpr double kBufc = 0.2, kKbufc = 0.001, kBufsr = 10.0, kKbufsr = 0.3;
constexpr double kBufss = 0.4, kKbufss = 0.00025;

// Epicardial rest state of the model publication, in state order.
__constant__ double kRest[19] = {
    -85.23, 0.000126, 3.64, 0.00036, 8.604, 136.89, 0.9073,
    0.00172, 0.7444, 0.7045, 0.00621, 0.4712, 0.0095,
    2.42e-8, 0.999998, 3.373e-5, 0.7888, 0.9755, 0.9953};

__device__ __forceinline__ double logistic(double x) { return 1.0 / (1.0 + exp(x)); }

// Steady state and time constant of every gate; calls sink(g, w_inf, tau)
// for g = 0..11 in state order (m, h, j, xr1, xr2, xs, r, s, d, f, f2, fCass).
template <class Sink>
__device__ __forceinline__ void gates(double V, double Ca_ss, Sink &&sink) {
  {  // m
    const double s = logistic((-56.86 - V) / 9.03);
    const double am = logistic((-60.0 - V) / 5.0);
    const double bm = 0.1 * logistic((V + 35.0) / 5.0) + 0.1 * logistic((V - 50.0) / 200.0);
    sink(0, s * s, am * bm);
  }
  const double sh = logistic((V + 71.55) / 7.43);
  const double hj_inf = sh * sh;
  if (V < -40.0) {
    const double ah = 0.057 * exp(-(V + 80.0) / 6.8);
    const double bh = 2.7 * exp(0.079 * V) + 3.1e5 * exp(0.3485 * V);
    sink(1, hj_inf, 1.0 / (ah + bh));
    const double aj = (-2.5428e4 * exp(0.2444 * V) - 6.948e-6 * exp(-0.04391 * V)) * (V + 37.78) /
                      (1.0 + exp(0.311 * (V + 79.23)));
    const double bj = 0.02424 * exp(-0.01052 * V) / (1.0 + exp(-0.1378 * (V + 40.14)));
    sink(2, hj_inf, 1.0 / (aj + bj));
  } else {
    const double bh = 0.77 / (0.13 * (1.0 + exp(-(V + 10.66) / 11.1)));
    sink(1, hj_inf, 1.0 / bh);
    const double bj = 0.6 * exp(0.057 * V) / (1.0 + exp(-0.1 * (V + 32.0)));
    sink(2, hj_inf, 1.0 / bj);
  }
  sink(3, logistic((-26.0 - V) / 7.0),
       (450.0 * logistic((-45.0 - V) / 10.0)) * (6.0 * logistic((V + 30.0) / 11.5)));
  sink(4, logistic((V + 88.0) / 24.0),
       (3.0 * logistic((-60.0 - V) / 20.0)) * (1.12 * logistic((V - 60.0) / 20.0)));
  {  // xs
    const double axs = 1400.0 / sqrt(1.0 + exp((5.0 - V) / 6.0));
    const double bxs = logistic((V - 35.0) / 15.0);
    sink(5, logistic((-5.0 - V) / 14.0), axs * bxs + 80.0);
  }
  {  // r, s (epicardium)
    const double v40 = V + 40.0, v45 = V + 45.0;
    sink(6, logistic((20.0 - V) / 6.0), 9.5 * exp(-(v40 * v40) / 1800.0) + 0.8);
    sink(7, logistic((V + 20.0) / 5.0),
         85.0 * exp(-(v45 * v45) / 320.0) + 5.0 * logistic((V - 20.0) / 5.0) + 3.0);
  }
  {  // d
    const double ad = 1.4 * logistic((-35.0 - V) / 13.0) + 0.25;
    const double bd = 1.4 * logistic((V + 5.0) / 5.0);
    const double gd = logistic((50.0 - V) / 20.0);
    sink(8, logistic((-8.0 - V) / 7.5), ad * bd + gd);
  }
  {  // f, f2
    const double v27 = V + 27.0, v25 = V + 25.0;
    sink(9, logistic((V + 20.0) / 7.0),
         1102.5 * exp(-(v27 * v27) / 225.0) + 200.0 * logistic((13.0 - V) / 10.0) +
             180.0 * logistic((V + 30.0) / 10.0) + 20.0);
    sink(10, 0.67 * logistic((V + 35.0) / 7.0) + 0.33,
         600.0 * exp(-(v25 * v25) / 170.0) + 31.0 * logistic((25.0 - V) / 10.0) +
             16.0 * logistic((V + 30.0) / 10.0));
  }
  {  // fCass
    const double q = (Ca_ss / 0.05) * (Ca_ss / 0.05);
    sink(11, 0.6 / (1.0 + q) + 0.4, 80.0 / (1.0 + q) + 2.0);
  }
}

// Total ionic current I_ion (pA/pF) and the auxiliary derivatives h_a
// (Ca_i, Ca_SR, Ca_ss, Na_i, K_i, Rbar).  gs scales G_Na, G_CaL, G_Kr.
__device__ __forceinline__ void currents(const double *y, double gs0, double gs1, double gs2,
                                         double &I_ion, double *ha) {
  const double V = y[0], Ca_i = y[1], Ca_sr = y[2], Ca_ss = y[3], Na_i = y[4], K_i = y[5];
  const double Rbar = y[6];
  const double m = y[7], h = y[8], jg = y[9], xr1 = y[10], xr2 = y[11], xs = y[12];
  const double r = y[13], s = y[14], d = y[15], f = y[16], f2 = y[17], fcass = y[18];

  const double E_Na = kRTF * log(kNao / Na_i);
  const double E_K = kRTF * log(kKo / K_i);
  const double E_Ks = kRTF * log((kKo + kPKNa * kNao) / (K_i + kPKNa * Na_i));
  const double E_Ca = 0.5 * kRTF * log(kCao / Ca_i);

  const double I_Na = gs0 * kGNa * (m * m * m) * h * jg * (V - E_Na);
  const double vek = V - E_K;
  const double a_k1 = 0.1 / (1.0 + exp(0.06 * (vek - 200.0)));
  const double b_k1 = (3.0 * exp(0.0002 * (vek + 100.0)) + exp(0.1 * (vek - 10.0))) /
                      (1.0 + exp(-0.5 * vek));
  const double sq = sqrt(kKo / 5.4);
  const double I_K1 = kGK1 * sq * (a_k1 / (a_k1 + b_k1)) * vek;
  const double I_to = kGto * r * s * vek;
  const double I_Kr = gs2 * kGKr * sq * xr1 * xr2 * vek;
  const double I_Ks = kGKs * xs * xs * (V - E_Ks);
  // L-type: (V - 15)/(e^u - 1) with u = 2 (V - 15)/RTF is (RTF/2) u/(e^u - 1),
  // written through expm1 so that u = 0 is regular.
  const double u = 2.0 * (V - 15.0) / kRTF;
  const double ratio = (u == 0.0) ? 1.0 : expm1(u) / u;
  const double I_CaL = gs1 * kGCaL * d * f * f2 * fcass * 4.0 * kF * (0.5 / ratio) *
                       (0.25 * Ca_ss * exp(u) - kCao);
  const double vfrt = V / kRTF;
  const double e_g = exp(kGammaNaCa * vfrt), e_g1 = exp((kGammaNaCa - 1.0) * vfrt);
  const double nai3 = Na_i * Na_i * Na_i;
  const double I_NaCa =
      kNaCa * (e_g * nai3 * kCao - e_g1 * (kNao * kNao * kNao) * Ca_i * kAlphaNaCa) /
      ((kKmNai * kKmNai * kKmNai + kNao * kNao * kNao) * (kKmCa + kCao) * (1.0 + kKsat * e_g1));
  const double I_NaK = kPNaK * kKo / (kKo + kKmK) * Na_i / (Na_i + kKmNa) /
                       (1.0 + 0.1245 * exp(-0.1 * vfrt) + 0.0353 * exp(-vfrt));
  const double I_pCa = kGpCa * Ca_i / (kKpCa + Ca_i);
  const double I_pK = kGpK * vek / (1.0 + exp((25.0 - V) / 5.98));
  const double I_bNa = kGbNa * (V - E_Na);
  const double I_bCa = kGbCa * (V - E_Ca);
  I_ion = I_Na + I_K1 + I_to + I_Kr + I_Ks + I_CaL + I_NaCa + I_NaK + I_pCa + I_pK + I_bNa + I_bCa;

  const double k_casr = kMaxSR - (kMaxSR - kMinSR) / (1.0 + (kEC / Ca_sr) * (kEC / Ca_sr));
  const double k1 = kK1p / k_casr, k2 = kK2p * k_casr;
  const double css2 = Ca_ss * Ca_ss;
  const double O = k1 * css2 * Rbar / (kK3 + k1 * css2);
  const double I_rel = kVrel * O * (Ca_sr - Ca_ss);
  const double I_up = kVmaxUp / (1.0 + (kKup * kKup) / (Ca_i * Ca_i));
  const double I_leak = kVleak * (Ca_sr - Ca_i);
  const double I_xfer = kVxfer * (Ca_ss - Ca_i);
  const double ci_k = Ca_i + kKbufc, csr_k = Ca_sr + kKbufsr, css_k = Ca_ss + kKbufss;
  const double buf_c = 1.0 / (1.0 + kBufc * kKbufc / (ci_k * ci_k));
  const double buf_sr = 1.0 / (1.0 + kBufsr * kKbufsr / (csr_k * csr_k));
  const double buf_ss = 1.0 / (1.0 + kBufss * kKbufss / (css_k * css_k));
  const double cvf = kCap / (kVc * kF);
  ha[0] = buf_c * ((I_leak - I_up) * kVsr / kVc + I_xfer -
                   (I_bCa + I_pCa - 2.0 * I_NaCa) * kCap / (2.0 * kVc * kF));
  ha[1] = buf_sr * (I_up - (I_rel + I_leak));
  ha[2] = buf_ss * (-I_CaL * kCap / (2.0 * kVss * kF) + I_rel * kVsr / kVss - I_xfer * kVc / kVss);
  ha[3] = -(I_Na + I_bNa + 3.0 * I_NaK + 3.0 * I_NaCa) * cvf;
  ha[4] = -(I_K1 + I_to + I_Kr + I_Ks - 2.0 * I_NaK + I_pK) * cvf;
  ha[5] = -k2 * Ca_ss * Rbar + kK4 * (1.0 - Rbar);
}

}  // namespace ttp06
