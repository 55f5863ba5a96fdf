// ttp06_device.h -- ten Tusscher-Panfilov 2006 epicardial cell model as
// device functions, one mesh node per lane, templated on the arithmetic type
// (double on the fine level, float on an FP32 coarse level).
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

template <class R>
__device__ __forceinline__ R logistic(R x) { return R(1) / (R(1) + exp(x)); }

// Divisions by model constants are written as products with the constant's
// reciprocal (folded at compile time), and quotients are combined where the
// algebra allows: an FP64 division costs about ten instructions, and the
// results differ from the printed forms by rounding only.

// Steady state and rate 1/tau of every gate; calls sink(g, w_inf, 1/tau) for
// g = 0..11 in state order (m, h, j, xr1, xr2, xs, r, s, d, f, f2, fCass).
// Exponentials of V with slopes 1/20, 1/10, 1/5 (e^{V/20} and its square and
// fourth power), 1/7 and -1/6 are formed once and scaled by constant factors
// e^{b} (written out below as literals): e^{aV + b} = e^{b} e^{aV}, and
// 1/(1 + e^{b} / E) = E / (E + e^{b}) needs no reciprocal of E.  An FP64
// exponential costs about thirty instructions, a product one.
// fCass, the one gate driven by Ca_ss alone: w_inf = 0.6 / (1 + q) + 0.4,
// tau = 80 / (1 + q) + 2, q = (Ca_ss / 0.05)^2.
template <class R>
__host__ __device__ __forceinline__ void fcass_gate(R Ca_ss, R &inf, R &rate) {
  const R q = (Ca_ss * R(20.0)) * (Ca_ss * R(20.0));
  const R iq = R(1.0) / (R(1.0) + q);
  inf = R(0.6) * iq + R(0.4);
  rate = (R(1.0) + q) / (R(82.0) + R(2.0) * q);
}

template <class R, class Sink>
__device__ __forceinline__ void gates(R V, R Ca_ss, Sink &&sink) {
  const R E20 = exp(V * R(0.05));  // e^{V/20}
  const R E10 = E20 * E20;         // e^{V/10}
  const R E5 = E10 * E10;          // e^{V/5}
  const R E7 = exp(V * R(1.0 / 7.0));
  const R E6m = exp(V * R(-1.0 / 6.0));
  {  // m: alpha = 1/(1 + e^{(-60 - V)/5}), beta's first term 0.1/(1 + e^{(V + 35)/5})
    const R s = logistic((-R(56.86) - V) * R(1.0 / 9.03));
    const R am = E5 / (E5 + R(6.14421235332821e-06));  // e^-12
    const R bm = R(0.1) / (R(1.0) + R(1096.6331584284585) * E5) +  // e^7
                 R(0.1) * logistic((V - R(50.0)) * R(0.005));
    sink(0, s * s, R(1.0) / (am * bm));
  }
  const R sh = logistic((V + R(71.55)) * R(1.0 / 7.43));
  const R hj_inf = sh * sh;
  if (V < -R(40.0)) {
    const R ah = R(0.057) * exp((V + R(80.0)) * R(-1.0 / 6.8));
    const R bh = R(2.7) * exp(R(0.079) * V) + R(3.1e5) * exp(R(0.3485) * V);
    sink(1, hj_inf, ah + bh);
    const R aj = (-R(2.5428e4) * exp(R(0.2444) * V) - R(6.948e-6) * exp(-R(0.04391) * V)) * (V + R(37.78)) /
                 (R(1.0) + exp(R(0.311) * (V + R(79.23))));
    const R bj = R(0.02424) * exp(-R(0.01052) * V) / (R(1.0) + exp(-R(0.1378) * (V + R(40.14))));
    sink(2, hj_inf, aj + bj);
  } else {
    // beta_h = 0.77 / (0.13 (1 + e^{-(V + 10.66)/11.1})), alpha_h = 0
    sink(1, hj_inf, R(0.77 / 0.13) / (R(1.0) + exp((V + R(10.66)) * R(-1.0 / 11.1))));
    // beta_j = 0.6 e^{0.057 V} / (1 + e^{-(V + 32)/10}), alpha_j = 0
    sink(2, hj_inf, R(0.6) * exp(R(0.057) * V) * E10 / (E10 + R(0.04076220397836621)));  // e^-3.2
  }
  // xr1: w_inf = 1/(1 + e^{(-26 - V)/7}); 1/tau = 1/(alpha beta) with alpha =
  // 450/(1 + e^{(-45 - V)/10}), beta = 6/(1 + e^{(V + 30)/11.5})
  sink(3, E7 / (E7 + R(0.0243728440732796)),  // e^{-26/7}
       (E10 + R(0.011108996538242306)) *      // e^-4.5
           (R(1.0) + exp((V + R(30.0)) * R(1.0 / 11.5))) / (R(2700.0) * E10));
  // xr2: alpha = 3/(1 + e^{(-60 - V)/20}), beta = 1.12/(1 + e^{(V - 60)/20})
  sink(4, logistic((V + R(88.0)) * R(1.0 / 24.0)),
       (E20 + R(0.049787068367863944)) * (R(1.0) + R(0.049787068367863944) * E20) /  // e^-3
           (R(3.36) * E20));
  {  // xs: alpha = 1400/sqrt(1 + e^{(5 - V)/6})
    const R axs = R(1400.0) / sqrt(R(1.0) + R(2.300975890892825) * E6m);  // e^{5/6}
    const R bxs = logistic((V - R(35.0)) * R(1.0 / 15.0));
    sink(5, logistic((-R(5.0) - V) * R(1.0 / 14.0)), R(1.0) / (axs * bxs + R(80.0)));
  }
  {  // r, s (epicardium)
    const R v40 = V + R(40.0), v45 = V + R(45.0);
    sink(6, R(1.0) / (R(1.0) + R(28.03162489452614) * E6m),  // e^{20/6}
         R(1.0) / (R(9.5) * exp((v40 * v40) * R(-1.0 / 1800.0)) + R(0.8)));
    sink(7, R(1.0) / (R(1.0) + R(54.598150033144236) * E5),  // e^4
         R(1.0) / (R(85.0) * exp((v45 * v45) * R(-1.0 / 320.0)) +
                   R(5.0) / (R(1.0) + R(0.01831563888873418) * E5) + R(3.0)));  // e^-4
  }
  {  // d: beta = 1.4/(1 + e^{(V + 5)/5}), gamma = 1/(1 + e^{(50 - V)/20})
    const R ad = R(1.4) * logistic((-R(35.0) - V) * R(1.0 / 13.0)) + R(0.25);
    const R bd = R(1.4) / (R(1.0) + R(2.718281828459045) * E5);  // e^1
    const R gd = E20 / (E20 + R(12.182493960703473));            // e^2.5
    sink(8, logistic((-R(8.0) - V) * R(1.0 / 7.5)), R(1.0) / (ad * bd + gd));
  }
  {  // f, f2: terms 1/(1 + e^{(13 - V)/10}), 1/(1 + e^{(25 - V)/10}), 1/(1 + e^{(V + 30)/10})
    const R v27 = V + R(27.0), v25 = V + R(25.0);
    const R l30 = R(1.0) / (R(1.0) + R(20.085536923187668) * E10);  // e^3
    sink(9, R(1.0) / (R(1.0) + R(17.41170806332765) * E7),         // e^{20/7}
         R(1.0) / (R(1102.5) * exp((v27 * v27) * R(-1.0 / 225.0)) +
                   R(200.0) * E10 / (E10 + R(3.6692966676192444)) +  // e^1.3
                   R(180.0) * l30 + R(20.0)));
    sink(10, R(0.67) / (R(1.0) + R(148.4131591025766) * E7) + R(0.33),  // e^5
         R(1.0) / (R(600.0) * exp((v25 * v25) * R(-1.0 / 170.0)) +
                   R(31.0) * E10 / (E10 + R(12.182493960703473)) +  // e^2.5
                   R(16.0) * l30));
  }
  {
    R inf, rate;
    fcass_gate(Ca_ss, inf, rate);
    sink(11, inf, rate);
  }
}

// Total ionic current I_ion (pA/pF) and the auxiliary derivatives h_a
// (Ca_i, Ca_SR, Ca_ss, Na_i, K_i, Rbar).  gs scales G_Na, G_CaL, G_Kr.
template <class R>
__host__ __device__ __forceinline__ void currents(const R *y, R gs0, R gs1, R gs2, R &I_ion,
                                                  R *ha) {
  const R V = y[0], Ca_i = y[1], Ca_sr = y[2], Ca_ss = y[3], Na_i = y[4], K_i = y[5];
  const R Rbar = y[6];
  const R m = y[7], h = y[8], jg = y[9], xr1 = y[10], xr2 = y[11], xs = y[12];
  const R r = y[13], s = y[14], d = y[15], f = y[16], f2 = y[17], fcass = y[18];

  const R E_Na = R(kRTF) * log(R(kNao) / Na_i);
  const R E_K = R(kRTF) * log(R(kKo) / K_i);
  const R E_Ks = R(kRTF) * log((R(kKo) + R(kPKNa) * R(kNao)) / (K_i + R(kPKNa) * Na_i));
  const R E_Ca = R(0.5) * R(kRTF) * log(R(kCao) / Ca_i);

  const R I_Na = gs0 * R(kGNa) * (m * m * m) * h * jg * (V - E_Na);
  const R vek = V - E_K;
  const R a_k1 = R(0.1) / (R(1.0) + exp(R(0.06) * (vek - R(200.0))));
  // beta_K1 = (3 e^{0.0002 (vek + 100)} + e^{0.1 (vek - 10)}) / (1 + e^{-0.5 vek}),
  // with e^{-0.5 vek} = 1 / EK^5, EK = e^{0.1 vek}
  const R EK = exp(R(0.1) * vek);
  const R EK2 = EK * EK;
  const R EK5 = EK2 * EK2 * EK;
  const R b_k1 = (R(3.0) * exp(R(0.0002) * (vek + R(100.0))) + R(0.36787944117144233) * EK) *  // e^-1
                 EK5 / (EK5 + R(1.0));
  const R sq = R(1.0);  // sqrt(K_o / 5.4) with K_o = 5.4 mM
  const R I_K1 = R(kGK1) * sq * (a_k1 / (a_k1 + b_k1)) * vek;
  const R I_to = R(kGto) * r * s * vek;
  const R I_Kr = gs2 * R(kGKr) * sq * xr1 * xr2 * vek;
  const R I_Ks = R(kGKs) * xs * xs * (V - E_Ks);
  // Ev = e^{V F/RT} serves three exponentials: e^u = Ev^2 e^{-30 F/RT} in
  // I_CaL, e^{(gamma - 1) V F/RT} = e^{gamma V F/RT} / Ev in I_NaCa and
  // e^{-V F/RT} = 1 / Ev in I_NaK (the quotients are cleared by multiplying
  // numerator and denominator by Ev).
  const R vfrt = V * R(1.0 / kRTF);
  const R Ev = exp(vfrt);
  // L-type: (V - 15)/(e^u - 1) with u = 2 (V - 15)/RTF is (RTF/2) u/(e^u - 1),
  // written through expm1 so that u = 0 is regular.
  const R u = (V - R(15.0)) * R(2.0 / kRTF);
  const R inv_ratio = (u == R(0.0)) ? R(1.0) : u / expm1(u);
  const R I_CaL = gs1 * R(kGCaL) * d * f * f2 * fcass * R(4.0) * R(kF) * (R(0.5) * inv_ratio) *
                       (R(0.25) * Ca_ss * (Ev * Ev) * R(0.3252969814969026) - R(kCao));  // e^{-30/RTF}
  const R e_g = exp(R(kGammaNaCa) * vfrt);
  const R nai3 = Na_i * Na_i * Na_i;
  const R I_NaCa =
      (e_g * nai3 * R(kCao) * Ev - e_g * (R(kNao) * R(kNao) * R(kNao)) * Ca_i * R(kAlphaNaCa)) *
      R(kNaCa / ((kKmNai * kKmNai * kKmNai + kNao * kNao * kNao) * (kKmCa + kCao))) /
      (Ev + R(kKsat) * e_g);
  const R I_NaK = R(kPNaK * kKo / (kKo + kKmK)) * Na_i * Ev /
                  ((Na_i + R(kKmNa)) * (Ev * (R(1.0) + R(0.1245) * exp(-R(0.1) * vfrt)) + R(0.0353)));
  const R I_pCa = R(kGpCa) * Ca_i / (R(kKpCa) + Ca_i);
  const R I_pK = R(kGpK) * vek / (R(1.0) + exp((R(25.0) - V) * R(1.0 / 5.98)));
  const R I_bNa = R(kGbNa) * (V - E_Na);
  const R I_bCa = R(kGbCa) * (V - E_Ca);
  I_ion = I_Na + I_K1 + I_to + I_Kr + I_Ks + I_CaL + I_NaCa + I_NaK + I_pCa + I_pK + I_bNa + I_bCa;

  // k_casr = max_SR - (max_SR - min_SR) / (1 + (EC / Ca_SR)^2)
  const R csr2 = Ca_sr * Ca_sr;
  const R k_casr = R(kMaxSR) - R(kMaxSR - kMinSR) * csr2 / (csr2 + R(kEC * kEC));
  const R k1 = R(kK1p) / k_casr, k2 = R(kK2p) * k_casr;
  const R css2 = Ca_ss * Ca_ss;
  const R O = k1 * css2 * Rbar / (R(kK3) + k1 * css2);
  const R I_rel = R(kVrel) * O * (Ca_sr - Ca_ss);
  const R ci2 = Ca_i * Ca_i;
  const R I_up = R(kVmaxUp) * ci2 / (ci2 + R(kKup * kKup));
  const R I_leak = R(kVleak) * (Ca_sr - Ca_i);
  const R I_xfer = R(kVxfer) * (Ca_ss - Ca_i);
  // buffer factors 1 / (1 + B K / (c + K)^2) = (c + K)^2 / ((c + K)^2 + B K)
  const R ci_k = Ca_i + R(kKbufc), csr_k = Ca_sr + R(kKbufsr), css_k = Ca_ss + R(kKbufss);
  const R ci_k2 = ci_k * ci_k, csr_k2 = csr_k * csr_k, css_k2 = css_k * css_k;
  const R buf_c = ci_k2 / (ci_k2 + R(kBufc * kKbufc));
  const R buf_sr = csr_k2 / (csr_k2 + R(kBufsr * kKbufsr));
  const R buf_ss = css_k2 / (css_k2 + R(kBufss * kKbufss));
  const R cvf = R(kCap / (kVc * kF));
  ha[0] = buf_c * ((I_leak - I_up) * R(kVsr / kVc) + I_xfer -
                   (I_bCa + I_pCa - R(2.0) * I_NaCa) * R(kCap / (2.0 * kVc * kF)));
  ha[1] = buf_sr * (I_up - (I_rel + I_leak));
  ha[2] = buf_ss * (I_CaL * R(-kCap / (2.0 * kVss * kF)) + I_rel * R(kVsr / kVss) - I_xfer * R(kVc / kVss));
  ha[3] = -(I_Na + I_bNa + R(3.0) * I_NaK + R(3.0) * I_NaCa) * cvf;
  ha[4] = -(I_K1 + I_to + I_Kr + I_Ks - R(2.0) * I_NaK + I_pK) * cvf;
  ha[5] = -k2 * Ca_ss * Rbar + R(kK4) * (R(1.0) - Rbar);
}

}  // namespace ttp06
