// ttp06_vjp.h -- the transposed Jacobian of the TTP06 currents (ttp06_device.h)
// applied to a cotangent, in one reverse pass: for the outputs I_ion and h_a
// (the auxiliary derivatives) and a cotangent (cI, ch[0..5]),
//   vx += d(cI I_ion + sum_k ch_k h_a,k)/dy,   vgs += the same w.r.t. the
// scalings of G_Na, G_CaL, G_Kr.
// I_ion is the sum of the currents and h_a are linear in them with factors
// that depend on the concentrations only (the buffer factors), so the adjoint
// of every current is known before any current is formed.  Each current is
// then formed and taken back through its own inputs in a block of its own,
// which keeps its intermediate values local; the fluxes that the buffer
// factors multiply are gathered on the way for the buffer factors' own
// derivatives at the end.
#pragma once

#include "ttp06_device.h"

namespace ttp06 {

template <class R>
__host__ __device__ __forceinline__ void currents_vjp(const R *y, R gs0, R gs1, R gs2, R cI,
                                                      const R *ch, R *vx, R *vgs) {
  const R V = y[0], Ca_i = y[1], Ca_sr = y[2], Ca_ss = y[3], Na_i = y[4], K_i = y[5];
  const R Rbar = y[6];
  const R iRTF = R(1.0 / kRTF);

  // ---- buffer factors c_k^2 / (c_k^2 + B K) and the currents' adjoints ----
  const R ci_k = Ca_i + R(kKbufc), csr_k = Ca_sr + R(kKbufsr), css_k = Ca_ss + R(kKbufss);
  const R ci_k2 = ci_k * ci_k, csr_k2 = csr_k * csr_k, css_k2 = css_k * css_k;
  const R bkc = R(kBufc * kKbufc), bksr = R(kBufsr * kKbufsr), bkss = R(kBufss * kKbufss);
  const R dbc = ci_k2 + bkc, dbsr = csr_k2 + bksr, dbss = css_k2 + bkss;
  const R cvf = R(kCap / (kVc * kF));
  const R c0 = R(kCap / (2.0 * kVc * kF));
  const R c2 = R(kCap / (2.0 * kVss * kF));
  const R a0 = ch[0] * ci_k2 / dbc, a1 = ch[1] * csr_k2 / dbsr, a2 = ch[2] * css_k2 / dbss;
  const R aNa = cI - ch[3] * cvf;                                   // I_Na, I_bNa
  const R aK = cI - ch[4] * cvf;                                    // I_K1, I_to, I_Kr, I_Ks, I_pK
  const R aNaK = cI - R(3.0) * ch[3] * cvf + R(2.0) * ch[4] * cvf;
  const R aNaCa = cI + R(2.0) * c0 * a0 - R(3.0) * ch[3] * cvf;
  const R aCaL = cI - c2 * a2;
  const R apCa = cI - c0 * a0;                                      // I_pCa, I_bCa

  // fluxes the buffer factors multiply: h_a,0..2 = buf X0..X2
  R X0 = R(0.0), X1 = R(0.0), X2 = R(0.0);
  R gV = R(0.0), gCi = R(0.0), gCsr = R(0.0), gCss = R(0.0), gNa = R(0.0), gK = R(0.0),
    gR = R(0.0);

  // I_Na = gs0 GNa m^3 h j (V - E_Na); I_bNa = GbNa (V - E_Na)
  {
    const R m = y[7], h = y[8], jg = y[9];
    const R vna = V - R(kRTF) * log(R(kNao) / Na_i);
    const R m3hj = (m * m * m) * h * jg;
    const R gna = gs0 * R(kGNa);
    const R t = aNa * (gna * m3hj + R(kGbNa));
    gV += t;
    gNa += t * R(kRTF) / Na_i;  // dE_Na/dNa_i = -RTF / Na_i
    vx[7] += aNa * gna * R(3.0) * m * m * h * jg * vna;
    vx[8] += aNa * gna * (m * m * m) * jg * vna;
    vx[9] += aNa * gna * (m * m * m) * h * vna;
    vgs[0] += aNa * R(kGNa) * m3hj * vna;
  }
  // the currents driven by V - E_K: I_K1, I_to, I_Kr, I_pK
  {
    const R vek = V - R(kRTF) * log(R(kKo) / K_i);
    R gvek;  // adjoint of vek
    {
      // I_K1 = GK1 x_k1 vek, x_k1 = a / (a + b)
      const R e1 = exp(R(0.06) * (vek - R(200.0)));
      const R a_k1 = R(0.1) / (R(1.0) + e1);
      const R EK = exp(R(0.1) * vek);
      const R EK2 = EK * EK;
      const R EK5 = EK2 * EK2 * EK;
      const R e2 = exp(R(0.0002) * (vek + R(100.0)));
      const R Ab = R(3.0) * e2 + R(0.36787944117144233) * EK;
      const R Bb = EK5 / (EK5 + R(1.0));
      const R b_k1 = Ab * Bb;
      const R ab = a_k1 + b_k1;
      const R da = -R(0.1) * R(0.06) * e1 / ((R(1.0) + e1) * (R(1.0) + e1));
      const R dAb = R(3.0) * R(0.0002) * e2 + R(0.36787944117144233) * R(0.1) * EK;
      const R dBb = R(0.5) * EK5 / ((EK5 + R(1.0)) * (EK5 + R(1.0)));
      const R db = dAb * Bb + Ab * dBb;
      const R dx = (da * b_k1 - a_k1 * db) / (ab * ab);
      gvek = aK * R(kGK1) * (dx * vek + a_k1 / ab);
    }
    {
      // I_to = Gto r s vek; I_Kr = gs2 GKr xr1 xr2 vek
      const R xr1 = y[10], xr2 = y[11], r = y[13], s = y[14];
      const R gto = aK * R(kGto);
      const R gkr = aK * gs2 * R(kGKr);
      gvek += gto * r * s + gkr * xr1 * xr2;
      vx[13] += gto * s * vek;
      vx[14] += gto * r * vek;
      vx[10] += gkr * xr2 * vek;
      vx[11] += gkr * xr1 * vek;
      vgs[2] += aK * R(kGKr) * xr1 * xr2 * vek;
    }
    {
      // I_pK = GpK vek / (1 + ep), ep = e^{(25 - V)/5.98}
      const R ep = exp((R(25.0) - V) * R(1.0 / 5.98));
      const R q = R(1.0) / (R(1.0) + ep);
      gvek += aK * R(kGpK) * q;
      gV += aK * R(kGpK) * vek * ep * q * q * R(1.0 / 5.98);
    }
    gV += gvek;
    gK += gvek * R(kRTF) / K_i;  // dE_K/dK_i = -RTF / K_i
  }
  // I_Ks = GKs xs^2 (V - E_Ks)
  {
    const R xs = y[12];
    const R ks_den = K_i + R(kPKNa) * Na_i;
    const R vks = V - R(kRTF) * log((R(kKo) + R(kPKNa) * R(kNao)) / ks_den);
    const R g = aK * R(kGKs);
    const R t = g * xs * xs;
    gV += t;
    gNa += t * R(kRTF) * R(kPKNa) / ks_den;
    gK += t * R(kRTF) / ks_den;
    vx[12] += g * R(2.0) * xs * vks;
  }
  // Ev = e^{V F/RT}, shared by I_CaL, I_NaCa and I_NaK as in currents
  const R vfrt = V * iRTF;
  const R Ev = exp(vfrt);
  // I_CaL = gs1 kcal d f f2 fCass ir(u) Qc
  {
    const R d = y[15], f = y[16], f2 = y[17], fcass = y[18];
    const R u = (V - R(15.0)) * R(2.0 / kRTF);
    R ir, dir;  // u / (e^u - 1) and its derivative in u
    if (fabs(u) < R(1e-4)) {
      ir = R(1.0) - u * R(0.5) + u * u * R(1.0 / 12.0);
      dir = -R(0.5) + u * R(1.0 / 6.0);
    } else {
      const R em1 = expm1(u);
      ir = u / em1;
      dir = (em1 - u * (em1 + R(1.0))) / (em1 * em1);
    }
    if (u == R(0.0)) ir = R(1.0);  // as in currents
    const R kcal = R(kGCaL) * R(4.0) * R(kF) * R(0.5);
    const R E2 = (Ev * Ev) * R(0.3252969814969026);
    const R Qc = R(0.25) * Ca_ss * E2 - R(kCao);
    const R dfff = d * f * f2 * fcass;
    const R irq = ir * Qc;
    X2 -= gs1 * kcal * dfff * irq * c2;
    const R g = aCaL * gs1 * kcal;
    vx[15] += g * f * f2 * fcass * irq;
    vx[16] += g * d * f2 * fcass * irq;
    vx[17] += g * d * f * fcass * irq;
    vx[18] += g * d * f * f2 * irq;
    vgs[1] += aCaL * kcal * dfff * irq;
    const R gd = g * dfff;
    gV += gd * (dir * R(2.0 / kRTF) * Qc + ir * R(0.5) * Ca_ss * E2 * iRTF);
    gCss += gd * ir * R(0.25) * E2;
  }
  // I_NaCa = knc e_g Wn / Den
  {
    const R e_g = exp(R(kGammaNaCa) * vfrt);
    const R nai3 = Na_i * Na_i * Na_i;
    const R knc = R(kNaCa / ((kKmNai * kKmNai * kKmNai + kNao * kNao * kNao) * (kKmCa + kCao)));
    const R Wn = nai3 * R(kCao) * Ev - (R(kNao) * R(kNao) * R(kNao)) * Ca_i * R(kAlphaNaCa);
    const R Num = e_g * Wn;
    const R Den = Ev + R(kKsat) * e_g;
    X0 += R(2.0) * c0 * knc * Num / Den;
    const R dEv = Ev * iRTF, deg = R(kGammaNaCa) * e_g * iRTF;
    const R dNum = deg * Wn + e_g * nai3 * R(kCao) * dEv;
    const R dDen = dEv + R(kKsat) * deg;
    const R g = aNaCa * knc;
    gV += g * (dNum * Den - Num * dDen) / (Den * Den);
    gNa += g * e_g * R(3.0) * Na_i * Na_i * R(kCao) * Ev / Den;
    gCi -= g * e_g * (R(kNao) * R(kNao) * R(kNao)) * R(kAlphaNaCa) / Den;
  }
  // I_NaK = cnak Na_i Ev / ((Na_i + KmNa) D2)
  {
    const R em = exp(-R(0.1) * vfrt);
    const R D2 = Ev * (R(1.0) + R(0.1245) * em) + R(0.0353);
    const R nak_n = Na_i + R(kKmNa);
    const R cnak = R(kPNaK * kKo / (kKo + kKmK));
    const R dEv = Ev * iRTF;
    const R dD2 = dEv * (R(1.0) + R(0.9) * R(0.1245) * em);
    const R g = aNaK * cnak;
    gV += g * Na_i / nak_n * (dEv * D2 - Ev * dD2) / (D2 * D2);
    gNa += g * Ev / D2 * R(kKmNa) / (nak_n * nak_n);
  }
  // I_pCa = GpCa Ca_i / (KpCa + Ca_i); I_bCa = GbCa (V - E_Ca)
  {
    const R kp = R(kKpCa) + Ca_i;
    const R I_pCa = R(kGpCa) * Ca_i / kp;
    const R I_bCa = R(kGbCa) * (V - R(0.5) * R(kRTF) * log(R(kCao) / Ca_i));
    X0 -= (I_bCa + I_pCa) * c0;
    gCi += apCa * R(kGpCa) * R(kKpCa) / (kp * kp);
    gV += apCa * R(kGbCa);
    gCi += apCa * R(kGbCa) * R(0.5) * R(kRTF) / Ca_i;  // dE_Ca/dCa_i = -RTF / (2 Ca_i)
  }
  // SR uptake, leak and the subspace transfer
  {
    const R aup = -R(kVsr / kVc) * a0 + a1;
    const R aleak = R(kVsr / kVc) * a0 - a1;
    const R axfer = a0 - R(kVc / kVss) * a2;
    const R ci2 = Ca_i * Ca_i;
    const R kup2 = R(kKup * kKup);
    const R I_up = R(kVmaxUp) * ci2 / (ci2 + kup2);
    const R I_leak = R(kVleak) * (Ca_sr - Ca_i);
    const R I_xfer = R(kVxfer) * (Ca_ss - Ca_i);
    X0 += (I_leak - I_up) * R(kVsr / kVc) + I_xfer;
    X1 += I_up - I_leak;
    X2 -= I_xfer * R(kVc / kVss);
    gCi += aup * R(kVmaxUp) * R(2.0) * Ca_i * kup2 / ((ci2 + kup2) * (ci2 + kup2));
    gCsr += aleak * R(kVleak);
    gCi -= aleak * R(kVleak);
    gCss += axfer * R(kVxfer);
    gCi -= axfer * R(kVxfer);
  }
  {
    // I_rel = Vrel O (Ca_SR - Ca_ss), O = T Rbar / (K3 + T), T = k1 Ca_ss^2,
    // k1 = K1p / k_casr, k2 = K2p k_casr (h_a,5 = -k2 Ca_ss Rbar + K4 (1 - Rbar))
    const R arel = -a1 + R(kVsr / kVss) * a2;
    const R csr2 = Ca_sr * Ca_sr;
    const R ec2 = R(kEC * kEC);
    const R k_casr = R(kMaxSR) - R(kMaxSR - kMinSR) * csr2 / (csr2 + ec2);
    const R k1 = R(kK1p) / k_casr, k2 = R(kK2p) * k_casr;
    const R css2 = Ca_ss * Ca_ss;
    const R T = k1 * css2;
    const R kt = R(kK3) + T;
    const R O = T * Rbar / kt;
    const R I_rel = R(kVrel) * O * (Ca_sr - Ca_ss);
    X1 -= I_rel;
    X2 += I_rel * R(kVsr / kVss);
    const R gO = arel * R(kVrel) * (Ca_sr - Ca_ss);
    gCsr += arel * R(kVrel) * O;
    gCss -= arel * R(kVrel) * O;
    const R gT = gO * Rbar * R(kK3) / (kt * kt);
    gR += gO * T / kt;
    gCss += gT * k1 * R(2.0) * Ca_ss;
    const R gk1 = gT * css2;
    const R gk2 = -ch[5] * Ca_ss * Rbar;
    gCss -= ch[5] * k2 * Rbar;
    gR -= ch[5] * (k2 * Ca_ss + R(kK4));
    const R gkc = -gk1 * R(kK1p) / (k_casr * k_casr) + gk2 * R(kK2p);
    const R den = csr2 + ec2;
    gCsr += gkc * (-R(kMaxSR - kMinSR) * R(2.0) * Ca_sr * ec2 / (den * den));
  }
  // the buffer factors' derivatives, 2 c_k B K / (c_k^2 + B K)^2
  gCi += ch[0] * X0 * R(2.0) * ci_k * bkc / (dbc * dbc);
  gCsr += ch[1] * X1 * R(2.0) * csr_k * bksr / (dbsr * dbsr);
  gCss += ch[2] * X2 * R(2.0) * css_k * bkss / (dbss * dbss);

  vx[0] += gV;
  vx[1] += gCi;
  vx[2] += gCsr;
  vx[3] += gCss;
  vx[4] += gNa;
  vx[5] += gK;
  vx[6] += gR;
}

}  // namespace ttp06
