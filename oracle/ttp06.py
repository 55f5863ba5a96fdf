"""ten Tusscher-Panfilov 2006 human ventricular (epicardial) cell model, written
out node-wise in FP64 numpy (TEST INFRASTRUCTURE ONLY, see package doc).

The paper uses this model with m1 = 6 auxiliary and m2 = 12 gating variables
(Sec. 5, model setup).  It does not print the equations; they are restated here
from the model's original publication (ten Tusscher & Panfilov, Am. J. Physiol.
Heart Circ. Physiol. 291:H1088, 2006), epicardial cell, rapid-buffering
formulation of Ca_i, Ca_SR and Ca_ss.  Agreement with that publication's traces
is parity unpinned (no trace is available); the HIP kernel is checked against
this module point by point.

State layout (one row per field, one column per mesh node):
    0 V (mV)
    1 Ca_i  2 Ca_SR  3 Ca_ss  4 Na_i  5 K_i (mM)  6 Rbar (-)      auxiliary w_a
    7 m  8 h  9 j  10 xr1  11 xr2  12 xs  13 r  14 s  15 d  16 f  17 f2
    18 fCass                                                       gates w_g
Currents are in pA/pF, time in ms.
"""
import numpy as np

NF = 19
NAUX = 6
NGATE = 12
AUX = slice(1, 7)
GATES = slice(7, 19)
FIELD_NAMES = ("V", "Ca_i", "Ca_SR", "Ca_ss", "Na_i", "K_i", "Rbar",
               "m", "h", "j", "xr1", "xr2", "xs", "r", "s", "d", "f", "f2",
               "fCass")

# physical constants
R_GAS = 8314.472      # mJ / (K mol)
T_K = 310.0           # K
FARADAY = 96485.3415  # C / mol
RTF = R_GAS * T_K / FARADAY
# cell geometry
CAP = 0.185           # uF, cell capacitance
V_C = 0.016404        # uL, cytoplasm
V_SR = 0.001094       # uL, sarcoplasmic reticulum
V_SS = 0.00005468     # uL, subspace
# extracellular concentrations
K_O, NA_O, CA_O = 5.4, 140.0, 2.0
# maximal conductances (epicardium)
G_NA = 14.838
G_K1 = 5.405
G_TO = 0.294
G_KR = 0.153
G_KS = 0.392
P_KNA = 0.03
G_CAL = 3.980e-5
K_NACA = 1000.0
GAMMA_NACA = 0.35
KM_CA = 1.38
KM_NAI = 87.5
K_SAT = 0.1
ALPHA_NACA = 2.5
P_NAK = 2.724
KM_K = 1.0
KM_NA = 40.0
G_PK = 0.0146
G_PCA = 0.1238
K_PCA = 0.0005
G_BNA = 0.00029
G_BCA = 0.000592
# calcium handling
VMAX_UP = 0.006375
K_UP = 0.00025
V_REL = 0.102
K1P = 0.15
K2P = 0.045
K3 = 0.060
K4 = 0.005
EC = 1.5
MAX_SR = 2.5
MIN_SR = 1.0
V_LEAK = 0.00036
V_XFER = 0.0038
BUF_C, K_BUFC = 0.2, 0.001
BUF_SR, K_BUFSR = 10.0, 0.3
BUF_SS, K_BUFSS = 0.4, 0.00025


def rest_state():
    """Epicardial initial (rest) state of the model publication, field order
    as in the module doc."""
    return np.array([
        -85.23,                                    # V
        0.000126, 3.64, 0.00036, 8.604, 136.89, 0.9073,  # Ca_i Ca_SR Ca_ss Na_i K_i Rbar
        0.00172, 0.7444, 0.7045,                   # m h j
        0.00621, 0.4712, 0.0095,                   # xr1 xr2 xs
        2.42e-8, 0.999998,                         # r s
        3.373e-5, 0.7888, 0.9755, 0.9953,          # d f f2 fCass
    ])


def _sig(x):
    return 1.0 / (1.0 + np.exp(x))


def gates(V, Ca_ss):
    """Steady states w_g,inf and time constants tau (ms) of the 12 gates.

    Returns (inf, tau), each of shape (12, N).  The relaxation form of the
    gating equations is dw/dt = (w_inf - w)/tau = Lambda_g (w - w_inf) with
    Lambda_g = -1/tau (eq. monodomain_g_lambda).  fCass depends on Ca_ss."""
    V = np.asarray(V, float)
    Ca_ss = np.asarray(Ca_ss, float)
    inf = np.empty((NGATE,) + V.shape)
    tau = np.empty((NGATE,) + V.shape)
    # m
    inf[0] = _sig((-56.86 - V) / 9.03) ** 2
    a_m = _sig((-60.0 - V) / 5.0)
    b_m = 0.1 * _sig((V + 35.0) / 5.0) + 0.1 * _sig((V - 50.0) / 200.0)
    tau[0] = a_m * b_m
    # h
    h_inf = _sig((V + 71.55) / 7.43) ** 2
    inf[1] = h_inf
    low = V < -40.0
    a_h = np.where(low, 0.057 * np.exp(-(V + 80.0) / 6.8), 0.0)
    b_h = np.where(low, 2.7 * np.exp(0.079 * V) + 3.1e5 * np.exp(0.3485 * V),
                   0.77 / (0.13 * (1.0 + np.exp(-(V + 10.66) / 11.1))))
    tau[1] = 1.0 / (a_h + b_h)
    # j
    inf[2] = h_inf
    a_j = np.where(low,
                   (-2.5428e4 * np.exp(0.2444 * V) - 6.948e-6 * np.exp(-0.04391 * V))
                   * (V + 37.78) / (1.0 + np.exp(0.311 * (V + 79.23))), 0.0)
    b_j = np.where(low,
                   0.02424 * np.exp(-0.01052 * V) / (1.0 + np.exp(-0.1378 * (V + 40.14))),
                   0.6 * np.exp(0.057 * V) / (1.0 + np.exp(-0.1 * (V + 32.0))))
    tau[2] = 1.0 / (a_j + b_j)
    # xr1
    inf[3] = _sig((-26.0 - V) / 7.0)
    tau[3] = (450.0 * _sig((-45.0 - V) / 10.0)) * (6.0 * _sig((V + 30.0) / 11.5))
    # xr2
    inf[4] = _sig((V + 88.0) / 24.0)
    tau[4] = (3.0 * _sig((-60.0 - V) / 20.0)) * (1.12 * _sig((V - 60.0) / 20.0))
    # xs
    inf[5] = _sig((-5.0 - V) / 14.0)
    a_xs = 1400.0 / np.sqrt(1.0 + np.exp((5.0 - V) / 6.0))
    b_xs = _sig((V - 35.0) / 15.0)
    tau[5] = a_xs * b_xs + 80.0
    # r
    inf[6] = _sig((20.0 - V) / 6.0)
    tau[6] = 9.5 * np.exp(-(V + 40.0) ** 2 / 1800.0) + 0.8
    # s (epicardium)
    inf[7] = _sig((V + 20.0) / 5.0)
    tau[7] = (85.0 * np.exp(-(V + 45.0) ** 2 / 320.0)
              + 5.0 * _sig((V - 20.0) / 5.0) + 3.0)
    # d
    inf[8] = _sig((-8.0 - V) / 7.5)
    a_d = 1.4 * _sig((-35.0 - V) / 13.0) + 0.25
    b_d = 1.4 * _sig((V + 5.0) / 5.0)
    g_d = _sig((50.0 - V) / 20.0)
    tau[8] = a_d * b_d + g_d
    # f
    inf[9] = _sig((V + 20.0) / 7.0)
    tau[9] = (1102.5 * np.exp(-(V + 27.0) ** 2 / 225.0)
              + 200.0 * _sig((13.0 - V) / 10.0)
              + 180.0 * _sig((V + 30.0) / 10.0) + 20.0)
    # f2
    inf[10] = 0.67 * _sig((V + 35.0) / 7.0) + 0.33
    tau[10] = (600.0 * np.exp(-(V + 25.0) ** 2 / 170.0)
               + 31.0 * _sig((25.0 - V) / 10.0)
               + 16.0 * _sig((V + 30.0) / 10.0))
    # fCass
    q = (Ca_ss / 0.05) ** 2
    inf[11] = 0.6 / (1.0 + q) + 0.4
    tau[11] = 80.0 / (1.0 + q) + 2.0
    return inf, tau


def currents(y, g_scale=(1.0, 1.0, 1.0)):
    """Membrane currents (pA/pF) at states y of shape (19, N).

    g_scale multiplies G_Na, G_CaL and G_Kr.  Returns a dict of arrays."""
    V, Ca_i, Ca_sr, Ca_ss, Na_i, K_i = y[0], y[1], y[2], y[3], y[4], y[5]
    m, h, j, xr1, xr2, xs, r, s, d, f, f2, fcass = (y[7 + k] for k in range(12))
    E_Na = RTF * np.log(NA_O / Na_i)
    E_K = RTF * np.log(K_O / K_i)
    E_Ks = RTF * np.log((K_O + P_KNA * NA_O) / (K_i + P_KNA * Na_i))
    E_Ca = 0.5 * RTF * np.log(CA_O / Ca_i)
    I = {}
    I["Na"] = g_scale[0] * G_NA * m ** 3 * h * j * (V - E_Na)
    a_k1 = 0.1 / (1.0 + np.exp(0.06 * (V - E_K - 200.0)))
    b_k1 = ((3.0 * np.exp(0.0002 * (V - E_K + 100.0)) + np.exp(0.1 * (V - E_K - 10.0)))
            / (1.0 + np.exp(-0.5 * (V - E_K))))
    I["K1"] = G_K1 * np.sqrt(K_O / 5.4) * (a_k1 / (a_k1 + b_k1)) * (V - E_K)
    I["to"] = G_TO * r * s * (V - E_K)
    I["Kr"] = g_scale[2] * G_KR * np.sqrt(K_O / 5.4) * xr1 * xr2 * (V - E_K)
    I["Ks"] = G_KS * xs ** 2 * (V - E_Ks)
    # L-type: 4 (V-15) F^2/(RT) (0.25 Ca_ss e^u - Ca_o)/(e^u - 1), u = 2 (V-15) F/(RT);
    # (V-15)/(e^u - 1) is written as (RT/(2F)) / ((e^u - 1)/u), regular at u = 0.
    u = 2.0 * (V - 15.0) / RTF
    safe_u = np.where(u == 0.0, 1.0, u)
    ratio = np.where(u == 0.0, 1.0, np.expm1(safe_u) / safe_u)  # (e^u - 1)/u
    I["CaL"] = (g_scale[1] * G_CAL * d * f * f2 * fcass * 4.0 * FARADAY
                * (0.5 / ratio) * (0.25 * Ca_ss * np.exp(u) - CA_O))
    vfrt = V / RTF
    I["NaCa"] = (K_NACA * (np.exp(GAMMA_NACA * vfrt) * Na_i ** 3 * CA_O
                           - np.exp((GAMMA_NACA - 1.0) * vfrt) * NA_O ** 3 * Ca_i * ALPHA_NACA)
                 / ((KM_NAI ** 3 + NA_O ** 3) * (KM_CA + CA_O)
                    * (1.0 + K_SAT * np.exp((GAMMA_NACA - 1.0) * vfrt))))
    I["NaK"] = (P_NAK * K_O / (K_O + KM_K) * Na_i / (Na_i + KM_NA)
                / (1.0 + 0.1245 * np.exp(-0.1 * vfrt) + 0.0353 * np.exp(-vfrt)))
    I["pCa"] = G_PCA * Ca_i / (K_PCA + Ca_i)
    I["pK"] = G_PK * (V - E_K) / (1.0 + np.exp((25.0 - V) / 5.98))
    I["bNa"] = G_BNA * (V - E_Na)
    I["bCa"] = G_BCA * (V - E_Ca)
    I["ion"] = (I["Na"] + I["K1"] + I["to"] + I["Kr"] + I["Ks"] + I["CaL"]
                + I["NaCa"] + I["NaK"] + I["pCa"] + I["pK"] + I["bNa"] + I["bCa"])
    return I


def aux_rhs(y, I):
    """h_a: time derivatives of Ca_i, Ca_SR, Ca_ss, Na_i, K_i, Rbar (shape (6, N))."""
    Ca_i, Ca_sr, Ca_ss, Na_i = y[1], y[2], y[3], y[4]
    Rbar = y[6]
    k_casr = MAX_SR - (MAX_SR - MIN_SR) / (1.0 + (EC / Ca_sr) ** 2)
    k1 = K1P / k_casr
    k2 = K2P * k_casr
    O = k1 * Ca_ss ** 2 * Rbar / (K3 + k1 * Ca_ss ** 2)
    I_rel = V_REL * O * (Ca_sr - Ca_ss)
    I_up = VMAX_UP / (1.0 + K_UP ** 2 / Ca_i ** 2)
    I_leak = V_LEAK * (Ca_sr - Ca_i)
    I_xfer = V_XFER * (Ca_ss - Ca_i)
    buf_c = 1.0 / (1.0 + BUF_C * K_BUFC / (Ca_i + K_BUFC) ** 2)
    buf_sr = 1.0 / (1.0 + BUF_SR * K_BUFSR / (Ca_sr + K_BUFSR) ** 2)
    buf_ss = 1.0 / (1.0 + BUF_SS * K_BUFSS / (Ca_ss + K_BUFSS) ** 2)
    out = np.empty((NAUX,) + Ca_i.shape)
    out[0] = buf_c * ((I_leak - I_up) * V_SR / V_C + I_xfer
                      - (I["bCa"] + I["pCa"] - 2.0 * I["NaCa"]) * CAP / (2.0 * V_C * FARADAY))
    out[1] = buf_sr * (I_up - (I_rel + I_leak))
    out[2] = buf_ss * (-I["CaL"] * CAP / (2.0 * V_SS * FARADAY)
                       + I_rel * V_SR / V_SS - I_xfer * V_C / V_SS)
    out[3] = -(I["Na"] + I["bNa"] + 3.0 * I["NaK"] + 3.0 * I["NaCa"]) * CAP / (V_C * FARADAY)
    out[4] = -(I["K1"] + I["to"] + I["Kr"] + I["Ks"] - 2.0 * I["NaK"] + I["pK"]) * CAP / (V_C * FARADAY)
    out[5] = -k2 * Ca_ss * Rbar + K4 * (1.0 - Rbar)
    return out


def evaluate(y, g_scale=(1.0, 1.0, 1.0)):
    """Node-wise ionic model at states y (19, N).

    Returns (I_ion (N,), h_a (6, N), Lambda_g (12, N), w_inf (12, N)) with
    Lambda_g = -1/tau the diagonal stiff matrix of eq. def_Lambda."""
    y = np.asarray(y, float)
    I = currents(y, g_scale)
    ha = aux_rhs(y, I)
    inf, tau = gates(y[0], y[3])
    return I["ion"], ha, -1.0 / tau, inf
