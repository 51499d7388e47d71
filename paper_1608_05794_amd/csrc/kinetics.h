// Device-side kinetics: NASA-7 thermodynamics (Eq. tfits, standard form),
// modified Arrhenius rates (Eq. kfor), equilibrium constants and reverse
// rates (Eqs. krev, kc), third-body and fall-off factors, and their
// temperature / concentration derivatives.  Shared by the lane-per-reactor
// and the wavefront-per-reactor kernels; species data are read through small
// accessor objects so each kernel keeps its own memory layout.
#pragma once

#include "ck_internal.h"

namespace ck {

struct Thermo {
    double cp, h, s, dcp;   // cp/R, H/(RT), S/R, d(cp/R)/dT
};

struct TPow {
    double T, invT, lnT, T2, T3, T4;
};

__device__ __forceinline__ TPow tpow(double T) {
    TPow p;
    p.T = T;
    p.invT = 1.0 / T;
    p.lnT = log(T);
    p.T2 = T * T;
    p.T3 = p.T2 * T;
    p.T4 = p.T3 * T;
    return p;
}

// Species k at temperature t: low range if T < Tmid, else high (per-lane select).
__device__ __forceinline__ Thermo species_thermo(const DevMech &M, int k, const TPow &t) {
    const int ns = M.nsp;
    const int off = (t.T < M.Tmid()[k]) ? 0 : 21;
    const double *c = M.thermo() + size_t(off) * ns + k;
    auto a = [&](int j) { return c[size_t(j) * ns]; };
    Thermo o;
    o.cp = a(0) + a(1) * t.T + a(2) * t.T2 + a(3) * t.T3 + a(4) * t.T4;
    o.h = a(5) + a(6) * t.T + a(7) * t.T2 + a(8) * t.T3 + a(9) * t.T4 + a(10) * t.invT;
    o.s = a(11) * t.lnT + a(12) * t.T + a(13) * t.T2 + a(14) * t.T3 + a(15) * t.T4 + a(16);
    o.dcp = a(17) + a(18) * t.T + a(19) * t.T2 + a(20) * t.T3;
    return o;
}

// x^n for n in 0..3
__device__ __forceinline__ double ipow(double x, int n) {
    const double x2 = x * x;
    return n == 0 ? 1.0 : (n == 1 ? x : (n == 2 ? x2 : x2 * x));
}

// The species slots of one reaction with their concentrations, in registers.
struct Slots {
    double c[kMaxSlots];
    int sp[kMaxSlots];
    int nu[kMaxSlots];     // 0 for unused slots
    int sgn[kMaxSlots];    // -1 reactant, +1 product, 0 unused
    int n, nre;
};

// nmax: a wave-uniform bound on the slot count (slots beyond it are skipped by scalar branches).
template <class Cget>
__device__ __forceinline__ void load_slots(const RxnRec &R, const Cget &C, Slots &S, int nmax) {
    S.n = rx_nslot(R.meta);
    S.nre = rx_nreac(R.meta);
#pragma unroll
    for (int s = 0; s < kMaxSlots; s++) {
        if (s >= nmax) {
            S.sp[s] = 0;
            S.nu[s] = 0;
            S.sgn[s] = 0;
            S.c[s] = 1.0;
            continue;
        }
        const bool used = s < S.n;
        S.sp[s] = rx_sp(R, s);
        S.nu[s] = used ? rx_nu(R, s) : 0;
        S.sgn[s] = used ? (s < S.nre ? -1 : 1) : 0;
        S.c[s] = C(used ? S.sp[s] : 0);
    }
}

// Everything one reaction contributes at (T, C).
struct Rate {
    double kf, kr;        // multiply the mass-action products; k_inf for fall-off
    double pf, pr;        // prod C^nu' and prod C^nu''
    double c;             // third-body / fall-off factor
    double dlnkf, dlnkr;  // d ln k / dT            (DERIV only)
    double dcdM, dcdT;    // d c / d[M], d c / dT   (DERIV only)
};

// Rate constants and factors of reaction R (Eqs. kfor, krev, kc; third-body and
// fall-off factor c).  Gget(k) returns g_k = H_k/(RT) - S_k/R, Hget(k) H_k/(RT).
template <bool DERIV, class Cget, class Gget, class Hget>
__device__ __forceinline__ void reaction_rate(const DevMech &M, const RxnRec &R, const Slots &S, int nmax,
                                              const TPow &t, double Ctot, const Cget &C, const Gget &G,
                                              const Hget &H, Rate &o) {
    const double lnkf = R.lnA + R.beta * t.lnT - R.EaR * t.invT;
    o.kf = exp(lnkf);
    if (DERIV) o.dlnkf = (R.beta + R.EaR * t.invT) * t.invT;
    o.pf = 1.0;
    o.pr = 1.0;
    double sg = 0.0, sh = 0.0;
#pragma unroll
    for (int s = 0; s < kMaxSlots; s++) {
        if (s >= nmax) break;
        const double p = ipow(S.c[s], S.nu[s]);
        if (S.sgn[s] < 0) o.pf *= p;
        else o.pr *= p;
        const int sp = S.sgn[s] != 0 ? S.sp[s] : 0;
        const double w = double(S.sgn[s] * S.nu[s]);
        sg += w * G(sp);
        if (DERIV) sh += w * H(sp);
    }
    const int meta = R.meta;
    if (rx_rev(meta)) {
        // ln Kc = -sum_j nu_j g_j + dnu ln(p0 / (R T)); kr = kf / Kc
        const double lnKc = -sg + R.dnu * (M.ln_p0_R - t.lnT);
        o.kr = exp(lnkf - lnKc);
        if (DERIV) o.dlnkr = o.dlnkf - (sh - R.dnu) * t.invT;
    } else {
        o.kr = 0.0;
        if (DERIV) o.dlnkr = 0.0;
    }
    o.c = 1.0;
    if (DERIV) {
        o.dcdM = 0.0;
        o.dcdT = 0.0;
    }
    const int ty = rx_type(meta);
    if (ty == kElementary) return;
    double Mc = Ctot;
    const int eb = R.eff_begin, ec = rx_neff(meta);
    for (int e = 0; e < ec; e++) {
        const EffRec E = M.eff[eb + e];
        Mc += E.am1 * C(E.sp);
    }
    if (ty == kThirdBody) {
        o.c = Mc;
        if (DERIV) o.dcdM = 1.0;
        return;
    }
    // fall-off: Pr = k0 [M] / k_inf, c = Pr / (1 + Pr) F
    const FallRec F = M.fall[R.fall];
    const double lnk0 = F.lnA0 + F.beta0 * t.lnT - F.Ea0R * t.invT;
    const double ratio = exp(lnk0 - lnkf);
    const double Pr = ratio * Mc;
    double Fb = 1.0, g = 0.0, dlogF_dL = 0.0, dFc_over_Fc = 0.0;
    if (ty == kTroe) {
        const double a = F.a;
        const double e3 = exp(-t.T * F.invT3);
        const double e1 = exp(-t.T * F.invT1);
        const double e2 = exp(-F.T2 * t.invT);
        const double Fc = (1.0 - a) * e3 + a * e1 + e2;
        const double L = log10(fmax(Fc, 1e-300));
        const double cc = -0.4 - 0.67 * L;
        const double nn = 0.75 - 1.27 * L;
        const double x = log10(fmax(Pr, 1e-300)) + cc;
        const double d = nn - 0.14 * x;
        const double f1 = x / d;
        const double u = 1.0 + f1 * f1;
        Fb = exp10(L / u);
        if (DERIV) {
            const double iu2 = 1.0 / (u * u);
            const double id2 = 1.0 / (d * d);
            g = L * (-2.0 * f1 * iu2) * (nn * id2);
            dlogF_dL = 1.0 / u - L * 2.0 * f1 * iu2 * ((-0.67 * nn + 1.27 * x) * id2);
            const double dFc = -(1.0 - a) * F.invT3 * e3 - a * F.invT1 * e1 + F.T2 * t.invT * t.invT * e2;
            dFc_over_Fc = dFc / Fc;
        }
    }
    const double onep = 1.0 + Pr;
    o.c = Pr / onep * Fb;
    if (DERIV) {
        const double dc_dPr = Fb / (onep * onep) + Fb * g / onep;
        const double dlnPr_dT = (F.beta0 + F.Ea0R * t.invT) * t.invT - o.dlnkf;
        o.dcdM = dc_dPr * ratio;
        o.dcdT = dc_dPr * Pr * dlnPr_dT;
        if (ty == kTroe) o.dcdT += Pr / onep * Fb * dlogF_dL * dFc_over_Fc;
    }
}

// d(prod over the side of slot s)/dC of slot s: nu_s C_s^(nu_s-1) times the side's other factors.
__device__ __forceinline__ double dprod_slot(const Slots &S, int s, int nmax) {
    double p = 1.0;
#pragma unroll
    for (int t = 0; t < kMaxSlots; t++) {
        if (t >= nmax) break;
        if (S.sgn[t] != S.sgn[s]) continue;
        const double ct = S.c[t];
        if (t == s)
            p *= S.nu[t] == 1 ? 1.0 : (S.nu[t] == 2 ? 2.0 * ct : 3.0 * ct * ct);
        else
            p *= ipow(ct, S.nu[t]);
    }
    return p;
}

// ROS4 coefficients (Appendix C; gamma as tabulated).
struct Ros4 {
    static constexpr double gamma = 0.57282;
    static constexpr double a21 = 2.0;
    static constexpr double a31 = 1.867943637803922, a32 = 0.2344449711399156;
    static constexpr double c21 = -7.137615036412310;
    static constexpr double c31 = 2.580708087951457, c32 = 0.6515950076447975;
    static constexpr double c41 = -2.137148994382534, c42 = -0.3214669691237626, c43 = -0.6949742501781779;
    static constexpr double m1 = 2.255570073418735, m2 = 0.2870493262186792, m3 = 0.4353179431840180,
                            m4 = 1.093502252409163;
    static constexpr double e1 = -0.2815431932141155, e2 = -0.07276199124938920, e3 = -0.1082196201495311,
                            e4 = -1.093502252409163;
};

// Runge--Kutta--Fehlberg 4(5) (Appendix B).
struct Rkf45 {
    static constexpr double a21 = 1.0 / 4.0;
    static constexpr double a31 = 3.0 / 32.0, a32 = 9.0 / 32.0;
    static constexpr double a41 = 1932.0 / 2197.0, a42 = -7200.0 / 2197.0, a43 = 7296.0 / 2197.0;
    static constexpr double a51 = 439.0 / 216.0, a52 = -8.0, a53 = 3680.0 / 513.0, a54 = -845.0 / 4104.0;
    static constexpr double a61 = -8.0 / 27.0, a62 = 2.0, a63 = -3544.0 / 2565.0, a64 = 1859.0 / 4104.0,
                            a65 = -11.0 / 40.0;
    static constexpr double b1 = 25.0 / 216.0, b3 = 1408.0 / 2565.0, b4 = 2197.0 / 4104.0, b5 = -1.0 / 5.0;
    static constexpr double d1 = 16.0 / 135.0 - 25.0 / 216.0, d3 = 6656.0 / 12825.0 - 1408.0 / 2565.0,
                            d4 = 28561.0 / 56430.0 - 2197.0 / 4104.0, d5 = -9.0 / 50.0 + 1.0 / 5.0,
                            d6 = 2.0 / 55.0;
};

// Step-size control shared by every integrator kernel (the paper leaves
// EstimateH0 and AdjustStepSize unspecified; this is the library's fixed
// specification: safety 0.9, factor in [0.2, 5], error exponent 1/q).
__device__ __forceinline__ double step_factor(double err, double q_inv, bool accepted) {
    if (accepted) return err == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(err, -q_inv)));
    return isfinite(err) ? fmax(0.2, 0.9 * pow(err, -q_inv)) : 0.2;
}

__device__ __forceinline__ double h_floor(double t) { return fmax(1e-30, 16.0 * 2.220446049250313e-16 * fabs(t)); }

}  // namespace ck
