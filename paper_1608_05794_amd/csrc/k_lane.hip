// Lane-per-reactor kernels: one reactor per SIMT lane, every intermediate in
// global memory as structure-of-arrays (slot e of reactor r at ws[e*S + r]),
// so each access of a wavefront is coalesced over 64 reactors.  This is the
// shallow-vectorisation design of Section 4 (Algorithm 2 with a 64-wide SIMD
// word): lanes of a wavefront run until the slowest one finishes.  It is the
// baseline the wavefront-per-reactor kernels are measured against.
#include "ck_internal.h"
#include "kinetics.h"
#include "launch.h"

namespace ck {

// Strided view: element e of one reactor at p[e * s].
struct SV {
    double *p;
    int64_t s;
    __device__ __forceinline__ double &operator[](int64_t e) const { return p[e * s]; }
};
struct CSV {
    const double *p;
    int64_t s;
    __device__ __forceinline__ double operator[](int64_t e) const { return p[e * s]; }
};

// Per-reactor scratch slots of the lane kernels.
struct LaneLayout {
    int nsp, N;
    int64_t C, G, H, CP, WD, JC, DWT, M, PIV, YT, F, U, YN, E, F0;
    int64_t total;
    __host__ __device__ LaneLayout(int nsp_, int N_, int stages) {
        nsp = nsp_;
        N = N_;
        int64_t o = 0;
        C = o; o += nsp;
        G = o; o += nsp;
        H = o; o += nsp;
        CP = o; o += nsp;
        WD = o; o += nsp;
        JC = o; o += int64_t(nsp) * nsp;
        DWT = o; o += nsp;
        M = o; o += int64_t(N) * N;
        PIV = o; o += N;
        YT = o; o += N;
        F = o; o += N;
        U = o; o += int64_t(stages) * N;
        YN = o; o += N;
        E = o; o += N;
        F0 = o; o += N;
        total = o;
    }
};

// Source term of one reactor (Section 3); y, f are views over the state.
template <class YV>
__device__ void rhs_lane(const DevMech &M, const YV &y, double P, SV f, SV w, const LaneLayout &L,
                         double *rho_out = nullptr, double *cp_out = nullptr) {
    const int ns = M.nsp;
    const double T = y[0];
    const TPow t = tpow(T);
    double S = 0.0;
    for (int k = 0; k < ns; k++) S += y[1 + k] * M.invW()[k];
    const double rho = P / (M.R * T * S);
    const double Ctot = P * t.invT / M.R;
    double cpm = 0.0;
    for (int k = 0; k < ns; k++) {
        const double Ck = rho * y[1 + k] * M.invW()[k];
        w[L.C + k] = Ck;
        const Thermo th = species_thermo(M, k, t);
        w[L.G + k] = th.h - th.s;
        w[L.H + k] = th.h;
        w[L.CP + k] = th.cp;
        w[L.WD + k] = 0.0;
        cpm += y[1 + k] * th.cp * M.invW()[k];
    }
    cpm *= M.R;
    auto Cg = [&](int k) { return w[L.C + k]; };
    auto Gg = [&](int k) { return w[L.G + k]; };
    auto Hg = [&](int k) { return w[L.H + k]; };
    for (int i = 0; i < M.nrxn; i++) {
        const RxnRec R = M.rx[i];
        Slots S;
        const int nmax = rx_nslot(R.meta);
        load_slots(R, Cg, S, nmax);
        Rate q;
        reaction_rate<false>(M, R, S, nmax, t, Ctot, Cg, Gg, Hg, q);
        const double qi = q.c * (q.kf * q.pf - q.kr * q.pr);
        for (int s = 0; s < S.n; s++) w[L.WD + S.sp[s]] += (S.sgn[s] * S.nu[s]) * qi;
    }
    double Q = 0.0;
    for (int k = 0; k < ns; k++) {
        const double wd = w[L.WD + k];
        f[1 + k] = M.W()[k] * wd / rho;
        Q += M.R * T * w[L.H + k] * wd;
    }
    f[0] = -Q / (rho * cpm);
    if (rho_out) *rho_out = rho;
    if (cp_out) *cp_out = cpm;
}

// Analytic Jacobian of one reactor into J (row-major N x N view); also f.
template <class YV>
__device__ void jac_lane(const DevMech &M, const YV &y, double P, SV J, SV f, SV w, const LaneLayout &L) {
    const int ns = M.nsp, N = M.N, nr = M.nrxn;
    double rho, cp;
    rhs_lane(M, y, P, f, w, L, &rho, &cp);
    const double T = y[0];
    const TPow t = tpow(T);
    const double Ctot = P * t.invT / M.R;
    double S = 0.0;
    for (int k = 0; k < ns; k++) S += y[1 + k] * M.invW()[k];
    const double Wbar = 1.0 / S;
    for (int64_t e = 0; e < int64_t(ns) * ns; e++) w[L.JC + e] = 0.0;
    for (int k = 0; k < ns; k++) w[L.DWT + k] = 0.0;
    auto Cg = [&](int k) { return w[L.C + k]; };
    auto Gg = [&](int k) { return w[L.G + k]; };
    auto Hg = [&](int k) { return w[L.H + k]; };
    for (int i = 0; i < nr; i++) {
        const RxnRec R = M.rx[i];
        Slots S;
        const int nmax = rx_nslot(R.meta);
        load_slots(R, Cg, S, nmax);
        Rate q;
        reaction_rate<true>(M, R, S, nmax, t, Ctot, Cg, Gg, Hg, q);
        const double Rn = q.kf * q.pf - q.kr * q.pr;
        const double dqT = q.c * (q.kf * q.dlnkf * q.pf - q.kr * q.dlnkr * q.pr) + Rn * q.dcdT;
        // mass-action part, slot pairs (row slot a, column slot b)
        for (int b = 0; b < S.n; b++) {
            const double d = dprod_slot(S, b, nmax);
            const double dq = q.c * (S.sgn[b] < 0 ? q.kf * d : -q.kr * d);
            for (int a = 0; a < S.n; a++) w[L.JC + int64_t(S.sp[a]) * ns + S.sp[b]] += (S.sgn[a] * S.nu[a]) * dq;
        }
        const int eb = R.eff_begin, ec = rx_neff(R.meta);
        for (int a = 0; a < S.n; a++) {
            const double v = S.sgn[a] * S.nu[a];
            w[L.DWT + S.sp[a]] += v * dqT;
            if (q.dcdM != 0.0) {
                // d[M]/dC_l = alpha_l = 1 + (alpha_l - 1)
                const double base = v * Rn * q.dcdM;
                for (int l = 0; l < ns; l++) w[L.JC + int64_t(S.sp[a]) * ns + l] += base;
                for (int e = 0; e < ec; e++) {
                    const EffRec E = M.eff[eb + e];
                    w[L.JC + int64_t(S.sp[a]) * ns + E.sp] += base * E.am1;
                }
            }
        }
    }
    // chain rule through C(T, Y) and rho(T, Y)
    double sumHJCC = 0.0, dQT = 0.0, sdcp = 0.0;
    for (int k = 0; k < ns; k++) {
        double jcc = 0.0;
        for (int l = 0; l < ns; l++) jcc += w[L.JC + int64_t(k) * ns + l] * w[L.C + l];
        const double Wk = M.W()[k];
        const double resid = w[L.WD + k] - jcc;
        const double a = Wk * Wbar * resid / rho;
        for (int j = 0; j < ns; j++) J[int64_t(1 + k) * N + 1 + j] = M.invW()[j] * (Wk * w[L.JC + int64_t(k) * ns + j] + a);
        J[int64_t(1 + k) * N] = (Wk / rho) * (w[L.DWT + k] + resid * t.invT);
        const double Hk = M.R * T * w[L.H + k];
        sumHJCC += Hk * jcc;
        dQT += M.R * w[L.CP + k] * w[L.WD + k] + Hk * (w[L.DWT + k] - jcc * t.invT);
        const Thermo th = species_thermo(M, k, t);
        sdcp += y[1 + k] * M.R * th.dcp * M.invW()[k];
    }
    const double D = rho * cp;
    const double fT = f[0];
    for (int j = 0; j < ns; j++) {
        double colH = 0.0;
        for (int k = 0; k < ns; k++) colH += M.R * T * w[L.H + k] * w[L.JC + int64_t(k) * ns + j];
        const double dQ = M.invW()[j] * (rho * colH - Wbar * sumHJCC);
        const double dD = rho * M.invW()[j] * (M.R * w[L.CP + j] - cp * Wbar);
        J[1 + j] = -(dQ + fT * dD) / D;
    }
    const double dDT = -rho * cp * t.invT + rho * sdcp;
    J[0] = -(dQT + fT * dDT) / D;
}

template <class YV>
__device__ double wrms_lane(int N, const SV &e, const YV &a, const SV &b, double rtol, double atol) {
    double s = 0.0;
    for (int i = 0; i < N; i++) {
        const double sc = atol + rtol * fmax(fabs(a[i]), fabs(b[i]));
        const double r = e[i] / sc;
        s += r * r;
    }
    return sqrt(s / N);
}

// LU with partial pivoting (first index of the largest |a_ik|) of the N x N view A.
__device__ int lu_lane(int N, SV A, SV piv) {
    for (int k = 0; k < N; k++) {
        int p = k;
        double best = fabs(A[int64_t(k) * N + k]);
        for (int i = k + 1; i < N; i++) {
            const double v = fabs(A[int64_t(i) * N + k]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (!(best > 0.0)) return k + 1;
        if (p != k)
            for (int j = 0; j < N; j++) {
                const double tmp = A[int64_t(k) * N + j];
                A[int64_t(k) * N + j] = A[int64_t(p) * N + j];
                A[int64_t(p) * N + j] = tmp;
            }
        const double inv = 1.0 / A[int64_t(k) * N + k];
        for (int i = k + 1; i < N; i++) {
            const double l = A[int64_t(i) * N + k] * inv;
            A[int64_t(i) * N + k] = l;
            for (int j = k + 1; j < N; j++) A[int64_t(i) * N + j] -= l * A[int64_t(k) * N + j];
        }
    }
    return 0;
}

__device__ void lu_solve_lane(int N, const SV &A, const SV &piv, SV b) {
    for (int k = 0; k < N; k++) {
        const int p = int(piv[k]);
        if (p != k) { const double t = b[k]; b[k] = b[p]; b[p] = t; }
    }
    for (int i = 0; i < N; i++) {
        double s = b[i];
        for (int j = 0; j < i; j++) s -= A[int64_t(i) * N + j] * b[j];
        b[i] = s;
    }
    for (int i = N - 1; i >= 0; i--) {
        double s = b[i];
        for (int j = i + 1; j < N; j++) s -= A[int64_t(i) * N + j] * b[j];
        b[i] = s / A[int64_t(i) * N + i];
    }
}

// ROS4 step (transformed Rosenbrock, Appendix C).  Returns false on a singular matrix.
__device__ bool ros4_step_lane(const DevMech &M, SV y, double P, double h, SV w, const LaneLayout &L) {
    const int N = M.N;
    SV Jm{&w[L.M], w.s}, piv{&w[L.PIV], w.s}, f{&w[L.F], w.s}, yt{&w[L.YT], w.s}, u{&w[L.U], w.s};
    jac_lane(M, y, P, Jm, f, w, L);
    const double dg = 1.0 / (Ros4::gamma * h);
    for (int64_t e = 0; e < int64_t(N) * N; e++) Jm[e] = -Jm[e];
    for (int i = 0; i < N; i++) Jm[int64_t(i) * N + i] += dg;
    if (lu_lane(N, Jm, piv)) return false;
    const double ih = 1.0 / h;
    // stage 1: f already holds f(y)
    for (int i = 0; i < N; i++) u[i] = f[i];
    lu_solve_lane(N, Jm, piv, SV{&u[0], w.s});
    // stage 2
    for (int i = 0; i < N; i++) yt[i] = y[i] + Ros4::a21 * u[i];
    rhs_lane(M, yt, P, f, w, L);
    for (int i = 0; i < N; i++) u[N + i] = f[i] + (Ros4::c21 * u[i]) * ih;
    lu_solve_lane(N, Jm, piv, SV{&u[N], w.s});
    // stage 3 (stage 4 uses the same argument)
    for (int i = 0; i < N; i++) yt[i] = y[i] + Ros4::a31 * u[i] + Ros4::a32 * u[N + i];
    rhs_lane(M, yt, P, f, w, L);
    for (int i = 0; i < N; i++) u[2 * N + i] = f[i] + (Ros4::c31 * u[i] + Ros4::c32 * u[N + i]) * ih;
    lu_solve_lane(N, Jm, piv, SV{&u[2 * N], w.s});
    for (int i = 0; i < N; i++)
        u[3 * N + i] = f[i] + (Ros4::c41 * u[i] + Ros4::c42 * u[N + i] + Ros4::c43 * u[2 * N + i]) * ih;
    lu_solve_lane(N, Jm, piv, SV{&u[3 * N], w.s});
    for (int i = 0; i < N; i++) {
        w[L.YN + i] = y[i] + Ros4::m1 * u[i] + Ros4::m2 * u[N + i] + Ros4::m3 * u[2 * N + i] + Ros4::m4 * u[3 * N + i];
        w[L.E + i] = Ros4::e1 * u[i] + Ros4::e2 * u[N + i] + Ros4::e3 * u[2 * N + i] + Ros4::e4 * u[3 * N + i];
    }
    return true;
}

// RKF45 step (Appendix B): k_i = h f(y + sum_j a_ij k_j).
__device__ bool rkf45_step_lane(const DevMech &M, SV y, double P, double h, SV w, const LaneLayout &L) {
    const int N = M.N;
    SV yt{&w[L.YT], w.s}, k{&w[L.U], w.s};
    auto stage = [&](int s) {
        SV ks{&k[int64_t(s) * N], w.s};
        rhs_lane(M, yt, P, ks, w, L);
        for (int i = 0; i < N; i++) ks[i] *= h;
    };
    for (int i = 0; i < N; i++) yt[i] = y[i];
    stage(0);
    for (int i = 0; i < N; i++) yt[i] = y[i] + Rkf45::a21 * k[i];
    stage(1);
    for (int i = 0; i < N; i++) yt[i] = y[i] + Rkf45::a31 * k[i] + Rkf45::a32 * k[N + i];
    stage(2);
    for (int i = 0; i < N; i++) yt[i] = y[i] + Rkf45::a41 * k[i] + Rkf45::a42 * k[N + i] + Rkf45::a43 * k[2 * N + i];
    stage(3);
    for (int i = 0; i < N; i++)
        yt[i] = y[i] + Rkf45::a51 * k[i] + Rkf45::a52 * k[N + i] + Rkf45::a53 * k[2 * N + i] + Rkf45::a54 * k[3 * N + i];
    stage(4);
    for (int i = 0; i < N; i++)
        yt[i] = y[i] + Rkf45::a61 * k[i] + Rkf45::a62 * k[N + i] + Rkf45::a63 * k[2 * N + i] +
                Rkf45::a64 * k[3 * N + i] + Rkf45::a65 * k[4 * N + i];
    stage(5);
    for (int i = 0; i < N; i++) {
        w[L.YN + i] = y[i] + Rkf45::b1 * k[i] + Rkf45::b3 * k[2 * N + i] + Rkf45::b4 * k[3 * N + i] + Rkf45::b5 * k[4 * N + i];
        w[L.E + i] = Rkf45::d1 * k[i] + Rkf45::d3 * k[2 * N + i] + Rkf45::d4 * k[3 * N + i] + Rkf45::d5 * k[4 * N + i] +
                     Rkf45::d6 * k[5 * N + i];
    }
    return true;
}

__global__ void __launch_bounds__(256) rhs_lane_kernel(DevMech M, int64_t n, const double *y, int64_t ld, const double *p,
                                                       double *dydt, double *ws, int64_t wsS) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    LaneLayout L(M.nsp, M.N, 0);
    rhs_lane(M, CSV{y + r, ld}, p[r], SV{dydt + r, ld}, SV{ws + r, wsS}, L);
}

__global__ void __launch_bounds__(256) jac_lane_kernel(DevMech M, int64_t n, const double *y, int64_t ld, const double *p,
                                                       double *jac, double *ws, int64_t wsS) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    LaneLayout L(M.nsp, M.N, 0);
    SV w{ws + r, wsS};
    jac_lane(M, CSV{y + r, ld}, p[r], SV{jac + r, ld}, SV{&w[L.F], wsS}, w, L);
}

template <int METHOD>   // 0 ROS4, 1 RKF45
__global__ void __launch_bounds__(64) integrate_lane_kernel(DevMech M, int64_t n, double *y, int64_t ld, const double *p,
                                                            const double *t_end, double *t_io, double *h_io, IntOpts o,
                                                            double *ws, int64_t wsS, int32_t *status, int32_t *nacc,
                                                            int32_t *nrej) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int N = M.N;
    LaneLayout L(M.nsp, N, METHOD == 0 ? 4 : 6);
    SV w{ws + r, wsS};
    SV yv{y + r, ld};
    const double P = p[r];
    const double te = t_end[r];
    const double qinv = METHOD == 0 ? 0.25 : 0.2;
    double t = t_io ? t_io[r] : 0.0;
    double h = h_io ? h_io[r] : 0.0;
    int st = CK_ST_OK;
    int na = 0, nj = 0;
    bool finite = true;
    for (int i = 0; i < N; i++) finite = finite && isfinite(yv[i]);
    if (!finite) {
        st = CK_ST_NONFINITE;
        h = 0.0;
    } else if (o.h_fixed > 0.0) {
        h = o.h_fixed;
    } else if (!(h > 0.0)) {
        if (o.h0 > 0.0) {
            h = o.h0;
        } else if (t < te) {
            // EstimateH0 (Hairer, Norsett & Wanner II.4, order 4)
            SV f0{&w[L.F0], wsS}, f1{&w[L.F], wsS}, yt{&w[L.YT], wsS};
            rhs_lane(M, yv, P, f0, w, L);
            bool ok = true;
            for (int i = 0; i < N; i++) ok = ok && isfinite(f0[i]);
            if (!ok) {
                st = CK_ST_NONFINITE;
                h = 0.0;
            } else {
                double d0 = 0.0, d1 = 0.0;
                for (int i = 0; i < N; i++) {
                    const double sc = o.atol + o.rtol * fabs(yv[i]);
                    d0 += (yv[i] / sc) * (yv[i] / sc);
                    d1 += (f0[i] / sc) * (f0[i] / sc);
                }
                d0 = sqrt(d0 / N);
                d1 = sqrt(d1 / N);
                const double span = te - t;
                double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
                h0 = fmin(h0, span);
                for (int i = 0; i < N; i++) yt[i] = yv[i] + h0 * f0[i];
                rhs_lane(M, yt, P, f1, w, L);
                double d2 = 0.0;
                for (int i = 0; i < N; i++) {
                    const double sc = o.atol + o.rtol * fabs(yv[i]);
                    const double v = (f1[i] - f0[i]) / sc;
                    d2 += v * v;
                }
                d2 = sqrt(d2 / N) / h0;
                const double dm = fmax(d1, d2);
                const double h1 = dm <= 1e-15 ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, 0.2);
                h = fmin(fmin(100.0 * h0, h1), span);
            }
        }
    }
    if (st == CK_ST_OK) {
        while (t < te) {
            if (int64_t(na) + nj >= o.max_steps) { st = CK_ST_MAX_STEPS; break; }
            const bool clipped = (t + h >= te);
            const double hs = clipped ? te - t : h;
            const bool ok = METHOD == 0 ? ros4_step_lane(M, yv, P, hs, w, L) : rkf45_step_lane(M, yv, P, hs, w, L);
            double err;
            SV yn{&w[L.YN], wsS}, ev{&w[L.E], wsS};
            if (o.h_fixed > 0.0) {
                err = 0.0;
            } else if (!ok) {
                err = INFINITY;
            } else {
                err = wrms_lane(N, ev, yv, yn, o.rtol, o.atol);
                bool fin = true;
                for (int i = 0; i < N; i++) fin = fin && isfinite(yn[i]);
                if (!fin) err = INFINITY;
            }
            const bool acc = err < 1.0;
            if (acc) {
                for (int i = 0; i < N; i++) yv[i] = yn[i];
                t = clipped ? te : t + hs;
                na++;
            } else {
                nj++;
            }
            const double fac = o.h_fixed > 0.0 ? 1.0 : step_factor(err, qinv, acc);
            h = hs * fac;
            if (t < te && h < h_floor(t)) { st = CK_ST_H_UNDERFLOW; break; }
        }
    }
    if (t_io) t_io[r] = t;
    if (h_io) h_io[r] = h;
    status[r] = st;
    nacc[r] = na;
    nrej[r] = nj;
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
int64_t lane_ws_doubles_per_reactor(const DevMech &M, int method) {
    return LaneLayout(M.nsp, M.N, method == 0 ? 4 : 6).total;
}

int launch_rhs_lane(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *dydt,
                    double *ws, int64_t wsS, hipStream_t s) {
    const int B = 256;
    rhs_lane_kernel<<<dim3(unsigned((n + B - 1) / B)), dim3(B), 0, s>>>(M, n, y, ld, p, dydt, ws, wsS);
    return hipGetLastError() == hipSuccess ? CK_OK : CK_EHIP;
}

int launch_jac_lane(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *jac,
                    double *ws, int64_t wsS, hipStream_t s) {
    const int B = 256;
    jac_lane_kernel<<<dim3(unsigned((n + B - 1) / B)), dim3(B), 0, s>>>(M, n, y, ld, p, jac, ws, wsS);
    return hipGetLastError() == hipSuccess ? CK_OK : CK_EHIP;
}

int launch_integrate_lane(int method, const DevMech &M, int64_t n, double *y, int64_t ld, const double *p,
                          const double *t_end, double *t, double *h, const IntOpts &o, double *ws, int64_t wsS,
                          int32_t *status, int32_t *nacc, int32_t *nrej, hipStream_t s) {
    const int B = 64;
    dim3 g(unsigned((n + B - 1) / B));
    if (method == 0)
        integrate_lane_kernel<0><<<g, dim3(B), 0, s>>>(M, n, y, ld, p, t_end, t, h, o, ws, wsS, status, nacc, nrej);
    else
        integrate_lane_kernel<1><<<g, dim3(B), 0, s>>>(M, n, y, ld, p, t_end, t, h, o, ws, wsS, status, nacc, nrej);
    return hipGetLastError() == hipSuccess ? CK_OK : CK_EHIP;
}

}  // namespace ck
