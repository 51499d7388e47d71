// Wavefront-per-reactor kernels.  One 64-lane wavefront owns one reactor:
//   - species phases run lane-per-species (lane l holds state component l,
//     i.e. T on lane 0 and Y_{l-1} on lane l; a second register slot holds
//     component l + 64 when N > 64);
//   - reaction phases run lane-per-reaction, scattering rates of progress
//     into per-species accumulators in LDS with FP64 LDS atomics;
//   - the Rosenbrock matrix (I/(gamma h) - J) lives in registers, one row
//     per lane, and is factored by a fully unrolled partial-pivoting LU.
// This is the deep-vectorisation design of Section 4 applied to a 64-wide
// wavefront.  Integrators pull reactors from a device work queue (the
// paper's global atomic counter, Section 5.2) one reactor per wavefront, so
// reactors with different step counts never hold each other up (the waste of
// Eq. waste is zero by construction).  Every workgroup is one wavefront.
#include "ck_internal.h"
#include "kinetics.h"
#include "launch.h"

extern "C" __device__ unsigned long long __ockl_wfred_max_u64(unsigned long long);
extern "C" __device__ double __ockl_wfred_add_f64(double);

namespace ck {
namespace {

__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ double wsum(double v) { return __ockl_wfred_add_f64(v); }
__device__ __forceinline__ double bcast(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ bool wave_all(bool v) { return __ballot(!v) == 0ull; }

// ---------------------------------------------------------------------------------------
// LDS layout of one wavefront (doubles):
//   C[ns+1] G[ns] H[ns] WD[ns] | IW[64] (1/W_j padded with zeros) |
//   JC[ns*ldj + 64] TB[ns] DWT[ns] TROW[ns + 64]   (Jacobian kernels only)
// ---------------------------------------------------------------------------------------
struct Lds {
    double *C, *G, *H, *WD, *IW, *JC, *TB, *DWT, *TROW;
    int ldj;
};

__host__ __device__ inline int ldj_of(int ns) { return ns | 1; }
__host__ __device__ inline size_t lds_doubles(int ns, bool jac) {
    size_t d = size_t(ns + 1) + 3 * size_t(ns) + 64;
    if (jac) d += size_t(ns) * ldj_of(ns) + 64 + 2 * size_t(ns) + size_t(ns) + 64;
    return d;
}

__device__ Lds carve(double *b, int ns, bool jac) {
    Lds L;
    L.ldj = ldj_of(ns);
    L.C = b; b += ns + 1;
    L.G = b; b += ns;
    L.H = b; b += ns;
    L.WD = b; b += ns;
    L.IW = b; b += 64;
    if (jac) {
        L.JC = b; b += size_t(ns) * L.ldj + 64;
        L.TB = b; b += ns;
        L.DWT = b; b += ns;
        L.TROW = b;
    } else {
        L.JC = L.TB = L.DWT = L.TROW = nullptr;
    }
    return L;
}

__device__ void init_lds(const DevMech &M, const Lds &L) {
    const int l = lane_id();
    L.IW[l] = l < M.nsp ? M.invW[l] : 0.0;
    L.C[M.nsp] = 1.0;
    if (L.TROW) {
        for (int e = l; e < M.nsp + 64; e += 64) L.TROW[e] = 0.0;
        for (int e = M.nsp * L.ldj + l; e < M.nsp * L.ldj + 64; e += 64) L.JC[e] = 0.0;
    }
    __syncthreads();
}

template <int RPL>
struct Mix {
    TPow t;
    double rho, Wbar, Ctot, cpm;
    double cp[RPL], h[RPL], dcp[RPL];
};

// Species index held by register slot c of this lane, or -1 (slot 0 of lane 0 is T).
__device__ __forceinline__ int slot_species(int c, int ns) {
    const int i = lane_id() + 64 * c;
    return (i >= 1 && i <= ns) ? i - 1 : -1;
}

// Mixture state and per-species thermodynamics (Section 3: ideal gas, Eq. tfits).
template <int RPL, bool JAC>
__device__ void species_pass(const DevMech &M, const double (&y)[RPL], double P, const Lds &L, Mix<RPL> &x) {
    const int ns = M.nsp;
    const double T = bcast(y[0], 0);
    x.t = tpow(T);
    double sy = 0.0;
#pragma unroll
    for (int c = 0; c < RPL; c++) {
        const int k = slot_species(c, ns);
        if (k >= 0) sy += y[c] * M.invW[k];
    }
    const double S = wsum(sy);
    x.rho = P / (M.R * T * S);
    x.Wbar = 1.0 / S;
    x.Ctot = P * x.t.invT / M.R;
    double cpp = 0.0;
#pragma unroll
    for (int c = 0; c < RPL; c++) {
        const int k = slot_species(c, ns);
        if (k >= 0) {
            L.C[k] = x.rho * y[c] * M.invW[k];
            const Thermo th = species_thermo(M, k, x.t);
            L.G[k] = th.h - th.s;
            L.H[k] = th.h;
            L.WD[k] = 0.0;
            x.cp[c] = th.cp;
            x.h[c] = th.h;
            x.dcp[c] = th.dcp;
            cpp += y[c] * th.cp * M.invW[k];
        } else {
            x.cp[c] = x.h[c] = x.dcp[c] = 0.0;
        }
    }
    x.cpm = wsum(cpp) * M.R;
    if (JAC) {
        const int l = lane_id();
        const int tot = ns * L.ldj;
        for (int e = l; e < tot; e += 64) L.JC[e] = 0.0;
        for (int e = l; e < ns; e += 64) {
            L.TB[e] = 0.0;
            L.DWT[e] = 0.0;
        }
    }
    __syncthreads();
}

// Rates of progress (Eqs. wdot, kfor, krev, kc), scattered into WD; with JAC
// also d wdot / dC (into JC, and the third-body rank-one part into TB) and
// d wdot / dT at fixed C (into DWT).
template <bool JAC>
__device__ void reaction_pass(const DevMech &M, const Lds &L, const TPow &t, double Ctot) {
    const int nr = M.nrxn;
    auto Cg = [&](int k) { return L.C[k]; };
    auto Gg = [&](int k) { return L.G[k]; };
    auto Hg = [&](int k) { return L.H[k]; };
    for (int i = lane_id(); i < nr; i += 64) {
        Rate q;
        reaction_rate<JAC>(M, i, t, Ctot, Cg, Gg, Hg, q);
        const double Rn = q.kf * q.pf - q.kr * q.pr;
        const double qi = q.c * Rn;
        const int nsl = M.nslot[i], nre = M.nreac[i];
        for (int s = 0; s < nsl; s++) {
            const int sp = M.slot_sp[size_t(s) * nr + i];
            const int nu = M.slot_nu[size_t(s) * nr + i];
            atomicAdd(&L.WD[sp], (s < nre ? -nu : nu) * qi);
        }
        if (JAC) {
            const double dqT = q.c * (q.kf * q.dlnkf * q.pf - q.kr * q.dlnkr * q.pr) + Rn * q.dcdT;
            for (int b = 0; b < nsl; b++) {
                const int spb = M.slot_sp[size_t(b) * nr + i];
                const double d = dprod_slot(M, i, b, Cg);
                const double dq = q.c * (b < nre ? q.kf * d : -q.kr * d);
                for (int a = 0; a < nsl; a++) {
                    const int spa = M.slot_sp[size_t(a) * nr + i];
                    const int nua = M.slot_nu[size_t(a) * nr + i];
                    atomicAdd(&L.JC[spa * L.ldj + spb], (a < nre ? -nua : nua) * dq);
                }
            }
            const int eb = M.eff_begin[i], ec = M.eff_count[i];
            for (int a = 0; a < nsl; a++) {
                const int spa = M.slot_sp[size_t(a) * nr + i];
                const int nua = M.slot_nu[size_t(a) * nr + i];
                const double v = (a < nre ? -nua : nua);
                atomicAdd(&L.DWT[spa], v * dqT);
                if (q.dcdM != 0.0) {
                    const double base = v * Rn * q.dcdM;
                    atomicAdd(&L.TB[spa], base);
                    for (int e = 0; e < ec; e++) atomicAdd(&L.JC[spa * L.ldj + M.eff_sp[eb + e]], base * M.eff_am1[eb + e]);
                }
            }
        }
    }
    __syncthreads();
}

// Eqs. ydot and tdot from the accumulated production rates.
template <int RPL>
__device__ void finish_rhs(const DevMech &M, const Lds &L, const Mix<RPL> &x, double (&f)[RPL]) {
    const int ns = M.nsp;
    double qp = 0.0;
#pragma unroll
    for (int c = 0; c < RPL; c++) {
        const int k = slot_species(c, ns);
        if (k >= 0) {
            const double wd = L.WD[k];
            f[c] = M.W[k] * wd / x.rho;
            qp += M.R * x.t.T * x.h[c] * wd;
        } else {
            f[c] = 0.0;
        }
    }
    const double Q = wsum(qp);
    if (lane_id() == 0) f[0] = -Q / (x.rho * x.cpm);
}

template <int RPL>
__device__ void rhs_wave(const DevMech &M, const Lds &L, const double (&y)[RPL], double P, double (&f)[RPL]) {
    Mix<RPL> x;
    species_pass<RPL, false>(M, y, P, L, x);
    reaction_pass<false>(M, L, x.t, x.Ctot);
    finish_rhs<RPL>(M, L, x, f);
    __syncthreads();
}

// Row of J owned by this lane: J[l][0] = c0, J[l][1 + j] = IW[j] * (alpha * src[j] + beta).
struct JRow {
    const double *src;
    double alpha, beta, c0;
};

// Chain rule from (d wdot/dC, d wdot/dT) to J = df/dy (N <= 64, one row per lane).
__device__ JRow jac_prepare(const DevMech &M, const Lds &L, const Mix<1> &x, double y0, double fT) {
    const int ns = M.nsp, lane = lane_id();
    const int k = slot_species(0, ns);
    const bool valid = k >= 0;
    const double T = x.t.T, RT = M.R * T;
    double jcc = 0.0, colH = 0.0, resid = 0.0, a = 0.0, col0 = 0.0, TBk = 0.0, WDk = 0.0, DWTk = 0.0;
    if (valid) {
        const double *row = &L.JC[k * L.ldj];
        for (int j = 0; j < ns; j++) {
            jcc += row[j] * L.C[j];
            colH += L.H[j] * L.JC[j * L.ldj + k];
        }
        TBk = L.TB[k];
        WDk = L.WD[k];
        DWTk = L.DWT[k];
        jcc += TBk * x.Ctot;
        colH *= RT;
        resid = WDk - jcc;
        a = M.W[k] * x.Wbar * resid / x.rho;
        col0 = (M.W[k] / x.rho) * (DWTk + resid * x.t.invT);
    }
    const double Hk = RT * x.h[0];
    const double sumHTB = wsum(valid ? Hk * TBk : 0.0);
    const double sumHJCC = wsum(valid ? Hk * jcc : 0.0);
    const double dQT = wsum(valid ? M.R * x.cp[0] * WDk + Hk * (DWTk - jcc * x.t.invT) : 0.0);
    const double sdcp = wsum(valid ? y0 * M.R * x.dcp[0] * M.invW[k] : 0.0);
    const double D = x.rho * x.cpm;
    if (valid) {
        const double dQ = M.invW[k] * (x.rho * (colH + sumHTB) - x.Wbar * sumHJCC);
        const double dD = x.rho * M.invW[k] * (M.R * x.cp[0] - x.cpm * x.Wbar);
        L.TROW[k] = -(dQ + fT * dD) / D * M.W[k];
    }
    const double J00 = -(dQT + fT * (-x.rho * x.cpm * x.t.invT + x.rho * sdcp)) / D;
    __syncthreads();
    JRow r;
    if (lane == 0) {
        r.src = L.TROW;
        r.alpha = 1.0;
        r.beta = 0.0;
        r.c0 = J00;
    } else if (valid) {
        r.src = &L.JC[k * L.ldj];
        r.alpha = M.W[k];
        r.beta = M.W[k] * TBk + a;
        r.c0 = col0;
    } else {
        r.src = L.TROW;
        r.alpha = 0.0;
        r.beta = 0.0;
        r.c0 = 0.0;
    }
    return r;
}

// f(y) and the Jacobian rows (registers) for N <= NP <= 64.
template <int NP>
__device__ void jac_rows(const DevMech &M, const Lds &L, double y, double P, double (&a)[NP], double &f) {
    Mix<1> x;
    const double yy[1] = {y};
    double ff[1];
    species_pass<1, true>(M, yy, P, L, x);
    reaction_pass<true>(M, L, x.t, x.Ctot);
    finish_rhs<1>(M, L, x, ff);
    f = ff[0];
    const JRow r = jac_prepare(M, L, x, y, bcast(ff[0], 0));
    a[0] = r.c0;
#pragma unroll
    for (int j = 1; j < NP; j++) a[j] = L.IW[j - 1] * (r.alpha * r.src[j - 1] + r.beta);
    __syncthreads();
}

// ---------------------------------------------------------------------------------------
// dense LU with partial pivoting, one row per lane, fully unrolled over NP columns
// ---------------------------------------------------------------------------------------
template <int NP>
struct LU {
    int piv[NP];      // lane holding the pivot row of column k (wave-uniform)
    int ord;          // this lane's pivot order
    double dinv;      // 1 / U[ord][ord]
    bool ok;
};

template <int NP>
__device__ void lu_factor(double (&a)[NP], LU<NP> &f) {
    const int lane = lane_id();
    bool done = false;
    f.ord = NP;
    f.dinv = 0.0;
    f.ok = true;
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const unsigned long long key = done ? 0ull : (unsigned long long)__double_as_longlong(fabs(a[k]));
        const unsigned long long mx = __ockl_wfred_max_u64(key);
        const int p = __builtin_ctzll(__ballot(!done && key == mx));
        f.piv[k] = p;
        f.ok = f.ok && (mx != 0ull);
        const double inv = 1.0 / bcast(a[k], p);
        if (lane == p) {
            done = true;
            f.ord = k;
            f.dinv = inv;
        }
        const double l = done ? 0.0 : a[k] * inv;
        if (!done) a[k] = l;
#pragma unroll
        for (int j = k + 1; j < NP; j++) a[j] = fma(-l, bcast(a[j], p), a[j]);
    }
}

// Solve (L U) x = P b in place; b and x distributed one component per lane.
template <int NP>
__device__ double lu_solve(const double (&a)[NP], const LU<NP> &f, double b) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const double yk = bcast(b, f.piv[k]);
        if (f.ord > k) b = fma(-a[k], yk, b);
    }
    double x = 0.0;
#pragma unroll
    for (int k = NP - 1; k >= 0; k--) {
        const double xk = bcast(b * f.dinv, f.piv[k]);
        if (lane == k) x = xk;
        if (f.ord < k) b = fma(-a[k], xk, b);
    }
    return x;
}

// ---------------------------------------------------------------------------------------
// one steps
// ---------------------------------------------------------------------------------------
template <int NP>
struct Ros4Wave {
    static constexpr double qinv = 0.25;
    __device__ static bool step(const DevMech &M, const Lds &L, double y, double P, double h, double &ynew,
                                double &e) {
        const int lane = lane_id();
        double a[NP];
        double f;
        jac_rows<NP>(M, L, y, P, a, f);
        const double dg = 1.0 / (Ros4::gamma * h);
#pragma unroll
        for (int j = 0; j < NP; j++) a[j] = (j == lane) ? dg - a[j] : -a[j];
        LU<NP> lu;
        lu_factor<NP>(a, lu);
        const double ih = 1.0 / h;
        const double u1 = lu_solve<NP>(a, lu, f);
        double yt[1] = {y + Ros4::a21 * u1}, ft[1];
        rhs_wave<1>(M, L, yt, P, ft);
        const double u2 = lu_solve<NP>(a, lu, ft[0] + (Ros4::c21 * u1) * ih);
        yt[0] = y + Ros4::a31 * u1 + Ros4::a32 * u2;
        rhs_wave<1>(M, L, yt, P, ft);
        const double u3 = lu_solve<NP>(a, lu, ft[0] + (Ros4::c31 * u1 + Ros4::c32 * u2) * ih);
        const double u4 = lu_solve<NP>(a, lu, ft[0] + (Ros4::c41 * u1 + Ros4::c42 * u2 + Ros4::c43 * u3) * ih);
        ynew = y + Ros4::m1 * u1 + Ros4::m2 * u2 + Ros4::m3 * u3 + Ros4::m4 * u4;
        e = Ros4::e1 * u1 + Ros4::e2 * u2 + Ros4::e3 * u3 + Ros4::e4 * u4;
        return lu.ok;
    }
};

template <int RPL>
struct Rkf45Wave {
    static constexpr double qinv = 0.2;
    __device__ static void stage(const DevMech &M, const Lds &L, const double (&yt)[RPL], double P, double h,
                                 double (&k)[RPL]) {
        rhs_wave<RPL>(M, L, yt, P, k);
#pragma unroll
        for (int c = 0; c < RPL; c++) k[c] *= h;
    }
    __device__ static bool step(const DevMech &M, const Lds &L, const double (&y)[RPL], double P, double h,
                                double (&ynew)[RPL], double (&e)[RPL]) {
        double k1[RPL], k2[RPL], k3[RPL], k4[RPL], k5[RPL], k6[RPL], yt[RPL];
        stage(M, L, y, P, h, k1);
#pragma unroll
        for (int c = 0; c < RPL; c++) yt[c] = y[c] + Rkf45::a21 * k1[c];
        stage(M, L, yt, P, h, k2);
#pragma unroll
        for (int c = 0; c < RPL; c++) yt[c] = y[c] + Rkf45::a31 * k1[c] + Rkf45::a32 * k2[c];
        stage(M, L, yt, P, h, k3);
#pragma unroll
        for (int c = 0; c < RPL; c++) yt[c] = y[c] + Rkf45::a41 * k1[c] + Rkf45::a42 * k2[c] + Rkf45::a43 * k3[c];
        stage(M, L, yt, P, h, k4);
#pragma unroll
        for (int c = 0; c < RPL; c++)
            yt[c] = y[c] + Rkf45::a51 * k1[c] + Rkf45::a52 * k2[c] + Rkf45::a53 * k3[c] + Rkf45::a54 * k4[c];
        stage(M, L, yt, P, h, k5);
#pragma unroll
        for (int c = 0; c < RPL; c++)
            yt[c] = y[c] + Rkf45::a61 * k1[c] + Rkf45::a62 * k2[c] + Rkf45::a63 * k3[c] + Rkf45::a64 * k4[c] +
                    Rkf45::a65 * k5[c];
        stage(M, L, yt, P, h, k6);
#pragma unroll
        for (int c = 0; c < RPL; c++) {
            ynew[c] = y[c] + Rkf45::b1 * k1[c] + Rkf45::b3 * k3[c] + Rkf45::b4 * k4[c] + Rkf45::b5 * k5[c];
            e[c] = Rkf45::d1 * k1[c] + Rkf45::d3 * k3[c] + Rkf45::d4 * k4[c] + Rkf45::d5 * k5[c] + Rkf45::d6 * k6[c];
        }
        return true;
    }
};

// ---------------------------------------------------------------------------------------
// per-reactor driver (Algorithm 1 on one wavefront)
// ---------------------------------------------------------------------------------------
template <int RPL>
__device__ double wrms_wave(int N, const double (&e)[RPL], const double (&a)[RPL], const double (&b)[RPL],
                            double rtol, double atol) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < RPL; c++) {
        const int i = lane_id() + 64 * c;
        if (i < N) {
            const double sc = atol + rtol * fmax(fabs(a[c]), fabs(b[c]));
            const double r = e[c] / sc;
            s += r * r;
        }
    }
    return sqrt(wsum(s) / N);
}

template <int RPL>
__device__ bool all_finite(int N, const double (&v)[RPL]) {
    bool ok = true;
#pragma unroll
    for (int c = 0; c < RPL; c++) ok = ok && (lane_id() + 64 * c >= N || isfinite(v[c]));
    return wave_all(ok);
}

// Step adapters with a common (array) interface.
template <int NP>
struct Ros4Adapter {
    static constexpr int RPL = 1;
    static constexpr double qinv = 0.25;
    __device__ static bool step(const DevMech &M, const Lds &L, const double (&y)[1], double P, double h,
                                double (&yn)[1], double (&e)[1]) {
        return Ros4Wave<NP>::step(M, L, y[0], P, h, yn[0], e[0]);
    }
};

template <class S>
__device__ void integrate_reactor(const DevMech &M, const Lds &L, int64_t r, double *y, int64_t ld, const double *p,
                                  const double *t_end, double *t_io, double *h_io, const IntOpts &o, int32_t *status,
                                  int32_t *nacc, int32_t *nrej) {
    constexpr int RPL = S::RPL;
    const int N = M.N;
    const int lane = lane_id();
    double yv[RPL];
#pragma unroll
    for (int c = 0; c < RPL; c++) {
        const int i = lane + 64 * c;
        yv[c] = i < N ? y[int64_t(i) * ld + r] : 0.0;
    }
    const double P = p[r];
    const double te = t_end[r];
    double t = t_io ? t_io[r] : 0.0;
    double h = h_io ? h_io[r] : 0.0;
    int st = CK_ST_OK;
    int na = 0, nj = 0;
    if (!all_finite<RPL>(N, yv)) {
        st = CK_ST_NONFINITE;
        h = 0.0;
    } else if (o.h_fixed > 0.0) {
        h = o.h_fixed;
    } else if (!(h > 0.0)) {
        if (o.h0 > 0.0) {
            h = o.h0;
        } else if (t < te) {
            // EstimateH0 (Hairer, Norsett & Wanner II.4, order 4)
            double f0[RPL], f1[RPL], yt[RPL];
            rhs_wave<RPL>(M, L, yv, P, f0);
            if (!all_finite<RPL>(N, f0)) {
                st = CK_ST_NONFINITE;
                h = 0.0;
            } else {
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int c = 0; c < RPL; c++) {
                    if (lane + 64 * c < N) {
                        const double sc = o.atol + o.rtol * fabs(yv[c]);
                        s0 += (yv[c] / sc) * (yv[c] / sc);
                        s1 += (f0[c] / sc) * (f0[c] / sc);
                    }
                }
                const double d0 = sqrt(wsum(s0) / N), d1 = sqrt(wsum(s1) / N);
                const double span = te - t;
                double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
                h0 = fmin(h0, span);
#pragma unroll
                for (int c = 0; c < RPL; c++) yt[c] = yv[c] + h0 * f0[c];
                rhs_wave<RPL>(M, L, yt, P, f1);
                double s2 = 0.0;
#pragma unroll
                for (int c = 0; c < RPL; c++) {
                    if (lane + 64 * c < N) {
                        const double sc = o.atol + o.rtol * fabs(yv[c]);
                        const double v = (f1[c] - f0[c]) / sc;
                        s2 += v * v;
                    }
                }
                const double d2 = sqrt(wsum(s2) / N) / h0;
                const double dm = fmax(d1, d2);
                const double h1 = dm <= 1e-15 ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, 0.2);
                h = fmin(fmin(100.0 * h0, h1), span);
            }
        }
    }
    if (st == CK_ST_OK) {
        while (t < te) {
            if (int64_t(na) + nj >= o.max_steps) {
                st = CK_ST_MAX_STEPS;
                break;
            }
            const bool clipped = (t + h >= te);
            const double hs = clipped ? te - t : h;
            double yn[RPL], e[RPL];
            const bool ok = S::step(M, L, yv, P, hs, yn, e);
            double err;
            if (o.h_fixed > 0.0)
                err = 0.0;
            else if (!ok)
                err = INFINITY;
            else {
                err = wrms_wave<RPL>(N, e, yv, yn, o.rtol, o.atol);
                if (!all_finite<RPL>(N, yn)) err = INFINITY;
            }
            const bool acc = err < 1.0;
            if (acc) {
#pragma unroll
                for (int c = 0; c < RPL; c++) yv[c] = yn[c];
                t = clipped ? te : t + hs;
                na++;
            } else {
                nj++;
            }
            const double fac = o.h_fixed > 0.0 ? 1.0 : step_factor(err, S::qinv, acc);
            h = hs * fac;
            if (t < te && h < h_floor(t)) {
                st = CK_ST_H_UNDERFLOW;
                break;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < RPL; c++) {
        const int i = lane + 64 * c;
        if (i < N) y[int64_t(i) * ld + r] = yv[c];
    }
    if (lane == 0) {
        if (t_io) t_io[r] = t;
        if (h_io) h_io[r] = h;
        status[r] = st;
        nacc[r] = na;
        nrej[r] = nj;
    }
}

template <int R>
struct Rkf45S {
    static constexpr int RPL = R;
    static constexpr double qinv = 0.2;
    __device__ static bool step(const DevMech &M, const Lds &L, const double (&y)[R], double P, double h,
                                double (&yn)[R], double (&e)[R]) {
        return Rkf45Wave<R>::step(M, L, y, P, h, yn, e);
    }
};

// Consecutive workgroups are dispatched round-robin over the 8 XCDs; map them so that
// the reactors handled on one XCD are contiguous (their state shares L2 lines).  The grid
// is a multiple of 8 workgroups, which makes the map a permutation of [0, nb).
__device__ __forceinline__ int64_t xcd_reactor(int64_t b, int64_t nb) {
    const int64_t per = nb / 8;
    const int64_t x = b % 8, i = b / 8;
    return x * per + i;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------------------
template <int RPL>
__global__ void __launch_bounds__(64) rhs_wave_kernel(DevMech M, int64_t n, const double *y, int64_t ld,
                                                      const double *p, double *dydt) {
    extern __shared__ double lds_raw[];
    const Lds L = carve(lds_raw, M.nsp, false);
    init_lds(M, L);
    const int N = M.N, lane = lane_id();
    const int64_t nb = int64_t(gridDim.x);
    const int64_t r = xcd_reactor(blockIdx.x, nb);
    if (r >= n) return;
    double yv[RPL], f[RPL];
#pragma unroll
    for (int c = 0; c < RPL; c++) {
        const int i = lane + 64 * c;
        yv[c] = i < N ? y[int64_t(i) * ld + r] : 0.0;
    }
    rhs_wave<RPL>(M, L, yv, p[r], f);
#pragma unroll
    for (int c = 0; c < RPL; c++) {
        const int i = lane + 64 * c;
        if (i < N) dydt[int64_t(i) * ld + r] = f[c];
    }
}

__global__ void __launch_bounds__(64) jac_wave_kernel(DevMech M, int64_t n, const double *y, int64_t ld,
                                                      const double *p, double *jac) {
    extern __shared__ double lds_raw[];
    const Lds L = carve(lds_raw, M.nsp, true);
    init_lds(M, L);
    const int N = M.N, lane = lane_id();
    const int64_t r = xcd_reactor(blockIdx.x, int64_t(gridDim.x));
    if (r >= n) return;
    const double yl = lane < N ? y[int64_t(lane) * ld + r] : 0.0;
    Mix<1> x;
    const double yy[1] = {yl};
    double ff[1];
    species_pass<1, true>(M, yy, p[r], L, x);
    reaction_pass<true>(M, L, x.t, x.Ctot);
    finish_rhs<1>(M, L, x, ff);
    const JRow row = jac_prepare(M, L, x, yl, bcast(ff[0], 0));
    if (lane < N) {
        double *out = jac + int64_t(lane) * N * ld + r;
        out[0] = row.c0;
        for (int j = 1; j < N; j++) out[int64_t(j) * ld] = L.IW[j - 1] * (row.alpha * row.src[j - 1] + row.beta);
    }
}

template <class S>
__global__ void __launch_bounds__(64) integrate_wave_kernel(DevMech M, int64_t n, double *y, int64_t ld,
                                                            const double *p, const double *t_end, double *t_io,
                                                            double *h_io, IntOpts o, unsigned *queue,
                                                            int32_t *status, int32_t *nacc, int32_t *nrej, bool jac) {
    extern __shared__ double lds_raw[];
    const Lds L = carve(lds_raw, M.nsp, jac);
    init_lds(M, L);
    for (;;) {
        unsigned v = 0;
        if (lane_id() == 0) v = atomicAdd(queue, 1u);
        const int64_t r = int64_t(unsigned(__builtin_amdgcn_readfirstlane(int(v))));
        if (r >= n) break;
        integrate_reactor<S>(M, L, r, y, ld, p, t_end, t_io, h_io, o, status, nacc, nrej);
        __syncthreads();
    }
}

__global__ void zero_u32_kernel(unsigned *q) { *q = 0u; }

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
namespace {
int pad_np(int N) { return ((N + 7) / 8) * 8; }

template <class S>
int launch_int(const DevMech &M, int64_t n, double *y, int64_t ld, const double *p, const double *t_end, double *t,
               double *h, const IntOpts &o, unsigned *queue, int32_t *status, int32_t *nacc, int32_t *nrej, bool jac,
               hipStream_t s) {
    const size_t lds = lds_doubles(M.nsp, jac) * sizeof(double);
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CK_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return CK_EHIP;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, integrate_wave_kernel<S>, 64, lds) != hipSuccess || per < 1)
        return CK_EHIP;
    int64_t grid = int64_t(cus) * per;
    if (grid > n) grid = n;
    zero_u32_kernel<<<1, 1, 0, s>>>(queue);
    integrate_wave_kernel<S><<<dim3(unsigned(grid)), dim3(64), lds, s>>>(M, n, y, ld, p, t_end, t, h, o, queue,
                                                                          status, nacc, nrej, jac);
    return hipGetLastError() == hipSuccess ? CK_OK : CK_EHIP;
}
}  // namespace

bool wave_supported(const DevMech &M, int method, int precision) {
    if (precision != CK_PREC_FP64) return false;
    if (method == 0) return M.N <= 64;
    return M.N <= 128;
}

size_t wave_ws_bytes(const DevMech &, int64_t) { return 256; }

int launch_rhs_wave(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *dydt,
                    hipStream_t s) {
    const size_t lds = lds_doubles(M.nsp, false) * sizeof(double);
    const unsigned grid = unsigned((n + 7) / 8 * 8);
    if (M.N <= 64)
        rhs_wave_kernel<1><<<dim3(grid), dim3(64), lds, s>>>(M, n, y, ld, p, dydt);
    else
        rhs_wave_kernel<2><<<dim3(grid), dim3(64), lds, s>>>(M, n, y, ld, p, dydt);
    return hipGetLastError() == hipSuccess ? CK_OK : CK_EHIP;
}

int launch_jac_wave(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *jac,
                    hipStream_t s) {
    if (M.N > 64) return CK_EUNSUPPORTED;
    const size_t lds = lds_doubles(M.nsp, true) * sizeof(double);
    const unsigned grid = unsigned((n + 7) / 8 * 8);
    jac_wave_kernel<<<dim3(grid), dim3(64), lds, s>>>(M, n, y, ld, p, jac);
    return hipGetLastError() == hipSuccess ? CK_OK : CK_EHIP;
}

int launch_integrate_wave(int method, const DevMech &M, int64_t n, double *y, int64_t ld, const double *p,
                          const double *t_end, double *t, double *h, const IntOpts &o, void *ws, int32_t *status,
                          int32_t *nacc, int32_t *nrej, hipStream_t s) {
    unsigned *q = static_cast<unsigned *>(ws);
    if (method == 1) {
        if (M.N <= 64) return launch_int<Rkf45S<1>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, false, s);
        return launch_int<Rkf45S<2>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, false, s);
    }
    switch (pad_np(M.N)) {
        case 8: return launch_int<Ros4Adapter<8>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, true, s);
        case 16: return launch_int<Ros4Adapter<16>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, true, s);
        case 24: return launch_int<Ros4Adapter<24>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, true, s);
        case 32: return launch_int<Ros4Adapter<32>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, true, s);
        case 40: return launch_int<Ros4Adapter<40>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, true, s);
        case 48: return launch_int<Ros4Adapter<48>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, true, s);
        case 56: return launch_int<Ros4Adapter<56>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, true, s);
        case 64: return launch_int<Ros4Adapter<64>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, true, s);
        default: return CK_EUNSUPPORTED;
    }
}

}  // namespace ck
