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
extern "C" __device__ unsigned __ockl_wfred_max_u32(unsigned);
extern "C" __device__ double __ockl_wfred_add_f64(double);

namespace ck {
namespace {

__device__ __forceinline__ int lane_id() { return __lane_id(); }
// Value the compiler cannot see through: keeps cheap per-phase values (lane masks, pivot
// lanes) from being hoisted across phases, where they would only occupy and spill SGPRs.
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ int lane_fresh() { return opaque(__lane_id()); }
// The same for a wave-uniform value, kept in a scalar register.
__device__ __forceinline__ int opaque_s(int v) {
    asm volatile("" : "+s"(v));
    return v;
}
__device__ __forceinline__ double wsum(double v) { return __ockl_wfred_add_f64(v); }
__device__ __forceinline__ double bcast(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ bool wave_all(bool v) { return __ballot(!v) == 0ull; }

// ---------------------------------------------------------------------------------------
// LDS layout of one wavefront (doubles):
//   C[ns+1] G[ns] H[ns] WD[ns] | IW[64] (1/W_j padded with zeros) | VX[64] (broadcast scratch) |
//   JC[ns*ldj + 64] TB[ns] DWT[ns] TROW[ns + 64]   (Jacobian kernels only)
// JC holds d wdot / dC for a window of `win` consecutive columns (all ns columns when the
// Jacobian is staged in one piece), leading dimension ldj = win | 1.
// ---------------------------------------------------------------------------------------
struct Lds {
    double *C, *G, *H, *WD, *IW, *VX, *JC, *TB, *DWT, *TROW;
    double *park;   // this wavefront's slice of the workspace for parked LU rows ([NP][64]), or null
    int ldj;
    int cv;         // 0: constant pressure (p = pressure); 1: constant volume (p = density)
};

__host__ __device__ inline int ldj_of(int win) { return win | 1; }
__host__ __device__ inline size_t lds_doubles(int ns, bool jac, int win) {
    size_t d = size_t(ns + 1) + 3 * size_t(ns) + 128;
    if (jac) d += size_t(ns) * ldj_of(win) + 64 + 2 * size_t(ns) + size_t(ns) + 64;
    return d;
}
__host__ __device__ inline size_t lds_doubles(int ns, bool jac) { return lds_doubles(ns, jac, ns); }

__device__ __forceinline__ Lds carve(double *b, int ns, bool jac, int win) {
    Lds L;
    L.ldj = ldj_of(win);
    L.C = b; b += ns + 1;
    L.G = b; b += ns;
    L.H = b; b += ns;
    L.WD = b; b += ns;
    L.IW = b; b += 64;
    L.VX = b; b += 64;
    if (jac) {
        L.JC = b; b += size_t(ns) * L.ldj + 64;
        L.TB = b; b += ns;
        L.DWT = b; b += ns;
        L.TROW = b;
    } else {
        L.JC = L.TB = L.DWT = L.TROW = nullptr;
    }
    L.park = nullptr;
    L.cv = 0;
    return L;
}
__device__ __forceinline__ Lds carve(double *b, int ns, bool jac) { return carve(b, ns, jac, ns); }

__device__ __forceinline__ void init_lds(const DevMech &M, const Lds &L) {
    const int l = lane_id();
    L.IW[l] = l < M.nsp ? M.invW()[l] : 0.0;
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
__device__ __forceinline__ int slot_species(int c, int ns, int lane) {
    const int i = lane + 64 * c;
    return (i >= 1 && i <= ns) ? i - 1 : -1;
}

// Mixture state and per-species thermodynamics (Section 3: ideal gas, Eq. tfits).
template <int RPL, bool JAC, bool ZERO_JC = true>
__device__ __forceinline__ void species_pass(const DevMech &M, const double (&y)[RPL], double P, const Lds &L, Mix<RPL> &x) {
    const int ns = M.nsp;
    const int lane = lane_fresh();
    const double T = bcast(y[0], 0);
    x.t = tpow(T);
    double sy = 0.0;
#pragma unroll
    for (int c = 0; c < RPL; c++) {
        const int k = slot_species(c, ns, lane);
        if (k >= 0) sy += y[c] * M.invW()[k];
    }
    const double S = wsum(sy);
    if (L.cv) {   // constant volume: P holds the (fixed) density
        x.rho = P;
        x.Ctot = P * S;
    } else {
        x.rho = P / (M.R * T * S);
        x.Ctot = P * x.t.invT / M.R;
    }
    x.Wbar = 1.0 / S;
    double cpp = 0.0;
#pragma unroll
    for (int c = 0; c < RPL; c++) {
        const int k = slot_species(c, ns, lane);
        if (k >= 0) {
            L.C[k] = x.rho * y[c] * M.invW()[k];
            const Thermo th = species_thermo(M, k, x.t);
            L.G[k] = th.h - th.s;
            L.H[k] = th.h;
            L.WD[k] = 0.0;
            x.cp[c] = th.cp;
            x.h[c] = th.h;
            x.dcp[c] = th.dcp;
            cpp += y[c] * th.cp * M.invW()[k];
        } else {
            x.cp[c] = x.h[c] = x.dcp[c] = 0.0;
        }
    }
    x.cpm = wsum(cpp) * M.R;
    if (JAC) {
        const int l = lane;
        const int tot = ns * L.ldj;
        if (ZERO_JC)
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
// d wdot / dT at fixed C (into DWT).  With a column window [c0, c0 + win) only
// those columns of d wdot / dC are accumulated, and WD, TB and DWT only when
// `first` is set.
// Column scatter of reaction i needs three scalars besides the concentrations: c k_f, c k_r and
// R_net dc/d[M].  mode 1 stores them in this lane's column of `cache` (entry (3 it + v) * 64 for
// the lane's it-th reaction); mode 2 reads them back instead of evaluating the rate constants, so
// a later column window costs a record load and the scatter only.
template <bool JAC>
__device__ __forceinline__ void reaction_pass(const DevMech &M, const Lds &L, const TPow &t, double Ctot, int c0, int win,
                              bool first, double *cache = nullptr, int mode = 0) {
    const int nr = M.nrxn;
    auto Cg = [&](int k) { return L.C[k]; };
    auto Gg = [&](int k) { return L.G[k]; };
    auto Hg = [&](int k) { return L.H[k]; };
    int it = 0;
    for (int i = lane_fresh(); i < nr; i += 64, it++) {
        const RxnRec R = M.rx[i];
        const int nmax = __builtin_amdgcn_readfirstlane(R.blk_slots);
        Slots S;
        load_slots(R, Cg, S, nmax);
        double ckf, ckr, rdm;
        if (JAC && mode == 2) {
            ckf = cache[(3 * it) * 64];
            ckr = cache[(3 * it + 1) * 64];
            rdm = cache[(3 * it + 2) * 64];
        } else {
            Rate q;
            reaction_rate<JAC>(M, R, S, nmax, t, Ctot, Cg, Gg, Hg, q);
            const double Rn = q.kf * q.pf - q.kr * q.pr;
            if (first) {
                const double qi = q.c * Rn;
#pragma unroll
                for (int s = 0; s < kMaxSlots; s++) {
                    if (s >= nmax) break;
                    if (S.sgn[s] != 0) atomicAdd(&L.WD[S.sp[s]], (S.sgn[s] * S.nu[s]) * qi);
                }
            }
            ckf = q.c * q.kf;
            ckr = q.c * q.kr;
            rdm = JAC ? Rn * q.dcdM : 0.0;
            if (JAC && first) {
                const double dqT = q.c * (q.kf * q.dlnkf * q.pf - q.kr * q.dlnkr * q.pr) + Rn * q.dcdT;
#pragma unroll
                for (int a = 0; a < kMaxSlots; a++) {
                    if (a >= nmax) break;
                    if (S.sgn[a] == 0) continue;
                    const double v = S.sgn[a] * S.nu[a];
                    atomicAdd(&L.DWT[S.sp[a]], v * dqT);
                    if (q.dcdM != 0.0) atomicAdd(&L.TB[S.sp[a]], v * rdm);
                }
            }
            if (JAC && mode == 1) {
                cache[(3 * it) * 64] = ckf;
                cache[(3 * it + 1) * 64] = ckr;
                cache[(3 * it + 2) * 64] = rdm;
            }
        }
        if (JAC) {
#pragma unroll
            for (int b = 0; b < kMaxSlots; b++) {
                if (b >= nmax) break;
                const int col = S.sp[b] - c0;
                if (S.sgn[b] == 0 || col < 0 || col >= win) continue;
                const double d = dprod_slot(S, b, nmax);
                const double dq = S.sgn[b] < 0 ? ckf * d : -ckr * d;
#pragma unroll
                for (int a = 0; a < kMaxSlots; a++) {
                    if (a >= nmax) break;
                    if (S.sgn[a] != 0) atomicAdd(&L.JC[S.sp[a] * L.ldj + col], (S.sgn[a] * S.nu[a]) * dq);
                }
            }
            if (rdm != 0.0) {
                const int eb = R.eff_begin, ec = rx_neff(R.meta);
#pragma unroll
                for (int a = 0; a < kMaxSlots; a++) {
                    if (a >= nmax) break;
                    if (S.sgn[a] == 0) continue;
                    const double base = (S.sgn[a] * S.nu[a]) * rdm;
                    for (int e = 0; e < ec; e++) {
                        const EffRec E = M.eff[eb + e];
                        const int col = E.sp - c0;
                        if (col >= 0 && col < win) atomicAdd(&L.JC[S.sp[a] * L.ldj + col], base * E.am1);
                    }
                }
            }
        }
    }
    __syncthreads();
}

template <bool JAC>
__device__ __forceinline__ void reaction_pass(const DevMech &M, const Lds &L, const TPow &t, double Ctot) {
    reaction_pass<JAC>(M, L, t, Ctot, 0, M.nsp, true);
}

// Eqs. ydot and tdot from the accumulated production rates.  Constant volume: internal energies
// U_k = H_k - R T and c_v = c_p - R / Wbar in place of H_k and c_p.
template <int RPL>
__device__ __forceinline__ void finish_rhs(const DevMech &M, const Lds &L, const Mix<RPL> &x, double (&f)[RPL]) {
    const int ns = M.nsp;
    const int lane = lane_fresh();
    const double shift = L.cv ? 1.0 : 0.0;
    double qp = 0.0;
#pragma unroll
    for (int c = 0; c < RPL; c++) {
        const int k = slot_species(c, ns, lane);
        if (k >= 0) {
            const double wd = L.WD[k];
            f[c] = M.W()[k] * wd / x.rho;
            qp += M.R * x.t.T * (x.h[c] - shift) * wd;
        } else {
            f[c] = 0.0;
        }
    }
    const double Q = wsum(qp);
    const double heat_cap = L.cv ? x.cpm - M.R / x.Wbar : x.cpm;
    if (lane == 0) f[0] = -Q / (x.rho * heat_cap);
}

template <int RPL>
__device__ __forceinline__ void rhs_wave(const DevMech &M, const Lds &L, const double (&y)[RPL], double P, double (&f)[RPL]) {
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

// Chain rule from (d wdot/dC at fixed T, d wdot/dT at fixed C) to J = df/dy, for the lane's
// species row k (lane k + 1) and the lane's entry of the temperature row.  Inputs: jcc =
// sum_l JC[k][l] C_l (third-body rank-one part excluded), colH = sum_r h_r JC[r][k] and colJ =
// sum_r JC[r][k] (h_r = H_r / (R T)).  The species row is J[k+1][0] = col0,
// J[k+1][1+j] = (alpha JC[k][j] + beta) / W_j; trow is J[0][1+k] and J00 = J[0][0].
// Constant pressure: C = rho Y / W with rho = P Wbar / (R T); constant volume: rho fixed, U_k and
// c_v in place of H_k and c_p.
struct Chain {
    double alpha, beta, col0, trow, J00;
};
__device__ __forceinline__ Chain chain_rule(const DevMech &M, const Lds &L, const Mix<1> &x, bool valid, int k,
                                            double y0, double fT, double jcc, double colH, double colJ) {
    const double RT = M.R * x.t.T;
    double TBk = 0.0, WDk = 0.0, DWTk = 0.0;
    if (valid) {
        TBk = L.TB[k];
        WDk = L.WD[k];
        DWTk = L.DWT[k];
    }
    const double Wk = valid ? M.W()[k] : 0.0, iWk = valid ? M.invW()[k] : 0.0;
    const double sdcp = wsum(valid ? y0 * M.R * x.dcp[0] * iWk : 0.0);
    Chain c;
    if (!L.cv) {
        jcc += TBk * x.Ctot;
        const double resid = WDk - jcc;
        const double Hk = RT * x.h[0];
        const double sumHTB = wsum(valid ? Hk * TBk : 0.0);
        const double sumHJCC = wsum(valid ? Hk * jcc : 0.0);
        const double dQT = wsum(valid ? M.R * x.cp[0] * WDk + Hk * (DWTk - jcc * x.t.invT) : 0.0);
        const double D = x.rho * x.cpm;
        const double dQ = iWk * (x.rho * (RT * colH + sumHTB) - x.Wbar * sumHJCC);
        const double dD = x.rho * iWk * (M.R * x.cp[0] - x.cpm * x.Wbar);
        c.trow = valid ? -(dQ + fT * dD) / D : 0.0;
        c.J00 = -(dQT + fT * (-x.rho * x.cpm * x.t.invT + x.rho * sdcp)) / D;
        c.alpha = Wk;
        c.beta = valid ? Wk * TBk + Wk * x.Wbar * resid / x.rho : 0.0;
        c.col0 = valid ? (Wk / x.rho) * (DWTk + resid * x.t.invT) : 0.0;
    } else {
        const double Uk = RT * (x.h[0] - 1.0);
        const double sumUTB = wsum(valid ? Uk * TBk : 0.0);
        const double dQT = wsum(valid ? M.R * (x.cp[0] - 1.0) * WDk + Uk * DWTk : 0.0);
        const double D = x.rho * (x.cpm - M.R / x.Wbar);
        const double dQ = iWk * x.rho * (RT * (colH - colJ) + sumUTB);
        const double dD = x.rho * iWk * M.R * (x.cp[0] - 1.0);
        c.trow = valid ? -(dQ + fT * dD) / D : 0.0;
        c.J00 = -(dQT + fT * x.rho * sdcp) / D;
        c.alpha = Wk;
        c.beta = Wk * TBk;
        c.col0 = valid ? (Wk / x.rho) * DWTk : 0.0;
    }
    return c;
}

// Row descriptor of J for N <= 64, one row per lane (Jacobian pieces staged whole in LDS).
__device__ __forceinline__ JRow jac_prepare(const DevMech &M, const Lds &L, const Mix<1> &x, double y0, double fT) {
    const int ns = M.nsp, lane = lane_fresh();
    const int k = slot_species(0, ns, lane);
    const bool valid = k >= 0;
    double jcc = 0.0, colH = 0.0, colJ = 0.0;
    if (valid) {
        const double *row = &L.JC[k * L.ldj];
        for (int j = 0; j < ns; j++) {
            jcc += row[j] * L.C[j];
            const double v = L.JC[j * L.ldj + k];
            colH += L.H[j] * v;
            colJ += v;
        }
    }
    const Chain c = chain_rule(M, L, x, valid, k, y0, fT, jcc, colH, colJ);
    if (valid) L.TROW[k] = c.trow * M.W()[k];
    __syncthreads();
    JRow r;
    if (lane == 0) {
        r.src = L.TROW;
        r.alpha = 1.0;
        r.beta = 0.0;
        r.c0 = c.J00;
    } else if (valid) {
        r.src = &L.JC[k * L.ldj];
        r.alpha = c.alpha;
        r.beta = c.beta;
        r.c0 = c.col0;
    } else {
        r.src = L.TROW;
        r.alpha = 0.0;
        r.beta = 0.0;
        r.c0 = 0.0;
    }
    return r;
}

// f(y) and this lane's row of the iteration matrix M = dg I - J (registers, element type T) for
// N <= NP <= 64.  The row descriptor jr stays valid (with the Jacobian pieces in LDS) until the
// next Jacobian, so J x products can be formed later without a stored FP64 matrix.
template <int NP, class T>
__device__ __forceinline__ void jac_rows(const DevMech &M, const Lds &L, double y, double P, double dg, T (&a)[NP], double &f,
                         JRow &jr) {
    Mix<1> x;
    const double yy[1] = {y};
    double ff[1];
    species_pass<1, true>(M, yy, P, L, x);
    reaction_pass<true>(M, L, x.t, x.Ctot);
    finish_rhs<1>(M, L, x, ff);
    f = ff[0];
    jr = jac_prepare(M, L, x, y, bcast(ff[0], 0));
    const int lane = lane_fresh();
    a[0] = T((lane == 0 ? dg : 0.0) - jr.c0);
#pragma unroll
    for (int j = 1; j < NP; j++) a[j] = T((lane == j ? dg : 0.0) - L.IW[j - 1] * (jr.alpha * jr.src[j - 1] + jr.beta));
    __syncthreads();
}

// f(y) and this lane's row of M = dg I - J (FP64 registers) for N <= NP <= 64, with d wdot/dC
// staged in NWIN column windows of WIN columns (NWIN * WIN >= ns).  The reaction pass runs once
// per window, which keeps JC at ns * (WIN | 1) doubles of LDS; the second window reuses the first
// window's rate constants when they fit the park slice (else it recomputes them).  Raw window
// entries wait in the park slice until the chain-rule scalars of the row are known.
template <int NP, int NWIN, int WIN>
__device__ __forceinline__ void jac_rows_win(const DevMech &M, const Lds &L, double y, double P, double dg, double (&a)[NP],
                             double &f) {
    Mix<1> x;
    const double yy[1] = {y};
    double ff[1];
    species_pass<1, true, false>(M, yy, P, L, x);
    const int ns = M.nsp;
    const int lane = lane_fresh();
    const int k = lane - 1;
    const bool valid = lane >= 1 && lane <= ns;
    double jcc = 0.0, colH = 0.0, colJ = 0.0;
    // per-reaction scatter scalars of the first window, kept in the park slice for the second
    static_assert(NWIN <= 2, "the scalar cache serves one later window");
    const bool keep = NWIN == 2 && 3 * ((M.nrxn + 63) / 64) <= NP;
    double *cache = L.park + lane_fresh();
#pragma unroll
    for (int w = 0; w < NWIN; w++) {
        const int c0 = w * WIN;
        const int tot = ns * L.ldj;
        for (int e = lane; e < tot; e += 64) L.JC[e] = 0.0;
        __syncthreads();
        reaction_pass<true>(M, L, x.t, x.Ctot, c0, WIN, w == 0, cache, keep ? (w == 0 ? 1 : 2) : 0);
        if (w == 0) finish_rhs<1>(M, L, x, ff);
        // raw d wdot_k / dC_(c0+j) into column 1 + c0 + j of the row registers; the chain-rule
        // scalars of the row are applied once every window is in
        // (every lane reads an in-range entry and keeps it under a bit mask, so that the reads
        // are not split into one masked branch each; the column tests use a scalar copy of ns
        // that the compiler cannot hoist out of the reactor loop, where the tests' results would
        // occupy and spill scalar registers)
        const double *row = &L.JC[(valid ? k : 0) * L.ldj];
        const int vkeep = opaque(valid ? -1 : 0);
        const int nsw = opaque_s(ns);
#pragma unroll
        for (int j = 0; j < WIN; j++) {
            if (1 + c0 + j >= NP) break;
            const bool in = c0 + j < nsw;
            const double e = row[j];
            const double v = __hiloint2double(__double2hiint(e) & vkeep, __double2loint(e) & vkeep);
            if (in) jcc += v * L.C[c0 + j];
            a[1 + c0 + j] = in ? v : 0.0;
        }
        if (valid && k >= c0 && k < c0 + WIN)
            for (int r = 0; r < ns; r++) {
                const double v = L.JC[r * L.ldj + (k - c0)];
                colH += L.H[r] * v;
                colJ += v;
            }
        __syncthreads();
    }
    f = ff[0];
    const Chain c = chain_rule(M, L, x, valid, k, y, bcast(f, 0), jcc, colH, colJ);
    if (valid) L.TROW[k] = c.trow;
    const double J00 = c.J00, col0 = c.col0, alpha = c.alpha, beta = c.beta;
    __syncthreads();
    a[0] = (lane == 0 ? dg : 0.0) - (lane == 0 ? J00 : col0);
#pragma unroll
    for (int j = 1; j < NP; j++) {
        const double Jv = lane == 0 ? L.TROW[j - 1] : L.IW[j - 1] * (alpha * a[j] + beta);
        a[j] = (lane == j ? dg : 0.0) - Jv;
    }
    __syncthreads();
}

// (J x) for x distributed one component per lane, from the Jacobian pieces in LDS.
__device__ __forceinline__ double jac_times(const DevMech &M, const Lds &L, const JRow &r, double x) {
    const int lane = lane_fresh();
    const int ns = M.nsp;
    const bool sp = lane >= 1 && lane <= ns;
    const double v = sp ? x * L.IW[lane - 1] : 0.0;      // x_{j+1} / W_j
    if (sp) L.VX[lane - 1] = v;
    const double Sv = wsum(v);
    const double x0 = bcast(x, 0);
    __syncthreads();
    double dot = 0.0;
    for (int j = 0; j < ns; j++) dot += r.src[j] * L.VX[j];
    __syncthreads();
    return r.c0 * x0 + r.alpha * dot + r.beta * Sv;
}

// ---------------------------------------------------------------------------------------
// dense LU with partial pivoting, one row per lane, fully unrolled over NP columns
// ---------------------------------------------------------------------------------------
template <int NP>
struct LU {
    int pivv;         // lane k holds the lane of the pivot row of column k
    int ord;          // this lane's pivot order
    double dinv;      // 1 / U[ord][ord]
    bool ok;
};

template <int NP>
__device__ __forceinline__ void lu_factor(double (&a)[NP], LU<NP> &f) {
    const int lane = lane_id();
    bool done = false;
    f.ord = NP;
    f.dinv = 0.0;
    f.ok = true;
    f.pivv = 0;
#pragma unroll
    for (int k = 0; k < NP; k++) {
        // pivot search on the high word of |a| (ordered like |a|; candidates within a relative 2^-20
        // of the largest may tie, and the first lane is taken)
        const unsigned key = done ? 0u : unsigned(__double2hiint(fabs(a[k])));
        const unsigned mx = __ockl_wfred_max_u32(key);
        const int p = __builtin_ctzll(__ballot(!done && key == mx));
        if (lane == k) f.pivv = p;
        f.ok = f.ok && (mx != 0u);
        // 1 / pivot: hardware reciprocal estimate refined by two Newton-Raphson steps (within an
        // ulp; a shorter dependency chain than the correctly rounded division)
        const double piv = bcast(a[k], p);
        double inv = __builtin_amdgcn_rcp(piv);
        inv = fma(fma(-piv, inv, 1.0), inv, inv);
        inv = fma(fma(-piv, inv, 1.0), inv, inv);
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

// Solve (L U) x = P b; b and x distributed one component per lane.
template <int NP>
__device__ __forceinline__ double lu_solve(const double (&a)[NP], const LU<NP> &f, double b) {
    const int lane = lane_fresh();
    const int pivv = opaque(f.pivv);
    const int ord = opaque(f.ord);
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const double yk = bcast(b, __builtin_amdgcn_readlane(pivv, k));
        if (ord > k) b = fma(-a[k], yk, b);
    }
    double x = 0.0;
#pragma unroll
    for (int k = NP - 1; k >= 0; k--) {
        const double xk = bcast(b * f.dinv, __builtin_amdgcn_readlane(pivv, k));
        if (lane == k) x = xk;
        if (ord < k) b = fma(-a[k], xk, b);
    }
    return x;
}

// ---------------------------------------------------------------------------------------
// one steps
// ---------------------------------------------------------------------------------------
// Window count and width of the staged d wdot/dC for a padded size NP, and whether the kernel
// uses a parking slice in the workspace (raw Jacobian window entries and the first window's
// per-reaction rate scalars; the forward-difference step also parks its Jacobian columns and
// its LU rows there).
template <int NP>
struct WaveShape {
    static constexpr int NWIN = NP > 32 ? 2 : 1;
    static constexpr int WIN = NWIN == 1 ? 0 : (NP - 1 + NWIN - 1) / NWIN;   // 0: all ns columns
    static constexpr bool PARK = NP > 32;
};

template <int NP>
__device__ __forceinline__ void park_rows(const Lds &L, const double (&a)[NP]) {
    double *r = L.park + lane_fresh();
#pragma unroll
    for (int j = 0; j < NP; j++) r[j * 64] = a[j];
}
template <int NP>
__device__ __forceinline__ void unpark_rows(const Lds &L, double (&a)[NP]) {
    const double *r = L.park + lane_fresh();
#pragma unroll
    for (int j = 0; j < NP; j++) a[j] = r[j * 64];
}

// FULLJC: d wdot/dC staged whole (the FP32-mode LDS layout), no column windows.
template <int NP, bool FULLJC = false>
struct Ros4Wave {
    using SH = WaveShape<NP>;
    static constexpr double qinv = 0.25;
    __device__ static __forceinline__ bool step(const DevMech &M, const Lds &L, double y, double P, double h, double &ynew,
                                double &e) {
        double a[NP];
        double f;
        const double dg = 1.0 / (Ros4::gamma * h);
        if (SH::NWIN == 1 || FULLJC) {
            JRow jr;
            jac_rows<NP, double>(M, L, y, P, dg, a, f, jr);
        } else {
            jac_rows_win<NP, SH::NWIN, SH::WIN>(M, L, y, P, dg, a, f);
        }
        LU<NP> lu;
        lu_factor<NP>(a, lu);
        const double ih = 1.0 / h;
        const double u1 = lu_solve<NP>(a, lu, f);
        // the factored rows stay in registers across the stage source terms (it fits without spills)
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

// ROS4 step with a forward-difference Jacobian (the paper's ROS4 set-up, Section 5): column j of
// J is (f(y + inc_j e_j) - f(y)) / inc_j, one source-term evaluation per column, with
//   inc_j = max(sqrt(eps) |y_j|, min_inc (rtol |y_j| + atol)),
//   min_inc = 1000 |h| eps N ||f(y)||_w (1 if that norm is 0), w_i = 1 / (rtol |y_i| + atol),
// as CVODE's dense difference quotient.  Columns are written to the parking slice (lane i holds
// row i), then loaded as the lane's row; f(y) doubles as the first stage's right-hand side.
template <int NP>
struct Ros4WaveFD {
    __device__ static __forceinline__ bool step(const DevMech &M, const Lds &L, double y, double P, double h,
                                                double &ynew, double &e, const IntOpts &o) {
        constexpr double eps = 2.220446049250313e-16;
        const int N = M.N;
        const int lane = lane_fresh();
        const bool comp = lane < N;
        double yy[1] = {y}, f0[1];
        rhs_wave<1>(M, L, yy, P, f0);
        const double r = comp ? f0[0] / (o.rtol * fabs(y) + o.atol) : 0.0;
        const double fnorm = sqrt(wsum(r * r) / N);
        const double min_inc = fnorm != 0.0 ? 1000.0 * fabs(h) * eps * N * fnorm : 1.0;
        {
            double *pk = L.park + lane_fresh();
            for (int j = 0; j < N; j++) {
                const double yj = bcast(y, j);
                const double wj = 1.0 / (o.rtol * fabs(yj) + o.atol);
                const double inc = fmax(sqrt(eps) * fabs(yj), min_inc / wj);
                double yp[1] = {lane == j ? yj + inc : y}, fj[1];
                rhs_wave<1>(M, L, yp, P, fj);
                pk[j * 64] = comp ? (fj[0] - f0[0]) / inc : 0.0;   // J[lane][j]
            }
        }
        const double dg = 1.0 / (Ros4::gamma * h);
        double a[NP];
        {
            const double *pk = L.park + lane_fresh();
#pragma unroll
            for (int j = 0; j < NP; j++) a[j] = (lane == j ? dg : 0.0) - (j < N ? pk[j * 64] : 0.0);
        }
        LU<NP> lu;
        lu_factor<NP>(a, lu);
        const double ih = 1.0 / h;
        const double u1 = lu_solve<NP>(a, lu, f0[0]);
        park_rows<NP>(L, a);
        double yt[1] = {y + Ros4::a21 * u1}, ft[1];
        rhs_wave<1>(M, L, yt, P, ft);
        unpark_rows<NP>(L, a);
        const double u2 = lu_solve<NP>(a, lu, ft[0] + (Ros4::c21 * u1) * ih);
        yt[0] = y + Ros4::a31 * u1 + Ros4::a32 * u2;
        rhs_wave<1>(M, L, yt, P, ft);
        unpark_rows<NP>(L, a);
        const double u3 = lu_solve<NP>(a, lu, ft[0] + (Ros4::c31 * u1 + Ros4::c32 * u2) * ih);
        const double u4 = lu_solve<NP>(a, lu, ft[0] + (Ros4::c41 * u1 + Ros4::c42 * u2 + Ros4::c43 * u3) * ih);
        ynew = y + Ros4::m1 * u1 + Ros4::m2 * u2 + Ros4::m3 * u3 + Ros4::m4 * u4;
        e = Ros4::e1 * u1 + Ros4::e2 * u2 + Ros4::e3 * u3 + Ros4::e4 * u4;
        return lu.ok;
    }
};

// ---------------------------------------------------------------------------------------
// FP32 factorisation with FP64 residual refinement
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ float bcastf(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double wmax_abs(double v) {
    return __longlong_as_double((long long)__ockl_wfred_max_u64((unsigned long long)__double_as_longlong(fabs(v))));
}

template <int NP>
struct LU32 {
    int pivv, ord;
    float dinv;
    bool ok;
};

template <int NP>
__device__ __forceinline__ void lu_factor32(float (&a)[NP], LU32<NP> &f) {
    const int lane = lane_id();
    bool done = false;
    f.ord = NP;
    f.dinv = 0.0f;
    f.ok = true;
    f.pivv = 0;
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const unsigned key = done ? 0u : __float_as_uint(fabsf(a[k]));
        const unsigned mx = __ockl_wfred_max_u32(key);
        const int p = __builtin_ctzll(__ballot(!done && key == mx));
        if (lane == k) f.pivv = p;
        f.ok = f.ok && (mx != 0u);
        const float inv = 1.0f / bcastf(a[k], p);
        if (lane == p) {
            done = true;
            f.ord = k;
            f.dinv = inv;
        }
        const float l = done ? 0.0f : a[k] * inv;
        if (!done) a[k] = l;
#pragma unroll
        for (int j = k + 1; j < NP; j++) a[j] = fmaf(-l, bcastf(a[j], p), a[j]);
    }
}

template <int NP>
__device__ __forceinline__ float lu_solve32(const float (&a)[NP], const LU32<NP> &f, float b) {
    const int lane = lane_fresh();
    const int pivv = opaque(f.pivv);
    const int ord = opaque(f.ord);
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const float yk = bcastf(b, __builtin_amdgcn_readlane(pivv, k));
        if (ord > k) b = fmaf(-a[k], yk, b);
    }
    float x = 0.0f;
#pragma unroll
    for (int k = NP - 1; k >= 0; k--) {
        const float xk = bcastf(b * f.dinv, __builtin_amdgcn_readlane(pivv, k));
        if (lane == k) x = xk;
        if (ord < k) b = fmaf(-a[k], xk, b);
    }
    return x;
}

// ROS4 step whose linear solves use an FP32 LU of M = I/(gamma h) - J, refined with FP64
// residuals r = b - M x (M x formed from the FP64 Jacobian pieces).  A solve is done once the
// correction is below 2^-48 of the solution.  If a correction fails to halve the previous one, or
// the allowed sweeps run out first, the FP32 step is abandoned and the reactor-step is done again
// in FP64 (rows formed in FP64 from the full staged d wdot/dC, FP64 LU); `fb` counts such steps.
// With zero sweeps the FP32 solutions are used as they are.
template <int NP>
struct Ros4Wave32 {
    __device__ static __forceinline__ bool step32(const DevMech &M, const Lds &L, double y, double P, double h,
                                                  double &ynew, double &e, int sweeps, bool &conv) {
        float a[NP];
        double f;
        JRow jr;
        const double dg = 1.0 / (Ros4::gamma * h);
        jac_rows<NP, float>(M, L, y, P, dg, a, f, jr);
        LU32<NP> lu;
        lu_factor32<NP>(a, lu);
        const bool ok = lu.ok;
        conv = true;
        auto solve = [&](double b) -> double {
            double x = double(lu_solve32<NP>(a, lu, float(b)));
            if (sweeps <= 0) return x;
            double dprev = INFINITY;
            for (int s = 0; s < sweeps; s++) {
                const double r = b - (dg * x - jac_times(M, L, jr, x));
                const double d = double(lu_solve32<NP>(a, lu, float(r)));
                x += d;
                const double dmax = wmax_abs(d), xmax = wmax_abs(x);
                if (dmax <= 0x1p-48 * xmax) return x;
                if (!(dmax <= 0.5 * dprev)) break;      // stagnation (or not finite)
                dprev = dmax;
            }
            conv = false;
            return x;
        };
        const double ih = 1.0 / h;
        const double u1 = solve(f);
        if (!conv) return ok;
        double yt[1] = {y + Ros4::a21 * u1}, ft[1];
        rhs_wave<1>(M, L, yt, P, ft);
        const double u2 = solve(ft[0] + (Ros4::c21 * u1) * ih);
        if (!conv) return ok;
        yt[0] = y + Ros4::a31 * u1 + Ros4::a32 * u2;
        rhs_wave<1>(M, L, yt, P, ft);
        const double u3 = solve(ft[0] + (Ros4::c31 * u1 + Ros4::c32 * u2) * ih);
        if (!conv) return ok;
        const double u4 = solve(ft[0] + (Ros4::c41 * u1 + Ros4::c42 * u2 + Ros4::c43 * u3) * ih);
        if (!conv) return ok;
        ynew = y + Ros4::m1 * u1 + Ros4::m2 * u2 + Ros4::m3 * u3 + Ros4::m4 * u4;
        e = Ros4::e1 * u1 + Ros4::e2 * u2 + Ros4::e3 * u3 + Ros4::e4 * u4;
        return ok;
    }
    __device__ static __forceinline__ bool step(const DevMech &M, const Lds &L, double y, double P, double h, double &ynew,
                                double &e, int sweeps, int &fb) {
        bool conv = true;
        const bool ok = step32(M, L, y, P, h, ynew, e, sweeps, conv);
        if (conv) return ok;
        fb++;
        return Ros4Wave<NP, true>::step(M, L, y, P, h, ynew, e);
    }
};

template <int RPL>
struct Rkf45Wave {
    static constexpr double qinv = 0.2;
    __device__ static __forceinline__ void stage(const DevMech &M, const Lds &L, const double (&yt)[RPL], double P, double h,
                                 double (&k)[RPL]) {
        rhs_wave<RPL>(M, L, yt, P, k);
#pragma unroll
        for (int c = 0; c < RPL; c++) k[c] *= h;
    }
    __device__ static __forceinline__ bool step(const DevMech &M, const Lds &L, const double (&y)[RPL], double P, double h,
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
__device__ __forceinline__ double wrms_wave(int N, const double (&e)[RPL], const double (&a)[RPL], const double (&b)[RPL],
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
__device__ __forceinline__ bool all_finite(int N, const double (&v)[RPL]) {
    bool ok = true;
#pragma unroll
    for (int c = 0; c < RPL; c++) ok = ok && (lane_id() + 64 * c >= N || isfinite(v[c]));
    return wave_all(ok);
}

// Step adapters with a common (array) interface.
template <int NP>
struct Ros4Adapter {
    static constexpr int RPL = 1;
    static constexpr int NSMAX = NP - 1;
    static constexpr bool JAC = true;
    static constexpr int WIN = WaveShape<NP>::WIN;
    static constexpr bool PARK = WaveShape<NP>::PARK;
    static constexpr int PARK_ROWS = NP;
    static constexpr double qinv = 0.25;
    __device__ static __forceinline__ bool step(const DevMech &M, const Lds &L, const double (&y)[1], double P, double h,
                                double (&yn)[1], double (&e)[1], const IntOpts &, int &) {
        return Ros4Wave<NP>::step(M, L, y[0], P, h, yn[0], e[0]);
    }
};

template <int NP>
struct Ros4AdapterFD {
    static constexpr int RPL = 1;
    static constexpr int NSMAX = NP - 1;
    static constexpr bool JAC = false;      // no d wdot/dC staging: only source-term evaluations
    static constexpr int WIN = 0;
    static constexpr bool PARK = true;
    static constexpr int PARK_ROWS = NP;
    static constexpr double qinv = 0.25;
    __device__ static __forceinline__ bool step(const DevMech &M, const Lds &L, const double (&y)[1], double P,
                                                double h, double (&yn)[1], double (&e)[1], const IntOpts &o, int &) {
        return Ros4WaveFD<NP>::step(M, L, y[0], P, h, yn[0], e[0], o);
    }
};

template <int NP>
struct Ros4Adapter32 {
    static constexpr int RPL = 1;
    static constexpr int NSMAX = NP - 1;
    static constexpr bool JAC = true;
    static constexpr int WIN = 0;
    static constexpr bool PARK = false;
    static constexpr int PARK_ROWS = 0;
    static constexpr double qinv = 0.25;
    __device__ static __forceinline__ bool step(const DevMech &M, const Lds &L, const double (&y)[1], double P, double h,
                                double (&yn)[1], double (&e)[1], const IntOpts &o, int &fb) {
        return Ros4Wave32<NP>::step(M, L, y[0], P, h, yn[0], e[0], o.refine_sweeps, fb);
    }
};

template <class S>
__device__ __forceinline__ void integrate_reactor(const DevMech &M, const Lds &L, int64_t r, double *y, int64_t ld, const double *p,
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
    int na = 0, nj = 0, fb = 0;
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
            const bool ok = S::step(M, L, yv, P, hs, yn, e, o, fb);
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
        if (o.n_fallback) o.n_fallback[r] = fb;
    }
}

template <int R>
struct Rkf45S {
    static constexpr int RPL = R;
    static constexpr int NSMAX = 64 * R - 1;
    static constexpr bool JAC = false;
    static constexpr int WIN = 0;
    static constexpr bool PARK = false;
    static constexpr int PARK_ROWS = 0;
    static constexpr double qinv = 0.2;
    __device__ static __forceinline__ bool step(const DevMech &M, const Lds &L, const double (&y)[R], double P, double h,
                                double (&yn)[R], double (&e)[R], const IntOpts &, int &) {
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
                                                      const double *p, double *dydt, int cv) {
    extern __shared__ double lds_raw[];
    Lds L = carve(lds_raw, M.nsp, false);
    L.cv = cv;
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
                                                      const double *p, double *jac, int cv) {
    extern __shared__ double lds_raw[];
    Lds L = carve(lds_raw, M.nsp, true);
    L.cv = cv;
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
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) integrate_wave_kernel(DevMech M, int64_t n, double *y, int64_t ld,
                                                            const double *p, const double *t_end, double *t_io,
                                                            double *h_io, IntOpts o, unsigned *queue,
                                                            double *park, int32_t *status, int32_t *nacc,
                                                            int32_t *nrej) {
    // LDS laid out for the largest species count of the instantiation: every offset is a
    // compile-time constant, so LDS addresses need no scalar registers
    extern __shared__ double lds_raw[];
    Lds L = carve(lds_raw, S::NSMAX, S::JAC, S::WIN > 0 ? S::WIN : S::NSMAX);
    L.cv = o.reactor;
    if (S::PARK) L.park = park + size_t(blockIdx.x) * (size_t(S::PARK_ROWS) * 64);
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

// Resident wavefronts per CU are capped so that parked LU rows fit the workspace.
constexpr int kWaveMaxPerCu = 8;

template <class S>
int launch_int(const DevMech &M, int64_t n, double *y, int64_t ld, const double *p, const double *t_end, double *t,
               double *h, const IntOpts &o, unsigned *queue, int32_t *status, int32_t *nacc, int32_t *nrej,
               hipStream_t s) {
    if (M.nsp > S::NSMAX) return CK_EUNSUPPORTED;
    const size_t lds = lds_doubles(S::NSMAX, S::JAC, S::WIN > 0 ? S::WIN : S::NSMAX) * sizeof(double);
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CK_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return CK_EHIP;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, integrate_wave_kernel<S>, 64, lds) != hipSuccess || per < 1)
        return CK_EHIP;
    if (o.blocks_per_cu > 0 && o.blocks_per_cu < per) per = o.blocks_per_cu;
    if (per > kWaveMaxPerCu) per = kWaveMaxPerCu;
    int64_t grid = int64_t(cus) * per;
    if (grid > n) grid = n;
    double *park = S::PARK ? reinterpret_cast<double *>(reinterpret_cast<char *>(queue) + 256) : nullptr;
    zero_u32_kernel<<<1, 1, 0, s>>>(queue);
    integrate_wave_kernel<S><<<dim3(unsigned(grid)), dim3(64), lds, s>>>(M, n, y, ld, p, t_end, t, h, o, queue,
                                                                          park, status, nacc, nrej);
    return hipGetLastError() == hipSuccess ? CK_OK : CK_EHIP;
}
}  // namespace

bool wave_supported(const DevMech &M, int method, int precision) {
    if (method == 0) return M.N <= 64;
    return precision == CK_PREC_FP64 && M.N <= 128;
}

size_t wave_ws_bytes(const DevMech &M, int cus) {
    // parked FP64 rows of every resident wavefront (FP64 ROS4 with NP > 32, or any NP <= 64 with
    // the forward-difference Jacobian)
    const int np = pad_np(M.N);
    if (np > 64) return 256;
    return 256 + size_t(cus) * kWaveMaxPerCu * size_t(np) * 64 * sizeof(double);
}

int launch_rhs_wave(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *dydt,
                    int cv, hipStream_t s) {
    const size_t lds = lds_doubles(M.nsp, false) * sizeof(double);
    const unsigned grid = unsigned((n + 7) / 8 * 8);
    if (M.N <= 64)
        rhs_wave_kernel<1><<<dim3(grid), dim3(64), lds, s>>>(M, n, y, ld, p, dydt, cv);
    else
        rhs_wave_kernel<2><<<dim3(grid), dim3(64), lds, s>>>(M, n, y, ld, p, dydt, cv);
    return hipGetLastError() == hipSuccess ? CK_OK : CK_EHIP;
}

int launch_jac_wave(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *jac,
                    int cv, hipStream_t s) {
    if (M.N > 64) return cv ? CK_EUNSUPPORTED : launch_jac_coop(M, n, y, ld, p, jac, s);
    const size_t lds = lds_doubles(M.nsp, true) * sizeof(double);
    const unsigned grid = unsigned((n + 7) / 8 * 8);
    jac_wave_kernel<<<dim3(grid), dim3(64), lds, s>>>(M, n, y, ld, p, jac, cv);
    return hipGetLastError() == hipSuccess ? CK_OK : CK_EHIP;
}

int launch_integrate_wave(int method, const DevMech &M, int64_t n, double *y, int64_t ld, const double *p,
                          const double *t_end, double *t, double *h, const IntOpts &o, void *ws, int32_t *status,
                          int32_t *nacc, int32_t *nrej, hipStream_t s) {
    unsigned *q = static_cast<unsigned *>(ws);
    if (method == 1) {
        if (M.N <= 64) return launch_int<Rkf45S<1>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
        return launch_int<Rkf45S<2>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
    }
    if (o.jacobian == CK_JAC_FD) {
        if (o.precision != CK_PREC_FP64) return CK_EUNSUPPORTED;
        switch (pad_np(M.N)) {
#define CK_CASEFD(NPV) \
    case NPV: return launch_int<Ros4AdapterFD<NPV>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
            CK_CASEFD(8) CK_CASEFD(16) CK_CASEFD(24) CK_CASEFD(32) CK_CASEFD(40) CK_CASEFD(48) CK_CASEFD(56)
            CK_CASEFD(64)
#undef CK_CASEFD
            default: return CK_EUNSUPPORTED;
        }
    }
    if (o.precision == CK_PREC_FP32_REFINE) {
        switch (pad_np(M.N)) {
#define CK_CASE32(NPV) \
    case NPV: return launch_int<Ros4Adapter32<NPV>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
            CK_CASE32(8) CK_CASE32(16) CK_CASE32(24) CK_CASE32(32) CK_CASE32(40) CK_CASE32(48) CK_CASE32(56)
            CK_CASE32(64)
#undef CK_CASE32
            default: return CK_EUNSUPPORTED;
        }
    }
    switch (pad_np(M.N)) {
        case 8: return launch_int<Ros4Adapter<8>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
        case 16: return launch_int<Ros4Adapter<16>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
        case 24: return launch_int<Ros4Adapter<24>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
        case 32: return launch_int<Ros4Adapter<32>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
        case 40: return launch_int<Ros4Adapter<40>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
        case 48: return launch_int<Ros4Adapter<48>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
        case 56: return launch_int<Ros4Adapter<56>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
        case 64: return launch_int<Ros4Adapter<64>>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
        default: return CK_EUNSUPPORTED;
    }
}

}  // namespace ck
