// Workgroup-cooperative ROS4: one reactor per workgroup.
//   - thread t holds state component t (T on thread 0, Y_{t-1} on thread t)
//     in the source-term phases: species phases thread-per-species, reaction
//     phases thread-per-reaction with LDS FP64 atomics, group-wide reductions
//     and broadcasts through LDS;
//   - the iteration matrix M = I/(gamma h) - J lives in registers and is
//     inverted in place by Gauss-Jordan elimination with partial pivoting.
//     Each elimination step rotates the rows left by one, so the pivot column
//     is always register 0 and one loop body serves every step.  The four
//     stage solves of a step are then matrix-vector products with no
//     sequential substitution;
//   - N <= 64: one wavefront, one matrix row per thread;
//   - N > 64: four wavefronts, each row split over a pair of adjacent threads
//     (half rows of N'/2 doubles), d wdot/dC staged in LDS in two column
//     windows (one per half), so two reactors fit in one CU's LDS and two
//     wavefronts fit each SIMD.  The inverse stays in registers across the
//     stage right-hand sides; a per-workgroup slice of the workspace carries
//     the first Jacobian window's per-reaction rate scalars to the second.
// Reactors come from the same device work queue as the wavefront kernels.
#include "ck_internal.h"
#include "kinetics.h"
#include "launch.h"

extern "C" __device__ unsigned long long __ockl_wfred_max_u64(unsigned long long);
extern "C" __device__ unsigned __ockl_wfred_max_u32(unsigned);
extern "C" __device__ double __ockl_wfred_add_f64(double);

namespace ck {
namespace coop {

__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ double readlane_d(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// LDS layout of one workgroup (doubles); WIN = Jacobian columns staged per window:
//   C[ns+1] G[ns] H[ns] WD[ns] | IW[128] | VX[128] | RED[16] | PB[2][128] BS[128] XS[128] |
//   JC[ns * ldj + 128] TB[ns] DWT[ns] TROW[ns + 128]
struct Lds {
    double *C, *G, *H, *WD, *IW, *VX, *RED, *PB, *BS, *XS, *JC, *TB, *DWT, *TROW;
    double *rows;   // this workgroup's park slice (global memory), or null
    // half-row kernel only: per-row chain-rule scalars and pivot orders, [128] each
    double *RA, *RB, *RC, *RJ;
    int *ORD;
    int ldj;
};

__host__ __device__ inline int ldj_of(int win) { return win | 1; }
// JC region: the staged d wdot/dC window, or at least jc_min doubles (the tile kernel reuses the
// region as scratch of its blocked elimination)
__host__ __device__ inline size_t jc_doubles(int ns, int win, size_t jc_min) {
    const size_t j = size_t(ns) * ldj_of(win) + 128;
    return j > jc_min ? j : jc_min;
}
__host__ __device__ inline size_t lds_doubles(int ns, int win, bool half = false, size_t jc_min = 0) {
    return size_t(ns + 1) + 3 * size_t(ns) + 128 + 128 + 16 + 2 * 128 + 128 + 128 + jc_doubles(ns, win, jc_min) +
           2 * size_t(ns) + size_t(ns) + 128 + (half ? 4 * 128 + 64 : 0);
}

__device__ __forceinline__ Lds carve(double *b, int ns, int win, bool half = false, size_t jc_min = 0) {
    Lds L;
    L.ldj = ldj_of(win);
    L.C = b; b += ns + 1;
    L.G = b; b += ns;
    L.H = b; b += ns;
    L.WD = b; b += ns;
    L.IW = b; b += 128;
    L.VX = b; b += 128;
    L.RED = b; b += 16;
    L.PB = b; b += 2 * 128;
    L.BS = b; b += 128;
    L.XS = b; b += 128;
    L.JC = b; b += jc_doubles(ns, win, jc_min);
    L.TB = b; b += ns;
    L.DWT = b; b += ns;
    L.TROW = b; b += ns + 128;
    L.rows = nullptr;
    L.RA = L.RB = L.RC = L.RJ = nullptr;
    L.ORD = nullptr;
    if (half) {
        L.RA = b; b += 128;
        L.RB = b; b += 128;
        L.RC = b; b += 128;
        L.RJ = b; b += 128;
        L.ORD = reinterpret_cast<int *>(b);
    }
    return L;
}

// Group primitives for W wavefronts.
template <int W>
struct Grp {
    static constexpr int T = 64 * W;
    __device__ static __forceinline__ int tid() { return opaque(int(threadIdx.x)); }
    __device__ static __forceinline__ int lane() { return int(threadIdx.x) & 63; }
    __device__ static __forceinline__ int wave() { return __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6); }
    __device__ static __forceinline__ double sum(double v, double *red) {
        const double s = __ockl_wfred_add_f64(v);
        if (W == 1) return s;
        if (lane() == 0) red[wave()] = s;
        __syncthreads();
        double t = red[0];
#pragma unroll
        for (int w = 1; w < W; w++) t += red[w];
        __syncthreads();
        return t;
    }
    // value of thread src (src uniform)
    __device__ static __forceinline__ double bcast(double v, int src, double *slot) {
        if (W == 1) return readlane_d(v, src);
        if (int(threadIdx.x) == src) *slot = v;
        __syncthreads();
        const double r = *slot;
        __syncthreads();
        return r;
    }
    // thread holding the largest key (lowest thread index on ties) and the key itself
    __device__ static __forceinline__ int argmax(unsigned long long key, double *xs, unsigned long long &best) {
        const unsigned long long mx = __ockl_wfred_max_u64(key);
        const int l = __builtin_ctzll(__ballot(key == mx));
        if (W == 1) {
            best = mx;
            return l;
        }
        unsigned long long *x = reinterpret_cast<unsigned long long *>(xs);
        if (lane() == 0) {
            x[2 * wave()] = mx;
            x[2 * wave() + 1] = (unsigned long long)(wave() * 64 + l);
        }
        __syncthreads();
        best = x[0];
        int bt = int(x[1]);
#pragma unroll
        for (int w = 1; w < W; w++)
            if (x[2 * w] > best) {
                best = x[2 * w];
                bt = int(x[2 * w + 1]);
            }
        __syncthreads();
        return __builtin_amdgcn_readfirstlane(bt);
    }
};

__device__ __forceinline__ void init_lds(const DevMech &M, const Lds &L, int tid, int nthreads) {
    for (int e = tid; e < 128; e += nthreads) {
        L.IW[e] = e < M.nsp ? M.invW()[e] : 0.0;
        L.VX[e] = 0.0;
    }
    for (int e = tid; e < M.nsp + 128; e += nthreads) L.TROW[e] = 0.0;
    __syncthreads();
}

struct Mix {
    TPow t;
    double rho, Wbar, Ctot, cpm, cp, h, dcp;
};

__device__ __forceinline__ int species_of(int tid, int ns) { return (tid >= 1 && tid <= ns) ? tid - 1 : -1; }

// Mixture state and species thermodynamics (Section 3); zeroes the accumulators.
template <int W, bool JAC>
__device__ __forceinline__ void species_pass(const DevMech &M, double y, double P, const Lds &L, Mix &x) {
    using G = Grp<W>;
    const int ns = M.nsp, tid = G::tid();
    const int k = species_of(tid, ns);
    const double T = G::bcast(y, 0, L.RED + 8);
    x.t = tpow(T);
    const double S = G::sum(k >= 0 ? y * M.invW()[k] : 0.0, L.RED);
    x.rho = P / (M.R * T * S);
    x.Wbar = 1.0 / S;
    x.Ctot = P * x.t.invT / M.R;
    double cpp = 0.0;
    if (k >= 0) {
        L.C[k] = x.rho * y * M.invW()[k];
        const Thermo th = species_thermo(M, k, x.t);
        L.G[k] = th.h - th.s;
        L.H[k] = th.h;
        L.WD[k] = 0.0;
        x.cp = th.cp;
        x.h = th.h;
        x.dcp = th.dcp;
        cpp = y * th.cp * M.invW()[k];
    } else {
        x.cp = x.h = x.dcp = 0.0;
    }
    x.cpm = G::sum(cpp, L.RED) * M.R;
    if (JAC)
        for (int e = tid; e < ns; e += G::T) {
            L.TB[e] = 0.0;
            L.DWT[e] = 0.0;
        }
    __syncthreads();
}

// Rates of progress into WD (FIRST window only) and d wdot/dC for columns [c0, c0 + win) into JC.
// The column scatter of a reaction needs c k_f, c k_r and R_net dc/d[M] besides the concentrations:
// mode 1 stores them in this thread's column of `cache` (entry (3 it + v) * T for the thread's it-th
// reaction), mode 2 reads them back instead of evaluating the rate constants again.
template <int W, bool JAC>
__device__ __forceinline__ void reaction_pass(const DevMech &M, const Lds &L, const TPow &t, double Ctot, int c0, int win,
                                              bool first, double *cache = nullptr, int mode = 0) {
    using G = Grp<W>;
    const int nr = M.nrxn, ns = M.nsp, tid = G::tid();
    if (JAC) {
        const int tot = ns * L.ldj;
        for (int e = tid; e < tot; e += G::T) L.JC[e] = 0.0;
        __syncthreads();
    }
    auto Cg = [&](int k) { return L.C[k]; };
    auto Gg = [&](int k) { return L.G[k]; };
    auto Hg = [&](int k) { return L.H[k]; };
    int it = 0;
    for (int i = tid; i < nr; i += G::T, it++) {
        const RxnRec R = M.rx[i];
        const int nmax = __builtin_amdgcn_readfirstlane(R.blk_slots);
        Slots S;
        load_slots(R, Cg, S, nmax);
        double ckf, ckr, rdm;
        if (JAC && mode == 2) {
            ckf = cache[(3 * it) * G::T];
            ckr = cache[(3 * it + 1) * G::T];
            rdm = cache[(3 * it + 2) * G::T];
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
                cache[(3 * it) * G::T] = ckf;
                cache[(3 * it + 1) * G::T] = ckr;
                cache[(3 * it + 2) * G::T] = rdm;
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

// Eqs. ydot and tdot.
template <int W>
__device__ __forceinline__ double finish_rhs(const DevMech &M, const Lds &L, const Mix &x) {
    using G = Grp<W>;
    const int tid = G::tid();
    const int k = species_of(tid, M.nsp);
    double f = 0.0, qp = 0.0;
    if (k >= 0) {
        const double wd = L.WD[k];
        f = M.W()[k] * wd / x.rho;
        qp = M.R * x.t.T * x.h * wd;
    }
    const double Q = G::sum(qp, L.RED);
    if (tid == 0) f = -Q / (x.rho * x.cpm);
    return f;
}

template <int W>
__device__ __forceinline__ double rhs(const DevMech &M, const Lds &L, double y, double P) {
    Mix x;
    species_pass<W, false>(M, y, P, L, x);
    reaction_pass<W, false>(M, L, x.t, x.Ctot, 0, 0, true);
    const double f = finish_rhs<W>(M, L, x);
    __syncthreads();
    return f;
}

// f(y) and this thread's row of M = dg I - J in registers (NP columns), d wdot/dC staged in NWIN
// column windows of width WIN.
template <int W, int NP, int NWIN, int WIN>
__device__ __forceinline__ void iteration_rows(const DevMech &M, const Lds &L, double y, double P, double dg, double (&a)[NP],
                               double &f) {
    using G = Grp<W>;
    const int ns = M.nsp;
    Mix x;
    species_pass<W, true>(M, y, P, L, x);
    const int tid = G::tid();
    const int k = species_of(tid, ns);
    const bool valid = k >= 0;
    double jcc = 0.0, colH = 0.0;
#pragma unroll
    for (int j = 0; j < NP; j++) a[j] = 0.0;
#pragma unroll
    for (int w = 0; w < NWIN; w++) {
        const int c0 = w * WIN;
        reaction_pass<W, true>(M, L, x.t, x.Ctot, c0, WIN, w == 0);
        if (w == 0) f = finish_rhs<W>(M, L, x);
        if (valid) {
            const double *row = &L.JC[k * L.ldj];
#pragma unroll
            for (int j = 0; j < WIN; j++) {
                if (c0 + j >= ns) break;
                const double v = row[j];
                a[1 + c0 + j] = v;                   // raw d wdot_k / dC_(c0+j) for now
                jcc += v * L.C[c0 + j];
            }
            if (k >= c0 && k < c0 + WIN)
                for (int r = 0; r < ns; r++) colH += L.H[r] * L.JC[r * L.ldj + (k - c0)];
        }
        __syncthreads();
    }
    // chain rule (as in the wavefront kernels)
    const double T = x.t.T, RT = M.R * T;
    double resid = 0.0, ra = 0.0, col0 = 0.0, TBk = 0.0, WDk = 0.0, DWTk = 0.0;
    if (valid) {
        TBk = L.TB[k];
        WDk = L.WD[k];
        DWTk = L.DWT[k];
        jcc += TBk * x.Ctot;
        colH *= RT;
        resid = WDk - jcc;
        ra = M.W()[k] * x.Wbar * resid / x.rho;
        col0 = (M.W()[k] / x.rho) * (DWTk + resid * x.t.invT);
    }
    const double Hk = RT * x.h;
    const double sumHTB = G::sum(valid ? Hk * TBk : 0.0, L.RED);
    const double sumHJCC = G::sum(valid ? Hk * jcc : 0.0, L.RED);
    const double dQT = G::sum(valid ? M.R * x.cp * WDk + Hk * (DWTk - jcc * x.t.invT) : 0.0, L.RED);
    const double sdcp = G::sum(valid ? y * M.R * x.dcp * M.invW()[k] : 0.0, L.RED);
    const double fT = G::bcast(f, 0, L.RED + 8);
    const double D = x.rho * x.cpm;
    if (valid) {
        const double dQ = M.invW()[k] * (x.rho * (colH + sumHTB) - x.Wbar * sumHJCC);
        const double dD = x.rho * M.invW()[k] * (M.R * x.cp - x.cpm * x.Wbar);
        L.TROW[k] = -(dQ + fT * dD) / D;
    }
    const double J00 = -(dQT + fT * (-x.rho * x.cpm * x.t.invT + x.rho * sdcp)) / D;
    __syncthreads();
    const double alpha = valid ? M.W()[k] : 0.0;
    const double beta = valid ? M.W()[k] * TBk + ra : 0.0;
    a[0] = (tid == 0 ? dg : 0.0) - (tid == 0 ? J00 : col0);
#pragma unroll
    for (int j = 1; j < NP; j++) {
        const double Jv = tid == 0 ? L.TROW[j - 1] : L.IW[j - 1] * (alpha * a[j] + beta);
        a[j] = (tid == j ? dg : 0.0) - Jv;
    }
    __syncthreads();
}

// In-place Gauss-Jordan inverse with partial pivoting and row rotation.  On return the thread
// whose pivot order is k holds row k of M^-1 with columns permuted: a[j] = Minv[k][p_j], p_j the
// thread that was pivot j.  Threads with index >= NP hold no row.
template <int W, int NP>
__device__ __forceinline__ bool gj_invert(double (&a)[NP], const Lds &L, int &ord) {
    using G = Grp<W>;
    const int tid = G::tid();
    bool done = tid >= NP;
    bool ok = true;
    ord = NP;
    for (int k = 0; k < NP; k++) {
        const double f = a[0];
        const unsigned long long key = done ? 0ull : (unsigned long long)__double_as_longlong(fabs(f));
        unsigned long long best;
        const int p = G::argmax(key, L.RED, best);
        ok = ok && best != 0ull;
        double *buf = L.PB + (k & 1) * 128;
        if (tid == p) {
            const double r = 1.0 / f;
#pragma unroll
            for (int j = 0; j < NP - 1; j++) a[j] = a[j + 1] * r;
            a[NP - 1] = r;
#pragma unroll
            for (int j = 0; j < NP; j++) buf[j] = a[j];
            done = true;
            ord = k;
        }
        __syncthreads();
        if (tid != p) {
#pragma unroll
            for (int j = 0; j < NP - 1; j++) a[j] = fma(-f, buf[j], a[j + 1]);
            a[NP - 1] = -f * buf[NP - 1];
        }
    }
    __syncthreads();
    return ok;
}

// x = M^-1 b with the rotated inverse; b and x one component per thread.
template <int W, int NP>
__device__ __forceinline__ double gj_apply(const double (&a)[NP], const Lds &L, int ord, double b) {
    using G = Grp<W>;
    const int tid = G::tid();
    if (ord < NP) L.BS[ord] = b;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NP; j++) s = fma(a[j], L.BS[j], s);
    if (ord < NP) L.XS[ord] = s;
    __syncthreads();
    const double x = tid < NP ? L.XS[tid] : 0.0;
    __syncthreads();
    return x;
}

template <int W, int NP, int NWIN, int WIN, bool PARK>
struct Ros4Coop {
    static constexpr double qinv = 0.25;
    static constexpr size_t kRows = size_t(NP) * 64 * W;   // parked doubles per workgroup
    static constexpr bool kHalf = false;
    static constexpr size_t kJcMin = 0;
    // the inverse rows go to the workspace while the stage source terms are evaluated and come
    // back as one batch of independent loads before the next products
    __device__ static __forceinline__ void park(const Lds &L, const double (&a)[NP]) {
        if (!PARK) return;
        double *r = L.rows + opaque(Grp<W>::tid());
#pragma unroll
        for (int j = 0; j < NP; j++) r[j * Grp<W>::T] = a[j];
    }
    __device__ static __forceinline__ void unpark(const Lds &L, double (&a)[NP]) {
        if (!PARK) return;
        const double *r = L.rows + opaque(Grp<W>::tid());
#pragma unroll
        for (int j = 0; j < NP; j++) a[j] = r[j * Grp<W>::T];
    }
    __device__ static __forceinline__ bool step(const DevMech &M, const Lds &L, double y, double P, double h, double &ynew,
                                double &e, const IntOpts &, int &) {
        double a[NP];
        double f;
        const double dg = 1.0 / (Ros4::gamma * h);
        iteration_rows<W, NP, NWIN, WIN>(M, L, y, P, dg, a, f);
        int ord;
        const bool ok = gj_invert<W, NP>(a, L, ord);
        const double ih = 1.0 / h;
        const double u1 = gj_apply<W, NP>(a, L, ord, f);
        park(L, a);
        double ft = rhs<W>(M, L, y + Ros4::a21 * u1, P);
        unpark(L, a);
        const double u2 = gj_apply<W, NP>(a, L, ord, ft + (Ros4::c21 * u1) * ih);
        ft = rhs<W>(M, L, y + Ros4::a31 * u1 + Ros4::a32 * u2, P);
        unpark(L, a);
        const double u3 = gj_apply<W, NP>(a, L, ord, ft + (Ros4::c31 * u1 + Ros4::c32 * u2) * ih);
        const double u4 = gj_apply<W, NP>(a, L, ord, ft + (Ros4::c41 * u1 + Ros4::c42 * u2 + Ros4::c43 * u3) * ih);
        ynew = y + Ros4::m1 * u1 + Ros4::m2 * u2 + Ros4::m3 * u3 + Ros4::m4 * u4;
        e = Ros4::e1 * u1 + Ros4::e2 * u2 + Ros4::e3 * u3 + Ros4::e4 * u4;
        return ok;
    }
};

// ---------------------------------------------------------------------------------------
// Half-row variant (N > 64): four wavefronts per reactor; row r of the iteration matrix is split
// over threads 2r (matrix columns [0, H)) and 2r + 1 (columns [H, 2H)), H = NP / 2, so a thread
// holds H doubles, leaving registers to batch the pivot-row reads and room for two wavefronts
// per SIMD.  Source-term phases keep the component mapping of the other kernels (thread i holds
// state component i); per-row scalars and pivot orders pass between the mappings through LDS.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double shfl_pair(double v) { return __shfl_xor(v, 1); }   // partner (lane ^ 1)

template <int NP>
__device__ __forceinline__ void iteration_rows_half(const DevMech &M, const Lds &L, double y, double P, double dg,
                                                    double (&a)[NP / 2], double &f) {
    constexpr int W = 4, H = NP / 2;
    using G = Grp<W>;
    const int ns = M.nsp;
    Mix x;
    species_pass<W, true>(M, y, P, L, x);
    const int tid = G::tid();
    const int k = species_of(tid, ns);              // component mapping
    const bool valid = k >= 0;
    const int row = tid >> 1, half = tid & 1;       // row mapping
    const int kr = row - 1;                         // species of the row (row 0 is T)
    const bool rvalid = row >= 1 && row <= ns;
    double colH = 0.0, jcp = 0.0;                   // jcp: this half's part of sum_l JC[kr][l] C_l
#pragma unroll
    for (int j = 0; j < H; j++) a[j] = 0.0;
    // the first window's per-reaction scatter scalars, kept for the second in this workgroup's park
    // slice
    const bool keep = L.rows != nullptr && 3 * ((M.nrxn + G::T - 1) / G::T) <= H;
    double *cache = keep ? L.rows + opaque(tid) : nullptr;
#pragma unroll
    for (int w = 0; w < 2; w++) {
        const int c0 = w * H - 1;                   // window w: matrix columns [w H, w H + H)
        reaction_pass<W, true>(M, L, x.t, x.Ctot, c0, H, w == 0, cache, keep ? (w == 0 ? 1 : 2) : 0);
        if (w == 0) f = finish_rhs<W>(M, L, x);
        if (rvalid && half == w) {
            const double *r = &L.JC[kr * L.ldj];
#pragma unroll
            for (int j = 0; j < H; j++) {
                const int jc = c0 + j;              // JC column of matrix column w H + j
                if (jc >= 0 && jc < ns) {
                    const double v = r[j];
                    a[j] = v;                       // raw d wdot_kr / dC_jc until the row scalars are known
                    jcp += v * L.C[jc];
                }
            }
        }
        if (valid && k + 1 >= w * H && k + 1 < w * H + H)
            for (int r = 0; r < ns; r++) colH += L.H[r] * L.JC[r * L.ldj + (k + 1 - w * H)];
        __syncthreads();
    }
    const double jrow = jcp + shfl_pair(jcp);
    if (half == 0 && rvalid) L.RJ[row] = jrow;
    __syncthreads();
    // chain rule in the component mapping (as iteration_rows)
    const double T = x.t.T, RT = M.R * T;
    double jcc = 0.0, resid = 0.0, ra = 0.0, col0 = 0.0, TBk = 0.0, WDk = 0.0, DWTk = 0.0;
    if (valid) {
        TBk = L.TB[k];
        WDk = L.WD[k];
        DWTk = L.DWT[k];
        jcc = L.RJ[tid] + TBk * x.Ctot;
        colH *= RT;
        resid = WDk - jcc;
        ra = M.W()[k] * x.Wbar * resid / x.rho;
        col0 = (M.W()[k] / x.rho) * (DWTk + resid * x.t.invT);
    }
    const double Hk = RT * x.h;
    const double sumHTB = G::sum(valid ? Hk * TBk : 0.0, L.RED);
    const double sumHJCC = G::sum(valid ? Hk * jcc : 0.0, L.RED);
    const double dQT = G::sum(valid ? M.R * x.cp * WDk + Hk * (DWTk - jcc * x.t.invT) : 0.0, L.RED);
    const double sdcp = G::sum(valid ? y * M.R * x.dcp * M.invW()[k] : 0.0, L.RED);
    const double fT = G::bcast(f, 0, L.RED + 8);
    const double D = x.rho * x.cpm;
    if (valid) {
        const double dQ = M.invW()[k] * (x.rho * (colH + sumHTB) - x.Wbar * sumHJCC);
        const double dD = x.rho * M.invW()[k] * (M.R * x.cp - x.cpm * x.Wbar);
        L.TROW[k] = -(dQ + fT * dD) / D;
    }
    if (tid < 128) {
        L.RA[tid] = valid ? M.W()[k] : 0.0;
        L.RB[tid] = valid ? M.W()[k] * TBk + ra : 0.0;
        L.RC[tid] = valid ? col0 : 0.0;
    }
    const double J00 = -(dQT + fT * (-x.rho * x.cpm * x.t.invT + x.rho * sdcp)) / D;
    __syncthreads();
    const double alpha = row < 128 ? L.RA[row] : 0.0;
    const double beta = row < 128 ? L.RB[row] : 0.0;
    const double c0r = row < 128 ? L.RC[row] : 0.0;
#pragma unroll
    for (int j = 0; j < H; j++) {
        const int c = half * H + j;                 // matrix column
        double v;
        if (c == 0) {
            v = (row == 0 ? dg : 0.0) - (row == 0 ? J00 : c0r);
        } else {
            const double Jv = row == 0 ? L.TROW[c - 1] : L.IW[c - 1] * (alpha * a[j] + beta);
            v = (row == c ? dg : 0.0) - Jv;
        }
        a[j] = v;
    }
    __syncthreads();
}

// Gauss-Jordan inverse on half rows (rotated as gj_invert): the pivot-column entry of a row is
// element 0 of its first half; each step shifts both halves left by one, the first half taking
// the partner's element 0.  On return ORD[r] is the pivot order of row r.
template <int NP>
__device__ __forceinline__ bool gj_invert_half(double (&a)[NP / 2], const Lds &L, int &ord) {
    constexpr int W = 4, H = NP / 2;
    using G = Grp<W>;
    const int tid = G::tid();
    const int row = tid >> 1, half = tid & 1;
    bool done = row >= NP;
    bool ok = true;
    ord = NP;
    for (int k = 0; k < NP; k++) {
        const double p0 = shfl_pair(a[0]);          // partner's element 0
        const double f = half ? p0 : a[0];          // the row's entry in the pivot column
        const unsigned long long key =
            (done || half) ? 0ull : (unsigned long long)__double_as_longlong(fabs(f));
        unsigned long long best;
        const int p = G::argmax(key, L.RED, best) >> 1;
        ok = ok && best != 0ull;
        double *buf = L.PB + (k & 1) * 128;
        if (row == p) {
            const double r = 1.0 / f;
#pragma unroll
            for (int j = 0; j < H - 1; j++) a[j] = a[j + 1] * r;
            a[H - 1] = (half ? 1.0 : p0) * r;
#pragma unroll
            for (int j = 0; j < H; j++) buf[half * H + j] = a[j];
            done = true;
            ord = k;
        }
        __syncthreads();
        if (row != p) {
            const double *pb = buf + half * H;
#pragma unroll
            for (int j = 0; j < H - 1; j++) a[j] = fma(-f, pb[j], a[j + 1]);
            a[H - 1] = half ? -f * pb[H - 1] : fma(-f, pb[H - 1], p0);
        }
    }
    if (half == 0 && row < NP) L.ORD[row] = ord;
    __syncthreads();
    return ok;
}

// x = M^-1 b with the half-row rotated inverse; b and x in the component mapping.
template <int NP>
__device__ __forceinline__ double gj_apply_half(const double (&a)[NP / 2], const Lds &L, int ord, double b) {
    constexpr int W = 4, H = NP / 2;
    using G = Grp<W>;
    const int tid = G::tid();
    const int row = tid >> 1, half = tid & 1;
    if (tid < NP && L.ORD[tid] < NP) L.BS[L.ORD[tid]] = b;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < H; j++) s = fma(a[j], L.BS[half * H + j], s);
    s += shfl_pair(s);
    if (half == 0 && row < NP && ord < NP) L.XS[ord] = s;
    __syncthreads();
    const double x = tid < NP ? L.XS[tid] : 0.0;
    __syncthreads();
    return x;
}

template <int NP>
struct Ros4CoopHalf {
    static constexpr double qinv = 0.25;
    static constexpr int H = NP / 2;
    static constexpr bool kHalf = true;
    static constexpr size_t kRows = size_t(H) * 256;   // park-slice doubles per workgroup
    static constexpr size_t kJcMin = 0;
    __device__ static __forceinline__ bool step(const DevMech &M, const Lds &L, double y, double P, double h,
                                                double &ynew, double &e, const IntOpts &, int &) {
        double a[H];
        double f;
        const double dg = 1.0 / (Ros4::gamma * h);
        iteration_rows_half<NP>(M, L, y, P, dg, a, f);
        int ord;
        const bool ok = gj_invert_half<NP>(a, L, ord);
        const double ih = 1.0 / h;
        const double u1 = gj_apply_half<NP>(a, L, ord, f);
        double ft = rhs<4>(M, L, y + Ros4::a21 * u1, P);
        const double u2 = gj_apply_half<NP>(a, L, ord, ft + (Ros4::c21 * u1) * ih);
        ft = rhs<4>(M, L, y + Ros4::a31 * u1 + Ros4::a32 * u2, P);
        const double u3 = gj_apply_half<NP>(a, L, ord, ft + (Ros4::c31 * u1 + Ros4::c32 * u2) * ih);
        const double u4 =
            gj_apply_half<NP>(a, L, ord, ft + (Ros4::c41 * u1 + Ros4::c42 * u2 + Ros4::c43 * u3) * ih);
        ynew = y + Ros4::m1 * u1 + Ros4::m2 * u2 + Ros4::m3 * u3 + Ros4::m4 * u4;
        e = Ros4::e1 * u1 + Ros4::e2 * u2 + Ros4::e3 * u3 + Ros4::e4 * u4;
        return ok;
    }
};

// ---------------------------------------------------------------------------------------
// Tile variant (N > 64): the iteration matrix lives in 16 x 16 tiles in the accumulator layout of
// the FP64 16x16x4 matrix-core instruction (lane l, register v of tile (I, J) holds entry
// (16 I + l / 16 + 4 v, 16 J + l % 16)); wavefront w owns tile rows w and w + 4.  The inverse
// comes from a blocked Gauss-Jordan elimination in panels of 16 columns: wavefront 0 eliminates
// the panel (all NP rows; partial pivoting over the rows not yet used as pivots), then every
// wavefront applies it to its tiles with matrix-core rank-16 updates
//     A[:, J] <- A[:, J] with the panel's pivot rows zeroed + T * U[:, J],
// T the eliminated panel (NP x 16) and U the panel's pivot rows before the update (16 x NP), both
// passed through LDS.  This is the arithmetic of 16 scalar Gauss-Jordan steps regrouped (sums of
// products in another order), so the result is the same inverse with the same pivots up to
// rounding; the pivot order of each row is kept for the solves, as in the other forms.
// ---------------------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));

typedef float f4 __attribute__((ext_vector_type(4)));

// Matrix row held in register v of lane group g (= lane / 16) of tile row I.  The FP64 16x16x4
// instruction interleaves the rows of its accumulator over the lane groups (row g + 4 v of the
// tile; measured on the device), where the FP32 one keeps them contiguous (4 g + v).  F32L selects
// the FP32 layout.
template <bool F32L = false>
__device__ __forceinline__ int tile_row(int I, int g, int v) { return F32L ? 16 * I + 4 * g + v : 16 * I + g + 4 * v; }

template <class T> struct TileT;
template <> struct TileT<double> {
    using V = d4;
    static constexpr bool F32L = false;
    __device__ static __forceinline__ V mfma(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // pivot-search key: the high word of |v| (ordered like |v|; values within a relative 2^-20 of
    // each other may tie, and then the first row in lane order is taken)
    __device__ static __forceinline__ unsigned key(double v) { return unsigned(__double2hiint(fabs(v))); }
    __device__ static __forceinline__ double readlane(double v, int src) { return readlane_d(v, src); }
    // 1 / x from the hardware estimate and two Newton-Raphson steps (within an ulp)
    __device__ static __forceinline__ double recip(double x) {
        double r = __builtin_amdgcn_rcp(x);
        r = fma(fma(-x, r, 1.0), r, r);
        return fma(fma(-x, r, 1.0), r, r);
    }
};
template <> struct TileT<float> {
    using V = f4;
    static constexpr bool F32L = true;
    __device__ static __forceinline__ V mfma(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ unsigned key(float v) { return __float_as_uint(fabsf(v)); }
    __device__ static __forceinline__ float readlane(float v, int src) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
    }
    __device__ static __forceinline__ float recip(float x) {
        const float r = __builtin_amdgcn_rcpf(x);
        return fmaf(fmaf(-x, r, 1.0f), r, r);
    }
};

template <int NP>
struct TileGeom {
    static_assert(NP % 16 == 0 && NP <= 128, "tile form: NP a multiple of 16, at most 128");
    static constexpr int TR = NP / 16;            // tile rows (and tile columns)
    static constexpr int RW = (TR + 3) / 4;       // tile rows per wavefront
    static constexpr int PLD = NP + 4;            // column stride of an LDS panel buffer (doubles)
    static constexpr int UBLD = NP;               // row stride of the pivot-row buffer
    // scratch carved from the JC region: panel buffers [2][16][PLD] and pivot rows [16][UBLD]
    static constexpr size_t kScratch = size_t(2) * 16 * PLD + size_t(16) * UBLD;
    // Tile row held in slot i by wavefront w (TR when none).  Up to seven tile rows, wavefront 0
    // (which also eliminates the panels) holds only row 0 and the others rows w and w + 3, so its
    // share of the updates is the smaller one; eight tile rows go two to each wavefront.
    static constexpr int STRIDE = TR <= 7 ? 3 : 4;
    __device__ static __forceinline__ int tile_of(int w, int i) {
        return (TR <= 7 && w == 0 && i > 0) ? TR : w + STRIDE * i;
    }
};

// Orders this wavefront's LDS accesses around an exchange between its own lanes (LDS operations
// of one wavefront complete in issue order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float row16_sum(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x124>(v);
    v += dpp_f<0x128>(v);
    return v;
}

// Sum over the 16 lanes of a DPP row, returned to every lane of the row.
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_d<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x124>(v);   // row_ror 4
    v += dpp_d<0x128>(v);   // row_ror 8
    return v;
}

// f(y) and this wavefront's tiles of M = dg I - J; d wdot/dC staged in two column windows (as
// iteration_rows_half, whose row-pair mapping still forms the row sums sum_l JC[k][l] C_l).
template <int NP, bool F32L = false>
__device__ __forceinline__ void iteration_tiles(const DevMech &M, const Lds &L, double y, double P, double dg,
                                                d4 (&m)[TileGeom<NP>::RW][TileGeom<NP>::TR], double &f) {
    constexpr int W = 4, H = NP / 2, TR = TileGeom<NP>::TR, RW = TileGeom<NP>::RW;
    using G = Grp<W>;
    const int ns = M.nsp;
    Mix x;
    species_pass<W, true>(M, y, P, L, x);
    const int tid = G::tid();
    const int k = species_of(tid, ns);              // component mapping
    const bool valid = k >= 0;
    const int row = tid >> 1, half = tid & 1;       // row-pair mapping (row sums)
    const int kr = row - 1;
    const bool rvalid = row >= 1 && row <= ns;
    const int wv = G::wave(), ln = G::lane(), g = ln >> 4, c16 = ln & 15;
    double colH = 0.0, jcp = 0.0;
#pragma unroll
    for (int i = 0; i < RW; i++)
#pragma unroll
        for (int J = 0; J < TR; J++) m[i][J] = d4{0.0, 0.0, 0.0, 0.0};
    const bool keep = L.rows != nullptr && 3 * ((M.nrxn + G::T - 1) / G::T) <= H;
    double *cache = keep ? L.rows + opaque(tid) : nullptr;
    // column sums sum_r H_r d wdot_r / dC_col accumulate in VX from the tiles; hr = H of the rows
    // this lane holds (0 for the temperature row and padding)
    if (tid < 128) L.VX[tid] = 0.0;
    double hr[RW][4];
#pragma unroll
    for (int i = 0; i < RW; i++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int r = tile_row<F32L>(TileGeom<NP>::tile_of(wv, i), g, v);
            hr[i][v] = (r >= 1 && r <= ns) ? L.H[r - 1] : 0.0;
        }
#pragma unroll
    for (int w = 0; w < 2; w++) {
        const int c0 = w * H - 1;                   // window w: matrix columns [w H, w H + H)
        reaction_pass<W, true>(M, L, x.t, x.Ctot, c0, H, w == 0, cache, keep ? (w == 0 ? 1 : 2) : 0);
        if (w == 0) f = finish_rhs<W>(M, L, x);
        if (rvalid && half == w) {
            const double *r = &L.JC[kr * L.ldj];
            for (int j = 0; j < H; j++) {
                const int jc = c0 + j;
                if (jc >= 0 && jc < ns) jcp += r[j] * L.C[jc];
            }
        }
        // raw window entries d wdot_(r-1) / dC_(col-1) into this wavefront's tiles
#pragma unroll
        for (int i = 0; i < RW; i++) {
            const int I = TileGeom<NP>::tile_of(wv, i);
            if (I >= TR) break;
#pragma unroll
            for (int J = 0; J < TR; J++) {
                if (16 * J + 15 < w * H || 16 * J >= w * H + H) continue;
                const int col = 16 * J + c16;
                const bool cin = col >= w * H && col < w * H + H && col >= 1 && col <= ns;
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int r = tile_row<F32L>(I, g, v);
                    if (cin && r >= 1 && r <= ns) m[i][J][v] = L.JC[(r - 1) * L.ldj + (col - w * H)];
                }
                if (cin) {
                    double part = 0.0;
#pragma unroll
                    for (int v = 0; v < 4; v++) part = fma(hr[i][v], m[i][J][v], part);
                    atomicAdd(&L.VX[col], part);
                }
            }
        }
        __syncthreads();
    }
    if (valid) colH = L.VX[k + 1];
    const double jrow = jcp + shfl_pair(jcp);
    if (half == 0 && rvalid) L.RJ[row] = jrow;
    __syncthreads();
    // chain rule in the component mapping (as iteration_rows)
    const double T = x.t.T, RT = M.R * T;
    double jcc = 0.0, resid = 0.0, ra = 0.0, col0 = 0.0, TBk = 0.0, WDk = 0.0, DWTk = 0.0;
    if (valid) {
        TBk = L.TB[k];
        WDk = L.WD[k];
        DWTk = L.DWT[k];
        jcc = L.RJ[tid] + TBk * x.Ctot;
        colH *= RT;
        resid = WDk - jcc;
        ra = M.W()[k] * x.Wbar * resid / x.rho;
        col0 = (M.W()[k] / x.rho) * (DWTk + resid * x.t.invT);
    }
    const double Hk = RT * x.h;
    const double sumHTB = G::sum(valid ? Hk * TBk : 0.0, L.RED);
    const double sumHJCC = G::sum(valid ? Hk * jcc : 0.0, L.RED);
    const double dQT = G::sum(valid ? M.R * x.cp * WDk + Hk * (DWTk - jcc * x.t.invT) : 0.0, L.RED);
    const double sdcp = G::sum(valid ? y * M.R * x.dcp * M.invW()[k] : 0.0, L.RED);
    const double fT = G::bcast(f, 0, L.RED + 8);
    const double D = x.rho * x.cpm;
    if (valid) {
        const double dQ = M.invW()[k] * (x.rho * (colH + sumHTB) - x.Wbar * sumHJCC);
        const double dD = x.rho * M.invW()[k] * (M.R * x.cp - x.cpm * x.Wbar);
        L.TROW[k] = -(dQ + fT * dD) / D;
    }
    if (tid < 128) {
        L.RA[tid] = valid ? M.W()[k] : 0.0;
        L.RB[tid] = valid ? M.W()[k] * TBk + ra : 0.0;
        L.RC[tid] = valid ? col0 : 0.0;
    }
    const double J00 = -(dQT + fT * (-x.rho * x.cpm * x.t.invT + x.rho * sdcp)) / D;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RW; i++) {
        const int I = TileGeom<NP>::tile_of(wv, i);
        if (I >= TR) break;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int r = tile_row<F32L>(I, g, v);
            const double alpha = L.RA[r], beta = L.RB[r], c0r = L.RC[r];
#pragma unroll
            for (int J = 0; J < TR; J++) {
                const int col = 16 * J + c16;
                double Jv;
                if (col == 0) Jv = r == 0 ? J00 : c0r;
                else if (r == 0) Jv = L.TROW[col - 1];
                else Jv = L.IW[col - 1] * (alpha * m[i][J][v] + beta);
                m[i][J][v] = (r == col ? dg : 0.0) - Jv;
            }
        }
    }
    __syncthreads();
}

// Rank-16 update of tile columns J0 <= J < J1 with eliminated panel p: A = the panel rows of this
// wavefront's tile rows (PNL, column-major), B = the panel's pivot rows (UB), on the matrix cores.
template <int J0, int J1, int NP, class T>
__device__ __forceinline__ void tile_update(typename TileT<T>::V (&m)[TileGeom<NP>::RW][TileGeom<NP>::TR],
                                            const T *PNL, const T *UB, int p, int wv, int g, int c16) {
    using TG = TileGeom<NP>;
    constexpr int TR = TG::TR, RW = TG::RW, PLD = TG::PLD, UBLD = TG::UBLD;
#pragma unroll
    for (int i = 0; i < RW; i++) {
        const int I = TG::tile_of(wv, i);
        if (I >= TR) break;
        T a[4];
#pragma unroll
        for (int s = 0; s < 4; s++) a[s] = PNL[(4 * s + g) * PLD + 16 * I + c16];
#pragma unroll
        for (int J = J0; J < J1; J++) {
            const int gJ = p + J < TR ? p + J : p + J - TR;
#pragma unroll
            for (int s = 0; s < 4; s++) {
                const T b = UB[(4 * s + g) * UBLD + 16 * gJ + c16];
                m[i][J] = TileT<T>::mfma(a[s], b, m[i][J]);
            }
        }
    }
}

// Tile column c of this wavefront's tile rows into an LDS panel buffer, column-major:
// PNL[col PLD + r] = A[r][16 c + col].
template <int NP, class T>
__device__ __forceinline__ void store_panel(const typename TileT<T>::V (&m)[TileGeom<NP>::RW][TileGeom<NP>::TR],
                                            int c, T *PNL, int wv, int g, int c16) {
    using TG = TileGeom<NP>;
#pragma unroll
    for (int i = 0; i < TG::RW; i++) {
        const int I = TG::tile_of(wv, i);
        if (I >= TG::TR) break;
#pragma unroll
        for (int v = 0; v < 4; v++) PNL[c16 * TG::PLD + tile_row<TileT<T>::F32L>(I, g, v)] = m[i][c][v];
    }
}

// Tile columns rotate by one: the next panel becomes column 0.
template <int NP, class V>
__device__ __forceinline__ void rotate_tiles(V (&m)[TileGeom<NP>::RW][TileGeom<NP>::TR]) {
#pragma unroll
    for (int i = 0; i < TileGeom<NP>::RW; i++) {
        const V t0 = m[i][0];
#pragma unroll
        for (int J = 0; J + 1 < TileGeom<NP>::TR; J++) m[i][J] = m[i][J + 1];
        m[i][TileGeom<NP>::TR - 1] = t0;
    }
}

// Blocked Gauss-Jordan inverse in place on the tiles.  On return L.ORD[r] is the pivot order of
// row r: tile entry (r, j) = Minv[ORD[r]][p_j], p_j the row that was pivot j.
//
// Panels of 16 columns with look-ahead: once panel p is eliminated and its pivot rows are in UB,
// every wavefront first applies it to tile column 1 (the next panel) and stores that column, then
// wavefront 0 eliminates panel p + 1 while the others apply panel p to the remaining columns;
// wavefront 0 holds the fewest tile rows, so its own remaining updates are the shortest.
template <int NP, class T = double>
__device__ __forceinline__ bool gj_invert_tiles(typename TileT<T>::V (&m)[TileGeom<NP>::RW][TileGeom<NP>::TR],
                                                const Lds &L) {
    using TG = TileGeom<NP>;
    using TT = TileT<T>;
    constexpr bool F32L = TT::F32L;
    constexpr int TR = TG::TR, RW = TG::RW, PLD = TG::PLD, UBLD = TG::UBLD;
    using G = Grp<4>;
    const int tid = G::tid(), wv = G::wave(), ln = G::lane(), g = ln >> 4, c16 = ln & 15;
    T *const JCT = reinterpret_cast<T *>(L.JC);
    T *const UB = JCT + 2 * 16 * PLD;
    if (tid < 128) L.ORD[tid] = NP;
    unsigned pmask = 0;          // wavefront 0: bit 0 (1) set once row l (l + 64) has been a pivot
    bool ok = true;
    // panel 0 (tile column 0) into the first panel buffer
    store_panel<NP, T>(m, 0, JCT, wv, g, c16);
    __syncthreads();
    for (int p = 0; p < TR; p++) {
        T *const PNL = JCT + (p & 1) * 16 * PLD;
        // (1) wavefront 0 eliminates panel p with one panel row per lane (rows l and l + 64): the
        //     pivot search is a wavefront reduction, the pivot row reaches every lane by lane reads
        //     (scalar operands of the updates), and the pivot reciprocal comes from the hardware
        //     estimate refined by Newton steps.  Meanwhile every wavefront finishes panel p - 1 on
        //     tile columns 2.. (column 1 of panel p - 1 was this panel) and rotates its columns.
        if (wv == 0) {
            const bool has1 = ln + 64 < NP;
            T R0[16], R1[16];
#pragma unroll
            for (int c = 0; c < 16; c++) {
                R0[c] = PNL[c * PLD + ln];
                R1[c] = has1 ? PNL[c * PLD + ln + 64] : T(0);
            }
#pragma unroll
            for (int c = 0; c < 16; c++) {
                const unsigned k0 = (pmask & 1u) ? 0u : TT::key(R0[c]);
                const unsigned k1 = ((pmask & 2u) || !has1) ? 0u : TT::key(R1[c]);
                const bool w1 = k1 > k0;
                const unsigned key = w1 ? k1 : k0;
                const unsigned mx = __ockl_wfred_max_u32(key);
                ok = ok && mx != 0u;
                const int src = __builtin_ctzll(__ballot(key == mx));
                const int sel1 = __builtin_amdgcn_readlane(int(w1), src);
                const bool piv = ln == src;
                // each pivot-row entry is read from the pivot lane just before its column is
                // updated (the pivot row itself becomes that entry times 1 / pivot)
                if (sel1) {
                    const T rp = TT::recip(TT::readlane(R1[c], src));
                    const T g0 = -R0[c] * rp, g1 = -R1[c] * rp;
#pragma unroll
                    for (int jj = 1; jj < 16; jj++) {
                        const int j = (c + jj) & 15;      // the next pivot column first
                        const T pj = TT::readlane(R1[j], src);
                        R0[j] = fma(g0, pj, R0[j]);
                        const T u = fma(g1, pj, R1[j]);
                        R1[j] = piv ? pj * rp : u;
                    }
                    R0[c] = g0;
                    R1[c] = piv ? rp : g1;
                    if (piv) pmask |= 2u;
                } else {
                    const T rp = TT::recip(TT::readlane(R0[c], src));
                    const T g0 = -R0[c] * rp, g1 = -R1[c] * rp;
#pragma unroll
                    for (int jj = 1; jj < 16; jj++) {
                        const int j = (c + jj) & 15;      // the next pivot column first
                        const T pj = TT::readlane(R0[j], src);
                        const T u = fma(g0, pj, R0[j]);
                        R0[j] = piv ? pj * rp : u;
                        R1[j] = fma(g1, pj, R1[j]);
                    }
                    R0[c] = piv ? rp : g0;
                    R1[c] = g1;
                    if (piv) pmask |= 1u;
                }
                if (ln == 0) L.ORD[src + 64 * sel1] = 16 * p + c;
            }
#pragma unroll
            for (int c = 0; c < 16; c++) {
                PNL[c * PLD + ln] = R0[c];
                if (has1) PNL[c * PLD + ln + 64] = R1[c];
            }
        }
        if (p > 0) {
            tile_update<2, TR, NP, T>(m, JCT + ((p - 1) & 1) * 16 * PLD, UB, p - 1, wv, g, c16);
            rotate_tiles<NP>(m);
        }
        __syncthreads();
        // (2) the eliminated panel into tile column 0; the pivot rows' entries of the other
        //     columns into UB (as U[order within the panel][column]) and zeroed in the tiles
#pragma unroll
        for (int i = 0; i < RW; i++) {
            const int I = TileGeom<NP>::tile_of(wv, i);
            if (I >= TR) break;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int r = tile_row<F32L>(I, g, v);
                m[i][0][v] = PNL[c16 * PLD + r];
                const int o = L.ORD[r] - 16 * p;
                if (o >= 0 && o < 16) {
#pragma unroll
                    for (int J = 1; J < TR; J++) {
                        const int gJ = p + J < TR ? p + J : p + J - TR;
                        UB[o * UBLD + 16 * gJ + c16] = m[i][J][v];
                        m[i][J][v] = T(0);
                    }
                }
            }
        }
        __syncthreads();
        // (3) look-ahead: panel p applied to tile column 1 (the next panel), which is then stored
        //     for its elimination
        if (p + 1 < TR) {
            tile_update<1, 2, NP, T>(m, PNL, UB, p, wv, g, c16);
            store_panel<NP, T>(m, 1, JCT + ((p + 1) & 1) * 16 * PLD, wv, g, c16);
            __syncthreads();
        }
    }
    // the last panel on every other tile column
    tile_update<1, TR, NP, T>(m, JCT + ((TR - 1) & 1) * 16 * PLD, UB, TR - 1, wv, g, c16);
    rotate_tiles<NP>(m);
    __syncthreads();
    return ok;
}

// x = M^-1 b with the tile inverse; b and x in the component mapping; ordr[i][v] = ORD of the
// row held in register v of tile row i.
template <int NP, class T = double>
__device__ __forceinline__ double gj_apply_tiles(const typename TileT<T>::V (&m)[TileGeom<NP>::RW][TileGeom<NP>::TR],
                                                 const Lds &L, const int (&ordr)[TileGeom<NP>::RW][4], double b) {
    constexpr int TR = TileGeom<NP>::TR, RW = TileGeom<NP>::RW;
    using G = Grp<4>;
    const int tid = G::tid(), wv = G::wave(), ln = G::lane(), c16 = ln & 15;
    if (tid < NP && L.ORD[tid] < NP) L.BS[L.ORD[tid]] = b;
    __syncthreads();
    T bs[TR];
#pragma unroll
    for (int J = 0; J < TR; J++) bs[J] = T(L.BS[16 * J + c16]);
#pragma unroll
    for (int i = 0; i < RW; i++) {
        if (TileGeom<NP>::tile_of(wv, i) >= TR) break;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            T z = T(0);
#pragma unroll
            for (int J = 0; J < TR; J++) z = fma(m[i][J][v], bs[J], z);
            z = row16_sum(z);
            if (c16 == 0 && ordr[i][v] < NP) L.XS[ordr[i][v]] = double(z);
        }
    }
    __syncthreads();
    const double xv = tid < NP ? L.XS[tid] : 0.0;
    __syncthreads();
    return xv;
}

// r = b - M x with the FP64 tiles of M (layout F32L); b and x in the component mapping.
template <int NP, bool F32L>
__device__ __forceinline__ double resid_tiles(const d4 (&m)[TileGeom<NP>::RW][TileGeom<NP>::TR], const Lds &L,
                                              double x, double b) {
    constexpr int TR = TileGeom<NP>::TR, RW = TileGeom<NP>::RW;
    using G = Grp<4>;
    const int tid = G::tid(), wv = G::wave(), ln = G::lane(), g = ln >> 4, c16 = ln & 15;
    if (tid < 128) L.VX[tid] = tid < NP ? x : 0.0;
    __syncthreads();
    double xs[TR];
#pragma unroll
    for (int J = 0; J < TR; J++) xs[J] = L.VX[16 * J + c16];
#pragma unroll
    for (int i = 0; i < RW; i++) {
        const int I = TileGeom<NP>::tile_of(wv, i);
        if (I >= TR) break;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            double z = 0.0;
#pragma unroll
            for (int J = 0; J < TR; J++) z = fma(m[i][J][v], xs[J], z);
            z = row16_sum(z);
            if (c16 == 0) L.XS[tile_row<F32L>(I, g, v)] = z;
        }
    }
    __syncthreads();
    const double r = tid < NP ? b - L.XS[tid] : 0.0;
    __syncthreads();
    return r;
}

__device__ __forceinline__ double group_max_abs(double v, double *red) {
    const double w = __longlong_as_double(
        (long long)__ockl_wfred_max_u64((unsigned long long)__double_as_longlong(fabs(v))));
    if (Grp<4>::lane() == 0) red[Grp<4>::wave()] = w;
    __syncthreads();
    const double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return r;
}

// Linear solves of the tile ROS4 step with the factorisation in FP32 (matrix-core FP32 updates) and
// FP64 residual refinement (RHS, Jacobian, error norm and control stay FP64): x = M32^-1 b, then up
// to `sweeps` corrections d = M32^-1 (b - M x), x += d, with M the FP64 matrix.  A solve is done
// once |d| <= 2^-48 |x| (max norms over the state); it fails when a correction stops shrinking by
// half or the sweeps run out first.
template <int NP>
__device__ __forceinline__ double refined_solve(const d4 (&m)[TileGeom<NP>::RW][TileGeom<NP>::TR],
                                                const f4 (&mf)[TileGeom<NP>::RW][TileGeom<NP>::TR], const Lds &L,
                                                const int (&ordr)[TileGeom<NP>::RW][4], int sweeps, double b,
                                                bool &conv) {
    double x = gj_apply_tiles<NP, float>(mf, L, ordr, b);
    conv = true;
    if (sweeps <= 0) return x;
    conv = false;
    double dprev = INFINITY;
    for (int s = 0; s < sweeps; s++) {
        const double r = resid_tiles<NP, true>(m, L, x, b);
        const double d = gj_apply_tiles<NP, float>(mf, L, ordr, r);
        x += d;
        const double dmax = group_max_abs(d, L.RED), xmax = group_max_abs(x, L.RED);
        if (dmax <= 0x1p-48 * xmax) {
            conv = true;
            break;
        }
        if (!(dmax <= 0.5 * dprev)) break;        // stagnation (or not finite)
        dprev = dmax;
    }
    return x;
}

template <int NP>
struct Ros4CoopTile {
    static constexpr double qinv = 0.25;
    static constexpr int H = NP / 2, TR = TileGeom<NP>::TR, RW = TileGeom<NP>::RW;
    static constexpr bool kHalf = true;
    static constexpr size_t kRows = size_t(H) * 256;   // park-slice doubles per workgroup
    static constexpr size_t kJcMin = TileGeom<NP>::kScratch;
    __device__ static __forceinline__ bool step(const DevMech &M, const Lds &L, double y, double P, double h,
                                                double &ynew, double &e, const IntOpts &, int &) {
        d4 m[RW][TR];
        double f;
        const double dg = 1.0 / (Ros4::gamma * h);
        iteration_tiles<NP>(M, L, y, P, dg, m, f);
        const bool ok = gj_invert_tiles<NP>(m, L);
        int ordr[RW][4];
        {
            const int wv = Grp<4>::wave(), g = Grp<4>::lane() >> 4;
#pragma unroll
            for (int i = 0; i < RW; i++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int I = TileGeom<NP>::tile_of(wv, i);
                    ordr[i][v] = I < TR ? L.ORD[tile_row(I, g, v)] : NP;
                }
        }
        const double ih = 1.0 / h;
        const double u1 = gj_apply_tiles<NP>(m, L, ordr, f);
        double ft = rhs<4>(M, L, y + Ros4::a21 * u1, P);
        const double u2 = gj_apply_tiles<NP>(m, L, ordr, ft + (Ros4::c21 * u1) * ih);
        ft = rhs<4>(M, L, y + Ros4::a31 * u1 + Ros4::a32 * u2, P);
        const double u3 = gj_apply_tiles<NP>(m, L, ordr, ft + (Ros4::c31 * u1 + Ros4::c32 * u2) * ih);
        const double u4 =
            gj_apply_tiles<NP>(m, L, ordr, ft + (Ros4::c41 * u1 + Ros4::c42 * u2 + Ros4::c43 * u3) * ih);
        ynew = y + Ros4::m1 * u1 + Ros4::m2 * u2 + Ros4::m3 * u3 + Ros4::m4 * u4;
        e = Ros4::e1 * u1 + Ros4::e2 * u2 + Ros4::e3 * u3 + Ros4::e4 * u4;
        return ok;
    }
};

// ROS4 step of the tile form with the linear solves in FP32 and FP64 refinement (refined_solve).
// If a solve fails to converge, the FP32 step is abandoned and this reactor-step is done again
// with the FP64 tile step (Jacobian, FP64 matrix-core inverse, solves); `fallback` counts it.
template <int NP>
struct Ros4CoopTile32 {
    static constexpr double qinv = 0.25;
    static constexpr int H = NP / 2, TR = TileGeom<NP>::TR, RW = TileGeom<NP>::RW;
    static constexpr bool kHalf = true;
    static constexpr size_t kRows = size_t(H) * 256;   // park-slice doubles per workgroup
    static constexpr size_t kJcMin = TileGeom<NP>::kScratch;
    __device__ static __forceinline__ bool step32(const DevMech &M, const Lds &L, double y, double P, double h,
                                                  double &ynew, double &e, int sweeps, bool &conv) {
        d4 m[RW][TR];
        f4 mf[RW][TR];
        double f;
        const double dg = 1.0 / (Ros4::gamma * h);
        iteration_tiles<NP, true>(M, L, y, P, dg, m, f);
#pragma unroll
        for (int i = 0; i < RW; i++)
#pragma unroll
            for (int J = 0; J < TR; J++)
#pragma unroll
                for (int v = 0; v < 4; v++) mf[i][J][v] = float(m[i][J][v]);
        const bool ok = gj_invert_tiles<NP, float>(mf, L);
        int ordr[RW][4];
        {
            const int wv = Grp<4>::wave(), g = Grp<4>::lane() >> 4;
#pragma unroll
            for (int i = 0; i < RW; i++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int I = TileGeom<NP>::tile_of(wv, i);
                    ordr[i][v] = I < TR ? L.ORD[tile_row<true>(I, g, v)] : NP;
                }
        }
        const double ih = 1.0 / h;
        const double u1 = refined_solve<NP>(m, mf, L, ordr, sweeps, f, conv);
        if (!conv) return ok;
        double ft = rhs<4>(M, L, y + Ros4::a21 * u1, P);
        const double u2 = refined_solve<NP>(m, mf, L, ordr, sweeps, ft + (Ros4::c21 * u1) * ih, conv);
        if (!conv) return ok;
        ft = rhs<4>(M, L, y + Ros4::a31 * u1 + Ros4::a32 * u2, P);
        const double u3 = refined_solve<NP>(m, mf, L, ordr, sweeps, ft + (Ros4::c31 * u1 + Ros4::c32 * u2) * ih, conv);
        if (!conv) return ok;
        const double u4 = refined_solve<NP>(m, mf, L, ordr, sweeps,
                                            ft + (Ros4::c41 * u1 + Ros4::c42 * u2 + Ros4::c43 * u3) * ih, conv);
        if (!conv) return ok;
        ynew = y + Ros4::m1 * u1 + Ros4::m2 * u2 + Ros4::m3 * u3 + Ros4::m4 * u4;
        e = Ros4::e1 * u1 + Ros4::e2 * u2 + Ros4::e3 * u3 + Ros4::e4 * u4;
        return ok;
    }
    __device__ static __forceinline__ bool step(const DevMech &M, const Lds &L, double y, double P, double h,
                                                double &ynew, double &e, const IntOpts &o, int &fallback) {
        bool conv = true;
        const bool ok = step32(M, L, y, P, h, ynew, e, o.refine_sweeps, conv);
        if (conv) return ok;
        fallback++;
        return Ros4CoopTile<NP>::step(M, L, y, P, h, ynew, e, o, fallback);
    }
};

// Algorithm 1 for one reactor on the group (same specification as the other kernels).
template <int W, class S>
__device__ __forceinline__ void integrate_reactor(const DevMech &M, const Lds &L, int64_t r, double *y, int64_t ld, const double *p,
                                  const double *t_end, double *t_io, double *h_io, const IntOpts &o, int32_t *status,
                                  int32_t *nacc, int32_t *nrej) {
    using G = Grp<W>;
    const int N = M.N;
    const int tid = G::tid();
    const bool mine = tid < N;
    double yv = mine ? y[int64_t(tid) * ld + r] : 0.0;
    const double P = p[r];
    const double te = t_end[r];
    double t = t_io ? t_io[r] : 0.0;
    double h = h_io ? h_io[r] : 0.0;
    int st = CK_ST_OK;
    int na = 0, nj = 0, fb = 0;
    auto all_finite = [&](double v) {
        return G::sum((mine && !isfinite(v)) ? 1.0 : 0.0, L.RED) == 0.0;
    };
    auto wsq = [&](double v) { return G::sum(mine ? v * v : 0.0, L.RED); };
    if (!all_finite(yv)) {
        st = CK_ST_NONFINITE;
        h = 0.0;
    } else if (o.h_fixed > 0.0) {
        h = o.h_fixed;
    } else if (!(h > 0.0)) {
        if (o.h0 > 0.0) {
            h = o.h0;
        } else if (t < te) {
            const double f0 = rhs<W>(M, L, yv, P);
            if (!all_finite(f0)) {
                st = CK_ST_NONFINITE;
                h = 0.0;
            } else {
                const double sc = o.atol + o.rtol * fabs(yv);
                const double d0 = sqrt(wsq(yv / sc) / N), d1 = sqrt(wsq(f0 / sc) / N);
                const double span = te - t;
                double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
                h0 = fmin(h0, span);
                const double f1 = rhs<W>(M, L, yv + h0 * f0, P);
                const double d2 = sqrt(wsq((f1 - f0) / sc) / N) / h0;
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
            double yn, e;
            const bool ok = S::step(M, L, yv, P, hs, yn, e, o, fb);
            double err;
            if (o.h_fixed > 0.0)
                err = 0.0;
            else if (!ok)
                err = INFINITY;
            else {
                const double sc = o.atol + o.rtol * fmax(fabs(yv), fabs(yn));
                err = sqrt(wsq(e / sc) / N);
                if (!all_finite(yn)) err = INFINITY;
            }
            const bool acc = err < 1.0;
            if (acc) {
                yv = yn;
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
    if (mine) y[int64_t(tid) * ld + r] = yv;
    if (tid == 0) {
        if (t_io) t_io[r] = t;
        if (h_io) h_io[r] = h;
        status[r] = st;
        nacc[r] = na;
        nrej[r] = nj;
        if (o.n_fallback) o.n_fallback[r] = fb;
    }
}

// WPE > 0: the register budget of WPE resident wavefronts per SIMD is imposed on the compiler.
template <int W, class S, int WIN, int WPE = 0>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1, WPE > 0 ? WPE : 10)))
coop_kernel(DevMech M, int64_t n, double *y, int64_t ld, const double *p, const double *t_end, double *t_io,
            double *h_io, IntOpts o, unsigned *queue, double *park, int32_t *status, int32_t *nacc, int32_t *nrej) {
    extern __shared__ double lds_raw[];
    Lds L = carve(lds_raw, M.nsp, WIN, S::kHalf, S::kJcMin);
    if (park) L.rows = park + size_t(blockIdx.x) * S::kRows;
    init_lds(M, L, int(threadIdx.x), 64 * W);
    __shared__ int64_t next;
    for (;;) {
        if (threadIdx.x == 0) next = int64_t(atomicAdd(queue, 1u));
        __syncthreads();
        const int64_t r = next;
        __syncthreads();
        if (r >= n) break;
        integrate_reactor<W, S>(M, L, r, y, ld, p, t_end, t_io, h_io, o, status, nacc, nrej);
        __syncthreads();
    }
}

// Standalone analytic Jacobian for N > 64 (deep vectorisation: one reactor per four-wavefront
// group, the half-row assembly of the integrator with dg = 0, so a = -J exactly).  Rates are
// evaluated again in the second column window (no park slice).  jac[(i N + j) ld + r] = dfi/dyj.
template <int NP>
__global__ void __launch_bounds__(256) jac_group_kernel(DevMech M, int64_t n, const double *y, int64_t ld,
                                                        const double *p, double *jac) {
    constexpr int H = NP / 2;
    extern __shared__ double lds_raw[];
    Lds L = carve(lds_raw, M.nsp, H, true);
    init_lds(M, L, int(threadIdx.x), 256);
    const int N = M.N, tid = int(threadIdx.x);
    const int row = tid >> 1, half = tid & 1;
    for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
        const double yv = tid < N ? y[int64_t(tid) * ld + r] : 0.0;
        double a[H];
        double f;
        iteration_rows_half<NP>(M, L, yv, p[r], 0.0, a, f);
        if (row < N) {
            double *out = jac + int64_t(row) * N * ld + r;
#pragma unroll
            for (int j = 0; j < H; j++) {
                const int c = half * H + j;
                if (c < N) out[int64_t(c) * ld] = -a[j];
            }
        }
        __syncthreads();
    }
}

__global__ void zero_queue_kernel(unsigned *q) { *q = 0u; }

// Workgroups per CU of a parking kernel are capped so that the parked rows fit the workspace.
constexpr int kParkBlocksPerCu = 2;

template <int W, class S, int WIN, bool PARK, int WPE = 0>
int launch_kernel(const DevMech &M, int64_t n, double *y, int64_t ld, const double *p, const double *t_end, double *t,
                  double *h, const IntOpts &o, unsigned *queue, int32_t *status, int32_t *nacc, int32_t *nrej,
                  hipStream_t s) {
    const size_t lds = lds_doubles(M.nsp, WIN, S::kHalf, S::kJcMin) * sizeof(double);
    auto kern = coop_kernel<W, S, WIN, WPE>;
    if (lds > 64 * 1024 && hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) != hipSuccess)
        return CK_EHIP;
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CK_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return CK_EHIP;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, 64 * W, lds) != hipSuccess || per < 1)
        return CK_EHIP;
    if (o.blocks_per_cu > 0 && o.blocks_per_cu < per) per = o.blocks_per_cu;
    if (PARK && per > kParkBlocksPerCu) per = kParkBlocksPerCu;
    int64_t grid = int64_t(cus) * per;
    if (grid > n) grid = n;
    double *park = PARK ? reinterpret_cast<double *>(reinterpret_cast<char *>(queue) + 256) : nullptr;
    zero_queue_kernel<<<1, 1, 0, s>>>(queue);
    kern<<<dim3(unsigned(grid)), dim3(64 * W), lds, s>>>(M, n, y, ld, p, t_end, t, h, o, queue, park, status, nacc,
                                                         nrej);
    return hipGetLastError() == hipSuccess ? CK_OK : CK_EHIP;
}

template <int W, int NP, int NWIN, int WIN>
int launch(const DevMech &M, int64_t n, double *y, int64_t ld, const double *p, const double *t_end, double *t,
           double *h, const IntOpts &o, unsigned *queue, int32_t *status, int32_t *nacc, int32_t *nrej,
           hipStream_t s) {
    constexpr bool PARK = W > 1;
    return launch_kernel<W, Ros4Coop<W, NP, NWIN, WIN, PARK>, WIN, PARK>(M, n, y, ld, p, t_end, t, h, o, queue,
                                                                         status, nacc, nrej, s);
}

template <int NP>
int launch_half(const DevMech &M, int64_t n, double *y, int64_t ld, const double *p, const double *t_end, double *t,
                double *h, const IntOpts &o, unsigned *queue, int32_t *status, int32_t *nacc, int32_t *nrej,
                hipStream_t s) {
    return launch_kernel<4, Ros4CoopHalf<NP>, NP / 2, true>(M, n, y, ld, p, t_end, t, h, o, queue, status, nacc,
                                                            nrej, s);
}

template <int NP>
int launch_tile(const DevMech &M, int64_t n, double *y, int64_t ld, const double *p, const double *t_end, double *t,
                double *h, const IntOpts &o, unsigned *queue, int32_t *status, int32_t *nacc, int32_t *nrej,
                hipStream_t s) {
    return launch_kernel<4, Ros4CoopTile<NP>, NP / 2, true, 2>(M, n, y, ld, p, t_end, t, h, o, queue, status, nacc,
                                                               nrej, s);
}

template <int NP>
int launch_tile32(const DevMech &M, int64_t n, double *y, int64_t ld, const double *p, const double *t_end,
                  double *t, double *h, const IntOpts &o, unsigned *queue, int32_t *status, int32_t *nacc,
                  int32_t *nrej, hipStream_t s) {
    return launch_kernel<4, Ros4CoopTile32<NP>, NP / 2, true, 2>(M, n, y, ld, p, t_end, t, h, o, queue, status,
                                                                 nacc, nrej, s);
}

}  // namespace coop

bool coop_supported(const DevMech &M) { return M.N <= 128; }
bool tile_supported(const DevMech &M) { return M.N > 64 && M.N <= 128; }

int launch_integrate_tile(const DevMech &M, int64_t n, double *y, int64_t ld, const double *p, const double *t_end,
                          double *t, double *h, const IntOpts &o, void *ws, int32_t *status, int32_t *nacc,
                          int32_t *nrej, hipStream_t s) {
    unsigned *q = static_cast<unsigned *>(ws);
    if (o.precision == CK_PREC_FP32_REFINE) {
        switch (((M.N + 15) / 16) * 16) {
#define CK_TILE32(NPV) \
    case NPV: return coop::launch_tile32<NPV>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
            CK_TILE32(80) CK_TILE32(96) CK_TILE32(112) CK_TILE32(128)
#undef CK_TILE32
            default: return CK_EUNSUPPORTED;
        }
    }
    switch (((M.N + 15) / 16) * 16) {
#define CK_TILE(NPV) \
    case NPV: return coop::launch_tile<NPV>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
        CK_TILE(80) CK_TILE(96) CK_TILE(112) CK_TILE(128)
#undef CK_TILE
        default: return CK_EUNSUPPORTED;
    }
}

namespace coop {
template <int NP>
int launch_jac_group(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *jac,
                     hipStream_t s) {
    const size_t lds = lds_doubles(M.nsp, NP / 2, true) * sizeof(double);
    auto kern = jac_group_kernel<NP>;
    if (lds > 64 * 1024 && hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) != hipSuccess)
        return CK_EHIP;
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CK_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return CK_EHIP;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, 256, lds) != hipSuccess || per < 1) return CK_EHIP;
    int64_t grid = int64_t(cus) * per;
    if (grid > n) grid = n;
    kern<<<dim3(unsigned(grid)), dim3(256), lds, s>>>(M, n, y, ld, p, jac);
    return hipGetLastError() == hipSuccess ? CK_OK : CK_EHIP;
}
}  // namespace coop

int launch_jac_coop(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *jac,
                    hipStream_t s) {
    switch (((M.N + 7) / 8) * 8) {
#define CK_JG(NPV) \
    case NPV: return coop::launch_jac_group<NPV>(M, n, y, ld, p, jac, s);
        CK_JG(72) CK_JG(80) CK_JG(88) CK_JG(96) CK_JG(104) CK_JG(112) CK_JG(120) CK_JG(128)
#undef CK_JG
        default: return CK_EUNSUPPORTED;
    }
}

size_t coop_ws_bytes(const DevMech &M, int cus) {
    if (M.N <= 64) return 256;
    // park slice per resident workgroup: (NP / 2) x 256 doubles, NP rounded up to 16 (the tile
    // form's padding; at least the half-row form's, rounded up to 8)
    const size_t np = size_t((M.N + 15) / 16) * 16;
    return 256 + size_t(cus) * coop::kParkBlocksPerCu * np * 128 * sizeof(double);
}

int launch_integrate_coop(const DevMech &M, int64_t n, double *y, int64_t ld, const double *p, const double *t_end,
                          double *t, double *h, const IntOpts &o, void *ws, int32_t *status, int32_t *nacc,
                          int32_t *nrej, hipStream_t s) {
    unsigned *q = static_cast<unsigned *>(ws);
    const int np = ((M.N + 7) / 8) * 8;
#define CK_COOP1(NPV) \
    case NPV: return coop::launch<1, NPV, 1, NPV>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
#define CK_COOP2(NPV) \
    case NPV: return coop::launch_half<NPV>(M, n, y, ld, p, t_end, t, h, o, q, status, nacc, nrej, s);
    switch (np) {
        CK_COOP1(8) CK_COOP1(16) CK_COOP1(24) CK_COOP1(32) CK_COOP1(40) CK_COOP1(48) CK_COOP1(56) CK_COOP1(64)
        CK_COOP2(72) CK_COOP2(80) CK_COOP2(88) CK_COOP2(96) CK_COOP2(104) CK_COOP2(112) CK_COOP2(120)
        CK_COOP2(128)
        default: return CK_EUNSUPPORTED;
    }
#undef CK_COOP1
#undef CK_COOP2
}

}  // namespace ck
