/*
 * ck_oracle.c -- plain FP64 CPU oracle for batched constant-pressure chemical
 * kinetics integration (Stone, Alferman & Niemeyer, "Accelerating finite-rate
 * chemical kinetics with coprocessors", arXiv 1608.05794).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness authority that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it; the product path never does.  It
 * shares no code with the GPU library: it has its own mechanism parser, its
 * own rate, Jacobian, LU and integrator code, written plainly and slowly.
 *
 * What it computes, by paper section:
 *   - Section 3 (Eqs. ydot, tdot, wdot, kfor, krev, kc, tfits): the source
 *     term f(y) for y = (T, Y_1..Y_n) at constant pressure.  Readings:
 *       * Eq. tdot carries the density: dT/dt = -sum_k H_k wdot_k / (rho cp),
 *         H_k molar enthalpy, cp mass-specific (the equation as printed drops
 *         rho; Eq. ydot's units require it);
 *       * Eq. tfits is garbled; the standard NASA seven-term forms of the
 *         cited database are used: cp/R = a1+a2T+a3T^2+a4T^3+a5T^4,
 *         H/(RT) = a1+a2T/2+a3T^2/3+a4T^3/4+a5T^4/5+a6/T,
 *         S/R = a1 lnT+a2T+a3T^2/2+a4T^3/3+a5T^4/4+a7; low range if T < Tmid;
 *       * the third-body/fall-off factor c_i, which the paper defers to a
 *         cited reference, takes the standard forms: [M] = sum_k alpha_ik C_k;
 *         fall-off k = k_inf * Pr/(1+Pr) * F with Pr = k0 [M] / k_inf,
 *         F = 1 (Lindemann) or the Troe broadening function;
 *       * the exponent of (p0/RT) in Eq. kc is the net mole change of the
 *         reaction, sum_j (nu''_j - nu'_j).
 *   - The analytic Jacobian J = df/dy (the paper uses forward differences and
 *     points to analytic forms as the better choice in its conclusions): the
 *     plain chain-rule derivative of the source term above.
 *   - Section 2 and Appendix C: the transformed four-stage Rosenbrock scheme
 *     (ROS4) with the tabulated a, c, m (printed as b) and E; gamma = 0.57282
 *     as in the table.  Stage 4 has a4j = a3j and a43 = 0, so its right-hand
 *     side equals stage 3's and is reused.
 *   - Section 2 and Appendix B: the Runge--Kutta--Fehlberg 4(5) pair; the
 *     fourth-order weights b propagate, the error estimate is
 *     sum (bhat_j - b_j) k_j.
 *   - Section 4, Algorithm 1: the per-reactor driver (EstimateH0, OneStep,
 *     accept if err < MaxError = 1, AdjustStepSize), loop while t < t_f.
 *     EstimateH0 and AdjustStepSize are not given in the paper; the choices
 *     (Hairer--Norsett--Wanner starting step, safety 0.9, factor bounds
 *     [0.2, 5]; (t, h, y) is the whole controller state) are a fixed specification
 *     shared with the GPU library.  Closed forms pin the starting step (its
 *     fallback for a zero right-hand side and its main branch on a stiff
 *     scalar problem), the factor bounds (5 on acceptance, 0.2 on rejection),
 *     the factor between them (exponent 1/q from a problem whose estimate is
 *     exactly C h^q; the safety factor 0.9 from the pair's error polynomial),
 *     clipping and termination.
 *   - Section 5.2: one reactor per OpenMP task, schedule(dynamic,1).
 *
 * Units: SI throughout (K, Pa, kg/mol, mol/m^3, J/mol, s).
 * Layouts: states are array-of-structures, y[r*N + i], N = n_species + 1,
 * i = 0 is T.  Jacobians are row-major per reactor: J[r*N*N + i*N + j] =
 * df_i/dy_j.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXSIDE 3

typedef struct {
    int type;                     /* 0 elementary, 1 third-body, 2 Lindemann, 3 Troe */
    int rev;
    int nr, np;
    int rsp[ORC_MAXSIDE], rnu[ORC_MAXSIDE];
    int psp[ORC_MAXSIDE], pnu[ORC_MAXSIDE];
    double A, beta, Ea;           /* high-pressure (or only) Arrhenius, SI */
    double A0, beta0, Ea0;        /* low-pressure Arrhenius for fall-off */
    double troe_a, troe_T3, troe_T1, troe_T2;
    double *alpha;                /* dense third-body efficiencies [n_species] or NULL */
} orc_rxn;

typedef struct {
    int nsp, nrxn, nel;
    double R, p0;
    double *W;                    /* [nsp] kg/mol */
    double *Tmid;                 /* [nsp] */
    double *alow, *ahigh;         /* [nsp*7] */
    int *comp;                    /* [nsp*nel] element counts */
    orc_rxn *rx;
} orc_mech;

/* ------------------------------------------------------------------------- */
/* mechanism file                                                            */
/* ------------------------------------------------------------------------- */
static int expect_word(FILE *f, const char *w)
{
    char buf[64];
    if (fscanf(f, "%63s", buf) != 1) return -1;
    return strcmp(buf, w) == 0 ? 0 : -1;
}

void orc_free(orc_mech *m)
{
    if (!m) return;
    if (m->rx)
        for (int i = 0; i < m->nrxn; i++) free(m->rx[i].alpha);
    free(m->rx); free(m->W); free(m->Tmid); free(m->alow); free(m->ahigh); free(m->comp);
    free(m);
}

int orc_load(const char *path, orc_mech **out)
{
    *out = NULL;
    FILE *f = fopen(path, "r");
    if (!f) return -2;
    orc_mech *m = calloc(1, sizeof(orc_mech));
    int ver = 0;
    char name[128];
    if (expect_word(f, "CKMECH") || fscanf(f, "%d", &ver) != 1 || ver != 1) goto bad;
    if (expect_word(f, "CONST") || fscanf(f, "%lf %lf", &m->R, &m->p0) != 2) goto bad;
    if (expect_word(f, "ELEMENTS") || fscanf(f, "%d", &m->nel) != 1 || m->nel < 1) goto bad;
    for (int e = 0; e < m->nel; e++) {
        double w;
        if (expect_word(f, "E") || fscanf(f, "%127s %lf", name, &w) != 2) goto bad;
    }
    if (expect_word(f, "SPECIES") || fscanf(f, "%d", &m->nsp) != 1 || m->nsp < 1) goto bad;
    m->W = calloc(m->nsp, sizeof(double));
    m->Tmid = calloc(m->nsp, sizeof(double));
    m->alow = calloc(7 * m->nsp, sizeof(double));
    m->ahigh = calloc(7 * m->nsp, sizeof(double));
    m->comp = calloc((size_t)m->nsp * m->nel, sizeof(int));
    for (int k = 0; k < m->nsp; k++) {
        int nc;
        double tl, th;
        if (expect_word(f, "S") || fscanf(f, "%127s %lf %d", name, &m->W[k], &nc) != 3) goto bad;
        for (int c = 0; c < nc; c++) {
            int e, cnt;
            if (fscanf(f, "%d %d", &e, &cnt) != 2 || e < 0 || e >= m->nel) goto bad;
            m->comp[k * m->nel + e] = cnt;
        }
        if (fscanf(f, "%lf %lf %lf", &tl, &m->Tmid[k], &th) != 3) goto bad;
        for (int j = 0; j < 7; j++)
            if (fscanf(f, "%lf", &m->alow[7 * k + j]) != 1) goto bad;
        for (int j = 0; j < 7; j++)
            if (fscanf(f, "%lf", &m->ahigh[7 * k + j]) != 1) goto bad;
    }
    if (expect_word(f, "REACTIONS") || fscanf(f, "%d", &m->nrxn) != 1 || m->nrxn < 0) goto bad;
    m->rx = calloc(m->nrxn > 0 ? m->nrxn : 1, sizeof(orc_rxn));
    for (int i = 0; i < m->nrxn; i++) {
        orc_rxn *r = &m->rx[i];
        if (expect_word(f, "R") || fscanf(f, "%d %d %d", &r->type, &r->rev, &r->nr) != 3) goto bad;
        if (r->type < 0 || r->type > 3 || r->nr < 1 || r->nr > ORC_MAXSIDE) goto bad;
        for (int j = 0; j < r->nr; j++)
            if (fscanf(f, "%d %d", &r->rsp[j], &r->rnu[j]) != 2 || r->rsp[j] < 0 || r->rsp[j] >= m->nsp) goto bad;
        if (fscanf(f, "%d", &r->np) != 1 || r->np < 1 || r->np > ORC_MAXSIDE) goto bad;
        for (int j = 0; j < r->np; j++)
            if (fscanf(f, "%d %d", &r->psp[j], &r->pnu[j]) != 2 || r->psp[j] < 0 || r->psp[j] >= m->nsp) goto bad;
        if (fscanf(f, "%lf %lf %lf", &r->A, &r->beta, &r->Ea) != 3) goto bad;
        if (r->type >= 2 && fscanf(f, "%lf %lf %lf", &r->A0, &r->beta0, &r->Ea0) != 3) goto bad;
        if (r->type == 3 && fscanf(f, "%lf %lf %lf %lf", &r->troe_a, &r->troe_T3, &r->troe_T1, &r->troe_T2) != 4) goto bad;
        if (r->type >= 1) {
            int ne;
            if (fscanf(f, "%d", &ne) != 1 || ne < 0) goto bad;
            r->alpha = malloc(sizeof(double) * m->nsp);
            for (int k = 0; k < m->nsp; k++) r->alpha[k] = 1.0;
            for (int j = 0; j < ne; j++) {
                int s;
                double a;
                if (fscanf(f, "%d %lf", &s, &a) != 2 || s < 0 || s >= m->nsp) goto bad;
                r->alpha[s] = a;
            }
        }
    }
    if (expect_word(f, "END")) goto bad;
    fclose(f);
    *out = m;
    return 0;
bad:
    fclose(f);
    orc_free(m);
    return -3;
}

int orc_info(const orc_mech *m, int *nsp, int *nrxn, int *nel)
{
    *nsp = m->nsp; *nrxn = m->nrxn; *nel = m->nel;
    return 0;
}

void orc_species_data(const orc_mech *m, double *W, int *comp)
{
    memcpy(W, m->W, sizeof(double) * m->nsp);
    memcpy(comp, m->comp, sizeof(int) * m->nsp * m->nel);
}

/* ------------------------------------------------------------------------- */
/* thermodynamics, Eq. tfits (standard NASA-7 reading)                        */
/* ------------------------------------------------------------------------- */
static const double *nasa_coeffs(const orc_mech *m, int k, double T)
{
    return (T < m->Tmid[k]) ? &m->alow[7 * k] : &m->ahigh[7 * k];
}

/* cp/R, H/(RT), S/R and d(cp/R)/dT of species k at T */
static void species_thermo(const orc_mech *m, int k, double T,
                           double *cp, double *h, double *s, double *dcp)
{
    const double *a = nasa_coeffs(m, k, T);
    double T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    *cp = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
    *h = a[0] + a[1] * T / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 + a[4] * T4 / 5.0 + a[5] / T;
    *s = a[0] * log(T) + a[1] * T + a[2] * T2 / 2.0 + a[3] * T3 / 3.0 + a[4] * T4 / 4.0 + a[6];
    *dcp = a[1] + 2.0 * a[2] * T + 3.0 * a[3] * T2 + 4.0 * a[4] * T3;
}

void orc_thermo(const orc_mech *m, double T, double *cp_R, double *h_RT, double *s_R)
{
    for (int k = 0; k < m->nsp; k++) {
        double d;
        species_thermo(m, k, T, &cp_R[k], &h_RT[k], &s_R[k], &d);
    }
}

/* ------------------------------------------------------------------------- */
/* reaction rates, Eqs. wdot, kfor, krev, kc                                  */
/* ------------------------------------------------------------------------- */
static double ipow(double x, int n)
{
    double p = 1.0;
    for (int i = 0; i < n; i++) p *= x;
    return p;
}

/* Everything the source term and its Jacobian need about one state. */
typedef struct {
    double T, P, rho, Wbar, cp_mass;
    double *C, *cpR, *hRT, *sR, *dcpR;
    double *wdot;
} orc_state;

/* Per-reaction quantities at (T, C). */
typedef struct {
    double kf, kr;            /* rate constants multiplying the mass-action products (k_inf for fall-off) */
    double c;                 /* third-body / fall-off factor c_i */
    double pf, pr;            /* prod C^nu', prod C^nu'' */
    double dlnkf_dT, dlnkr_dT;
    double dc_dM;             /* d c_i / d [M] at fixed T */
    double dc_dT;             /* d c_i / d T at fixed C */
} orc_rate;

static double arrhenius(double A, double beta, double Ea, double R, double T)
{
    return A * pow(T, beta) * exp(-Ea / (R * T));
}

static void reaction_rate(const orc_mech *m, const orc_rxn *r, const orc_state *st, orc_rate *q)
{
    const double T = st->T, R = m->R;
    double kf = arrhenius(r->A, r->beta, r->Ea, R, T);
    q->dlnkf_dT = (r->beta + r->Ea / (R * T)) / T;
    if (r->rev) {
        /* ln Kc = sum_j nu_j (S_j/R - H_j/(RT)) + (sum_j nu_j) ln(p0/(R T)), nu = nu'' - nu' */
        double lnKc = 0.0, dnu = 0.0, dlnKc = 0.0;
        for (int j = 0; j < r->np; j++) {
            int s = r->psp[j];
            lnKc += r->pnu[j] * (st->sR[s] - st->hRT[s]);
            dlnKc += r->pnu[j] * st->hRT[s];
            dnu += r->pnu[j];
        }
        for (int j = 0; j < r->nr; j++) {
            int s = r->rsp[j];
            lnKc -= r->rnu[j] * (st->sR[s] - st->hRT[s]);
            dlnKc -= r->rnu[j] * st->hRT[s];
            dnu -= r->rnu[j];
        }
        lnKc += dnu * log(m->p0 / (R * T));
        double Kc = exp(lnKc);
        q->kr = kf / Kc;
        /* d lnKc/dT = (sum_j nu_j h_j - dnu) / T, since d(g_j)/dT = -h_j/T */
        q->dlnkr_dT = q->dlnkf_dT - (dlnKc - dnu) / T;
    } else {
        q->kr = 0.0;
        q->dlnkr_dT = 0.0;
    }
    q->kf = kf;
    q->pf = 1.0;
    for (int j = 0; j < r->nr; j++) q->pf *= ipow(st->C[r->rsp[j]], r->rnu[j]);
    q->pr = 1.0;
    for (int j = 0; j < r->np; j++) q->pr *= ipow(st->C[r->psp[j]], r->pnu[j]);

    q->c = 1.0; q->dc_dM = 0.0; q->dc_dT = 0.0;
    if (r->type == 0) return;
    double M = 0.0;
    for (int k = 0; k < m->nsp; k++) M += r->alpha[k] * st->C[k];
    if (r->type == 1) {
        q->c = M;
        q->dc_dM = 1.0;
        return;
    }
    /* fall-off: Pr = k0 [M] / k_inf, c = Pr/(1+Pr) F */
    double k0 = arrhenius(r->A0, r->beta0, r->Ea0, R, T);
    double ratio = k0 / kf;
    double Pr = ratio * M;
    double dlnPr_dT = (r->beta0 + r->Ea0 / (R * T)) / T - q->dlnkf_dT;
    double F = 1.0, g = 0.0, dlogF_dL = 0.0, dFcent = 0.0, Fcent = 1.0;
    if (r->type == 3) {
        double a = r->troe_a;
        Fcent = (1.0 - a) * exp(-T / r->troe_T3) + a * exp(-T / r->troe_T1) + exp(-r->troe_T2 / T);
        dFcent = -(1.0 - a) / r->troe_T3 * exp(-T / r->troe_T3) - a / r->troe_T1 * exp(-T / r->troe_T1)
                 + r->troe_T2 / (T * T) * exp(-r->troe_T2 / T);
        double L = log10(Fcent > 1e-300 ? Fcent : 1e-300);
        double cc = -0.4 - 0.67 * L;
        double nn = 0.75 - 1.27 * L;
        double x = log10(Pr > 1e-300 ? Pr : 1e-300) + cc;
        double d = nn - 0.14 * x;
        double f1 = x / d;
        double u = 1.0 + f1 * f1;
        double logF = L / u;
        F = pow(10.0, logF);
        /* g = d log10 F / d log10 Pr */
        g = L * (-2.0 * f1 / (u * u)) * (nn / (d * d));
        /* d log10 F / d L at fixed Pr */
        dlogF_dL = 1.0 / u - L * 2.0 * f1 / (u * u) * ((-0.67 * nn + 1.27 * x) / (d * d));
    }
    double onep = 1.0 + Pr;
    q->c = Pr / onep * F;
    /* dc/dPr = F/(1+Pr)^2 + F g/(1+Pr) */
    double dc_dPr = F / (onep * onep) + F * g / onep;
    q->dc_dM = dc_dPr * ratio;
    q->dc_dT = dc_dPr * Pr * dlnPr_dT;
    if (r->type == 3)
        q->dc_dT += Pr / onep * F * dlogF_dL * dFcent / Fcent;
}

/* Mixture state: rho, C, thermo, cp (Section 3, ideal gas closure). */
static void mixture_state(const orc_mech *m, const double *y, double P, orc_state *st)
{
    const int n = m->nsp;
    const double T = y[0];
    st->T = T;
    st->P = P;
    double S = 0.0;
    for (int k = 0; k < n; k++) S += y[1 + k] / m->W[k];
    st->Wbar = 1.0 / S;
    st->rho = P / (m->R * T * S);
    st->cp_mass = 0.0;
    for (int k = 0; k < n; k++) {
        st->C[k] = st->rho * y[1 + k] / m->W[k];
        species_thermo(m, k, T, &st->cpR[k], &st->hRT[k], &st->sR[k], &st->dcpR[k]);
        st->cp_mass += y[1 + k] * st->cpR[k] * m->R / m->W[k];
    }
}

typedef struct {
    double *buf;
    orc_state st;
    orc_rate *rates;
    double *dq;               /* [nsp] scratch for dq_i/dC */
} orc_work;

static void work_init(const orc_mech *m, orc_work *w)
{
    int n = m->nsp;
    w->buf = calloc(7 * (size_t)n, sizeof(double));
    w->st.C = w->buf;
    w->st.cpR = w->buf + n;
    w->st.hRT = w->buf + 2 * n;
    w->st.sR = w->buf + 3 * n;
    w->st.dcpR = w->buf + 4 * n;
    w->st.wdot = w->buf + 5 * n;
    w->dq = w->buf + 6 * n;
    w->rates = calloc(m->nrxn > 0 ? m->nrxn : 1, sizeof(orc_rate));
}

static void work_free(orc_work *w)
{
    free(w->buf);
    free(w->rates);
}

/* f(y): Eqs. ydot and tdot with wdot from Eq. wdot. */
static void source_term(const orc_mech *m, orc_work *w, const double *y, double P, double *f)
{
    const int n = m->nsp;
    orc_state *st = &w->st;
    mixture_state(m, y, P, st);
    for (int k = 0; k < n; k++) st->wdot[k] = 0.0;
    for (int i = 0; i < m->nrxn; i++) {
        const orc_rxn *r = &m->rx[i];
        orc_rate *q = &w->rates[i];
        reaction_rate(m, r, st, q);
        double qi = q->c * (q->kf * q->pf - q->kr * q->pr);
        for (int j = 0; j < r->nr; j++) st->wdot[r->rsp[j]] -= r->rnu[j] * qi;
        for (int j = 0; j < r->np; j++) st->wdot[r->psp[j]] += r->pnu[j] * qi;
    }
    double Q = 0.0;
    for (int k = 0; k < n; k++) {
        f[1 + k] = m->W[k] * st->wdot[k] / st->rho;
        Q += m->R * st->T * st->hRT[k] * st->wdot[k];
    }
    f[0] = -Q / (st->rho * st->cp_mass);
}

/* Net stoichiometric coefficient of species k in reaction r. */
static int net_nu(const orc_rxn *r, int k)
{
    int v = 0;
    for (int j = 0; j < r->nr; j++) if (r->rsp[j] == k) v -= r->rnu[j];
    for (int j = 0; j < r->np; j++) if (r->psp[j] == k) v += r->pnu[j];
    return v;
}

/* d(prod_j C_j^nu_j)/dC_l, as the product with one factor lowered (no division). */
static double dprod(const double *C, const int *sp, const int *nu, int ns, int l)
{
    int found = 0;
    double p = 1.0;
    for (int j = 0; j < ns; j++) {
        if (sp[j] == l) {
            found = 1;
            p *= nu[j] * ipow(C[l], nu[j] - 1);
        } else {
            p *= ipow(C[sp[j]], nu[j]);
        }
    }
    return found ? p : 0.0;
}

/* JC[k][l] = d wdot_k / d C_l at fixed T and dwT[k] = d wdot_k / dT at fixed C, from the
 * per-reaction quantities of the last source-term evaluation (w->rates, w->st). */
static void rate_derivatives(const orc_mech *m, orc_work *w, double *JC, double *dwT)
{
    const int n = m->nsp;
    orc_state *st = &w->st;
    for (int i = 0; i < m->nrxn; i++) {
        const orc_rxn *r = &m->rx[i];
        const orc_rate *q = &w->rates[i];
        double Rnet = q->kf * q->pf - q->kr * q->pr;
        /* dq_i/dC_l */
        for (int l = 0; l < n; l++) {
            double d = q->c * (q->kf * dprod(st->C, r->rsp, r->rnu, r->nr, l)
                               - q->kr * dprod(st->C, r->psp, r->pnu, r->np, l));
            if (r->type >= 1) d += Rnet * q->dc_dM * r->alpha[l];
            w->dq[l] = d;
        }
        double dqT = q->c * (q->kf * q->dlnkf_dT * q->pf - q->kr * q->dlnkr_dT * q->pr) + Rnet * q->dc_dT;
        for (int k = 0; k < n; k++) {
            int v = net_nu(r, k);
            if (v == 0) continue;
            for (int l = 0; l < n; l++) JC[k * n + l] += v * w->dq[l];
            dwT[k] += v * dqT;
        }
    }
}

/* Analytic Jacobian J = df/dy (row-major N x N) at y; also returns f. */
static void jacobian(const orc_mech *m, orc_work *w, const double *y, double P, double *J, double *f)
{
    const int n = m->nsp, N = n + 1;
    orc_state *st = &w->st;
    source_term(m, w, y, P, f);
    const double T = st->T, rho = st->rho, Wbar = st->Wbar, cp = st->cp_mass, R = m->R;
    double *JC = calloc((size_t)n * n, sizeof(double));
    double *dwT = calloc(n, sizeof(double));
    rate_derivatives(m, w, JC, dwT);
    /* chain rule through C(T, Y) and rho(T, Y) */
    double *JCC = calloc(n, sizeof(double));     /* sum_l JC[k][l] C_l */
    for (int k = 0; k < n; k++) {
        double s = 0.0;
        for (int l = 0; l < n; l++) s += JC[k * n + l] * st->C[l];
        JCC[k] = s;
    }
    /* species rows */
    for (int k = 0; k < n; k++) {
        double Wk = m->W[k];
        double resid = st->wdot[k] - JCC[k];
        for (int j = 0; j < n; j++)
            J[(1 + k) * N + 1 + j] = (Wk / m->W[j]) * JC[k * n + j] + Wk * Wbar / (rho * m->W[j]) * resid;
        J[(1 + k) * N + 0] = (Wk / rho) * (dwT[k] + resid / T);
    }
    /* temperature row: fT = -Q / D, Q = sum_k H_k wdot_k, D = rho cp */
    double D = rho * cp;
    double fT = f[0];
    for (int j = 0; j < n; j++) {
        double dQ = 0.0;
        for (int k = 0; k < n; k++) {
            double dw = JC[k * n + j] * rho / m->W[j] - (Wbar / m->W[j]) * JCC[k];
            dQ += R * T * st->hRT[k] * dw;
        }
        double dD = -cp * rho * Wbar / m->W[j] + rho * st->cpR[j] * R / m->W[j];
        J[0 * N + 1 + j] = -(dQ + fT * dD) / D;
    }
    {
        double dQ = 0.0, sdcp = 0.0;
        for (int k = 0; k < n; k++) {
            dQ += R * st->cpR[k] * st->wdot[k] + R * T * st->hRT[k] * (dwT[k] - JCC[k] / T);
            sdcp += y[1 + k] * R * st->dcpR[k] / m->W[k];
        }
        double dD = -rho * cp / T + rho * sdcp;
        J[0] = -(dQ + fT * dD) / D;
    }
    free(JC); free(dwT); free(JCC);
}

/* Constant-volume reactor (Section 3: the constant-volume form uses c_v and the internal energies
 * in place of c_p and the enthalpies).  State (T, Y); the density rho is fixed and the pressure
 * follows from the ideal gas:
 *   C_k = rho Y_k / W_k,  f_Yk = W_k wdot_k / rho,
 *   f_T = -sum_k U_k wdot_k / (rho c_v),  U_k = H_k - R T,  c_v = sum_k Y_k (cp_k - R) / W_k. */
static void mixture_state_cv(const orc_mech *m, const double *y, double rho, orc_state *st)
{
    const int n = m->nsp;
    const double T = y[0];
    double S = 0.0;
    for (int k = 0; k < n; k++) S += y[1 + k] / m->W[k];
    st->T = T;
    st->rho = rho;
    st->Wbar = 1.0 / S;
    st->P = rho * m->R * T * S;
    st->cp_mass = 0.0;   /* holds c_v in this form */
    for (int k = 0; k < n; k++) {
        st->C[k] = rho * y[1 + k] / m->W[k];
        species_thermo(m, k, T, &st->cpR[k], &st->hRT[k], &st->sR[k], &st->dcpR[k]);
        st->cp_mass += y[1 + k] * (st->cpR[k] - 1.0) * m->R / m->W[k];
    }
}

static void source_term_cv(const orc_mech *m, orc_work *w, const double *y, double rho, double *f)
{
    const int n = m->nsp;
    orc_state *st = &w->st;
    mixture_state_cv(m, y, rho, st);
    for (int k = 0; k < n; k++) st->wdot[k] = 0.0;
    for (int i = 0; i < m->nrxn; i++) {
        const orc_rxn *r = &m->rx[i];
        orc_rate *q = &w->rates[i];
        reaction_rate(m, r, st, q);
        double qi = q->c * (q->kf * q->pf - q->kr * q->pr);
        for (int j = 0; j < r->nr; j++) st->wdot[r->rsp[j]] -= r->rnu[j] * qi;
        for (int j = 0; j < r->np; j++) st->wdot[r->psp[j]] += r->pnu[j] * qi;
    }
    double Q = 0.0;
    for (int k = 0; k < n; k++) {
        f[1 + k] = m->W[k] * st->wdot[k] / rho;
        Q += m->R * st->T * (st->hRT[k] - 1.0) * st->wdot[k];
    }
    f[0] = -Q / (rho * st->cp_mass);
}

/* Analytic Jacobian of the constant-volume form.  With rho fixed, C depends on Y only:
 *   dC_k/dY_j = delta_kj rho / W_k,  dC/dT = 0,
 *   df_Yk/dY_j = (W_k / W_j) JC[k][j],  df_Yk/dT = (W_k / rho) dwT[k],
 *   df_T/dY_j = -[(rho / W_j) sum_k U_k JC[k][j] + f_T rho R (cp_j/R - 1) / W_j] / (rho c_v),
 *   df_T/dT   = -[sum_k R (cp_k/R - 1) wdot_k + sum_k U_k dwT[k] + f_T rho sum_k Y_k R dcp_k/W_k] / (rho c_v). */
static void jacobian_cv(const orc_mech *m, orc_work *w, const double *y, double rho, double *J, double *f)
{
    const int n = m->nsp, N = n + 1;
    orc_state *st = &w->st;
    source_term_cv(m, w, y, rho, f);
    const double T = st->T, cv = st->cp_mass, R = m->R;
    double *JC = calloc((size_t)n * n, sizeof(double));
    double *dwT = calloc(n, sizeof(double));
    rate_derivatives(m, w, JC, dwT);
    for (int k = 0; k < n; k++) {
        for (int j = 0; j < n; j++) J[(1 + k) * N + 1 + j] = (m->W[k] / m->W[j]) * JC[k * n + j];
        J[(1 + k) * N + 0] = (m->W[k] / rho) * dwT[k];
    }
    const double D = rho * cv, fT = f[0];
    for (int j = 0; j < n; j++) {
        double s = 0.0;
        for (int k = 0; k < n; k++) s += R * T * (st->hRT[k] - 1.0) * JC[k * n + j];
        const double dQ = (rho / m->W[j]) * s;
        const double dD = rho * R * (st->cpR[j] - 1.0) / m->W[j];
        J[0 * N + 1 + j] = -(dQ + fT * dD) / D;
    }
    {
        double dQ = 0.0, sdcp = 0.0;
        for (int k = 0; k < n; k++) {
            dQ += R * (st->cpR[k] - 1.0) * st->wdot[k] + R * T * (st->hRT[k] - 1.0) * dwT[k];
            sdcp += y[1 + k] * R * st->dcpR[k] / m->W[k];
        }
        J[0] = -(dQ + fT * rho * sdcp) / D;
    }
    free(JC); free(dwT);
}

/* ------------------------------------------------------------------------- */
/* problems: chemistry or a dense linear test system y' = A y                */
/* ------------------------------------------------------------------------- */
typedef struct {
    int N;
    const orc_mech *m;        /* chemistry if non-NULL */
    double P;
    orc_work *w;
    const double *A;          /* linear system if m == NULL */
    long nfev, njev;
    int jac_fd;               /* ROS4 Jacobian: 0 analytic, 1 forward differences */
    double rtol, atol;        /* error weights of the difference increments */
    int cv;                   /* chemistry: 0 constant pressure (P = pressure), 1 constant volume (P = density) */
} orc_problem;

static void prob_f(orc_problem *p, const double *y, double *f)
{
    p->nfev++;
    if (p->m) {
        if (p->cv)
            source_term_cv(p->m, p->w, y, p->P, f);
        else
            source_term(p->m, p->w, y, p->P, f);
        return;
    }
    for (int i = 0; i < p->N; i++) {
        double s = 0.0;
        for (int j = 0; j < p->N; j++) s += p->A[i * p->N + j] * y[j];
        f[i] = s;
    }
}

static void prob_jac(orc_problem *p, const double *y, double *J)
{
    p->njev++;
    if (p->m) {
        double *f = malloc(sizeof(double) * p->N);
        if (p->cv)
            jacobian_cv(p->m, p->w, y, p->P, J, f);
        else
            jacobian(p->m, p->w, y, p->P, J, f);
        free(f);
        return;
    }
    memcpy(J, p->A, sizeof(double) * p->N * p->N);
}

/* Forward-difference Jacobian, one extra source-term evaluation per column (the
 * paper's ROS4 set-up, Section 5: first-order forward differences as in
 * CVODE's dense difference-quotient Jacobian).  Increment of column j:
 *   inc_j = max(sqrt(eps) |y_j|, min_inc / w_j),  w_j = 1 / (rtol |y_j| + atol),
 *   min_inc = 1000 |h| eps N ||f(y)||_w  (1 if that norm is 0),
 * ||.||_w the weighted RMS norm with the weights w; J_ij = (f_i(y + inc_j e_j) - f_i(y)) / inc_j. */
static void jacobian_fd(orc_problem *p, const double *y, double h, double *J)
{
    const int N = p->N;
    const double eps = 2.220446049250313e-16;
    double *f0 = malloc(sizeof(double) * N), *f1 = malloc(sizeof(double) * N);
    double *yp = malloc(sizeof(double) * N);
    p->njev++;
    prob_f(p, y, f0);
    double s = 0.0;
    for (int i = 0; i < N; i++) {
        double r = f0[i] / (p->rtol * fabs(y[i]) + p->atol);
        s += r * r;
    }
    const double fnorm = sqrt(s / N);
    const double min_inc = (fnorm != 0.0) ? 1000.0 * fabs(h) * eps * N * fnorm : 1.0;
    memcpy(yp, y, sizeof(double) * N);
    for (int j = 0; j < N; j++) {
        const double wj = 1.0 / (p->rtol * fabs(y[j]) + p->atol);
        const double inc = fmax(sqrt(eps) * fabs(y[j]), min_inc / wj);
        yp[j] = y[j] + inc;
        prob_f(p, yp, f1);
        for (int i = 0; i < N; i++) J[i * N + j] = (f1[i] - f0[i]) / inc;
        yp[j] = y[j];
    }
    free(f0); free(f1); free(yp);
}

/* ------------------------------------------------------------------------- */
/* dense LU with partial pivoting (first index of the largest |a_ik|)         */
/* ------------------------------------------------------------------------- */
static int lu_factor(int N, double *a, int *piv)
{
    for (int k = 0; k < N; k++) {
        int p = k;
        double best = fabs(a[k * N + k]);
        for (int i = k + 1; i < N; i++)
            if (fabs(a[i * N + k]) > best) { best = fabs(a[i * N + k]); p = i; }
        piv[k] = p;
        if (best == 0.0) return k + 1;
        if (p != k)
            for (int j = 0; j < N; j++) { double t = a[k * N + j]; a[k * N + j] = a[p * N + j]; a[p * N + j] = t; }
        for (int i = k + 1; i < N; i++) {
            double l = a[i * N + k] / a[k * N + k];
            a[i * N + k] = l;
            for (int j = k + 1; j < N; j++) a[i * N + j] -= l * a[k * N + j];
        }
    }
    return 0;
}

static void lu_solve(int N, const double *a, const int *piv, double *b)
{
    for (int k = 0; k < N; k++)
        if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int i = 0; i < N; i++) {
        double s = b[i];
        for (int j = 0; j < i; j++) s -= a[i * N + j] * b[j];
        b[i] = s;
    }
    for (int i = N - 1; i >= 0; i--) {
        double s = b[i];
        for (int j = i + 1; j < N; j++) s -= a[i * N + j] * b[j];
        b[i] = s / a[i * N + i];
    }
}

/* exported for tests: factor + solve one system (row-major a, overwritten) */
int orc_lu_solve(int N, double *a, double *b)
{
    int *piv = malloc(sizeof(int) * N);
    int info = lu_factor(N, a, piv);
    if (!info) lu_solve(N, a, piv, b);
    free(piv);
    return info;
}

/* ------------------------------------------------------------------------- */
/* one-step methods                                                           */
/* ------------------------------------------------------------------------- */
/* Appendix C (ROS4, Hairer & Wanner); gamma as tabulated. */
static const double ROS_GAMMA = 0.57282;
static const double ROS_A[4][3] = {
    {0.0, 0.0, 0.0},
    {2.0, 0.0, 0.0},
    {1.867943637803922, 0.2344449711399156, 0.0},
    {1.867943637803922, 0.2344449711399156, 0.0},
};
static const double ROS_C[4][3] = {
    {0.0, 0.0, 0.0},
    {-7.137615036412310, 0.0, 0.0},
    {2.580708087951457, 0.6515950076447975, 0.0},
    {-2.137148994382534, -0.3214669691237626, -0.6949742501781779},
};
static const double ROS_M[4] = {2.255570073418735, 0.2870493262186792, 0.4353179431840180, 1.093502252409163};
static const double ROS_E[4] = {-0.2815431932141155, -0.07276199124938920, -0.1082196201495311, -1.093502252409163};

/* Appendix B (Runge--Kutta--Fehlberg). */
static const double RKF_A[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0 / 4.0, 0, 0, 0, 0},
    {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0},
};
static const double RKF_B[6] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0, -1.0 / 5.0, 0.0};
static const double RKF_BH[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0, 2.0 / 55.0};

typedef struct {
    double *ytmp, *f, *u, *M, *e;   /* u: 6*N stage storage; M: N*N */
    int *piv;
} step_work;

/* ROS4 step (Section 2, transformed Rosenbrock; Appendix C).  Returns 0, or
 * the LU breakdown column + 1 (then the step counts as rejected). */
static int ros4_step(orc_problem *p, step_work *sw, const double *y, double h, double *ynew, double *err_vec)
{
    const int N = p->N;
    double *u = sw->u, *M = sw->M, *ytmp = sw->ytmp, *f = sw->f;
    if (p->jac_fd)
        jacobian_fd(p, y, h, M);
    else
        prob_jac(p, y, M);
    for (int i = 0; i < N * N; i++) M[i] = -M[i];
    for (int i = 0; i < N; i++) M[i * N + i] += 1.0 / (ROS_GAMMA * h);
    int info = lu_factor(N, M, sw->piv);
    if (info) return info;
    for (int s = 0; s < 4; s++) {
        double *us = u + s * N;
        if (s < 3) {   /* stage 4's argument equals stage 3's (a4j = a3j, a43 = 0) */
            for (int i = 0; i < N; i++) {
                double v = y[i];
                for (int j = 0; j < s; j++) v += ROS_A[s][j] * u[j * N + i];
                ytmp[i] = v;
            }
            prob_f(p, ytmp, f);
        }
        for (int i = 0; i < N; i++) {
            double v = 0.0;
            for (int j = 0; j < s; j++) v += ROS_C[s][j] * u[j * N + i];
            us[i] = f[i] + v / h;
        }
        lu_solve(N, M, sw->piv, us);
    }
    for (int i = 0; i < N; i++) {
        double v = y[i], e = 0.0;
        for (int s = 0; s < 4; s++) {
            v += ROS_M[s] * u[s * N + i];
            e += ROS_E[s] * u[s * N + i];
        }
        ynew[i] = v;
        err_vec[i] = e;
    }
    return 0;
}

/* RKF45 step (Section 2; Appendix B): k_i = h f(y + sum_j a_ij k_j). */
static int rkf45_step(orc_problem *p, step_work *sw, const double *y, double h, double *ynew, double *err_vec)
{
    const int N = p->N;
    double *k = sw->u, *ytmp = sw->ytmp;
    for (int s = 0; s < 6; s++) {
        for (int i = 0; i < N; i++) {
            double v = y[i];
            for (int j = 0; j < s; j++) v += RKF_A[s][j] * k[j * N + i];
            ytmp[i] = v;
        }
        prob_f(p, ytmp, k + s * N);
        for (int i = 0; i < N; i++) k[s * N + i] *= h;
    }
    for (int i = 0; i < N; i++) {
        double v = y[i], e = 0.0;
        for (int s = 0; s < 6; s++) {
            v += RKF_B[s] * k[s * N + i];
            e += (RKF_BH[s] - RKF_B[s]) * k[s * N + i];
        }
        ynew[i] = v;
        err_vec[i] = e;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* driver (Algorithm 1)                                                       */
/* ------------------------------------------------------------------------- */
typedef struct {
    double rtol, atol;
    double h0;          /* > 0: initial step given */
    double h_fixed;     /* > 0: fixed-step mode, every step accepted */
    int64_t max_steps;  /* attempted steps */
    int32_t jac_fd;     /* ROS4 Jacobian: 0 analytic, 1 forward differences */
    int32_t cv;         /* 0 constant pressure, 1 constant volume (the P array then holds densities) */
} orc_opts;

enum { ST_OK = 0, ST_MAX_STEPS = 1, ST_H_UNDERFLOW = 2, ST_NONFINITE = 3 };

/* weighted RMS norm of e with weights atol + rtol * max(|a|,|b|) */
static double wrms(int N, const double *e, const double *a, const double *b, double rtol, double atol)
{
    double s = 0.0;
    for (int i = 0; i < N; i++) {
        double sc = atol + rtol * fmax(fabs(a[i]), fabs(b[i]));
        double r = e[i] / sc;
        s += r * r;
    }
    return sqrt(s / N);
}

static int all_finite(int N, const double *v)
{
    for (int i = 0; i < N; i++) if (!isfinite(v[i])) return 0;
    return 1;
}

/* EstimateH0 (Hairer, Norsett & Wanner, Solving ODEs I, II.4; order 4). */
static double estimate_h0(orc_problem *p, const double *y0, const double *f0, double span,
                          double rtol, double atol, double *ytmp, double *f1)
{
    const int N = p->N;
    double d0 = wrms(N, y0, y0, y0, rtol, atol);
    double d1 = wrms(N, f0, y0, y0, rtol, atol);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    if (h0 > span) h0 = span;
    for (int i = 0; i < N; i++) ytmp[i] = y0[i] + h0 * f0[i];
    prob_f(p, ytmp, f1);
    for (int i = 0; i < N; i++) ytmp[i] = f1[i] - f0[i];
    double d2 = wrms(N, ytmp, y0, y0, rtol, atol) / h0;
    double dm = fmax(d1, d2);
    double h1 = (dm <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, 1.0 / 5.0);
    double h = fmin(100.0 * h0, h1);
    return fmin(h, span);
}

/* Integrate one system from *t to t_end.  method 0 = ROS4, 1 = RKF45. */
static int integrate_one(orc_problem *p, int method, double *y, double *t_io, double *h_io, double t_end,
                         const orc_opts *o, int32_t *nacc, int32_t *nrej)
{
    const int N = p->N;
    const double q = (method == 0) ? 4.0 : 5.0;   /* error estimate is O(h^q) */
    p->jac_fd = o->jac_fd;
    p->cv = p->m ? o->cv : 0;
    p->rtol = o->rtol;
    p->atol = o->atol;
    step_work sw;
    sw.ytmp = malloc(sizeof(double) * N);
    sw.f = malloc(sizeof(double) * N);
    sw.u = malloc(sizeof(double) * 6 * N);
    sw.M = malloc(sizeof(double) * N * N);
    sw.e = malloc(sizeof(double) * N);
    sw.piv = malloc(sizeof(int) * N);
    double *ynew = malloc(sizeof(double) * N);
    double *f0 = malloc(sizeof(double) * N);
    int status = ST_OK;
    double t = t_io ? *t_io : 0.0;
    double h;
    *nacc = 0;
    *nrej = 0;

    if (!all_finite(N, y)) { status = ST_NONFINITE; h = 0.0; goto done; }
    if (o->h_fixed > 0.0) {
        h = o->h_fixed;
    } else if (h_io && *h_io > 0.0) {
        h = *h_io;
    } else if (o->h0 > 0.0) {
        h = o->h0;
    } else if (t < t_end) {
        prob_f(p, y, f0);
        if (!all_finite(N, f0)) { status = ST_NONFINITE; h = 0.0; goto done; }
        h = estimate_h0(p, y, f0, t_end - t, o->rtol, o->atol, sw.ytmp, sw.f);
    } else {
        h = 0.0;
    }

    while (t < t_end) {
        if ((int64_t)(*nacc) + (int64_t)(*nrej) >= o->max_steps) { status = ST_MAX_STEPS; break; }
        int clipped = (t + h >= t_end);
        double hs = clipped ? (t_end - t) : h;
        int info = (method == 0) ? ros4_step(p, &sw, y, hs, ynew, sw.e) : rkf45_step(p, &sw, y, hs, ynew, sw.e);
        double err;
        if (o->h_fixed > 0.0) {
            err = 0.0;
        } else if (info) {
            err = INFINITY;
        } else {
            err = wrms(N, sw.e, y, ynew, o->rtol, o->atol);
            if (!all_finite(N, ynew)) err = INFINITY;
        }
        double fac;
        if (err < 1.0) {
            memcpy(y, ynew, sizeof(double) * N);
            t = clipped ? t_end : t + hs;
            (*nacc)++;
            fac = (err == 0.0) ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(err, -1.0 / q)));
        } else {
            (*nrej)++;
            fac = isfinite(err) ? fmax(0.2, 0.9 * pow(err, -1.0 / q)) : 0.2;
        }
        if (o->h_fixed > 0.0) fac = 1.0;
        h = hs * fac;
        if (t < t_end && h < fmax(1e-30, 16.0 * 2.220446049250313e-16 * fabs(t))) { status = ST_H_UNDERFLOW; break; }
    }
done:
    if (t_io) *t_io = t;
    if (h_io) *h_io = h;
    free(sw.ytmp); free(sw.f); free(sw.u); free(sw.M); free(sw.e); free(sw.piv); free(ynew); free(f0);
    return status;
}

/* ------------------------------------------------------------------------- */
/* batch entry points (one reactor per OpenMP task, schedule(dynamic,1))      */
/* ------------------------------------------------------------------------- */
static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_rhs(const orc_mech *m, int64_t n, const double *y, const double *P, double *dydt, int nthreads)
{
    const int N = m->nsp + 1;
    set_threads(nthreads);
#pragma omp parallel
    {
        orc_work w;
        work_init(m, &w);
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < n; r++) source_term(m, &w, y + r * N, P[r], dydt + r * N);
        work_free(&w);
    }
}

/* Constant-volume source term and Jacobian (rho[r]: density of reactor r, kg/m^3). */
void orc_rhs_cv(const orc_mech *m, int64_t n, const double *y, const double *rho, double *dydt, int nthreads)
{
    const int N = m->nsp + 1;
    set_threads(nthreads);
#pragma omp parallel
    {
        orc_work w;
        work_init(m, &w);
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < n; r++) source_term_cv(m, &w, y + r * N, rho[r], dydt + r * N);
        work_free(&w);
    }
}

void orc_jac_cv(const orc_mech *m, int64_t n, const double *y, const double *rho, double *jac, int nthreads)
{
    const int N = m->nsp + 1;
    set_threads(nthreads);
#pragma omp parallel
    {
        orc_work w;
        work_init(m, &w);
        double *f = malloc(sizeof(double) * N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < n; r++) jacobian_cv(m, &w, y + r * N, rho[r], jac + r * (int64_t)N * N, f);
        free(f);
        work_free(&w);
    }
}

void orc_jac(const orc_mech *m, int64_t n, const double *y, const double *P, double *jac, int nthreads)
{
    const int N = m->nsp + 1;
    set_threads(nthreads);
#pragma omp parallel
    {
        orc_work w;
        work_init(m, &w);
        double *f = malloc(sizeof(double) * N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < n; r++) jacobian(m, &w, y + r * N, P[r], jac + r * (int64_t)N * N, f);
        free(f);
        work_free(&w);
    }
}

/* Forward and reverse gross rates of progress q_f = c kf prod C^nu', q_r = c kr prod C^nu''
 * (per reaction) and the thermo of one state; used by the tests' scaled error metric. */
/* Forward-difference Jacobian of each reactor (AoS, as orc_jac), increments for step h and
 * tolerances rtol / atol (see jacobian_fd). */
void orc_jac_fd(const orc_mech *m, int64_t n, const double *y, const double *P, double rtol, double atol,
                double h, double *jac, int nthreads)
{
    const int N = m->nsp + 1;
    set_threads(nthreads);
#pragma omp parallel
    {
        orc_work w;
        work_init(m, &w);
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < n; r++) {
            orc_problem p = {N, m, P[r], &w, NULL, 0, 0, 1, rtol, atol, 0};
            jacobian_fd(&p, y + r * N, h, jac + r * N * N);
        }
        work_free(&w);
    }
}

void orc_rates(const orc_mech *m, const double *y, double P, double *qf, double *qr, double *rho, double *cp_mass, double *h_RT)
{
    orc_work w;
    work_init(m, &w);
    double *f = malloc(sizeof(double) * (m->nsp + 1));
    source_term(m, &w, y, P, f);
    for (int i = 0; i < m->nrxn; i++) {
        qf[i] = w.rates[i].c * w.rates[i].kf * w.rates[i].pf;
        qr[i] = w.rates[i].c * w.rates[i].kr * w.rates[i].pr;
    }
    *rho = w.st.rho;
    *cp_mass = w.st.cp_mass;
    for (int k = 0; k < m->nsp; k++) h_RT[k] = w.st.hRT[k];
    free(f);
    work_free(&w);
}

void orc_stoich(const orc_mech *m, int *nu /* [nsp*nrxn] */)
{
    for (int k = 0; k < m->nsp; k++)
        for (int i = 0; i < m->nrxn; i++) nu[k * m->nrxn + i] = net_nu(&m->rx[i], k);
}

int orc_integrate(const orc_mech *m, int method, int64_t n, double *y, const double *P, const double *t_end,
                  double *t, double *h, const orc_opts *o, int32_t *status, int32_t *nacc, int32_t *nrej,
                  int nthreads)
{
    const int N = m->nsp + 1;
    set_threads(nthreads);
#pragma omp parallel
    {
        orc_work w;
        work_init(m, &w);
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < n; r++) {
            orc_problem p = {N, m, P[r], &w, NULL, 0, 0, 0, 0.0, 0.0, 0};
            status[r] = integrate_one(&p, method, y + r * N, t ? t + r : NULL, h ? h + r : NULL, t_end[r], o,
                                      nacc + r, nrej + r);
        }
        work_free(&w);
    }
    return 0;
}

/* Linear test problem y' = A y (dense, row-major N x N), J = A. */
int orc_integrate_linear(int method, int N, const double *A, double *y, double t_end, double *t, double *h,
                         const orc_opts *o, int32_t *status, int32_t *nacc, int32_t *nrej, long *nfev)
{
    orc_problem p = {N, NULL, 0.0, NULL, A, 0, 0, 0, 0.0, 0.0, 0};
    *status = integrate_one(&p, method, y, t, h, t_end, o, nacc, nrej);
    if (nfev) *nfev = p.nfev;
    return 0;
}

/* One step of either method on y' = A y from y (no control): returns y* and the error vector. */
int orc_step_linear(int method, int N, const double *A, const double *y, double h, double *ynew, double *err)
{
    orc_problem p = {N, NULL, 0.0, NULL, A, 0, 0, 0, 0.0, 0.0, 0};
    step_work sw;
    sw.ytmp = malloc(sizeof(double) * N);
    sw.f = malloc(sizeof(double) * N);
    sw.u = malloc(sizeof(double) * 6 * N);
    sw.M = malloc(sizeof(double) * N * N);
    sw.e = malloc(sizeof(double) * N);
    sw.piv = malloc(sizeof(int) * N);
    int info = (method == 0) ? ros4_step(&p, &sw, y, h, ynew, err) : rkf45_step(&p, &sw, y, h, ynew, err);
    free(sw.ytmp); free(sw.f); free(sw.u); free(sw.M); free(sw.e); free(sw.piv);
    return info;
}
