/*
 * ck.h -- C ABI of the MI355X (gfx950) batched chemical-kinetics library.
 *
 * The library integrates many independent constant-pressure homogeneous
 * reactors (Stone, Alferman & Niemeyer, arXiv 1608.05794).  Each reactor is
 * the autonomous ODE system du/dt = f(u) of Section 2 (Eq. ode) with state
 * u = (T, Y_1 .. Y_n), N = n + 1, and the source term of Section 3
 * (Eqs. ydot, tdot, wdot, kfor, krev, kc, tfits).
 *
 * Conventions for every call below
 *   - Units are SI: K, Pa, kg/mol, mol/m^3, J/mol, s.
 *   - States are structure-of-arrays float64: y[i * ld + r] is component i
 *     (i = 0 temperature, i = 1 + k mass fraction of species k) of reactor r,
 *     0 <= r < n, ld >= n.  Consecutive reactors are adjacent in memory.
 *   - All array arguments are DEVICE pointers owned by the caller; the
 *     library never frees them.  `stream` is a hipStream_t (NULL = the
 *     null stream).  Calls are asynchronous on that stream; the return code
 *     covers argument validation and kernel launch only.
 *   - Return codes: CK_OK or a negative CK_E* value (see ck_strerror).
 *   - A mechanism handle's tables are immutable after ck_mechanism_load; the
 *     handle may be used from several host threads and streams at once.
 *     Calls that pass no workspace use a library-owned buffer per (mechanism,
 *     stream), so concurrent calls on different streams never share one;
 *     calls on one stream run in stream order.  A caller-supplied workspace
 *     must not be in use by another call that may overlap in time.
 */
#ifndef CK_H
#define CK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ck_mech ck_mech;

enum {
    CK_OK = 0,
    CK_EINVAL = -1,        /* bad argument (null pointer, negative size, ld < n, bad tolerance) */
    CK_EIO = -2,           /* mechanism file cannot be opened */
    CK_EPARSE = -3,        /* mechanism file malformed */
    CK_ENOMEM = -4,        /* device or host allocation failed */
    CK_EHIP = -5,          /* HIP runtime error (launch, copy) */
    CK_EUNSUPPORTED = -6,  /* option combination not implemented for this mechanism size */
    CK_ETOOBIG = -7        /* the call needs more workspace than the allocation-free entry point holds */
};

/* Per-reactor integration outcome (status[] array). */
enum {
    CK_ST_OK = 0,          /* reached t_end */
    CK_ST_MAX_STEPS = 1,   /* attempted-step budget exhausted before t_end */
    CK_ST_H_UNDERFLOW = 2, /* step size fell below max(1e-30 s, 16 eps |t|) */
    CK_ST_NONFINITE = 3    /* initial state or its source term not finite */
};

/* Kernel choice for the integrators. */
enum {
    CK_KERNEL_AUTO = 0,    /* ROS4: WAVE if N <= 64, else GROUP_TILE if N <= 128; RKF45: WAVE if N <= 128 */
    CK_KERNEL_LANE = 1,    /* one reactor per lane, all scratch in global memory (Algorithm 2 analogue) */
    CK_KERNEL_WAVE = 2,    /* one reactor per 64-lane wavefront, persistent work queue, LU in registers */
    CK_KERNEL_GROUP = 3,   /* ROS4 only: one reactor per workgroup of 1 (N <= 64) or 4 (N <= 128, matrix
                              rows split over thread pairs) wavefronts, persistent work queue,
                              Gauss-Jordan inverse in registers.  With 4 wavefronts the reaction
                              contributions are summed with LDS atomics in an order that varies
                              between runs: results agree to rounding, not bit for bit.  Every other
                              kernel gives bitwise identical results for identical inputs, whatever
                              the batch a reactor is in */
    CK_KERNEL_GROUP_TILE = 4 /* ROS4 only, 64 < N <= 128: the four-wavefront workgroup with the
                              iteration matrix in 16x16 tiles and a blocked Gauss-Jordan inverse
                              (panels of 16 columns, partial pivoting) whose rank-16 updates run on
                              the FP64 matrix cores (MFMA).  Same pivots and results as GROUP up to
                              rounding; the same summation caveat applies */
};

/* Reactor form (Section 3).  Constant pressure: p[] holds pressures (Pa); the density follows
 * the state.  Constant volume: p[] holds densities (kg/m^3), fixed per reactor; the energy
 * equation uses c_v and the internal energies (wavefront kernels, N <= 64 for the Jacobian and
 * ROS4). */
enum {
    CK_REACTOR_CONST_P = 0,
    CK_REACTOR_CONST_V = 1
};

/* Jacobian used by ROS4. */
enum {
    CK_JAC_ANALYTIC = 0,   /* analytic Jacobian (chain rule through the rates of progress) */
    CK_JAC_FD = 1          /* forward differences, one source-term evaluation per column (the
                              paper's set-up, Section 5; increments as CVODE's dense difference
                              quotient); wavefront kernel, FP64, N <= 64 */
};

/* Precision of the Rosenbrock linear solves. */
enum {
    CK_PREC_FP64 = 0,      /* FP64 LU and triangular solves */
    CK_PREC_FP32_REFINE = 1 /* FP32 factorisation with FP64 residual refinement (RHS, Jacobian, error
                              norm and control stay FP64): FP32 LU in the wavefront kernel (N <= 64),
                              FP32 matrix-core Gauss-Jordan in the tile workgroup kernel
                              (64 < N <= 128).  Each solve: x = M32^-1 b, then up to refine_sweeps
                              corrections with FP64 residuals b - M x, done once the correction is
                              below 2^-48 of the solution; if a correction fails to halve or the
                              sweeps run out, that step is refactored in FP64 (counted in
                              n_fallback).  refine_sweeps = 0: plain FP32 solves */
};

typedef struct {
    double rtol;           /* relative tolerance, > 0 unless h_fixed > 0 */
    double atol;           /* absolute tolerance, >= 0 */
    double h0;             /* > 0: initial step for reactors whose h[] entry is not > 0; 0: estimate */
    double h_fixed;        /* > 0: fixed-step mode (every step accepted, no control) */
    int64_t max_steps;     /* attempted (accepted + rejected) steps per reactor and call */
    int32_t kernel;        /* CK_KERNEL_* */
    int32_t precision;     /* CK_PREC_* (ROS4 only) */
    int32_t refine_sweeps; /* FP32 mode: maximum FP64 refinement sweeps, 0..3 */
    int32_t blocks_per_cu; /* persistent kernels (WAVE, GROUP): resident workgroups per compute unit;
                              0 = as many as registers and LDS allow (larger values are clamped) */
    int32_t jacobian;      /* CK_JAC_* (ROS4 only) */
    int32_t reactor;       /* CK_REACTOR_*: with CK_REACTOR_CONST_V the p array holds densities */
    int32_t *n_fallback;   /* CK_PREC_FP32_REFINE only, optional (NULL: not reported): device array
                              [n] receiving, per reactor and call, the attempted steps whose FP64
                              refinement stagnated or ran out of sweeps and that were refactored in
                              FP64 (that step's remaining solves use the FP64 factors) */
} ck_opts;

/* Fills *o with the defaults: rtol 1e-8, atol 1e-12, h0 0, h_fixed 0, max_steps 1e6,
 * CK_KERNEL_AUTO, CK_PREC_FP64, refine_sweeps 3, blocks_per_cu 0, CK_JAC_ANALYTIC, CK_REACTOR_CONST_P,
 * n_fallback NULL. */
void ck_opts_default(ck_opts *o);

const char *ck_strerror(int code);

/*
 * Mechanism staging (Section 3; the paper preprocesses its mechanisms into a
 * binary database that its source-term code reads).  Parses the text file at
 * `path` (format: CKMECH 1, written by the package's synth module), packs the
 * species NASA-7 data and the per-reaction Arrhenius, stoichiometry,
 * third-body and fall-off parameters, and uploads them to `device`.
 * On success *out receives a handle; free it with ck_mechanism_free.
 * Errors: CK_EIO, CK_EPARSE, CK_ENOMEM, CK_EHIP, CK_EINVAL.
 */
int ck_mechanism_load(const char *path, int device, ck_mech **out);
void ck_mechanism_free(ck_mech *m);
int ck_mechanism_info(const ck_mech *m, int *n_species, int *n_reactions, int *n_elements);

/*
 * Source term f(y) (Section 3, Eqs. ydot and tdot with Eq. wdot):
 * dY_k/dt = W_k wdot_k / rho and dT/dt = -sum_k H_k wdot_k / (rho cp), at
 * constant pressure p[r] (Pa).  y and dydt are [N][ld] (they may not
 * alias); p is [n].  n = 0 is a no-op.
 */
int ck_rhs_eval(const ck_mech *m, int64_t n, const double *y, int64_t ld, const double *p,
                double *dydt, void *stream);

/*
 * Analytic Jacobian J = df/dy of the source term above (the derivative the
 * paper approximates by forward differences in Section 5; analytic forms are
 * its recommended improvement).  jac is [N*N][ld]: jac[(i*N + j)*ld + r] =
 * df_i/dy_j of reactor r, i.e. row-major per reactor, reactor-minor.
 */
int ck_jacobian_eval(const ck_mech *m, int64_t n, const double *y, int64_t ld, const double *p,
                     double *jac, void *stream);

/*
 * Bytes of device workspace that ck_integrate_* needs for n reactors with
 * options o (NULL = defaults).  Pass a buffer at least this large as
 * `workspace`, or NULL to let the library allocate its own: one per stream
 * the mechanism is called on, kept (and grown when a call needs more, which
 * waits for the device) until ck_mechanism_free.
 * Lane kernel: per-reactor scratch, linear in n.  Wavefront kernel: a
 * 256-byte queue counter, plus for 32 < N' <= 64 (N' = N rounded up to a
 * multiple of 8) a parking slice of 64 N' doubles per resident wavefront (8
 * per compute unit of the mechanism's device).  Workgroup kernel with N > 64:
 * the counter plus a parking slice of 128 N' doubles per resident workgroup
 * (2 per compute unit).  Independent of n except for the lane kernel.
 * Returns 0 on a device query error.
 */
size_t ck_workspace_bytes(const ck_mech *m, int64_t n, const ck_opts *o);

/*
 * Integrate every reactor from t[r] (0 if t == NULL) to t_end[r] with the
 * four-stage L-stable Rosenbrock method of Section 2 / Appendix C (ROS4) and
 * adaptive steps (Algorithm 1 per reactor: EstimateH0, OneStep, accept if the
 * weighted RMS error < 1, AdjustStepSize).
 *   y        [N][ld] in/out state.
 *   p        [n] pressures (Pa).
 *   t_end    [n] end times.
 *   t, h     optional [n] in/out: start time / last proposed step; pass them
 *            back to resume exactly where a call stopped.  h[r] > 0 on input
 *            is used as the first step.
 *   status, n_accept, n_reject   [n] outputs (int32).
 *   workspace  device buffer of ck_workspace_bytes(), or NULL.
 * A reactor whose status is not CK_ST_OK keeps its last accepted (t, h, y).
 */
int ck_integrate_ros4(const ck_mech *m, int64_t n, double *y, int64_t ld, const double *p,
                      const double *t_end, double *t, double *h, const ck_opts *o, void *workspace,
                      int32_t *status, int32_t *n_accept, int32_t *n_reject, void *stream);

/* Same contract with the embedded Runge--Kutta--Fehlberg 4(5) pair of
 * Section 2 / Appendix B (fourth-order solution propagated). */
int ck_integrate_rkf45(const ck_mech *m, int64_t n, double *y, int64_t ld, const double *p,
                       const double *t_end, double *t, double *h, const ck_opts *o, void *workspace,
                       int32_t *status, int32_t *n_accept, int32_t *n_reject, void *stream);

/*
 * Graph-driven step loop (the persistent-kernel batch of Section 5.2 / Algorithm 2 with the host
 * out of the per-launch path).  Integrates every reactor from t[r] to t_end[r] with method 0
 * (ROS4) or 1 (RKF45) as a sequence of bounded launches of the integrator chosen by o (at most
 * launch_steps attempted steps per reactor each, resuming from (t, h)).  launches_per_graph such
 * launches, each followed by a small kernel that adds its step counts into n_accept / n_reject and
 * updates status[], are captured once into a HIP graph together with a device-side count of the
 * reactors still short of t_end; the graph is replayed on `stream` and the host reads that count
 * once per replay (one host synchronisation per launches_per_graph launches).  The loop ends when
 * no reactor is left or when replays * launches_per_graph * launch_steps >= o->max_steps (the
 * budget is rounded up to whole replays).  A reactor that ends with CK_ST_H_UNDERFLOW or
 * CK_ST_NONFINITE is frozen for the remaining launches and keeps that status.
 *   t, h     required [n] in/out (start time and step; zeros start from t = 0 with EstimateH0).
 *   status, n_accept, n_reject   [n] outputs: totals over every launch.
 *   replays  optional out: graph replays run.
 *   workspace  device buffer of ck_graph_workspace_bytes(), or NULL (library-owned, per stream).
 * Synchronous: returns after the last replay has completed.  Results equal those of the same
 * launches issued one by one (bitwise for every kernel but CK_KERNEL_GROUP at N > 64).
 * launch_steps >= 1, 1 <= launches_per_graph <= 64.
 */
int ck_integrate_graph(const ck_mech *m, int32_t method, int64_t n, double *y, int64_t ld, const double *p,
                       const double *t_end, double *t, double *h, const ck_opts *o, int32_t launch_steps,
                       int32_t launches_per_graph, void *workspace, int32_t *status, int32_t *n_accept,
                       int32_t *n_reject, int32_t *replays, void *stream);
size_t ck_graph_workspace_bytes(const ck_mech *m, int64_t n, const ck_opts *o);

/*
 * Allocation-free ROS4, for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same contract as
 * ck_integrate_ros4 with the workspace taken from a fixed array of the library, CK_NOALLOC_BYTES
 * per device (held until the process ends; its address on each device is looked up once, on the
 * first call on that device).  The call allocates nothing and returns CK_ETOOBIG when
 * ck_workspace_bytes(m, n, o) exceeds CK_NOALLOC_BYTES (the one-reactor-per-lane kernel needs
 * scratch linear in n; the persistent kernels need at most 64 MiB on a 256-CU device for
 * N <= 120).  Every call on one device shares that device's array, and each call clears what it
 * needs (its queue counter) itself: calls that overlap in time on one device race and must not be
 * issued (serialise them on one stream).
 */
#define CK_NOALLOC_BYTES ((size_t)64 << 20)
int ck_integrate_ros4_noalloc(const ck_mech *m, int64_t n, double *y, int64_t ld, const double *p,
                              const double *t_end, double *t, double *h, const ck_opts *o, int32_t *status,
                              int32_t *n_accept, int32_t *n_reject, void *stream);

/*
 * Variants of ck_rhs_eval / ck_jacobian_eval with an explicit kernel family
 * (CK_KERNEL_LANE: one reactor per lane, coalesced; CK_KERNEL_WAVE: one
 * reactor per wavefront, the family the wavefront integrators use;
 * CK_KERNEL_AUTO: the library's choice).  ck_rhs_eval and ck_jacobian_eval
 * use CK_KERNEL_AUTO, which is the deep-vectorised family (Section 4) for
 * N <= 128.  A CK_KERNEL_WAVE Jacobian runs one reactor per wavefront for
 * N <= 64 and one reactor per four-wavefront workgroup (matrix rows split
 * over thread pairs, as in the N > 64 integrator) for 64 < N <= 128
 * (constant pressure only there; CK_EUNSUPPORTED otherwise).  The lane family
 * uses a library-owned scratch buffer sized for n.  reactor:
 * CK_REACTOR_CONST_P (p = pressures) or CK_REACTOR_CONST_V (p = densities;
 * wavefront family only, N <= 64, CK_EUNSUPPORTED with CK_KERNEL_LANE).
 */
int ck_rhs_eval_ex(const ck_mech *m, int64_t n, const double *y, int64_t ld, const double *p, double *dydt,
                   int32_t kernel, int32_t reactor, void *stream);
int ck_jacobian_eval_ex(const ck_mech *m, int64_t n, const double *y, int64_t ld, const double *p, double *jac,
                        int32_t kernel, int32_t reactor, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CK_H */
