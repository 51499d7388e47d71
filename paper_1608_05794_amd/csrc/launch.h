// Launchers of the two kernel families (internal to the library).
#pragma once

#include "ck_internal.h"

namespace ck {

// Integration options as the kernels see them (validated copy of ck_opts).
struct IntOpts {
    double rtol, atol, h0, h_fixed;
    int64_t max_steps;
    int32_t precision, refine_sweeps, blocks_per_cu, jacobian;
    int32_t reactor;   // 0 constant pressure, 1 constant volume
    int32_t *n_fallback;   // optional [n]: FP32-mode steps refactored in FP64 (written per call)
};

// lane-per-reactor family (k_lane.hip)
int64_t lane_ws_doubles_per_reactor(const DevMech &M, int method);
int launch_rhs_lane(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *dydt,
                    double *ws, int64_t wsS, hipStream_t s);
int launch_jac_lane(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *jac,
                    double *ws, int64_t wsS, hipStream_t s);
int launch_integrate_lane(int method, const DevMech &M, int64_t n, double *y, int64_t ld, const double *p,
                          const double *t_end, double *t, double *h, const IntOpts &o, double *ws, int64_t wsS,
                          int32_t *status, int32_t *nacc, int32_t *nrej, hipStream_t s);

// wavefront-per-reactor family (k_wave.hip)
bool wave_supported(const DevMech &M, int method, int precision);
size_t wave_ws_bytes(const DevMech &M, int cus);   // queue counter + parked LU rows
int launch_rhs_wave(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *dydt,
                    int cv, hipStream_t s);
int launch_jac_wave(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *jac,
                    int cv, hipStream_t s);
int launch_integrate_wave(int method, const DevMech &M, int64_t n, double *y, int64_t ld, const double *p,
                          const double *t_end, double *t, double *h, const IntOpts &o, void *ws,
                          int32_t *status, int32_t *nacc, int32_t *nrej, hipStream_t s);

// workgroup-cooperative ROS4 (k_coop.hip)
bool coop_supported(const DevMech &M);
size_t coop_ws_bytes(const DevMech &M, int cus);   // queue counter + parked inverse rows
int launch_integrate_coop(const DevMech &M, int64_t n, double *y, int64_t ld, const double *p, const double *t_end,
                          double *t, double *h, const IntOpts &o, void *ws, int32_t *status, int32_t *nacc,
                          int32_t *nrej, hipStream_t s);
// tile form of the four-wavefront ROS4 (64 < N <= 128): blocked Gauss-Jordan on the matrix cores
bool tile_supported(const DevMech &M);
int launch_integrate_tile(const DevMech &M, int64_t n, double *y, int64_t ld, const double *p, const double *t_end,
                          double *t, double *h, const IntOpts &o, void *ws, int32_t *status, int32_t *nacc,
                          int32_t *nrej, hipStream_t s);
// standalone Jacobian for 64 < N <= 128: one reactor per four-wavefront group
int launch_jac_coop(const DevMech &M, int64_t n, const double *y, int64_t ld, const double *p, double *jac,
                    hipStream_t s);

}  // namespace ck
