// C-ABI entry points: argument validation, workspace management and kernel
// selection.  Every compute step runs in the kernels of k_lane.hip,
// k_wave.hip and k_coop.hip.
#include <climits>
#include <cmath>

#include "ck_internal.h"
#include "launch.h"

using namespace ck;

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = (prev == dev) || hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (ok && prev >= 0) hipSetDevice(prev);
    }
};

// Library-owned workspace of a mechanism for calls on `s` that pass none.  Each stream gets its
// own buffer: two streams running the persistent kernels at once must not share a queue counter.
// Growing a buffer waits for that stream (the only one that uses it) before freeing the old one.
int cached_ws(ck_mech *m, hipStream_t s, size_t bytes, void **out) {
    std::lock_guard<std::mutex> lk(m->ws_mutex);
    ck_mech::StreamWs *e = nullptr;
    for (auto &w : m->ws)
        if (w.stream == s) e = &w;
    if (!e) {
        m->ws.push_back({s, nullptr, 0});
        e = &m->ws.back();
    }
    if (e->bytes < bytes) {
        if (e->ptr) {
            if (hipStreamSynchronize(s) != hipSuccess) return CK_EHIP;
            hipFree(e->ptr);
            e->ptr = nullptr;
            e->bytes = 0;
        }
        if (hipMalloc(&e->ptr, bytes) != hipSuccess) return CK_ENOMEM;
        e->bytes = bytes;
    }
    *out = e->ptr;
    return CK_OK;
}

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

bool check_state_args(const ck_mech *m, int64_t n, const void *y, int64_t ld, const void *p, const void *out) {
    if (!m || n < 0 || n > INT32_MAX) return false;
    if (n == 0) return true;
    return y && p && out && ld >= n;
}

int validate_opts(const ck_opts *o, IntOpts &io) {
    ck_opts d;
    ck_opts_default(&d);
    if (!o) o = &d;
    if (!(o->h_fixed >= 0.0) || !(o->h0 >= 0.0)) return CK_EINVAL;
    if (o->h_fixed == 0.0 && !(o->rtol > 0.0)) return CK_EINVAL;
    if (!(o->atol >= 0.0) || o->max_steps < 1) return CK_EINVAL;
    if (o->kernel < CK_KERNEL_AUTO || o->kernel > CK_KERNEL_GROUP_TILE) return CK_EINVAL;
    if (o->precision != CK_PREC_FP64 && o->precision != CK_PREC_FP32_REFINE) return CK_EINVAL;
    if (o->refine_sweeps < 0 || o->refine_sweeps > 3) return CK_EINVAL;
    if (o->blocks_per_cu < 0) return CK_EINVAL;
    if (o->jacobian != CK_JAC_ANALYTIC && o->jacobian != CK_JAC_FD) return CK_EINVAL;
    if (o->reactor != CK_REACTOR_CONST_P && o->reactor != CK_REACTOR_CONST_V) return CK_EINVAL;
    io.rtol = o->rtol;
    io.atol = o->atol;
    io.h0 = o->h0;
    io.h_fixed = o->h_fixed;
    io.max_steps = o->max_steps;
    io.precision = o->precision;
    io.refine_sweeps = o->refine_sweeps;
    io.blocks_per_cu = o->blocks_per_cu;
    io.jacobian = o->jacobian;
    io.reactor = o->reactor;
    io.n_fallback = o->precision == CK_PREC_FP32_REFINE ? o->n_fallback : nullptr;
    return CK_OK;
}

// Kernel family an integrate call will use (CK_KERNEL_LANE / WAVE / GROUP), or an error.
int choose_kernel(const ck_mech *m, int method, const ck_opts *o) {
    ck_opts d;
    ck_opts_default(&d);
    if (!o) o = &d;
    const bool fp64 = o->precision == CK_PREC_FP64;
    const bool wave_ok = wave_supported(m->dev, method, o->precision);
    if (o->reactor == CK_REACTOR_CONST_V) {
        // constant volume: wavefront kernels only
        if (!wave_ok || (o->kernel != CK_KERNEL_AUTO && o->kernel != CK_KERNEL_WAVE)) return CK_EUNSUPPORTED;
        return CK_KERNEL_WAVE;
    }
    if (method == 0 && o->jacobian == CK_JAC_FD) {
        // forward-difference Jacobian: wavefront kernel, FP64 only
        if (!fp64 || !wave_ok || (o->kernel != CK_KERNEL_AUTO && o->kernel != CK_KERNEL_WAVE))
            return CK_EUNSUPPORTED;
        return CK_KERNEL_WAVE;
    }
    const bool group_ok = method == 0 && fp64 && coop_supported(m->dev);
    const bool tile_ok = method == 0 && tile_supported(m->dev);     // FP64 or FP32 with refinement
    switch (o->kernel) {
        case CK_KERNEL_WAVE: return wave_ok ? CK_KERNEL_WAVE : CK_EUNSUPPORTED;
        case CK_KERNEL_GROUP: return group_ok ? CK_KERNEL_GROUP : CK_EUNSUPPORTED;
        case CK_KERNEL_GROUP_TILE: return tile_ok ? CK_KERNEL_GROUP_TILE : CK_EUNSUPPORTED;
        case CK_KERNEL_LANE: return fp64 ? CK_KERNEL_LANE : CK_EUNSUPPORTED;
        default:
            if (wave_ok) return CK_KERNEL_WAVE;
            if (tile_ok) return CK_KERNEL_GROUP_TILE;
            if (group_ok) return CK_KERNEL_GROUP;
            return fp64 ? CK_KERNEL_LANE : CK_EUNSUPPORTED;
    }
}

size_t lane_bytes(const ck_mech *m, int64_t n, int method) {
    return size_t(lane_ws_doubles_per_reactor(m->dev, method)) * size_t(round_up(std::max<int64_t>(n, 1), 64)) *
           sizeof(double);
}

int integrate(int method, const ck_mech *mc, int64_t n, double *y, int64_t ld, const double *p, const double *t_end,
              double *t, double *h, const ck_opts *o, void *workspace, int32_t *status, int32_t *nacc, int32_t *nrej,
              void *stream) {
    ck_mech *m = const_cast<ck_mech *>(mc);
    if (!check_state_args(m, n, y, ld, p, y)) return CK_EINVAL;
    IntOpts io;
    int rc = validate_opts(o, io);
    if (rc != CK_OK) return rc;
    if (n == 0) return CK_OK;
    if (!t_end || !status || !nacc || !nrej) return CK_EINVAL;
    const int kern = choose_kernel(m, method, o);
    if (kern < 0) return kern;
    DeviceGuard g(m->device);
    if (!g.ok) return CK_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t need = ck_workspace_bytes(m, n, o);
    void *ws = workspace;
    if (!ws) {
        rc = cached_ws(m, s, need, &ws);
        if (rc != CK_OK) return rc;
    }
    if (kern == CK_KERNEL_WAVE)
        return launch_integrate_wave(method, m->dev, n, y, ld, p, t_end, t, h, io, ws, status, nacc, nrej, s);
    if (kern == CK_KERNEL_GROUP)
        return launch_integrate_coop(m->dev, n, y, ld, p, t_end, t, h, io, ws, status, nacc, nrej, s);
    if (kern == CK_KERNEL_GROUP_TILE)
        return launch_integrate_tile(m->dev, n, y, ld, p, t_end, t, h, io, ws, status, nacc, nrej, s);
    const int64_t S = round_up(n, 64);
    return launch_integrate_lane(method, m->dev, n, y, ld, p, t_end, t, h, io, static_cast<double *>(ws), S, status,
                                 nacc, nrej, s);
}

}  // namespace

extern "C" void ck_opts_default(ck_opts *o) {
    if (!o) return;
    o->rtol = 1e-8;
    o->atol = 1e-12;
    o->h0 = 0.0;
    o->h_fixed = 0.0;
    o->max_steps = 1000000;
    o->kernel = CK_KERNEL_AUTO;
    o->precision = CK_PREC_FP64;
    o->refine_sweeps = 3;
    o->blocks_per_cu = 0;
    o->jacobian = CK_JAC_ANALYTIC;
    o->reactor = CK_REACTOR_CONST_P;
    o->n_fallback = nullptr;
}

extern "C" const char *ck_strerror(int code) {
    switch (code) {
        case CK_OK: return "ok";
        case CK_EINVAL: return "invalid argument";
        case CK_EIO: return "cannot open mechanism file";
        case CK_EPARSE: return "malformed mechanism file";
        case CK_ENOMEM: return "out of memory";
        case CK_EHIP: return "HIP runtime error";
        case CK_EUNSUPPORTED: return "unsupported option for this mechanism";
        case CK_ETOOBIG: return "workspace needed exceeds the allocation-free maximum (CK_NOALLOC_BYTES)";
        default: return "unknown error";
    }
}

extern "C" int ck_rhs_eval_ex(const ck_mech *mc, int64_t n, const double *y, int64_t ld, const double *p, double *dydt,
                              int32_t kernel, int32_t reactor, void *stream) {
    ck_mech *m = const_cast<ck_mech *>(mc);
    if (!check_state_args(m, n, y, ld, p, dydt)) return CK_EINVAL;
    if (kernel < CK_KERNEL_AUTO || kernel > CK_KERNEL_WAVE) return CK_EINVAL;
    if (reactor != CK_REACTOR_CONST_P && reactor != CK_REACTOR_CONST_V) return CK_EINVAL;
    if (reactor == CK_REACTOR_CONST_V && kernel == CK_KERNEL_LANE) return CK_EUNSUPPORTED;
    if (n == 0) return CK_OK;
    DeviceGuard g(m->device);
    if (!g.ok) return CK_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (kernel == CK_KERNEL_LANE) {
        void *ws = nullptr;
        int rc = cached_ws(m, s, lane_bytes(m, n, 0), &ws);
        if (rc != CK_OK) return rc;
        return launch_rhs_lane(m->dev, n, y, ld, p, dydt, static_cast<double *>(ws), round_up(n, 64), s);
    }
    return launch_rhs_wave(m->dev, n, y, ld, p, dydt, reactor, s);
}

extern "C" int ck_rhs_eval(const ck_mech *m, int64_t n, const double *y, int64_t ld, const double *p, double *dydt,
                           void *stream) {
    return ck_rhs_eval_ex(m, n, y, ld, p, dydt, CK_KERNEL_AUTO, CK_REACTOR_CONST_P, stream);
}

extern "C" int ck_jacobian_eval_ex(const ck_mech *mc, int64_t n, const double *y, int64_t ld, const double *p,
                                   double *jac, int32_t kernel, int32_t reactor, void *stream) {
    ck_mech *m = const_cast<ck_mech *>(mc);
    if (!check_state_args(m, n, y, ld, p, jac)) return CK_EINVAL;
    if (kernel < CK_KERNEL_AUTO || kernel > CK_KERNEL_WAVE) return CK_EINVAL;
    if (reactor != CK_REACTOR_CONST_P && reactor != CK_REACTOR_CONST_V) return CK_EINVAL;
    if (reactor == CK_REACTOR_CONST_V) {
        if (kernel == CK_KERNEL_LANE) return CK_EUNSUPPORTED;
        kernel = CK_KERNEL_WAVE;
    }
    // default: the deep-vectorised family (one reactor per wavefront, or per four-wavefront group
    // for 64 < N <= 128); the lane kernel beyond that
    if (kernel == CK_KERNEL_AUTO) kernel = m->dev.N <= 128 ? CK_KERNEL_WAVE : CK_KERNEL_LANE;
    if (n == 0) return CK_OK;
    DeviceGuard g(m->device);
    if (!g.ok) return CK_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (kernel == CK_KERNEL_WAVE) return launch_jac_wave(m->dev, n, y, ld, p, jac, reactor, s);
    void *ws = nullptr;
    int rc = cached_ws(m, s, lane_bytes(m, n, 0), &ws);
    if (rc != CK_OK) return rc;
    return launch_jac_lane(m->dev, n, y, ld, p, jac, static_cast<double *>(ws), round_up(n, 64), s);
}

extern "C" int ck_jacobian_eval(const ck_mech *m, int64_t n, const double *y, int64_t ld, const double *p, double *jac,
                                void *stream) {
    return ck_jacobian_eval_ex(m, n, y, ld, p, jac, CK_KERNEL_AUTO, CK_REACTOR_CONST_P, stream);
}

extern "C" size_t ck_workspace_bytes(const ck_mech *m, int64_t n, const ck_opts *o) {
    if (!m || n < 0) return 0;
    size_t best = 256;
    for (int method = 0; method < 2; method++) {
        const int k = choose_kernel(m, method, o);
        size_t b = 256;
        if (k == CK_KERNEL_LANE) b = lane_bytes(m, n, method);
        else if (k == CK_KERNEL_WAVE || k == CK_KERNEL_GROUP || k == CK_KERNEL_GROUP_TILE) {
            int cus = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess)
                return 0;
            b = k == CK_KERNEL_WAVE ? wave_ws_bytes(m->dev, cus) : coop_ws_bytes(m->dev, cus);
        }
        if (b > best) best = b;
    }
    return best;
}

extern "C" int ck_integrate_ros4(const ck_mech *m, int64_t n, double *y, int64_t ld, const double *p,
                                 const double *t_end, double *t, double *h, const ck_opts *o, void *workspace,
                                 int32_t *status, int32_t *n_accept, int32_t *n_reject, void *stream) {
    return integrate(0, m, n, y, ld, p, t_end, t, h, o, workspace, status, n_accept, n_reject, stream);
}

extern "C" int ck_integrate_rkf45(const ck_mech *m, int64_t n, double *y, int64_t ld, const double *p,
                                  const double *t_end, double *t, double *h, const ck_opts *o, void *workspace,
                                  int32_t *status, int32_t *n_accept, int32_t *n_reject, void *stream) {
    return integrate(1, m, n, y, ld, p, t_end, t, h, o, workspace, status, n_accept, n_reject, stream);
}

// ---------------------------------------------------------------------------------------
// Graph-driven step loop: bounded launches captured K at a time in a HIP graph
// ---------------------------------------------------------------------------------------
namespace {

// Bookkeeping of the graph loop, after the integrator's own workspace (256-byte aligned pieces).
struct GraphWs {
    size_t kernel_bytes, te, st, acc, rej, remaining, total;
    GraphWs(size_t kbytes, int64_t n) {
        auto up = [](size_t v) { return (v + 255) / 256 * 256; };
        const size_t nn = size_t(std::max<int64_t>(n, 1));
        kernel_bytes = up(kbytes);
        te = kernel_bytes;
        st = te + up(nn * sizeof(double));
        acc = st + up(nn * sizeof(int32_t));
        rej = acc + up(nn * sizeof(int32_t));
        remaining = rej + up(nn * sizeof(int32_t));
        total = remaining + 256;
    }
};

__global__ void graph_init_kernel(int64_t n, const double *t_end, double *te, int32_t *status, int32_t *nacc,
                                  int32_t *nrej) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    te[i] = t_end[i];
    status[i] = CK_ST_OK;
    nacc[i] = 0;
    nrej[i] = 0;
}

__global__ void graph_zero_kernel(unsigned *c) { *c = 0u; }

// Folds one bounded launch into the totals.  A reactor that ended with H_UNDERFLOW or NONFINITE is
// frozen: its working end time becomes its current time, so later launches leave it unchanged, and
// its status is kept.  With `count`, reactors still short of t_end (MAX_STEPS) are counted.
__global__ void graph_merge_kernel(int64_t n, const double *t, double *te, const int32_t *st_k, const int32_t *acc_k,
                                   const int32_t *rej_k, int32_t *status, int32_t *nacc, int32_t *nrej,
                                   unsigned *remaining, int count) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    bool open = false;
    if (i < n) {
        nacc[i] += acc_k[i];
        nrej[i] += rej_k[i];
        const int prev = status[i];
        if (prev != CK_ST_H_UNDERFLOW && prev != CK_ST_NONFINITE) {
            const int sk = st_k[i];
            status[i] = sk;
            if (sk == CK_ST_H_UNDERFLOW || sk == CK_ST_NONFINITE) te[i] = t[i];
            open = sk == CK_ST_MAX_STEPS;
        }
    }
    if (count) {
        const unsigned long long b = __ballot(open);
        if (b && __lane_id() == __ffsll((long long)b) - 1) atomicAdd(remaining, unsigned(__popcll(b)));
    }
}

struct StreamHolder {
    hipStream_t s = nullptr;
    ~StreamHolder() {
        if (s) hipStreamDestroy(s);
    }
};
struct GraphHolder {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    ~GraphHolder() {
        if (e) hipGraphExecDestroy(e);
        if (g) hipGraphDestroy(g);
    }
};

}  // namespace

extern "C" size_t ck_graph_workspace_bytes(const ck_mech *m, int64_t n, const ck_opts *o) {
    const size_t k = ck_workspace_bytes(m, n, o);
    if (k == 0) return 0;
    return GraphWs(k, n).total;
}

extern "C" int ck_integrate_graph(const ck_mech *mc, int32_t method, int64_t n, double *y, int64_t ld,
                                  const double *p, const double *t_end, double *t, double *h, const ck_opts *o,
                                  int32_t launch_steps, int32_t launches_per_graph, void *workspace,
                                  int32_t *status, int32_t *n_accept, int32_t *n_reject, int32_t *replays,
                                  void *stream) {
    ck_mech *m = const_cast<ck_mech *>(mc);
    if (method != 0 && method != 1) return CK_EINVAL;
    if (!check_state_args(m, n, y, ld, p, y)) return CK_EINVAL;
    IntOpts io;
    int rc = validate_opts(o, io);
    if (rc != CK_OK) return rc;
    if (launch_steps < 1 || launches_per_graph < 1 || launches_per_graph > 64) return CK_EINVAL;
    if (replays) *replays = 0;
    if (n == 0) return CK_OK;
    if (!t_end || !t || !h || !status || !n_accept || !n_reject) return CK_EINVAL;
    rc = choose_kernel(m, method, o);
    if (rc < 0) return rc;
    ck_opts d;
    ck_opts_default(&d);
    ck_opts lo = o ? *o : d;                 // per-launch options: a bounded attempted-step budget
    const int64_t budget = lo.max_steps;
    lo.max_steps = launch_steps;
    DeviceGuard g(m->device);
    if (!g.ok) return CK_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const GraphWs L(ck_workspace_bytes(m, n, &lo), n);
    if (L.kernel_bytes == 0) return CK_EHIP;
    char *ws = static_cast<char *>(workspace);
    if (!ws) {
        void *v = nullptr;
        rc = cached_ws(m, s, L.total, &v);
        if (rc != CK_OK) return rc;
        ws = static_cast<char *>(v);
    }
    double *te = reinterpret_cast<double *>(ws + L.te);
    int32_t *st_k = reinterpret_cast<int32_t *>(ws + L.st);
    int32_t *acc_k = reinterpret_cast<int32_t *>(ws + L.acc);
    int32_t *rej_k = reinterpret_cast<int32_t *>(ws + L.rej);
    unsigned *rem = reinterpret_cast<unsigned *>(ws + L.remaining);
    const dim3 blk(256), grd(unsigned((n + 255) / 256));

    // capture K launches (+ bookkeeping) on a private stream; the graph is replayed on `s`
    StreamHolder cs;
    CK_HIP_TRY(hipStreamCreateWithFlags(&cs.s, hipStreamNonBlocking));
    GraphHolder gh;
    CK_HIP_TRY(hipStreamBeginCapture(cs.s, hipStreamCaptureModeRelaxed));
    int crc = CK_OK;
    for (int k = 0; k < launches_per_graph && crc == CK_OK; k++) {
        crc = integrate(method, m, n, y, ld, p, te, t, h, &lo, ws, st_k, acc_k, rej_k, cs.s);
        if (crc != CK_OK) break;
        const bool last = k == launches_per_graph - 1;
        if (last) graph_zero_kernel<<<1, 1, 0, cs.s>>>(rem);
        graph_merge_kernel<<<grd, blk, 0, cs.s>>>(n, t, te, st_k, acc_k, rej_k, status, n_accept, n_reject, rem,
                                                   last ? 1 : 0);
    }
    const hipError_t ec = hipStreamEndCapture(cs.s, &gh.g);
    if (crc != CK_OK) return crc;
    if (ec != hipSuccess || hipGetLastError() != hipSuccess) return CK_EHIP;
    CK_HIP_TRY(hipGraphInstantiate(&gh.e, gh.g, nullptr, nullptr, 0));

    graph_init_kernel<<<grd, blk, 0, s>>>(n, t_end, te, status, n_accept, n_reject);
    CK_HIP_TRY(hipGetLastError());
    int32_t done = 0;
    for (;;) {
        CK_HIP_TRY(hipGraphLaunch(gh.e, s));
        done++;
        unsigned left = 0;
        CK_HIP_TRY(hipMemcpyAsync(&left, rem, sizeof(left), hipMemcpyDeviceToHost, s));
        CK_HIP_TRY(hipStreamSynchronize(s));
        if (left == 0 || int64_t(done) * launches_per_graph * launch_steps >= budget) break;
    }
    if (replays) *replays = done;
    return CK_OK;
}

// ---------------------------------------------------------------------------------------
// Allocation-free ROS4: the workspace is a fixed device array of the library
// ---------------------------------------------------------------------------------------
namespace {

__device__ __align__(256) unsigned char scratch[CK_NOALLOC_BYTES];

// Device address of `scratch` on each device (each device holds its own copy), resolved once per
// device with that device current.  The host-side symbol is not a device address.
int scratch_ptr(int device, void **out) {
    static std::mutex mu;
    static std::vector<void *> ptr;
    std::lock_guard<std::mutex> lk(mu);
    if (device < 0) return CK_EINVAL;
    if (int(ptr.size()) <= device) ptr.resize(size_t(device) + 1, nullptr);
    if (!ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CK_EHIP;
        ptr[device] = p;
    }
    *out = ptr[device];
    return CK_OK;
}

}  // namespace

extern "C" int ck_integrate_ros4_noalloc(const ck_mech *m, int64_t n, double *y, int64_t ld, const double *p,
                                         const double *t_end, double *t, double *h, const ck_opts *o,
                                         int32_t *status, int32_t *n_accept, int32_t *n_reject, void *stream) {
    if (!m) return CK_EINVAL;
    if (!check_state_args(m, n, y, ld, p, y)) return CK_EINVAL;
    IntOpts io;
    const int rc = validate_opts(o, io);
    if (rc != CK_OK) return rc;
    if (n == 0) return CK_OK;
    const int kern = choose_kernel(m, 0, o);
    if (kern < 0) return kern;
    DeviceGuard g(m->device);
    if (!g.ok) return CK_EHIP;
    const size_t need = ck_workspace_bytes(m, n, o);
    if (need == 0) return CK_EHIP;
    if (need > CK_NOALLOC_BYTES) return CK_ETOOBIG;
    void *ws = nullptr;
    const int sr = scratch_ptr(m->device, &ws);
    if (sr != CK_OK) return sr;
    return integrate(0, m, n, y, ld, p, t_end, t, h, o, ws, status, n_accept, n_reject, stream);
}
