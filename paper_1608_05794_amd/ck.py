"""Python binding of libck.so (ctypes).  Argument marshalling only.

Device memory and streams come from PyTorch (ROCm build): every array is a
float64 / int32 device tensor, and calls are enqueued on torch's current
stream unless a stream is given.  Every computation runs in the library's
HIP kernels; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libck.so")

KERNELS = {"auto": 0, "lane": 1, "wave": 2, "group": 3, "tile": 4}
PRECISIONS = {"fp64": 0, "fp32_refine": 1}
JACOBIANS = {"analytic": 0, "fd": 1}
REACTORS = {"cp": 0, "cv": 1}   # constant pressure (p = pressures, Pa) / constant volume (p = densities, kg/m^3)
STATUS = {0: "ok", 1: "max_steps", 2: "h_underflow", 3: "nonfinite"}


class CkError(RuntimeError):
    pass


class Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("h0", C.c_double), ("h_fixed", C.c_double),
                ("max_steps", C.c_int64), ("kernel", C.c_int32), ("precision", C.c_int32),
                ("refine_sweeps", C.c_int32), ("blocks_per_cu", C.c_int32), ("jacobian", C.c_int32), ("reactor", C.c_int32),
                ("n_fallback", C.c_void_p)]


_lib = None

EXPORTS = ["ck_opts_default", "ck_strerror", "ck_mechanism_load", "ck_mechanism_free", "ck_mechanism_info",
           "ck_rhs_eval", "ck_rhs_eval_ex", "ck_jacobian_eval", "ck_jacobian_eval_ex", "ck_workspace_bytes",
           "ck_integrate_ros4", "ck_integrate_rkf45", "ck_integrate_graph",
           "ck_graph_workspace_bytes", "ck_integrate_ros4_noalloc"]


def lib():
    """Load libck.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CkError(f"{LIB_PATH} is missing: build it with paper_1608_05794_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i64, dp, i32p = C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p
        L.ck_opts_default.argtypes = [C.POINTER(Opts)]
        L.ck_strerror.argtypes = [C.c_int]
        L.ck_strerror.restype = C.c_char_p
        L.ck_mechanism_load.argtypes = [C.c_char_p, C.c_int, C.POINTER(vp)]
        L.ck_mechanism_free.argtypes = [vp]
        L.ck_mechanism_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.ck_rhs_eval.argtypes = [vp, i64, dp, i64, dp, dp, vp]
        L.ck_rhs_eval_ex.argtypes = [vp, i64, dp, i64, dp, dp, C.c_int32, C.c_int32, vp]
        L.ck_jacobian_eval.argtypes = [vp, i64, dp, i64, dp, dp, vp]
        L.ck_jacobian_eval_ex.argtypes = [vp, i64, dp, i64, dp, dp, C.c_int32, C.c_int32, vp]
        L.ck_workspace_bytes.argtypes = [vp, i64, C.POINTER(Opts)]
        L.ck_workspace_bytes.restype = C.c_size_t
        sig = [vp, i64, dp, i64, dp, dp, dp, dp, C.POINTER(Opts), vp, i32p, i32p, i32p, vp]
        L.ck_integrate_ros4.argtypes = sig
        L.ck_integrate_rkf45.argtypes = sig
        L.ck_integrate_graph.argtypes = [vp, C.c_int32, i64, dp, i64, dp, dp, dp, dp, C.POINTER(Opts), C.c_int32,
                                         C.c_int32, vp, i32p, i32p, i32p, C.POINTER(C.c_int32), vp]
        L.ck_integrate_ros4_noalloc.argtypes = [vp, i64, dp, i64, dp, dp, dp, dp, C.POINTER(Opts), i32p, i32p, i32p, vp]
        L.ck_graph_workspace_bytes.argtypes = [vp, i64, C.POINTER(Opts)]
        L.ck_graph_workspace_bytes.restype = C.c_size_t
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise CkError(f"ck error {rc}: {lib().ck_strerror(rc).decode()}")


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _state(y, N):
    if y.dtype != torch.float64 or not y.is_cuda or y.dim() != 2 or y.shape[0] != N:
        raise CkError(f"state must be a float64 device tensor of shape [{N}, n]")
    if y.stride(1) != 1:
        raise CkError("state must be reactor-contiguous (stride 1 along reactors)")
    return y.stride(0)


def _vec(v, n, dev, name, dtype=torch.float64):
    """Check a per-reactor vector argument: `dtype`, on the state's device, stride 1, >= n entries."""
    if v is None:
        return None
    if not torch.is_tensor(v) or v.dtype != dtype or v.device != dev or v.dim() != 1:
        raise CkError(f"{name} must be a 1-d {dtype} tensor on {dev}")
    if v.numel() < n or (v.numel() > 1 and v.stride(0) != 1):
        raise CkError(f"{name} must be contiguous with at least {n} entries")
    return v


def make_opts(rtol=1e-8, atol=1e-12, h0=0.0, h_fixed=0.0, max_steps=1_000_000, kernel="auto", precision="fp64",
              refine_sweeps=3, blocks_per_cu=0, jacobian="analytic", reactor="cp", n_fallback=None):
    o = Opts()
    lib().ck_opts_default(C.byref(o))
    o.rtol, o.atol, o.h0, o.h_fixed, o.max_steps = rtol, atol, h0, h_fixed, max_steps
    o.kernel = KERNELS[kernel]
    o.precision = PRECISIONS[precision]
    o.refine_sweeps = refine_sweeps
    o.blocks_per_cu = blocks_per_cu
    o.jacobian = JACOBIANS[jacobian]
    o.reactor = REACTORS[reactor]
    o.n_fallback = n_fallback.data_ptr() if n_fallback is not None else None
    return o


class Mechanism:
    """A mechanism staged on one device (ck_mechanism_load)."""

    def __init__(self, path, device=0):
        h = C.c_void_p()
        _check(lib().ck_mechanism_load(os.fspath(path).encode(), int(device), C.byref(h)))
        self._h = h
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        _check(lib().ck_mechanism_info(h, C.byref(a), C.byref(b), C.byref(c)))
        self.n_species, self.n_reactions, self.n_elements = a.value, b.value, c.value
        self.N = self.n_species + 1
        self.device = torch.device("cuda", device)

    def close(self):
        if getattr(self, "_h", None):
            lib().ck_mechanism_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self, n, **opts):
        o = make_opts(**opts)
        return int(lib().ck_workspace_bytes(self._h, int(n), C.byref(o)))

    def graph_workspace_bytes(self, n, **opts):
        o = make_opts(**opts)
        return int(lib().ck_graph_workspace_bytes(self._h, int(n), C.byref(o)))


def rhs(mech, y, p, out=None, kernel=None, stream=None, reactor="cp"):
    """dy/dt for every reactor (ck_rhs_eval / ck_rhs_eval_ex); y [N, n] float64, p [n]: pressures (Pa)
    for reactor="cp", densities (kg/m^3) for "cv"."""
    _state(y, mech.N)
    n = y.shape[1]
    _vec(p, n, y.device, "p")
    if out is None:
        # the library writes out[i ld + r] with the state's leading dimension: pass a compact state
        # so that a fresh compact output matches it
        y = y.contiguous()
        out = torch.empty_like(y)
    ld = _state(y, mech.N)
    if out.dtype != torch.float64 or out.device != y.device or out.shape != y.shape or \
            out.stride(0) != ld or out.stride(1) != 1:
        raise CkError("output must be a float64 tensor with the state's shape, device and strides")
    if kernel is None and reactor == "cp":
        _check(lib().ck_rhs_eval(mech.handle, n, _ptr(y), ld, _ptr(p), _ptr(out), _stream(stream)))
    else:
        _check(lib().ck_rhs_eval_ex(mech.handle, n, _ptr(y), ld, _ptr(p), _ptr(out), KERNELS[kernel or "auto"],
                                    REACTORS[reactor], _stream(stream)))
    return out


def jac(mech, y, p, kernel=None, stream=None, reactor="cp"):
    """Analytic Jacobian (ck_jacobian_eval / _ex): returns [N*N, n] with row (i*N + j) = df_i/dy_j."""
    _state(y, mech.N)
    n = y.shape[1]
    _vec(p, n, y.device, "p")
    # the library writes jac[(i N + j) ld + r] with the state's leading dimension: pass a compact state
    # so that ld = n matches the [N*N, n] output
    y = y.contiguous()
    ld = _state(y, mech.N)
    out = torch.empty((mech.N * mech.N, n), dtype=torch.float64, device=y.device)
    if kernel is None and reactor == "cp":
        _check(lib().ck_jacobian_eval(mech.handle, n, _ptr(y), ld, _ptr(p), _ptr(out), _stream(stream)))
    else:
        _check(lib().ck_jacobian_eval_ex(mech.handle, n, _ptr(y), ld, _ptr(p), _ptr(out), KERNELS[kernel or "auto"],
                                         REACTORS[reactor], _stream(stream)))
    return out


def integrate(mech, y, p, t_end, method="ros4", t=None, h=None, workspace=None, stream=None, inplace=False,
              **opts):
    """Integrate every reactor to t_end (ck_integrate_ros4 / ck_integrate_rkf45).

    Returns dict(y, t, h, status, n_accept, n_reject) of device tensors.  t and h
    (float64 [n]) are updated in place when given, so a later call resumes exactly.
    """
    _state(y, mech.N)
    n = y.shape[1]
    dev = y.device
    # a copy is compact whatever the input's strides: take the leading dimension from what is passed
    yy = y if inplace else y.clone(memory_format=torch.contiguous_format)
    ld = _state(yy, mech.N)
    _vec(p, n, dev, "p")
    _vec(t, n, dev, "t")
    _vec(h, n, dev, "h")
    te = t_end if torch.is_tensor(t_end) else torch.full((n,), float(t_end), dtype=torch.float64, device=dev)
    _vec(te, n, dev, "t_end")
    _vec(opts.get("n_fallback"), n, dev, "n_fallback", dtype=torch.int32)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    na = torch.empty(n, dtype=torch.int32, device=dev)
    nr = torch.empty(n, dtype=torch.int32, device=dev)
    o = make_opts(**opts)
    if workspace is not None:
        need = int(lib().ck_workspace_bytes(mech.handle, n, C.byref(o)))
        if not torch.is_tensor(workspace) or workspace.device != dev or not workspace.is_contiguous() or \
                workspace.numel() * workspace.element_size() < need:
            raise CkError(f"workspace must be a contiguous tensor on {dev} of at least {need} bytes")
    fn = {"ros4": lib().ck_integrate_ros4, "rkf45": lib().ck_integrate_rkf45}[method]
    _check(fn(mech.handle, n, _ptr(yy), ld, _ptr(p), _ptr(te), _ptr(t), _ptr(h), C.byref(o), _ptr(workspace),
              _ptr(st), _ptr(na), _ptr(nr), _stream(stream)))
    return dict(y=yy, t=t, h=h, status=st, n_accept=na, n_reject=nr)


def integrate_noalloc(mech, y, p, t_end, t=None, h=None, stream=None, **opts):
    """ROS4 through the allocation-free entry point (ck_integrate_ros4_noalloc), in place on y: the
    library takes its workspace from a fixed device array.  Outputs (status, counters) are allocated
    here by the caller side.  Returns dict(y, t, h, status, n_accept, n_reject)."""
    ld = _state(y, mech.N)
    n = y.shape[1]
    dev = y.device
    _vec(p, n, dev, "p")
    _vec(t, n, dev, "t")
    _vec(h, n, dev, "h")
    te = t_end if torch.is_tensor(t_end) else torch.full((n,), float(t_end), dtype=torch.float64, device=dev)
    _vec(te, n, dev, "t_end")
    st = torch.empty(n, dtype=torch.int32, device=dev)
    na = torch.empty(n, dtype=torch.int32, device=dev)
    nr = torch.empty(n, dtype=torch.int32, device=dev)
    o = make_opts(**opts)
    _check(lib().ck_integrate_ros4_noalloc(mech.handle, n, _ptr(y), ld, _ptr(p), _ptr(te), _ptr(t), _ptr(h),
                                           C.byref(o), _ptr(st), _ptr(na), _ptr(nr), _stream(stream)))
    return dict(y=y, t=t, h=h, status=st, n_accept=na, n_reject=nr)


def integrate_graph(mech, y, p, t_end, method="ros4", launch_steps=500, launches_per_graph=8, t=None, h=None,
                    workspace=None, stream=None, inplace=False, **opts):
    """Integrate to t_end with the graph-driven step loop (ck_integrate_graph): bounded launches of
    `launch_steps` attempted steps, captured `launches_per_graph` at a time in a HIP graph and replayed
    until no reactor is left (or opts' max_steps is spent).  Synchronous.  Returns dict(y, t, h, status,
    n_accept, n_reject, replays); t and h are allocated (zeros) when not given."""
    _state(y, mech.N)
    n = y.shape[1]
    dev = y.device
    yy = y if inplace else y.clone(memory_format=torch.contiguous_format)
    ld = _state(yy, mech.N)
    _vec(p, n, dev, "p")
    t = torch.zeros(n, dtype=torch.float64, device=dev) if t is None else _vec(t, n, dev, "t")
    h = torch.zeros(n, dtype=torch.float64, device=dev) if h is None else _vec(h, n, dev, "h")
    te = t_end if torch.is_tensor(t_end) else torch.full((n,), float(t_end), dtype=torch.float64, device=dev)
    _vec(te, n, dev, "t_end")
    _vec(opts.get("n_fallback"), n, dev, "n_fallback", dtype=torch.int32)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    na = torch.empty(n, dtype=torch.int32, device=dev)
    nr = torch.empty(n, dtype=torch.int32, device=dev)
    o = make_opts(**opts)
    if workspace is not None:
        need = int(lib().ck_graph_workspace_bytes(mech.handle, n, C.byref(o)))
        if not torch.is_tensor(workspace) or workspace.device != dev or not workspace.is_contiguous() or \
                workspace.numel() * workspace.element_size() < need:
            raise CkError(f"workspace must be a contiguous tensor on {dev} of at least {need} bytes")
    reps = C.c_int32(0)
    _check(lib().ck_integrate_graph(mech.handle, {"ros4": 0, "rkf45": 1}[method], n, _ptr(yy), ld, _ptr(p),
                                    _ptr(te), _ptr(t), _ptr(h), C.byref(o), int(launch_steps),
                                    int(launches_per_graph), _ptr(workspace), _ptr(st), _ptr(na), _ptr(nr),
                                    C.byref(reps), _stream(stream)))
    return dict(y=yy, t=t, h=h, status=st, n_accept=na, n_reject=nr, replays=reps.value)
