"""ctypes binding of the lbfft C ABI (include/lbfft.h).

Argument marshalling only: every step of the method runs in the HIP library
(paper_1403_3746_amd/liblbfft.so).  PyTorch supplies the device workspace and the stream.
Functions keep the C names; ``Sim`` is a convenience owner of a context and its workspace.
If the library is missing, loading raises -- there is no fallback path.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBFFT_LIB", os.path.join(_PKG, "liblbfft.so"))

LB_OK, LB_E_ARG, LB_E_SIZE, LB_E_NOMEM, LB_E_HIP, LB_E_NONFINITE, LB_E_STATE = 0, -1, -2, -3, -4, -5, -6
LB_FP64, LB_FP32 = 0, 1
_STATUS = {0: "LB_OK", -1: "LB_E_ARG", -2: "LB_E_SIZE", -3: "LB_E_NOMEM", -4: "LB_E_HIP",
           -5: "LB_E_NONFINITE", -6: "LB_E_STATE"}

EXPORTS = ("lb_workspace_bytes", "lb_init", "lb_step", "lb_sync", "lb_moments", "lb_conservation", "lb_conservation_history",
           "lb_get_f", "lb_set_f", "lb_set_moments", "lb_force_coefficients", "lb_rhs", "lb_derivative",
           "lb_step_timed", "lb_plan_info", "lb_free", "lb_last_error", "lb_derivative_noalloc")
PASS_NAMES = ("moments", "macro_x1", "macro_y1", "stress", "macro_x2", "macro_y2", "finalize",
              "pop_x", "pop_y")


class lb_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double),
                ("dt", ctypes.c_double), ("tau", ctypes.c_double), ("K", ctypes.c_double),
                ("H", ctypes.c_double), ("zeta", ctypes.c_double), ("q", ctypes.c_double),
                ("b_dof", ctypes.c_double), ("vdw_a", ctypes.c_double), ("vdw_b", ctypes.c_double),
                ("hist_len", ctypes.c_int32)]


class lb_dvm(ctypes.Structure):
    _fields_ = [("va", ctypes.c_double), ("vb", ctypes.c_double), ("vc", ctypes.c_double),
                ("vd", ctypes.c_double), ("eta0", ctypes.c_double)]


class LBError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load liblbfft.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"lbfft HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, D, I, V = ctypes.POINTER(lb_params), ctypes.POINTER(lb_dvm), ctypes.c_int, ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    dpp = ctypes.POINTER(dp)
    lib.lb_workspace_bytes.argtypes = [I, P, I]
    lib.lb_workspace_bytes.restype = ctypes.c_size_t
    lib.lb_init.argtypes = [ctypes.POINTER(V), I, P, D, I, dpp, dpp, dpp, dpp, V, ctypes.c_size_t, V]
    lib.lb_step.argtypes = [V, I]
    lib.lb_sync.argtypes = [V]
    lib.lb_moments.argtypes = [V, I, dp, dp, dp, dp]
    lib.lb_conservation.argtypes = [V, I, dp]
    lib.lb_conservation_history.argtypes = [V, I, I, dp, ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_longlong)]
    lib.lb_get_f.argtypes = [V, I, dp]
    lib.lb_set_f.argtypes = [V, I, dp]
    lib.lb_set_moments.argtypes = [V, I, dp, dp, dp, dp]
    lib.lb_force_coefficients.argtypes = [V, I, dp, dp, dp]
    lib.lb_rhs.argtypes = [V, I, dp]
    lib.lb_derivative.argtypes = [V, I, I, I, dp, dp]
    lib.lb_step_timed.argtypes = [V, I, dp]
    lib.lb_plan_info.argtypes = [V, I, ctypes.POINTER(ctypes.c_int), I]
    lib.lb_free.argtypes = [V]
    lib.lb_free.restype = None
    lib.lb_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("lb_workspace_bytes", "lb_free", "lb_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def lb_last_error():
    return load().lb_last_error().decode()


def _check(status):
    if status != LB_OK:
        raise LBError(status, lb_last_error())


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def make_params(p, nx, ny):
    """lb_params from a parameter dict (keys dx, dt, tau, K, H, zeta, q, b, a, bw)."""
    return lb_params(nx, ny, p["dx"], p["dt"], p["tau"], p["K"], p["H"], p["zeta"], p["q"],
                     p["b"], p["a"], p["bw"], int(p.get("hist", 0)))


def make_dvm(d=None):
    d = d or {}
    return lb_dvm(d.get("va", 1.0), d.get("vb", 0.5), d.get("vc", 2.0), d.get("vd", 1.0),
                  d.get("eta0", 2.5))


def lb_workspace_bytes(params, prec):
    arr = (lb_params * len(params))(*params)
    return load().lb_workspace_bytes(len(params), arr, prec)


def lb_init(params, dvm, prec, rho0, ux0, uy0, T0, d_workspace, ws_bytes, hip_stream):
    lib = load()
    n = len(params)
    arr = (lb_params * n)(*params)
    keep = []

    def plist(fields):
        out = (ctypes.POINTER(ctypes.c_double) * n)()
        for k, f in enumerate(fields):
            a = np.ascontiguousarray(f, dtype=np.float64)
            keep.append(a)
            out[k] = _dptr(a)
        return out

    ctx = ctypes.c_void_p()
    st = lib.lb_init(ctypes.byref(ctx), n, arr, ctypes.byref(dvm) if dvm is not None else None, prec,
                     plist(rho0), plist(ux0), plist(uy0), plist(T0), ctypes.c_void_p(d_workspace),
                     ws_bytes, ctypes.c_void_p(hip_stream))
    _check(st)
    return ctx


def lb_step(ctx, n_steps):
    _check(load().lb_step(ctx, n_steps))


def lb_sync(ctx):
    _check(load().lb_sync(ctx))


def lb_moments(ctx, inst, shape):
    out = [np.empty(shape) for _ in range(4)]
    _check(load().lb_moments(ctx, inst, *[_dptr(a) for a in out]))
    return out


def lb_conservation(ctx, inst):
    out = np.empty(4)
    _check(load().lb_conservation(ctx, inst, _dptr(out)))
    return out


def lb_conservation_history(ctx, inst, max_entries, allow_nonfinite=False):
    """(first_step, array[n, 4]) of the per-step conservation integrals kept on the GPU.  With
    allow_nonfinite the entries are returned even if some are NaN/Inf (a run that blew up)."""
    out = np.empty((max(max_entries, 1), 4))
    n = ctypes.c_int()
    first = ctypes.c_longlong()
    st = load().lb_conservation_history(ctx, inst, max_entries, _dptr(out), ctypes.byref(n),
                                        ctypes.byref(first))
    if not (allow_nonfinite and st == LB_E_NONFINITE):
        _check(st)
    return first.value, out[: n.value].copy()


def lb_get_f(ctx, inst, shape):
    f = np.empty((16,) + tuple(shape))
    _check(load().lb_get_f(ctx, inst, _dptr(f)))
    return f


def lb_set_f(ctx, inst, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _check(load().lb_set_f(ctx, inst, _dptr(f)))


def lb_set_moments(ctx, inst, rho, ux, uy, T):
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (rho, ux, uy, T)]
    _check(load().lb_set_moments(ctx, inst, *(_dptr(x) for x in a)))


def lb_force_coefficients(ctx, inst, shape):
    out = [np.empty(shape) for _ in range(3)]
    _check(load().lb_force_coefficients(ctx, inst, *[_dptr(a) for a in out]))
    return out


def lb_rhs(ctx, inst, shape):
    R = np.empty((16,) + tuple(shape))
    _check(load().lb_rhs(ctx, inst, _dptr(R)))
    return R


def lb_derivative(ctx, inst, axis, order, g):
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.empty_like(g)
    _check(load().lb_derivative(ctx, inst, axis, order, _dptr(g), _dptr(out)))
    return out


def lb_derivative_noalloc(nx, ny, dx, prec, axis, order, d_g, d_out, hip_stream):
    """Windowed-FFT derivative of the float64 device field at address d_g ([ny][nx]) into d_out,
    with no device allocation (the library's static scratch array)."""
    lib = load()
    fn = lib.lb_derivative_noalloc
    fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    fn.restype = ctypes.c_int
    _check(fn(nx, ny, dx, prec, axis, order, ctypes.c_void_p(d_g), ctypes.c_void_p(d_out),
              ctypes.c_void_p(hip_stream)))


def lb_step_timed(ctx, n_steps):
    """Mean milliseconds per launch of each pass kind (dict keyed by PASS_NAMES)."""
    ms = np.zeros(len(PASS_NAMES))
    _check(load().lb_step_timed(ctx, n_steps, _dptr(ms)))
    return dict(zip(PASS_NAMES, ms.tolist()))


def lb_plan_info(ctx, inst):
    out = (ctypes.c_int * 5)()
    _check(load().lb_plan_info(ctx, inst, out, 5))
    return dict(pops_per_block_x=out[0], size_classes=out[1], pop_y_plan=out[2], macro_y_plan=out[3],
                pop_x_plan=out[4])


def lb_free(ctx):
    if ctx:
        load().lb_free(ctx)


class Sim:
    """A batch of instances on the current CUDA (HIP) device and stream.

    instances: list of (param_dict, (rho0, ux0, uy0, T0)) with [ny][nx] float64 arrays.
    precision: "fp64" or "fp32".
    """

    def __init__(self, instances, precision="fp64", dvm=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("lbfft needs a HIP device")
        self.prec = LB_FP64 if precision == "fp64" else LB_FP32
        self.shapes = [ic[0].shape for _, ic in instances]
        self.params = [make_params(p, ic[0].shape[1], ic[0].shape[0]) for p, ic in instances]
        self.ws_bytes = lb_workspace_bytes(self.params, self.prec)
        if self.ws_bytes == 0:
            raise LBError(LB_E_ARG, "invalid parameters or grid size")
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.stream = torch.cuda.current_stream()
        self.ctx = lb_init(self.params, make_dvm(dvm), self.prec,
                           [ic[0] for _, ic in instances], [ic[1] for _, ic in instances],
                           [ic[2] for _, ic in instances], [ic[3] for _, ic in instances],
                           self.workspace.data_ptr(), self.ws_bytes, self.stream.cuda_stream)

    def step(self, n=1):
        lb_step(self.ctx, n)

    def sync(self):
        lb_sync(self.ctx)

    def moments(self, inst=0):
        return lb_moments(self.ctx, inst, self.shapes[inst])

    def conservation(self, inst=0):
        return lb_conservation(self.ctx, inst)

    def history(self, inst=0, max_entries=1 << 20, allow_nonfinite=False):
        return lb_conservation_history(self.ctx, inst, max_entries, allow_nonfinite)

    def get_f(self, inst=0):
        return lb_get_f(self.ctx, inst, self.shapes[inst])

    def set_f(self, f, inst=0):
        lb_set_f(self.ctx, inst, f)

    def set_moments(self, rho, ux, uy, T, inst=0):
        shape = self.shapes[inst]
        a = [np.broadcast_to(np.asarray(x, dtype=np.float64), shape) for x in (rho, ux, uy, T)]
        lb_set_moments(self.ctx, inst, *a)

    def force_coefficients(self, inst=0):
        return lb_force_coefficients(self.ctx, inst, self.shapes[inst])

    def rhs(self, inst=0):
        return lb_rhs(self.ctx, inst, self.shapes[inst])

    def derivative(self, g, axis, order=1, inst=0):
        return lb_derivative(self.ctx, inst, axis, order, g)

    def step_timed(self, n):
        return lb_step_timed(self.ctx, n)

    def plan(self, inst=0):
        return lb_plan_info(self.ctx, inst)

    def close(self):
        if getattr(self, "ctx", None):
            lb_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
