"""ctypes binding of libionic_sdc.so (the C ABI in include/ionic_sdc.h).

Argument marshalling only: every step of the reaction + SDC stage runs in the
library's HIP kernels.  The functions below carry the C entry points' names
and raise IonicError on a non-zero status.  PyTorch provides device memory
(uint8 tensors for the state, float64 tensors for inputs) and streams.  The
library must be built (``__graft_entry__.build()``); without it every call
fails loudly -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

LR91, TT06_EPI, TEST_LINEAR, TEST_LOGISTIC = 1, 2, 90, 91
FP64, MIXED = 0, 1
PRED_NEWTON, PRED_ROS2, PRED_RUSH_LARSEN = 0, 1, 2
PREDICTORS = {"newton": PRED_NEWTON, "ros2": PRED_ROS2, "rush_larsen": PRED_RUSH_LARSEN}
MODEL_IDS = {"LR91": LR91, "TT06": TT06_EPI, "TEST_LINEAR": TEST_LINEAR, "TEST_LOGISTIC": TEST_LOGISTIC}
PRECISIONS = {"fp64": FP64, "mixed": MIXED}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libionic_sdc.so")


class IonicError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("ionic status %d: %s" % (status, message))
        self.status = status


class ionic_config(ctypes.Structure):
    _fields_ = [
        ("n_vertices", c_int64),
        ("model", c_int32),
        ("precision", c_int32),
        ("newton_tol", c_double),
        ("newton_maxit", c_int32),
        ("n_params", c_int32),
        ("params", POINTER(c_double)),
    ]


class ionic_stats(ctypes.Structure):
    _fields_ = [
        ("vertex_steps", c_int64),
        ("newton_iters", c_int64),
        ("newton_solves", c_int64),
        ("n_nonconverged", c_int64),
        ("n_nonfinite", c_int64),
        ("newton_it_max", c_int32),
        ("reserved", c_int32),
    ]


class ionic_adapt_result(ctypes.Structure):
    _fields_ = [
        ("t", c_double),
        ("dt_next", c_double),
        ("err_last", c_double),
        ("accepted", c_int64),
        ("rejected", c_int64),
        ("reached", c_int32),
        ("failed", c_int32),
    ]


class ionic_grid(ctypes.Structure):
    _fields_ = [("nx", c_int64), ("ny", c_int64), ("nz", c_int64), ("h", c_double),
                ("sigma", c_double)]


class ionic_bidomain_grid(ctypes.Structure):
    _fields_ = [("nx", c_int64), ("ny", c_int64), ("nz", c_int64), ("h", c_double),
                ("sigma_i", c_double * 3), ("sigma_e", c_double * 3)]


class ionic_implicit_info(ctypes.Structure):
    _fields_ = [("steps", c_int64), ("inner_passes", c_int64), ("cg_iterations", c_int64),
                ("krylov_iterations", c_int64), ("last_change", c_double),
                ("inner_max", c_int32), ("converged", c_int32), ("krylov_max", c_int32),
                ("krylov_converged", c_int32)]


class ionic_elliptic_info(ctypes.Structure):
    _fields_ = [("cg_iterations", c_int64), ("relative_residual", c_double),
                ("converged", c_int32), ("reserved", c_int32)]


def make_bidomain_grid(nx, ny=1, nz=1, h=0.01, sigma_i=(1.5e-3,) * 3, sigma_e=(1.5e-3,) * 3):
    g = ionic_bidomain_grid()
    g.nx, g.ny, g.nz, g.h = int(nx), int(ny), int(nz), float(h)
    for a in range(3):
        g.sigma_i[a] = float(sigma_i[a])
        g.sigma_e[a] = float(sigma_e[a])
    return g


def make_grid(nx, ny=1, nz=1, h=0.01, sigma=0.75e-3):
    g = ionic_grid()
    g.nx, g.ny, g.nz, g.h, g.sigma = int(nx), int(ny), int(nz), float(h), float(sigma)
    return g


_SIGNATURES = {
    "ionic_n_states": (c_int, [c_int]),
    "ionic_n_fp64_states": (c_int, [c_int]),
    "ionic_state_name": (ctypes.c_char_p, [c_int, c_int]),
    "ionic_n_params": (c_int, [c_int]),
    "ionic_param_name": (ctypes.c_char_p, [c_int, c_int]),
    "ionic_plane_stride": (c_int64, [c_int64]),
    "ionic_state_bytes": (c_size_t, [c_int, c_int, c_int64]),
    "ionic_lobatto": (c_int, [c_int, POINTER(c_double), POINTER(c_double)]),
    "ionic_init": (c_int, [POINTER(c_void_p), POINTER(ionic_config), c_void_p, c_size_t,
                           c_void_p, c_int, c_void_p]),
    "ionic_destroy": (None, [c_void_p]),
    "reaction_sdc_step": (c_int, [c_void_p, c_double, c_double, c_int, c_int, c_int, c_void_p,
                                  c_double, c_double, c_void_p, c_void_p]),
    "ionic_set_predictor": (c_int, [c_void_p, c_int]),
    "ionic_set_vertex_order": (c_int, [c_void_p, c_void_p, c_int64]),
    "reaction_sdc_adaptive": (c_int, [c_void_p, c_double, c_double, c_double, c_double, c_double,
                                      c_int, c_int, c_void_p, c_double, c_double, c_void_p,
                                      c_void_p, c_size_t, c_int64, c_void_p,
                                      POINTER(ionic_adapt_result), c_void_p]),
    "ionic_diffusion_current": (c_int, [c_void_p, POINTER(ionic_grid), c_void_p, c_void_p]),
    "reaction_diffusion_step": (c_int, [c_void_p, POINTER(ionic_grid), c_double, c_double, c_int,
                                        c_int, c_int, c_void_p, c_double, c_double, c_void_p,
                                        c_void_p]),
    "ionic_multigrid_levels": (c_int, [c_int64, c_int64, c_int64]),
    "ionic_elliptic_work_bytes": (c_size_t, [c_int64, c_int64, c_int64, c_int]),
    "ionic_elliptic_solve": (c_int, [c_void_p, POINTER(ionic_bidomain_grid), c_void_p, c_void_p,
                                     c_size_t, c_double, c_int, POINTER(ionic_elliptic_info),
                                     c_void_p]),
    "reaction_bidomain_step": (c_int, [c_void_p, POINTER(ionic_bidomain_grid), c_double, c_double,
                                       c_int, c_int, c_int, c_void_p, c_double, c_double,
                                       c_void_p, c_void_p, c_size_t, c_double, c_int, c_void_p,
                                       POINTER(ionic_elliptic_info), c_void_p]),
    "ionic_implicit_work_bytes": (c_size_t, [c_int, c_int64, c_int64, c_int64, c_int]),
    "reaction_bidomain_implicit_step": (c_int, [c_void_p, POINTER(ionic_bidomain_grid), c_double,
                                                c_double, c_int, c_void_p, c_double, c_double,
                                                c_void_p, c_void_p, c_size_t, c_double, c_double,
                                                c_double, c_int, c_int,
                                                POINTER(ionic_implicit_info), c_void_p]),
    "ionic_set_inputs": (c_int, [c_void_p, c_double, c_double, c_int, c_int, c_void_p, c_double,
                                 c_double, c_void_p]),
    "reaction_sdc_step_batch": (c_int, [POINTER(c_void_p), POINTER(c_int), c_int, c_void_p]),
    "state_readback": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_int, c_void_p]),
    "state_readback_noalloc": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_void_p]),
    "ionic_gates_to_steady_state": (c_int, [c_void_p, c_void_p]),
    "ionic_get_stats": (c_int, [c_void_p, POINTER(ionic_stats)]),
    "ionic_reset_stats": (c_int, [c_void_p]),
    "ionic_debug_jacobian": (c_int, [c_void_p, c_int64, c_double, c_double, POINTER(c_double),
                                     POINTER(c_double), c_void_p]),
    "ionic_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("%s is missing: build it with __graft_entry__.build()" % LIB_PATH)
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(status):
    if status != 0:
        raise IonicError(status, lib().ionic_last_error().decode())
    return status


def _ptr(x):
    """Device/host address of a torch tensor, an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---- entry points with the C names -------------------------------------------------
def ionic_n_states(model):
    n = lib().ionic_n_states(model)
    if n < 0:
        _check(n)
    return n


def ionic_n_fp64_states(model):
    n = lib().ionic_n_fp64_states(model)
    if n < 0:
        _check(n)
    return n


def ionic_state_name(model, idx):
    s = lib().ionic_state_name(model, idx)
    return None if s is None else s.decode()


def ionic_n_params(model):
    n = lib().ionic_n_params(model)
    if n < 0:
        _check(n)
    return n


def ionic_param_name(model, idx):
    s = lib().ionic_param_name(model, idx)
    return None if s is None else s.decode()


def ionic_plane_stride(n):
    return lib().ionic_plane_stride(n)


def ionic_state_bytes(model, precision, n):
    return lib().ionic_state_bytes(model, precision, n)


def ionic_lobatto(n_nodes):
    c = (c_double * n_nodes)()
    S = (c_double * ((n_nodes - 1) * n_nodes))()
    _check(lib().ionic_lobatto(n_nodes, c, S))
    return np.array(c[:]), np.array(S[:]).reshape(n_nodes - 1, n_nodes)


def make_config(model, n_vertices, precision=FP64, newton_tol=1e-10, newton_maxit=10, params=None):
    cfg = ionic_config()
    cfg.n_vertices = int(n_vertices)
    cfg.model = int(model)
    cfg.precision = int(precision)
    cfg.newton_tol = float(newton_tol)
    cfg.newton_maxit = int(newton_maxit)
    if params is not None and len(params) > 0:
        arr = (c_double * len(params))(*[float(p) for p in params])
        cfg.n_params = len(params)
        cfg.params = ctypes.cast(arr, POINTER(c_double))
        cfg._keep = arr
    else:
        cfg.n_params = 0
        cfg.params = None
    return cfg


def ionic_init(cfg, state_ptr, state_bytes, x0, x0_on_device=False, stream=None):
    """Returns the opaque handle (an int).  x0: host numpy (n, N) float64, a device
    address / tensor (x0_on_device=True), or None for the model's resting state."""
    h = c_void_p()
    if x0 is None:
        x0p = None
        keep = None
    elif x0_on_device:
        x0p = _ptr(x0)
        keep = None
    else:
        keep = np.ascontiguousarray(x0, dtype=np.float64)
        x0p = keep.ctypes.data
    _check(lib().ionic_init(ctypes.byref(h), ctypes.byref(cfg), state_ptr, state_bytes, x0p,
                            1 if x0_on_device else 0, _stream(stream)))
    del keep
    return h.value


def ionic_destroy(handle):
    lib().ionic_destroy(handle)


def reaction_sdc_step(handle, t0, dt, n_steps, n_nodes, n_sweeps, i_stim=None, stim_t_on=0.0,
                      stim_t_off=0.0, i_diff=None, stream=None):
    _check(lib().reaction_sdc_step(handle, t0, dt, n_steps, n_nodes, n_sweeps, _ptr(i_stim),
                                   stim_t_on, stim_t_off, _ptr(i_diff), _stream(stream)))


def ionic_set_predictor(handle, predictor):
    _check(lib().ionic_set_predictor(handle, PREDICTORS.get(predictor, predictor)))


def ionic_set_vertex_order(handle, order, n):
    """order: a device int32 tensor holding a permutation of range(n), kept alive
    by the caller while the handle steps, or None for the identity order."""
    import torch
    if order is None:
        _check(lib().ionic_set_vertex_order(handle, None, 0))
        return
    if order.dtype != torch.int32 or not order.is_cuda or not order.is_contiguous():
        raise ValueError("order must be a contiguous int32 device tensor")
    _check(lib().ionic_set_vertex_order(handle, c_void_p(order.data_ptr()), int(order.numel())))


def reaction_sdc_adaptive(handle, t0, t_end, dt_init, dt_max, err_tol, n_nodes, n_sweeps,
                          work, work_bytes, max_attempts, i_stim=None, stim_t_on=0.0,
                          stim_t_off=0.0, i_diff=None, history=None, stream=None):
    """Returns the ionic_adapt_result fields as a dict (synchronises the stream)."""
    out = ionic_adapt_result()
    _check(lib().reaction_sdc_adaptive(handle, t0, t_end, dt_init, dt_max, err_tol, n_nodes,
                                       n_sweeps, _ptr(i_stim), stim_t_on, stim_t_off, _ptr(i_diff),
                                       _ptr(work), work_bytes, int(max_attempts), _ptr(history),
                                       ctypes.byref(out), _stream(stream)))
    return {name: getattr(out, name) for name, _ in ionic_adapt_result._fields_}


def ionic_diffusion_current(handle, grid, out, stream=None):
    _check(lib().ionic_diffusion_current(handle, ctypes.byref(grid), _ptr(out), _stream(stream)))
    return out


def reaction_diffusion_step(handle, grid, t0, dt, n_steps, n_nodes, n_sweeps, work, i_stim=None,
                            stim_t_on=0.0, stim_t_off=0.0, stream=None):
    _check(lib().reaction_diffusion_step(handle, ctypes.byref(grid), t0, dt, n_steps, n_nodes,
                                         n_sweeps, _ptr(i_stim), stim_t_on, stim_t_off, _ptr(work),
                                         _stream(stream)))


def ionic_multigrid_levels(nx, ny, nz):
    n = lib().ionic_multigrid_levels(nx, ny, nz)
    if n < 0:
        _check(n)
    return n


def ionic_elliptic_work_bytes(nx, ny, nz, max_iter):
    return lib().ionic_elliptic_work_bytes(nx, ny, nz, max_iter)


def _info_dict(info):
    return {name: getattr(info, name) for name, _ in ionic_elliptic_info._fields_
            if name != "reserved"}


def ionic_elliptic_solve(handle, grid, u, work, work_bytes, rtol=1e-8, max_iter=1000,
                         stream=None):
    info = ionic_elliptic_info()
    _check(lib().ionic_elliptic_solve(handle, ctypes.byref(grid), _ptr(u), _ptr(work), work_bytes,
                                      rtol, max_iter, ctypes.byref(info), _stream(stream)))
    return _info_dict(info)


def reaction_bidomain_step(handle, grid, t0, dt, n_steps, n_nodes, n_sweeps, u, work, work_bytes,
                           i_diff_work, i_stim=None, stim_t_on=0.0, stim_t_off=0.0, rtol=1e-8,
                           max_iter=1000, stream=None):
    info = ionic_elliptic_info()
    _check(lib().reaction_bidomain_step(handle, ctypes.byref(grid), t0, dt, n_steps, n_nodes,
                                        n_sweeps, _ptr(i_stim), stim_t_on, stim_t_off, _ptr(u),
                                        _ptr(work), work_bytes, rtol, max_iter, _ptr(i_diff_work),
                                        ctypes.byref(info), _stream(stream)))
    return _info_dict(info)


def ionic_implicit_work_bytes(model, nx, ny, nz, max_iter):
    return lib().ionic_implicit_work_bytes(MODEL_IDS.get(model, model), nx, ny, nz, max_iter)


def reaction_bidomain_implicit_step(handle, grid, t0, dt, n_steps, u, work, work_bytes,
                                    i_stim=None, stim_t_on=0.0, stim_t_off=0.0,
                                    elliptic_rtol=1e-10, krylov_rtol=1e-10, inner_tol=1e-8,
                                    max_inner=30, max_iter=1000, stream=None):
    info = ionic_implicit_info()
    _check(lib().reaction_bidomain_implicit_step(handle, ctypes.byref(grid), t0, dt, n_steps,
                                                 _ptr(i_stim), stim_t_on, stim_t_off, _ptr(u),
                                                 _ptr(work), work_bytes, elliptic_rtol, krylov_rtol,
                                                 inner_tol, max_inner, max_iter,
                                                 ctypes.byref(info), _stream(stream)))
    return {name: getattr(info, name) for name, _ in ionic_implicit_info._fields_}


def ionic_set_inputs(handle, t0, dt, n_nodes, n_sweeps, i_stim=None, stim_t_on=0.0,
                     stim_t_off=0.0, i_diff=None):
    _check(lib().ionic_set_inputs(handle, t0, dt, n_nodes, n_sweeps, _ptr(i_stim), stim_t_on,
                                  stim_t_off, _ptr(i_diff)))


def reaction_sdc_step_batch(handles, n_steps, stream=None):
    n = len(handles)
    hs = (c_void_p * n)(*handles)
    ns = (c_int * n)(*[int(k) for k in n_steps])
    _check(lib().reaction_sdc_step_batch(hs, ns, n, _stream(stream)))


def state_readback(handle, n_states, first, count, out=None, stream=None):
    """Returns a host (n_states, count) float64 array, or fills a device tensor `out`."""
    if out is not None:
        _check(lib().state_readback(handle, _ptr(out), first, count, 1, _stream(stream)))
        return out
    host = np.empty((n_states, count), dtype=np.float64)
    _check(lib().state_readback(handle, host.ctypes.data, first, count, 0, _stream(stream)))
    return host


def state_readback_noalloc(handle, n_states, first, count, stream=None):
    """Host (n_states, count) float64 array, staged through the library's
    static device buffer (no allocation; at most 8 MiB per call)."""
    host = np.empty((n_states, count), dtype=np.float64)
    _check(lib().state_readback_noalloc(handle, host.ctypes.data, first, count, _stream(stream)))
    return host


def ionic_gates_to_steady_state(handle, stream=None):
    _check(lib().ionic_gates_to_steady_state(handle, _stream(stream)))


def ionic_get_stats(handle):
    st = ionic_stats()
    _check(lib().ionic_get_stats(handle, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in ionic_stats._fields_ if name != "reserved"}


def ionic_reset_stats(handle):
    _check(lib().ionic_reset_stats(handle))


def ionic_debug_jacobian(handle, n_states, vertex, i_stim=0.0, i_diff=0.0, stream=None):
    F = (c_double * n_states)()
    J = (c_double * (n_states * n_states))()
    _check(lib().ionic_debug_jacobian(handle, vertex, i_stim, i_diff, F, J, _stream(stream)))
    return np.array(F[:]), np.array(J[:]).reshape(n_states, n_states)


# ---- convenience wrapper ----------------------------------------------------------------
class Simulation:
    """One simulation: a device state buffer (torch uint8 tensor) plus its handle."""

    def __init__(self, model, x0, precision=FP64, newton_tol=1e-10, newton_maxit=10, params=None,
                 stream=None, device="cuda", n_vertices=None):
        """x0: host (n_states, N) array, a device float64 tensor of that shape
        (converted on the GPU, asynchronously), or None with n_vertices for the
        model's resting state."""
        import torch
        model = MODEL_IDS.get(model, model)
        precision = PRECISIONS.get(precision, precision)
        self.model, self.precision = model, precision
        self.n_states = ionic_n_states(model)
        on_device = isinstance(x0, torch.Tensor) and x0.is_cuda
        if x0 is None:
            if n_vertices is None:
                raise ValueError("x0 = None needs n_vertices")
            self.n = int(n_vertices)
        else:
            if on_device:
                if x0.dtype != torch.float64 or not x0.is_contiguous():
                    raise ValueError("a device x0 must be a contiguous float64 tensor")
            else:
                x0 = np.asarray(x0, dtype=np.float64)
            if x0.ndim != 2 or x0.shape[0] != self.n_states:
                raise ValueError("x0 must have shape (%d, N)" % self.n_states)
            self.n = int(x0.shape[1])
        nbytes = ionic_state_bytes(model, precision, self.n)
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.config = make_config(model, self.n, precision, newton_tol, newton_maxit, params)
        self._x0_keep = x0 if on_device else None  # alive until the conversion has run
        self.handle = ionic_init(self.config, self.state.data_ptr(), nbytes, x0, on_device, stream)

    def step(self, t0, dt, n_steps, n_nodes, n_sweeps, i_stim=None, stim_t_on=0.0, stim_t_off=0.0,
             i_diff=None, stream=None):
        reaction_sdc_step(self.handle, t0, dt, n_steps, n_nodes, n_sweeps, i_stim, stim_t_on,
                          stim_t_off, i_diff, stream)

    def set_predictor(self, predictor):
        ionic_set_predictor(self.handle, predictor)

    def set_vertex_order(self, order):
        """order: a permutation of range(n) (numpy or device tensor) or None."""
        import torch
        if order is None:
            self._order = None
            ionic_set_vertex_order(self.handle, None, 0)
            return
        t = torch.as_tensor(np.ascontiguousarray(order, dtype=np.int32)).cuda() \
            if not isinstance(order, torch.Tensor) else order
        ionic_set_vertex_order(self.handle, t, self.n)
        self._order = t   # the library reads it on every later launch

    def adaptive(self, t0, t_end, dt_init, dt_max, err_tol, n_nodes=2, n_sweeps=1, i_stim=None,
                 stim_t_on=0.0, stim_t_off=0.0, i_diff=None, max_attempts=100000,
                 history=False, stream=None):
        """Adaptive run from t0 to t_end (ROS2 predictor).  Returns the result
        dict; with history=True also the (attempts, 4) array of (t, tau, err,
        accepted) rows."""
        import torch
        nbytes = ionic_state_bytes(self.model, self.precision, self.n)
        if getattr(self, "_work", None) is None or self._work.numel() < nbytes:
            self._work = torch.empty(nbytes, dtype=torch.uint8, device=self.state.device)
        hist = (torch.zeros((int(max_attempts), 4), dtype=torch.float64, device=self.state.device)
                if history else None)
        res = reaction_sdc_adaptive(self.handle, t0, t_end, dt_init, dt_max, err_tol, n_nodes,
                                    n_sweeps, self._work, nbytes, max_attempts, i_stim, stim_t_on,
                                    stim_t_off, i_diff, hist, stream)
        if history:
            n = res["accepted"] + res["rejected"]
            return res, hist[:n].cpu().numpy()
        return res

    def readback(self, first=0, count=None, stream=None):
        count = self.n - first if count is None else count
        return state_readback(self.handle, self.n_states, first, count, stream=stream)

    def stats(self):
        return ionic_get_stats(self.handle)

    def debug_jacobian(self, vertex, i_stim=0.0, i_diff=0.0):
        return ionic_debug_jacobian(self.handle, self.n_states, vertex, i_stim, i_diff)

    def close(self):
        if getattr(self, "handle", None):
            ionic_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
