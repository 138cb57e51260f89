"""Python binding of libfpn (include/fpn.h): argument marshalling only.

Every step of the solver runs in the library's HIP kernels; PyTorch is used here
for device memory and streams.  Importing this package fails loudly when the
compiled library is missing (build it with ``python paper_2106_08040_amd/build.py``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FPN_LIB") or os.path.join(_HERE, "libfpn.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libfpn.so not built at {LIB_PATH}; run `python paper_2106_08040_amd/build.py`")

# PyTorch's HIP runtime must be the one in the process before libfpn is loaded, so that the
# library binds to it (same SONAME) instead of loading a second HIP/HSA runtime.
try:
    import torch as _torch_mod  # noqa: F401
except ImportError:  # host-only helpers still work without torch
    _torch_mod = None

_lib = ctypes.CDLL(LIB_PATH)

FPN_OK, FPN_E_ARG, FPN_E_RANGE, FPN_E_DEVICE, FPN_E_NOMEM, FPN_E_UNSUPPORTED, FPN_E_IO = 0, -1, -2, -3, -4, -7, -8
FPN_INST_OK, FPN_INST_BAD_PARAM, FPN_INST_NONFINITE, FPN_INST_SINGULAR, FPN_INST_UNRESOLVED, FPN_INST_TOL_UNMET = \
    0, 1, 2, 3, 4, 5
FPN_OUT_M, FPN_OUT_HARM, FPN_HARM_Z, FPN_OUT_DMDT = 1, 2, 4, 8
FPN_MAX_L = 24
FPN_STATIC_MAX_N, FPN_STATIC_MAX_NS = 128, 2048
FPN_NPARAM = 5  # sensitivities: D, K, alpha, easy-axis polar angle, azimuth

EXPORTED = ["fpn_status_string", "fpn_last_error", "fpn_create", "fpn_destroy", "fpn_solve",
            "fpn_stationary", "fpn_truncation_estimate", "fpn_select_degree", "fpn_last_steps", "fpn_timing_enable", "fpn_timing_read", "fpn_host_operator", "fpn_host_frame",
            "fpn_host_table_nnz", "fpn_mlp_create", "fpn_mlp_destroy", "fpn_mlp_num_params", "fpn_mlp_params",
            "fpn_mlp_set_input_norm", "fpn_mlp_forward", "fpn_mlp_gradient", "fpn_mlp_train_step",
            "fpn_surrogate_features", "fpn_surrogate_predict", "fpn_plan_create", "fpn_plan_launch",
            "fpn_plan_graph_launch", "fpn_plan_steps", "fpn_plan_destroy", "fpn_solve_tangent", "fpn_adjoint",
            "fpn_stepper_wave_options", "fpn_set_stepper_waves", "fpn_autotune", "fpn_equilibrium",
            "fpn_solve_static", "fpn_mlp_shape", "fpn_surrogate_init", "fpn_surrogate_create", "fpn_surrogate_save",
            "fpn_surrogate_destroy", "fpn_surrogate_member", "fpn_surrogate_set_scales", "fpn_surrogate_view",
            "fpn_surrogate_infer", "fpn_surrogate_train_step", "fpn_fit_rows", "fpn_nrmse_global",
            "fpn_mixing_order", "fpn_frequency_index_set", "fpn_m2_system", "fpn_m2_weights", "fpn_m2_model",
            "fpn_rows_error", "fpn_surrogate_add_residual", "fpn_surrogate_set_residual_scale"]


class fpn_drive(ctypes.Structure):
    _fields_ = [("amp", ctypes.c_double * 3), ("freq", ctypes.c_double * 3),
                ("phase", ctypes.c_double * 3), ("period", ctypes.c_double)]


class fpn_solve_opts(ctypes.Structure):
    _fields_ = [("samples_per_period", ctypes.c_int32), ("settle_periods", ctypes.c_int32),
                ("n_harm", ctypes.c_int32), ("substeps", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("tol", ctypes.c_double)]


class fpn_batch(ctypes.Structure):
    _fields_ = [("D", ctypes.c_void_p), ("Ms", ctypes.c_void_p), ("K", ctypes.c_void_p),
                ("alpha", ctypes.c_void_p), ("temp", ctypes.c_void_p), ("easy_axis", ctypes.c_void_p),
                ("offset", ctypes.c_void_p), ("L", ctypes.POINTER(ctypes.c_int32))]


_vp = ctypes.c_void_p
_lib.fpn_status_string.restype = ctypes.c_char_p
_lib.fpn_status_string.argtypes = [ctypes.c_int32]
_lib.fpn_last_error.restype = ctypes.c_char_p
_lib.fpn_last_error.argtypes = []
_lib.fpn_create.restype = ctypes.c_int32
_lib.fpn_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int]
_lib.fpn_destroy.restype = ctypes.c_int32
_lib.fpn_destroy.argtypes = [_vp]
_lib.fpn_solve.restype = ctypes.c_int32
_lib.fpn_solve.argtypes = [_vp, ctypes.POINTER(fpn_drive), ctypes.POINTER(fpn_solve_opts),
                           ctypes.POINTER(fpn_batch), ctypes.c_int64, _vp, _vp, _vp, _vp, _vp]
_lib.fpn_solve_static.restype = ctypes.c_int32
_lib.fpn_solve_static.argtypes = [_vp, ctypes.POINTER(fpn_drive), ctypes.POINTER(fpn_solve_opts),
                                  ctypes.POINTER(fpn_batch), ctypes.c_int64, _vp, _vp, _vp, _vp]
_lib.fpn_equilibrium.restype = ctypes.c_int32
_lib.fpn_equilibrium.argtypes = [_vp, ctypes.POINTER(fpn_drive), ctypes.POINTER(fpn_solve_opts),
                                 ctypes.POINTER(fpn_batch), ctypes.c_int64, _vp, _vp, _vp, _vp]
_lib.fpn_stationary.restype = ctypes.c_int32
_lib.fpn_stationary.argtypes = [_vp, ctypes.POINTER(fpn_batch), ctypes.c_int64, _vp, _vp, _vp, _vp]
_lib.fpn_select_degree.restype = ctypes.c_int32
_lib.fpn_select_degree.argtypes = [_vp, ctypes.POINTER(fpn_batch), ctypes.c_int64, ctypes.POINTER(fpn_drive),
                                   ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _vp, _vp, _vp, _vp]
_lib.fpn_truncation_estimate.restype = ctypes.c_int32
_lib.fpn_truncation_estimate.argtypes = [_vp, ctypes.POINTER(fpn_batch), ctypes.c_int64, ctypes.POINTER(fpn_drive),
                                         ctypes.c_int32, _vp, _vp, _vp]
_lib.fpn_last_steps.restype = ctypes.c_int32
_lib.fpn_last_steps.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
_lib.fpn_timing_enable.restype = ctypes.c_int32
_lib.fpn_timing_enable.argtypes = [_vp, ctypes.c_int]
_lib.fpn_timing_read.restype = ctypes.c_int32
_lib.fpn_timing_read.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
_lib.fpn_host_operator.restype = ctypes.c_int32
_lib.fpn_host_operator.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
_lib.fpn_host_frame.restype = ctypes.c_int32
_lib.fpn_host_frame.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.fpn_host_table_nnz.restype = ctypes.c_int64
_lib.fpn_host_table_nnz.argtypes = [ctypes.c_int32]
_lib.fpn_mlp_create.restype = ctypes.c_int32
_lib.fpn_mlp_create.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_uint64,
                                ctypes.POINTER(_vp)]
_lib.fpn_mlp_destroy.restype = ctypes.c_int32
_lib.fpn_mlp_destroy.argtypes = [_vp]
_lib.fpn_mlp_num_params.restype = ctypes.c_int64
_lib.fpn_mlp_num_params.argtypes = [_vp]
_lib.fpn_mlp_params.restype = ctypes.c_int32
_lib.fpn_mlp_params.argtypes = [_vp, _vp, _vp, _vp]
_lib.fpn_mlp_set_input_norm.restype = ctypes.c_int32
_lib.fpn_mlp_set_input_norm.argtypes = [_vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
_lib.fpn_mlp_shape.restype = ctypes.c_int32
_lib.fpn_mlp_shape.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
_lib.fpn_mlp_forward.restype = ctypes.c_int32
_lib.fpn_mlp_forward.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp]
_lib.fpn_mlp_gradient.restype = ctypes.c_int32
_lib.fpn_mlp_gradient.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp, _vp]
_lib.fpn_mlp_train_step.restype = ctypes.c_int32
_lib.fpn_mlp_train_step.argtypes = [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_float, _vp, _vp]


_lib.fpn_solve_tangent.restype = ctypes.c_int32
_lib.fpn_solve_tangent.argtypes = [_vp, ctypes.POINTER(fpn_drive), ctypes.POINTER(fpn_solve_opts),
                                   ctypes.POINTER(fpn_batch), ctypes.c_int64, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.fpn_adjoint.restype = ctypes.c_int32
_lib.fpn_adjoint.argtypes = [_vp, ctypes.POINTER(fpn_drive), ctypes.POINTER(fpn_solve_opts),
                             ctypes.POINTER(fpn_batch), ctypes.c_int64, _vp, _vp, _vp, _vp, _vp]
_lib.fpn_stepper_wave_options.restype = ctypes.c_int32
_lib.fpn_stepper_wave_options.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
_lib.fpn_set_stepper_waves.restype = ctypes.c_int32
_lib.fpn_set_stepper_waves.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32]
_lib.fpn_autotune.restype = ctypes.c_int32
_lib.fpn_autotune.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
_lib.fpn_plan_create.restype = ctypes.c_int32
_lib.fpn_plan_create.argtypes = [_vp, ctypes.POINTER(fpn_drive), ctypes.POINTER(fpn_solve_opts),
                                 ctypes.POINTER(fpn_batch), ctypes.c_int64, ctypes.POINTER(ctypes.c_float), _vp, _vp,
                                 _vp, ctypes.POINTER(_vp)]
_lib.fpn_plan_launch.restype = ctypes.c_int32
_lib.fpn_plan_launch.argtypes = [_vp, _vp]
_lib.fpn_plan_graph_launch.restype = ctypes.c_int32
_lib.fpn_plan_graph_launch.argtypes = [_vp, _vp]
_lib.fpn_plan_steps.restype = ctypes.c_int32
_lib.fpn_plan_steps.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32)]
_lib.fpn_plan_destroy.restype = ctypes.c_int32
_lib.fpn_plan_destroy.argtypes = [_vp]


class fpn_surrogate(ctypes.Structure):
    _fields_ = [("net", _vp * 2), ("out_scale", ctypes.c_float), ("err_calib", ctypes.c_float),
                ("res", _vp * 2), ("res_scale", ctypes.c_float)]


_lib.fpn_surrogate_features.restype = ctypes.c_int32
_lib.fpn_surrogate_features.argtypes = [_vp, ctypes.POINTER(fpn_batch), ctypes.c_int64, _vp, _vp, _vp]
_lib.fpn_surrogate_init.restype = ctypes.c_int32
_lib.fpn_surrogate_init.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint64),
                                    ctypes.POINTER(_vp)]
_lib.fpn_surrogate_create.restype = ctypes.c_int32
_lib.fpn_surrogate_create.argtypes = [_vp, ctypes.c_char_p, ctypes.POINTER(_vp)]
_lib.fpn_surrogate_save.restype = ctypes.c_int32
_lib.fpn_surrogate_save.argtypes = [_vp, ctypes.c_char_p]
_lib.fpn_surrogate_destroy.restype = ctypes.c_int32
_lib.fpn_surrogate_destroy.argtypes = [_vp]
_lib.fpn_surrogate_member.restype = ctypes.c_int32
_lib.fpn_surrogate_member.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(_vp)]
_lib.fpn_surrogate_add_residual.restype = ctypes.c_int32
_lib.fpn_surrogate_add_residual.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_uint64)]
_lib.fpn_surrogate_set_residual_scale.restype = ctypes.c_int32
_lib.fpn_surrogate_set_residual_scale.argtypes = [_vp, ctypes.c_float]
_lib.fpn_surrogate_set_scales.restype = ctypes.c_int32
_lib.fpn_surrogate_set_scales.argtypes = [_vp, ctypes.c_float, ctypes.c_float]
_lib.fpn_surrogate_view.restype = ctypes.c_int32
_lib.fpn_surrogate_view.argtypes = [_vp, ctypes.POINTER(fpn_surrogate)]
_lib.fpn_surrogate_infer.restype = ctypes.c_int32
_lib.fpn_surrogate_infer.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp, _vp]
_lib.fpn_surrogate_train_step.restype = ctypes.c_int32
_lib.fpn_surrogate_train_step.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_float, _vp, _vp]
_lib.fpn_fit_rows.restype = ctypes.c_int32
_lib.fpn_fit_rows.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _vp, _vp,
                              _vp, _vp, _vp]
_lib.fpn_nrmse_global.restype = ctypes.c_int32
_lib.fpn_nrmse_global.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp,
                                  ctypes.c_int32, _vp, _vp, _vp]
_lib.fpn_m2_system.restype = ctypes.c_int32
_lib.fpn_m2_system.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp, _vp, _vp]
_lib.fpn_m2_weights.restype = ctypes.c_int32
_lib.fpn_m2_weights.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_int32)]
_lib.fpn_m2_model.restype = ctypes.c_int32
_lib.fpn_m2_model.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_int32, _vp, _vp]
_lib.fpn_rows_error.restype = ctypes.c_int32
_lib.fpn_rows_error.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _vp, _vp]
_lib.fpn_mixing_order.restype = ctypes.c_int32
_lib.fpn_mixing_order.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32)]
_lib.fpn_frequency_index_set.restype = ctypes.c_int32
_lib.fpn_frequency_index_set.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
_lib.fpn_surrogate_predict.restype = ctypes.c_int32
_lib.fpn_surrogate_predict.argtypes = [_vp, ctypes.POINTER(fpn_surrogate), ctypes.c_double, ctypes.POINTER(fpn_drive),
                                       ctypes.POINTER(fpn_solve_opts), ctypes.POINTER(fpn_batch), ctypes.c_int64,
                                       _vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_int64), _vp]


class FpnError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.fpn_status_string(code).decode()
        detail = _lib.fpn_last_error().decode()
        super().__init__(f"{where}: {msg} ({code}): {detail}")
        self.code = code


def _check(code, where):
    if code != FPN_OK:
        raise FpnError(code, where)


def fpn_status_string(code):
    return _lib.fpn_status_string(code).decode()


def fpn_last_error():
    return _lib.fpn_last_error().decode()


# ------------------------------------------------------------------ host helpers ---

def fpn_host_operator(L, D, Ms, K, alpha, T, field_easy):
    """Dense Galerkin operator (1/s, SH order) built from the library's tables."""
    N = (L + 1) ** 2
    A = np.zeros((N, N), dtype=np.float64)
    f = (ctypes.c_double * 3)(*[float(x) for x in field_easy])
    _check(_lib.fpn_host_operator(int(L), D, Ms, K, alpha, T, f,
                                  A.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "fpn_host_operator")
    return A


def fpn_host_frame(n):
    R = np.zeros(9, dtype=np.float64)
    nn = (ctypes.c_double * 3)(*[float(x) for x in n])
    _check(_lib.fpn_host_frame(nn, R.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "fpn_host_frame")
    return R.reshape(3, 3)


def fpn_host_table_nnz(L):
    return int(_lib.fpn_host_table_nnz(int(L)))


# ------------------------------------------------------------------ device calls ---

def fpn_stepper_wave_options(L):
    """Workgroup sizes (instances per workgroup) compiled for degree L (fpn_stepper_wave_options)."""
    w = (ctypes.c_int32 * 3)()
    c = ctypes.c_int32()
    _check(_lib.fpn_stepper_wave_options(int(L), w, ctypes.byref(c)), "fpn_stepper_wave_options")
    return [int(w[k]) for k in range(c.value)]


def mixing_order(k, n_dens=16):
    """fpn_mixing_order: (mx, my) of bin k (Eq. mix)."""
    mx, my = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.fpn_mixing_order(int(k), int(n_dens), ctypes.byref(mx), ctypes.byref(my)), "fpn_mixing_order")
    return mx.value, my.value


def frequency_index_set(Mx, My, n_dens=16):
    """fpn_frequency_index_set: the graded bins I_freq as an int32 array."""
    c = ctypes.c_int32()
    out = (ctypes.c_int32 * ((Mx + 1) * (My + 1)))()
    _check(_lib.fpn_frequency_index_set(int(Mx), int(My), int(n_dens), out, ctypes.byref(c)), "fpn_frequency_index_set")
    return np.array(out[:c.value], dtype=np.int32)


def m2_weights(G, b, yy, s=0):
    """fpn_m2_weights (host): G [J, J] and b [J] complex (numpy), yy float; returns
    (w [J], ||M w - y||^2, truncated objective, singular values kept)."""
    G = np.ascontiguousarray(np.asarray(G, dtype=np.complex128))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.complex128))
    J = b.size
    w = np.zeros(J)
    full, red, rank = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    pd = ctypes.POINTER(ctypes.c_double)
    _check(_lib.fpn_m2_weights(J, G.view(np.float64).ctypes.data_as(pd), b.view(np.float64).ctypes.data_as(pd),
                               float(yy), int(s), w.ctypes.data_as(pd), ctypes.byref(full), ctypes.byref(red),
                               ctypes.byref(rank)), "fpn_m2_weights")
    return w, full.value, red.value, rank.value


def _torch():
    import torch
    return torch


def _dev_f64(x, device):
    torch = _torch()
    t = torch.as_tensor(x, dtype=torch.float64, device=device)
    return t.contiguous()


def make_drive(amp, freq, period, phase=(0.0, 0.0, 0.0)):
    d = fpn_drive()
    d.amp[:] = [float(a) for a in amp]
    d.freq[:] = [float(f) for f in freq]
    d.phase[:] = [float(p) for p in phase]
    d.period = float(period)
    return d


class Context:
    """Owns an fpn context on one HIP device (tables, drive tables, workspace)."""

    def __init__(self, device=0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the fpn library needs an MI355X (gfx950)")
        self.device = device
        self._h = _vp()
        torch.cuda.set_device(device)
        _check(_lib.fpn_create(ctypes.byref(self._h), int(device)), "fpn_create")

    def close(self):
        if self._h:
            _lib.fpn_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _batch(self, inst, L):
        """inst: dict of D, Ms, K, alpha, T, easy_axis [n,3], offset [n,3]; kept alive by the caller."""
        dev = f"cuda:{self.device}"
        t = {k: _dev_f64(inst[k], dev) for k in ("D", "Ms", "K", "alpha", "T", "easy_axis")}
        t["offset"] = _dev_f64(inst["offset"], dev) if inst.get("offset") is not None else None
        Lh = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.int32), (t["D"].numel(),)))
        b = fpn_batch(t["D"].data_ptr(), t["Ms"].data_ptr(), t["K"].data_ptr(), t["alpha"].data_ptr(),
                      t["T"].data_ptr(), t["easy_axis"].data_ptr(),
                      t["offset"].data_ptr() if t["offset"] is not None else None,
                      Lh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        return b, t, Lh

    def solve(self, inst, L, drive, samples, settle, n_harm, substeps=0, want_m=True, want_harm=True,
              harm_z=False, stream=None, out=None, tol=0.0, want_dmdt=False):
        """Run fpn_solve.  Returns (m [n,3,Ns] float32, harm [n,ch,Kh+1] complex64, status [n] int32)
        as torch tensors on the device (None for outputs not requested), and dm/dt [n,3,Ns] float32
        as a fourth element when want_dmdt is set."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        b, keep, Lh = self._batch(inst, L)
        n = keep["D"].numel()
        ch = 3 if harm_z else 2
        if out is None:
            out = {}
        m = out.get("m") if want_m else None
        if want_m and m is None:
            m = torch.empty((n, 3, samples), dtype=torch.float32, device=dev)
        hm = out.get("harm") if want_harm else None
        if want_harm and hm is None:
            hm = torch.empty((n, ch, n_harm + 1, 2), dtype=torch.float32, device=dev)
        st = out.get("status")
        if st is None:
            st = torch.empty((n,), dtype=torch.int32, device=dev)
        dd = out.get("dmdt") if want_dmdt else None
        if want_dmdt and dd is None:
            dd = torch.empty((n, 3, samples), dtype=torch.float32, device=dev)
        opts = fpn_solve_opts(samples, settle, n_harm, substeps,
                              (FPN_OUT_M if want_m else 0) | (FPN_OUT_HARM if want_harm else 0) |
                              (FPN_HARM_Z if harm_z else 0) | (FPN_OUT_DMDT if want_dmdt else 0), float(tol))
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        code = _lib.fpn_solve(self._h, ctypes.byref(drive), ctypes.byref(opts), ctypes.byref(b), n,
                              m.data_ptr() if m is not None else None, dd.data_ptr() if dd is not None else None,
                              hm.data_ptr() if hm is not None else None, st.data_ptr(), s.cuda_stream)
        _check(code, "fpn_solve")
        self._keep = (keep, Lh)  # inputs alive until the next call on this context
        harm = torch.view_as_complex(hm) if hm is not None else None
        return (m, harm, st, dd) if want_dmdt else (m, harm, st)

    def solve_static(self, inst, L, drive, samples, settle, n_harm, substeps=0, want_m=True, want_harm=True,
                     harm_z=False, stream=None, out=None, tol=0.0):
        """fpn_solve_static (no device allocation inside the library; one degree L <= 16, at most
        FPN_STATIC_MAX_N instances): (m, harm, status) as fpn_solve.  Pass `out` (dict of preallocated
        tensors "m", "harm" [n,ch,Kh+1,2] float32, "status") to allocate nothing on this side either."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        b, keep, Lh = self._batch(inst, L)
        n = keep["D"].numel()
        ch = 3 if harm_z else 2
        out = out or {}
        m = out.get("m") if want_m else None
        if want_m and m is None:
            m = torch.empty((n, 3, samples), dtype=torch.float32, device=dev)
        hm = out.get("harm") if want_harm else None
        if want_harm and hm is None:
            hm = torch.empty((n, ch, n_harm + 1, 2), dtype=torch.float32, device=dev)
        st = out.get("status")
        if st is None:
            st = torch.empty((n,), dtype=torch.int32, device=dev)
        opts = fpn_solve_opts(samples, settle, n_harm, substeps,
                              (FPN_OUT_M if want_m else 0) | (FPN_OUT_HARM if want_harm else 0) |
                              (FPN_HARM_Z if harm_z else 0), float(tol))
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        code = _lib.fpn_solve_static(self._h, ctypes.byref(drive), ctypes.byref(opts), ctypes.byref(b), n,
                                     m.data_ptr() if m is not None else None,
                                     hm.data_ptr() if hm is not None else None, st.data_ptr(), s.cuda_stream)
        _check(code, "fpn_solve_static")
        self._keep = (keep, Lh)
        return m, (torch.view_as_complex(hm) if hm is not None else None), st

    def equilibrium(self, inst, drive, samples, settle, n_harm, want_m=True, harm_z=False, stream=None):
        """fpn_equilibrium (model M0): (m [n,3,Ns] float32 or None, harm [n,ch,Kh+1] complex64, status)."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        n = np.asarray(inst["D"]).shape[0] if not hasattr(inst["D"], "numel") else inst["D"].numel()
        b, keep, Lh = self._batch(inst, np.ones(n, np.int32))
        ch = 3 if harm_z else 2
        m = torch.empty((n, 3, samples), dtype=torch.float32, device=dev) if want_m else None
        hm = torch.empty((n, ch, n_harm + 1, 2), dtype=torch.float32, device=dev)
        st = torch.empty((n,), dtype=torch.int32, device=dev)
        opts = fpn_solve_opts(samples, settle, n_harm, 0, (FPN_OUT_M if want_m else 0) | FPN_OUT_HARM |
                              (FPN_HARM_Z if harm_z else 0), 0.0)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(_lib.fpn_equilibrium(self._h, ctypes.byref(drive), ctypes.byref(opts), ctypes.byref(b), n,
                                    m.data_ptr() if m is not None else None, hm.data_ptr(), st.data_ptr(),
                                    s.cuda_stream), "fpn_equilibrium")
        self._keep = (keep, Lh)
        return m, torch.view_as_complex(hm), st

    def set_stepper_waves(self, L, waves):
        """fpn_set_stepper_waves: workgroup size of degree L for this context (0: the default)."""
        _check(_lib.fpn_set_stepper_waves(self._h, int(L), int(waves)), "fpn_set_stepper_waves")

    def autotune(self, L):
        """fpn_autotune: time every workgroup size of degree L, keep the fastest.
        Returns (chosen size, {size: ns per instance-step})."""
        w = ctypes.c_int32()
        ns = (ctypes.c_double * 3)()
        _check(_lib.fpn_autotune(self._h, int(L), ctypes.byref(w), ns), "fpn_autotune")
        opts = fpn_stepper_wave_options(L)
        return int(w.value), {opts[k]: float(ns[k]) for k in range(len(opts))}

    def last_steps(self):
        """Time steps taken by the most recent solve, tangent solve or adjoint, summed over instances."""
        v = ctypes.c_int64()
        _check(_lib.fpn_last_steps(self._h, ctypes.byref(v)), "fpn_last_steps")
        return int(v.value)

    TIMING_KERNELS = ("instance_prep", "stationary", "stepper", "harmonics")

    def timing_enable(self, on=True):
        _check(_lib.fpn_timing_enable(self._h, 1 if on else 0), "fpn_timing_enable")

    def timing_read(self):
        """{kernel: (total_ms, launches)} accumulated since timing_enable(True)."""
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_int64 * 4)()
        _check(_lib.fpn_timing_read(self._h, ms, cnt), "fpn_timing_read")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.TIMING_KERNELS)}

    def solve_tangent(self, inst, L, drive, samples, settle, n_harm, substeps=0, want_m=True, want_harm=True,
                      harm_z=False, tol=0.0):
        """fpn_solve_tangent: (m, harm, dm [n,5,3,Ns], dharm [n,5,ch,Kh+1] complex, status)."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        b, keep, Lh = self._batch(inst, L)
        n = keep["D"].numel()
        ch = 3 if harm_z else 2
        m = torch.empty((n, 3, samples), dtype=torch.float32, device=dev) if want_m else None
        dm = torch.empty((n, FPN_NPARAM, 3, samples), dtype=torch.float32, device=dev) if want_m else None
        hm = torch.empty((n, ch, n_harm + 1, 2), dtype=torch.float32, device=dev) if want_harm else None
        dh = torch.empty((n, FPN_NPARAM, ch, n_harm + 1, 2), dtype=torch.float32, device=dev) if want_harm else None
        st = torch.empty((n,), dtype=torch.int32, device=dev)
        opts = fpn_solve_opts(samples, settle, n_harm, substeps,
                              (FPN_OUT_M if want_m else 0) | (FPN_OUT_HARM if want_harm else 0) |
                              (FPN_HARM_Z if harm_z else 0), float(tol))
        s = torch.cuda.current_stream(self.device)
        ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        _check(_lib.fpn_solve_tangent(self._h, ctypes.byref(drive), ctypes.byref(opts), ctypes.byref(b), n, ptr(m),
                                      ptr(hm), ptr(dm), ptr(dh), st.data_ptr(), s.cuda_stream), "fpn_solve_tangent")
        self._keep = (keep, Lh)
        cv = torch.view_as_complex
        return m, (cv(hm) if hm is not None else None), dm, (cv(dh) if dh is not None else None), st

    def adjoint(self, inst, L, drive, samples, settle, n_harm, dL_dharm, substeps=0, harm_z=False, tol=0.0,
                want_harm=True):
        """fpn_adjoint: dL_dharm real [n, ch, Kh+1, 2] (d loss / d (Re, Im) Phi).  Returns (grad [n,5] float64,
        harm [n,ch,Kh+1,2] float32 or None, status)."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        b, keep, Lh = self._batch(inst, L)
        n = keep["D"].numel()
        ch = 3 if harm_z else 2
        g = _f32(dL_dharm, dev).reshape(n, ch, n_harm + 1, 2).contiguous()
        grad = torch.empty((n, FPN_NPARAM), dtype=torch.float64, device=dev)
        hm = torch.empty((n, ch, n_harm + 1, 2), dtype=torch.float32, device=dev) if want_harm else None
        st = torch.empty((n,), dtype=torch.int32, device=dev)
        opts = fpn_solve_opts(samples, settle, n_harm, substeps, FPN_HARM_Z if harm_z else 0, float(tol))
        s = torch.cuda.current_stream(self.device)
        _check(_lib.fpn_adjoint(self._h, ctypes.byref(drive), ctypes.byref(opts), ctypes.byref(b), n, g.data_ptr(),
                                grad.data_ptr(), hm.data_ptr() if hm is not None else None, st.data_ptr(),
                                s.cuda_stream), "fpn_adjoint")
        self._keep = (keep, Lh, g)
        return grad, hm, st

    def plan(self, inst, L, drive, samples, settle, n_harm, substeps=0, want_m=True, want_harm=True, harm_z=False,
             tol=0.0, cost_hint=None):
        """A reusable solve schedule bound to these inputs and to freshly allocated outputs (fpn_plan_*)."""
        return Plan(self, inst, L, drive, samples, settle, n_harm, substeps, want_m, want_harm, harm_z, tol, cost_hint)

    def surrogate_features(self, inst):
        """Network input features [n, 8] (float32, device) and status [n] (fpn_surrogate_features)."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        b, keep, Lh = self._batch(inst, 1)
        n = keep["D"].numel()
        x = torch.empty((n, 8), dtype=torch.float32, device=dev)
        st = torch.empty((n,), dtype=torch.int32, device=dev)
        s = torch.cuda.current_stream(self.device)
        _check(_lib.fpn_surrogate_features(self._h, ctypes.byref(b), n, x.data_ptr(), st.data_ptr(), s.cuda_stream),
               "fpn_surrogate_features")
        self._keep = (keep, Lh)
        return x, st

    def surrogate_predict(self, model, tol, inst, L, drive, samples, settle, n_harm, substeps=0, solver_tol=0.0):
        """fpn_surrogate_predict with a SurrogateModel: returns (harm [n,2,Kh+1] complex64, err [n],
        used_solver [n], status [n], n_fallback)."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        b, keep, Lh = self._batch(inst, L)
        n = keep["D"].numel()
        sur = fpn_surrogate()
        _check(_lib.fpn_surrogate_view(model._h, ctypes.byref(sur)), "fpn_surrogate_view")
        opts = fpn_solve_opts(samples, settle, n_harm, substeps, FPN_OUT_HARM, float(solver_tol))
        hm = torch.empty((n, 2, n_harm + 1, 2), dtype=torch.float32, device=dev)
        err = torch.empty((n,), dtype=torch.float32, device=dev)
        used = torch.empty((n,), dtype=torch.int32, device=dev)
        st = torch.empty((n,), dtype=torch.int32, device=dev)
        nf = ctypes.c_int64()
        s = torch.cuda.current_stream(self.device)
        _check(_lib.fpn_surrogate_predict(self._h, ctypes.byref(sur), float(tol), ctypes.byref(drive),
                                          ctypes.byref(opts), ctypes.byref(b), n, hm.data_ptr(), err.data_ptr(),
                                          used.data_ptr(), st.data_ptr(), ctypes.byref(nf), s.cuda_stream),
               "fpn_surrogate_predict")
        self._keep = (keep, Lh)
        return torch.view_as_complex(hm), err, used, st, int(nf.value)

    def fit_rows(self, phi, S, pair_phi, pair_s):
        """fpn_fit_rows: phi [n_phi, n_pos, n_ch, n_bins] and S [n_S, n_pos, n_ch, n_bins] complex64 (device);
        returns (a [n_pairs, n_ch, n_bins] complex64, err [n_pairs, n_ch, n_bins] float32)."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        phi = phi.contiguous()
        S = S.contiguous()
        _, n_pos, n_ch, n_bins = phi.shape
        assert S.shape[1:] == phi.shape[1:]
        pp = torch.as_tensor(pair_phi, dtype=torch.int32, device=dev).contiguous()
        ps = torch.as_tensor(pair_s, dtype=torch.int32, device=dev).contiguous()
        assert pp.numel() == ps.numel()
        assert int(pp.min()) >= 0 and int(pp.max()) < phi.shape[0] and int(ps.min()) >= 0 and int(ps.max()) < S.shape[0]
        n = pp.numel()
        a = torch.empty((n, n_ch, n_bins, 2), dtype=torch.float32, device=dev)
        err = torch.empty((n, n_ch, n_bins), dtype=torch.float32, device=dev)
        s = torch.cuda.current_stream(self.device)
        _check(_lib.fpn_fit_rows(self._h, torch.view_as_real(phi).data_ptr(), torch.view_as_real(S).data_ptr(), n_pos,
                                 n_ch, n_bins, n, pp.data_ptr(), ps.data_ptr(), a.data_ptr(), err.data_ptr(),
                                 s.cuda_stream), "fpn_fit_rows")
        return torch.view_as_complex(a), err

    def nrmse_global(self, err, n_ang, kset):
        """fpn_nrmse_global: err [n_groups * n_ang, n_ch, n_bins] (device float32), kset bins; returns
        (eps_freq [n_groups, n_k], eps_global [n_groups])."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        err = err.contiguous()
        n_pairs, n_ch, n_bins = err.shape
        assert n_pairs % n_ang == 0
        ks = torch.as_tensor(kset, dtype=torch.int32, device=dev).contiguous()
        assert int(ks.min()) >= 0 and int(ks.max()) < n_bins
        g = n_pairs // n_ang
        ef = torch.empty((g, ks.numel()), dtype=torch.float32, device=dev)
        eg = torch.empty((g,), dtype=torch.float32, device=dev)
        s = torch.cuda.current_stream(self.device)
        _check(_lib.fpn_nrmse_global(self._h, err.data_ptr(), g, n_ang, n_ch, n_bins, ks.data_ptr(), ks.numel(),
                                     ef.data_ptr(), eg.data_ptr(), s.cuda_stream), "fpn_nrmse_global")
        return ef, eg

    def m2_system(self, phi, a, S, n_ang, kset):
        """fpn_m2_system: phi [J * n_ang, n_pos, n_ch, n_bins] and S [n_ang, ...] complex64, a [J * n_ang,
        n_ch, n_bins] complex64 (device); returns (G [J, J] complex128, b [J] complex128, ||y||^2) on the device."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        phi, a, S = phi.contiguous(), a.contiguous(), S.contiguous()
        n_el, n_pos, n_ch, n_bins = phi.shape
        assert n_el % n_ang == 0 and S.shape == (n_ang, n_pos, n_ch, n_bins) and a.shape == (n_el, n_ch, n_bins)
        J = n_el // n_ang
        ks = torch.as_tensor(kset, dtype=torch.int32, device=dev).contiguous()
        assert int(ks.min()) >= 0 and int(ks.max()) < n_bins
        G = torch.empty((J, J, 2), dtype=torch.float64, device=dev)
        b = torch.empty((J, 2), dtype=torch.float64, device=dev)
        yy = torch.empty((1,), dtype=torch.float64, device=dev)
        s = torch.cuda.current_stream(self.device)
        _check(_lib.fpn_m2_system(self._h, torch.view_as_real(phi).data_ptr(), torch.view_as_real(a).data_ptr(),
                                  torch.view_as_real(S).data_ptr(), n_pos, n_ch, n_bins, J, n_ang, ks.data_ptr(),
                                  ks.numel(), G.data_ptr(), b.data_ptr(), yy.data_ptr(), s.cuda_stream), "fpn_m2_system")
        return torch.view_as_complex(G), torch.view_as_complex(b), yy

    def m2_model(self, phi, a, w, n_ang):
        """fpn_m2_model: S_model [n_ang, n_pos, n_ch, n_bins] complex64 from weights w [J] (float64)."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        phi, a = phi.contiguous(), a.contiguous()
        n_el, n_pos, n_ch, n_bins = phi.shape
        J = n_el // n_ang
        wt = torch.as_tensor(w, dtype=torch.float64, device=dev).contiguous()
        assert wt.numel() == J
        out = torch.empty((n_ang, n_pos, n_ch, n_bins, 2), dtype=torch.float32, device=dev)
        s = torch.cuda.current_stream(self.device)
        _check(_lib.fpn_m2_model(self._h, torch.view_as_real(phi).data_ptr(), torch.view_as_real(a).data_ptr(),
                                 wt.data_ptr(), n_pos, n_ch, n_bins, J, n_ang, out.data_ptr(), s.cuda_stream),
               "fpn_m2_model")
        return torch.view_as_complex(out)

    def rows_error(self, model, S):
        """fpn_rows_error: Eq. error1 rows [n_mat, n_ch, n_bins] of model against S (same shapes)."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        model, S = model.contiguous(), S.contiguous()
        n_mat, n_pos, n_ch, n_bins = S.shape
        assert model.shape == S.shape
        err = torch.empty((n_mat, n_ch, n_bins), dtype=torch.float32, device=dev)
        s = torch.cuda.current_stream(self.device)
        _check(_lib.fpn_rows_error(self._h, torch.view_as_real(model).data_ptr(), torch.view_as_real(S).data_ptr(),
                                   n_pos, n_ch, n_bins, n_mat, err.data_ptr(), s.cuda_stream), "fpn_rows_error")
        return err

    def stationary(self, inst, L, field):
        torch = _torch()
        dev = f"cuda:{self.device}"
        b, keep, Lh = self._batch(inst, L)
        n = keep["D"].numel()
        f = _dev_f64(field, dev)
        m = torch.empty((n, 3), dtype=torch.float64, device=dev)
        st = torch.empty((n,), dtype=torch.int32, device=dev)
        s = torch.cuda.current_stream(self.device)
        _check(_lib.fpn_stationary(self._h, ctypes.byref(b), n, f.data_ptr(), m.data_ptr(), st.data_ptr(),
                                   s.cuda_stream), "fpn_stationary")
        torch.cuda.synchronize(self.device)
        return m, st

    def select_degree(self, inst, L_min, drive, samples, tol, L_max=FPN_MAX_L):
        """fpn_select_degree: per instance the smallest degree in L_min[i]..L_max whose truncation
        estimate is <= tol.  Returns (L [n] int32 numpy, est [n] float64 device, status [n] int32 device)."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        b, keep, Lh = self._batch(inst, L_min)
        n = keep["D"].numel()
        Lout = np.empty(n, dtype=np.int32)
        est = torch.empty((n,), dtype=torch.float64, device=dev)
        st = torch.empty((n,), dtype=torch.int32, device=dev)
        s = torch.cuda.current_stream(self.device)
        _check(_lib.fpn_select_degree(self._h, ctypes.byref(b), n, ctypes.byref(drive), int(samples), float(tol),
                                      int(L_max), Lout.ctypes.data, est.data_ptr(), st.data_ptr(), s.cuda_stream),
               "fpn_select_degree")
        return Lout, est, st

    def truncation_estimate(self, inst, L, drive, samples):
        """|m_L - m_{L-2}| of the stationary moments under each instance's largest sampled field
        (fpn_truncation_estimate): an upper estimate of the degree-L truncation error.  Returns
        (est [n] float64, status [n] int32) on the device."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        b, keep, Lh = self._batch(inst, L)
        n = keep["D"].numel()
        est = torch.empty((n,), dtype=torch.float64, device=dev)
        st = torch.empty((n,), dtype=torch.int32, device=dev)
        s = torch.cuda.current_stream(self.device)
        _check(_lib.fpn_truncation_estimate(self._h, ctypes.byref(b), n, ctypes.byref(drive), int(samples),
                                            est.data_ptr(), st.data_ptr(), s.cuda_stream), "fpn_truncation_estimate")
        return est, st


def _f32(x, device):
    torch = _torch()
    return torch.as_tensor(x, dtype=torch.float32, device=device).contiguous()


class MLP:
    """A surrogate network owned by the library (fpn_mlp_*): FP32 master parameters, BF16 matrix-core
    products.  Parameters are exchanged as one flat FP32 tensor (per layer W [out, in], then b [out]).
    A member of a SurrogateModel is a borrowed handle (``handle`` given): the model frees it."""

    def __init__(self, ctx, widths, seed=0, handle=None):
        self.ctx = ctx
        self.widths = [int(w) for w in widths]
        self._owned = handle is None
        self._h = _vp()
        if handle is not None:
            self._h = handle
        else:
            w = (ctypes.c_int32 * len(self.widths))(*self.widths)
            _check(_lib.fpn_mlp_create(ctx._h, len(self.widths) - 1, w, int(seed), ctypes.byref(self._h)),
                   "fpn_mlp_create")
        self.n_params = int(_lib.fpn_mlp_num_params(self._h))

    def close(self):
        if self._h and self._owned:
            _lib.fpn_mlp_destroy(self._h)
        self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _dev(self):
        return f"cuda:{self.ctx.device}"

    def _stream(self):
        return _torch().cuda.current_stream(self.ctx.device).cuda_stream

    def get_params(self):
        p = _torch().empty(self.n_params, dtype=_torch().float32, device=self._dev)
        _check(_lib.fpn_mlp_params(self._h, p.data_ptr(), None, self._stream()), "fpn_mlp_params")
        return p

    def set_params(self, flat):
        t = _f32(flat, self._dev)
        assert t.numel() == self.n_params
        _check(_lib.fpn_mlp_params(self._h, None, t.data_ptr(), self._stream()), "fpn_mlp_params")
        _torch().cuda.synchronize(self.ctx.device)

    def unflatten(self, flat):
        """Split a flat parameter vector (numpy) into lists of W [out, in] and b [out]."""
        flat = np.asarray(flat)
        Ws, bs, o = [], [], 0
        for i, j in zip(self.widths[:-1], self.widths[1:]):
            Ws.append(flat[o:o + i * j].reshape(j, i))
            o += i * j
            bs.append(flat[o:o + j])
            o += j
        return Ws, bs

    def set_input_norm(self, mean, std):
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(std, dtype=np.float32)
        _check(_lib.fpn_mlp_set_input_norm(self._h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                           s.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), "fpn_mlp_set_input_norm")

    def forward(self, x, out=None):
        torch = _torch()
        x = _f32(x, self._dev)
        n = x.shape[0]
        y = out if out is not None else torch.empty((n, self.widths[-1]), dtype=torch.float32, device=self._dev)
        _check(_lib.fpn_mlp_forward(self._h, x.data_ptr(), n, y.data_ptr(), self._stream()), "fpn_mlp_forward")
        return y

    def gradient(self, x, t):
        torch = _torch()
        x, t = _f32(x, self._dev), _f32(t, self._dev)
        g = torch.empty(self.n_params, dtype=torch.float32, device=self._dev)
        loss = torch.empty(1, dtype=torch.float64, device=self._dev)
        _check(_lib.fpn_mlp_gradient(self._h, x.data_ptr(), t.data_ptr(), x.shape[0], g.data_ptr(), loss.data_ptr(),
                                     self._stream()), "fpn_mlp_gradient")
        return g, loss / (x.shape[0] * self.widths[-1])

    def train_step(self, x, t, lr, loss_out=None):
        """One Adam step; returns the device tensor holding the loss sum (before the update)."""
        torch = _torch()
        loss = loss_out if loss_out is not None else torch.empty(1, dtype=torch.float64, device=self._dev)
        _check(_lib.fpn_mlp_train_step(self._h, x.data_ptr(), t.data_ptr(), x.shape[0], float(lr), loss.data_ptr(),
                                       self._stream()), "fpn_mlp_train_step")
        return loss


class SurrogateModel:
    """fpn_sur_model: a two-member ensemble with its output scale and error calibration, trainable,
    evaluable and savable (fpn_surrogate_init / _create / _save / _infer / _train_step / _destroy)."""

    def __init__(self, ctx, widths=None, seeds=(1, 2), path=None):
        self.ctx = ctx
        self._h = _vp()
        if path is not None:
            _check(_lib.fpn_surrogate_create(ctx._h, os.fsencode(path), ctypes.byref(self._h)), "fpn_surrogate_create")
        else:
            ws = [int(w) for w in widths]
            w = (ctypes.c_int32 * len(ws))(*ws)
            sd = (ctypes.c_uint64 * 2)(*[int(x) for x in seeds])
            _check(_lib.fpn_surrogate_init(ctx._h, len(ws) - 1, w, sd, ctypes.byref(self._h)), "fpn_surrogate_init")
        self._refresh()

    def _refresh(self):
        sur = fpn_surrogate()
        _check(_lib.fpn_surrogate_view(self._h, ctypes.byref(sur)), "fpn_surrogate_view")
        self.out_scale, self.err_calib = float(sur.out_scale), float(sur.err_calib)
        self.res_scale = float(sur.res_scale)
        self.members, self.residual = [], []
        for k in range(4 if sur.res[0] else 2):
            h = _vp()
            _check(_lib.fpn_surrogate_member(self._h, k, ctypes.byref(h)), "fpn_surrogate_member")
            nl = ctypes.c_int32()
            wb = (ctypes.c_int32 * 17)()
            _check(_lib.fpn_mlp_shape(h, ctypes.byref(nl), wb), "fpn_mlp_shape")
            (self.members if k < 2 else self.residual).append(MLP(self.ctx, list(wb[:nl.value + 1]), handle=h))
        self.widths = self.members[0].widths

    def add_residual(self, seeds=(3, 4)):
        """fpn_surrogate_add_residual: a second stage of two networks trained on the members' residuals."""
        sd = (ctypes.c_uint64 * 2)(*[int(x) for x in seeds])
        _check(_lib.fpn_surrogate_add_residual(self.ctx._h, self._h, sd), "fpn_surrogate_add_residual")
        self._refresh()

    def set_residual_scale(self, res_scale):
        _check(_lib.fpn_surrogate_set_residual_scale(self._h, float(res_scale)), "fpn_surrogate_set_residual_scale")
        self._refresh()

    def close(self):
        for m in getattr(self, "members", []) + getattr(self, "residual", []):
            m.close()
        if self._h:
            _lib.fpn_surrogate_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_scales(self, out_scale, err_calib):
        _check(_lib.fpn_surrogate_set_scales(self._h, float(out_scale), float(err_calib)), "fpn_surrogate_set_scales")
        sur = fpn_surrogate()
        _check(_lib.fpn_surrogate_view(self._h, ctypes.byref(sur)), "fpn_surrogate_view")
        self.out_scale, self.err_calib = float(sur.out_scale), float(sur.err_calib)   # as stored (FP32)

    def save(self, path):
        _check(_lib.fpn_surrogate_save(self._h, os.fsencode(path)), "fpn_surrogate_save")

    def _stream(self):
        return _torch().cuda.current_stream(self.ctx.device).cuda_stream

    def infer(self, x):
        """(y [n, W], err_est [n]) from features x [n, 8] (device float32)."""
        torch = _torch()
        dev = f"cuda:{self.ctx.device}"
        x = _f32(x, dev)
        n = x.shape[0]
        y = torch.empty((n, self.widths[-1]), dtype=torch.float32, device=dev)
        e = torch.empty((n,), dtype=torch.float32, device=dev)
        _check(_lib.fpn_surrogate_infer(self.ctx._h, self._h, x.data_ptr(), n, y.data_ptr(), e.data_ptr(),
                                        self._stream()), "fpn_surrogate_infer")
        return y, e

    def train_step(self, x, y_true, lr):
        """One Adam step of both members on (x, y_true); returns the device tensor of the two loss sums."""
        torch = _torch()
        dev = f"cuda:{self.ctx.device}"
        x, y_true = _f32(x, dev), _f32(y_true, dev)
        loss = torch.empty(2, dtype=torch.float64, device=dev)
        _check(_lib.fpn_surrogate_train_step(self.ctx._h, self._h, x.data_ptr(), y_true.data_ptr(), x.shape[0],
                                             float(lr), loss.data_ptr(), self._stream()), "fpn_surrogate_train_step")
        return loss


class Plan:
    """fpn_plan: one solve bound to its inputs and outputs, launched eagerly or as a HIP graph."""

    def __init__(self, ctx, inst, L, drive, samples, settle, n_harm, substeps, want_m, want_harm, harm_z, tol,
                 cost_hint):
        torch = _torch()
        dev = f"cuda:{ctx.device}"
        self.ctx = ctx
        self._b, self._keep, self._Lh = ctx._batch(inst, L)
        n = self._keep["D"].numel()
        self.n = n
        ch = 3 if harm_z else 2
        self.m = torch.empty((n, 3, samples), dtype=torch.float32, device=dev) if want_m else None
        self._hm = torch.empty((n, ch, n_harm + 1, 2), dtype=torch.float32, device=dev) if want_harm else None
        self.status = torch.empty((n,), dtype=torch.int32, device=dev)
        self._drive = drive
        self._opts = fpn_solve_opts(samples, settle, n_harm, substeps,
                                    (FPN_OUT_M if want_m else 0) | (FPN_OUT_HARM if want_harm else 0) |
                                    (FPN_HARM_Z if harm_z else 0), float(tol))
        hint = None
        if cost_hint is not None:
            self._hint = np.ascontiguousarray(cost_hint, dtype=np.float32)
            hint = self._hint.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._h = _vp()
        _check(_lib.fpn_plan_create(ctx._h, ctypes.byref(drive), ctypes.byref(self._opts), ctypes.byref(self._b), n,
                                    hint, self.m.data_ptr() if self.m is not None else None,
                                    self._hm.data_ptr() if self._hm is not None else None, self.status.data_ptr(),
                                    ctypes.byref(self._h)), "fpn_plan_create")

    @property
    def harm(self):
        return _torch().view_as_complex(self._hm) if self._hm is not None else None

    def _stream(self, stream):
        return (stream if stream is not None else _torch().cuda.current_stream(self.ctx.device)).cuda_stream

    def launch(self, stream=None):
        _check(_lib.fpn_plan_launch(self._h, self._stream(stream)), "fpn_plan_launch")

    def graph_launch(self, stream=None):
        _check(_lib.fpn_plan_graph_launch(self._h, self._stream(stream)), "fpn_plan_graph_launch")

    def steps(self):
        out = np.zeros(self.n, dtype=np.int32)
        _check(_lib.fpn_plan_steps(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "fpn_plan_steps")
        return out

    def close(self):
        if self._h:
            _lib.fpn_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
