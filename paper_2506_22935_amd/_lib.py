"""ctypes binding of libgraf_af.so (argument marshalling only).

Mirrors include/graf_af.h.  Loading fails loudly when the library is missing:
there is no CPU fallback.
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# GRAF_AF_LIB points at another build of the same library (e.g. an
# instrumented one); the default is the in-tree build.
LIB_PATH = os.environ.get("GRAF_AF_LIB") or os.path.join(_PKG, "libgraf_af.so")

AF_OK = 0
STATUS = {0: "AF_OK", -1: "AF_ERR_INVALID_ARG", -2: "AF_ERR_UNSUPPORTED", -3: "AF_ERR_BUDGET",
          -4: "AF_ERR_HIP", -5: "AF_ERR_WORKSPACE", -6: "AF_ERR_NO_DEVICE"}


AF_WAVE_PERIODIC = 1  # af_wave.flags: the periodic (circular) AF


class AfWave(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("max_lag", ctypes.c_int32),
                ("h_tau", ctypes.c_int32), ("h_k", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("s_off", ctypes.c_int64), ("grid_off", ctypes.c_int64)]


class AfPlanOpts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_float), ("store_mode", ctypes.c_int32),
                ("budget_bytes", ctypes.c_int64), ("variant", ctypes.c_int32),
                ("segment_iters", ctypes.c_int32), ("loss_passes", ctypes.c_int32),
                ("launch_mode", ctypes.c_int32)]


class AfLossParams(ctypes.Structure):
    _fields_ = [("w_isl", ctypes.c_float), ("w_psl", ctypes.c_float), ("psl_temp", ctypes.c_float),
                ("band_w", ctypes.c_void_p), ("psl_hard", ctypes.c_int32), ("w_spec", ctypes.c_float),
                ("match_target", ctypes.c_void_p), ("w_match", ctypes.c_float), ("w_width", ctypes.c_float),
                ("gamma", ctypes.c_float), ("w_const", ctypes.c_float), ("w_smooth", ctypes.c_float),
                ("cell_w", ctypes.c_void_p), ("w_cell", ctypes.c_float)]


class AfAdamParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class AfPlanSummary(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_int64), ("store_bytes", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("segments", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("variant", ctypes.c_int32), ("stores", ctypes.c_int32)]


# name -> (restype, argtypes); every entry point declared in graf_af.h
_VP, _I32, _I64, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
SIGNATURES = {
    "af_plan_create": (ctypes.c_int, [_I32, ctypes.POINTER(AfWave), ctypes.POINTER(AfPlanOpts),
                                      ctypes.POINTER(_VP)]),
    "af_plan_destroy": (None, [_VP]),
    "af_plan_workspace_size": (ctypes.c_int, [_VP, ctypes.POINTER(_SZ)]),
    "af_plan_get_summary": (ctypes.c_int, [_VP, ctypes.POINTER(AfPlanSummary)]),
    "af_plan_autotune": (ctypes.c_int, [_VP, _VP, _VP, _SZ, _VP, ctypes.POINTER(_I32),
                                        ctypes.POINTER(ctypes.c_float)]),
    "af_forward": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "af_backward": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "af_loss": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(AfLossParams), _VP, _VP, _VP, _VP, _SZ, _VP]),
    "af_loss_no_alloc": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(AfLossParams), _VP, _VP, _VP, _VP]),
    "af_loss_stage": (ctypes.c_int, [_VP, _I32, _VP, ctypes.POINTER(AfLossParams), _VP, _VP, _VP, _VP, _SZ,
                                     _VP]),
    "af_phase_to_signal": (ctypes.c_int, [_VP, _VP, _I64, _VP]),
    "af_spectral_variance": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "af_project": (ctypes.c_int, [_VP, _VP, _VP, _I32, _VP, _VP]),
    "af_scenario_combine": (ctypes.c_int, [_VP, _I32, _VP, _VP, _VP, _VP]),
    "af_cross_workspace_size": (ctypes.c_int, [_VP, ctypes.POINTER(_SZ)]),
    "af_cross_forward": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "af_cross_backward": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "af_optim_step": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(AfLossParams),
                                     ctypes.POINTER(AfAdamParams), _VP, _VP, _SZ, _VP]),
    "af_gemm_config": (ctypes.c_int, [_I32, _I32, _I32, _I32, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                      ctypes.POINTER(_SZ)]),
    "af_gemm_bf16": (ctypes.c_int, [_I32, _I32, _I32, _I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _I32, _I32, _VP,
                                    _SZ, _VP]),
    "af_colsum_workspace_size": (ctypes.c_int, [_I32, _I32, ctypes.POINTER(_SZ)]),
    "af_colsum": (ctypes.c_int, [_I32, _I32, _VP, _VP, _VP, _SZ, _VP]),
    "af_adam_update": (ctypes.c_int, [_I64, _VP, _VP, _VP, _VP, _I32, ctypes.POINTER(AfAdamParams), _VP, _VP]),
    "af_to_bf16": (ctypes.c_int, [_I64, _VP, _VP, _VP]),
    "af_phase_grad": (ctypes.c_int, [_I64, _VP, _VP, _VP, _VP, _VP]),
    "af_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "af_version": (_I32, []),
}

_lib = None


class AfError(RuntimeError):
    def __init__(self, fn, code):
        name = STATUS.get(code, str(code))
        msg = "%s failed: %s" % (fn, name)
        if _lib is not None:
            try:
                msg += " (%s)" % _lib.af_status_string(code).decode()
            except Exception:
                pass
        super().__init__(msg)
        self.code = code


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libgraf_af.so is not built (%s); run __graft_entry__.build() or "
                "python -m paper_2506_22935_amd.build" % LIB_PATH)
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def check(fn, code):
    if code != AF_OK:
        raise AfError(fn, code)
