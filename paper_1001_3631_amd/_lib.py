"""ctypes binding of libteuk.so: the C ABI of include/teuk.h, names unchanged.

Argument marshalling only; every computation runs in the HIP library.  The
library is loaded from this package directory; a missing library raises.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libteuk.so")

TEUK_OK = 0
TEUK_EINVAL = -1
TEUK_EDEVICE = -2
TEUK_ENONFINITE = -3
TEUK_ENOMEM = -4
TEUK_ESTATE = -5

_ERRNAMES = {TEUK_EINVAL: "TEUK_EINVAL", TEUK_EDEVICE: "TEUK_EDEVICE",
             TEUK_ENONFINITE: "TEUK_ENONFINITE", TEUK_ENOMEM: "TEUK_ENOMEM",
             TEUK_ESTATE: "TEUK_ESTATE"}


class TeukError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class GridDesc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_double), ("a", ctypes.c_double),
                ("s", ctypes.c_int32), ("m", ctypes.c_int32),
                ("nr", ctypes.c_int32), ("nth", ctypes.c_int32),
                ("rs_min", ctypes.c_double), ("rs_max", ctypes.c_double),
                ("cfl", ctypes.c_double), ("rs_extract", ctypes.c_double),
                ("ko_eps", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("h_r", ctypes.c_double), ("h_th", ctypes.c_double),
                ("r_plus", ctypes.c_double), ("r_minus", ctypes.c_double),
                ("i_ext", ctypes.c_int32), ("nr", ctypes.c_int32), ("nth", ctypes.c_int32),
                ("row_pitch", ctypes.c_int32), ("steps_done", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("seg_rows", ctypes.c_int32), ("k_steps", ctypes.c_int32), ("adj_seg_rows", ctypes.c_int32)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("seg_rows", ctypes.c_int32), ("k_steps", ctypes.c_int32), ("batch_mode", ctypes.c_int32),
                ("us_per_iteration", ctypes.c_double)]


# teuk_batch modes
BATCH_PERSISTENT = 0
BATCH_PER_ITERATION = 1


class SourceDesc(ctypes.Structure):
    _fields_ = [("amplitude", ctypes.c_double), ("sigma_r_cells", ctypes.c_double),
                ("sigma_th_cells", ctypes.c_double), ("cutoff_sigmas", ctypes.c_double),
                ("nsamples", ctypes.c_int64), ("orbit", ctypes.POINTER(ctypes.c_double)),
                ("orbit_dev", ctypes.c_void_p)]


class FluxDesc(ctypes.Structure):
    _fields_ = [("nmodes", ctypes.c_int32), ("m", ctypes.POINTER(ctypes.c_int32)),
                ("waves", ctypes.POINTER(ctypes.c_void_p)), ("nsteps", ctypes.c_int64),
                ("nth", ctypes.c_int32), ("dt", ctypes.c_double)]


class WsRequest(ctypes.Structure):
    _fields_ = [("sigma_r_cells", ctypes.c_double), ("sigma_th_cells", ctypes.c_double),
                ("cutoff_sigmas", ctypes.c_double), ("adjoint", ctypes.c_int32)]


class GradPlan(ctypes.Structure):
    _fields_ = [("nsteps", ctypes.c_int64), ("interval", ctypes.c_int64), ("snapshots", ctypes.c_int64),
                ("state_weight", ctypes.c_double),
                ("i0", ctypes.c_int32), ("i1", ctypes.c_int32), ("j0", ctypes.c_int32), ("j1", ctypes.c_int32),
                ("n_lo", ctypes.c_int64), ("n_hi", ctypes.c_int64), ("force_recompute", ctypes.c_int32),
                ("ckpt_dev", ctypes.c_void_p), ("ckpt_bytes", ctypes.c_uint64)]


_P = ctypes.c_void_p
_CTX = ctypes.c_void_p

# name -> (restype, argtypes); the exported symbol set of include/teuk.h
SIGNATURES = {
    "teuk_workspace_size": (ctypes.c_int, [ctypes.POINTER(GridDesc), ctypes.POINTER(WsRequest),
                                           ctypes.POINTER(ctypes.c_size_t)]),
    "teuk_init_grid": (ctypes.c_int, [ctypes.POINTER(GridDesc), ctypes.POINTER(WsRequest), _P, _P,
                                      ctypes.c_size_t, ctypes.POINTER(_CTX)]),
    "teuk_init_grid_static": (ctypes.c_int, [ctypes.POINTER(GridDesc), ctypes.POINTER(WsRequest), _P,
                                             ctypes.POINTER(_CTX)]),
    "teuk_destroy": (ctypes.c_int, [_CTX]),
    "teuk_get_info": (ctypes.c_int, [_CTX, ctypes.POINTER(Info)]),
    "teuk_set_state": (ctypes.c_int, [_CTX, _P, _P]),
    "teuk_get_state": (ctypes.c_int, [_CTX, _P, _P]),
    "teuk_init_pulse": (ctypes.c_int, [_CTX, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "teuk_set_source": (ctypes.c_int, [_CTX, ctypes.POINTER(SourceDesc)]),
    "teuk_set_amplitude": (ctypes.c_int, [_CTX, ctypes.c_double]),
    "teuk_orbit_circular": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_double)]),
    "teuk_orbit_eccentric": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    "teuk_step_n": (ctypes.c_int, [_CTX, ctypes.c_int64, _P]),
    "teuk_extract_waveform": (ctypes.c_int, [_CTX, _P]),
    "teuk_checkpoint_size": (ctypes.c_int, [_CTX, ctypes.POINTER(GradPlan), ctypes.POINTER(ctypes.c_size_t)]),
    "teuk_checkpoint_schedule": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "teuk_forward_checkpointed": (ctypes.c_int, [_CTX, ctypes.POINTER(GradPlan), _P,
                                                 ctypes.POINTER(ctypes.c_double)]),
    "teuk_backward_checkpointed": (ctypes.c_int, [_CTX, ctypes.POINTER(GradPlan), _P, ctypes.c_double, _P, _P,
                                                  ctypes.POINTER(ctypes.c_double)]),
    "teuk_adjoint_begin": (ctypes.c_int, [_CTX, _P, _P, ctypes.c_int64, _P]),
    "teuk_adjoint_step_n": (ctypes.c_int, [_CTX, ctypes.c_int64, _P]),
    "teuk_adjoint_add_state": (ctypes.c_int, [_CTX, _P, _P]),
    "teuk_adjoint_get": (ctypes.c_int, [_CTX, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "teuk_check_finite": (ctypes.c_int, [_CTX]),
    "teuk_set_tuning": (ctypes.c_int, [_CTX, ctypes.POINTER(Tuning)]),
    "teuk_get_tuning": (ctypes.c_int, [_CTX, ctypes.POINTER(Tuning)]),
    "teuk_autotune": (ctypes.c_int, [_CTX, ctypes.c_char_p, ctypes.POINTER(TuneEntry), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32)]),
    "teuk_batch_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(GridDesc),
                                                 ctypes.POINTER(WsRequest), ctypes.POINTER(ctypes.c_size_t)]),
    "teuk_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(GridDesc), ctypes.POINTER(WsRequest), _P,
                                         _P, ctypes.c_size_t, ctypes.POINTER(_CTX)]),
    "teuk_batch_destroy": (ctypes.c_int, [_CTX]),
    "teuk_batch_instance": (ctypes.c_int, [_CTX, ctypes.c_int32, ctypes.POINTER(_CTX)]),
    "teuk_batch_set_tuning": (ctypes.c_int, [_CTX, ctypes.c_int32]),
    "teuk_batch_get_tuning": (ctypes.c_int, [_CTX, ctypes.POINTER(ctypes.c_int32)]),
    "teuk_batch_set_mode": (ctypes.c_int, [_CTX, ctypes.c_int32]),
    "teuk_batch_get_mode": (ctypes.c_int, [_CTX, ctypes.POINTER(ctypes.c_int32)]),
    "teuk_batch_get_groups": (ctypes.c_int, [_CTX, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int32)]),
    "teuk_batch_step_n": (ctypes.c_int, [_CTX, ctypes.c_int64, ctypes.POINTER(_P)]),
    "teuk_batch_sync": (ctypes.c_int, [_CTX]),
    "teuk_batch_set_wait_limit": (ctypes.c_int, [_CTX, ctypes.c_double]),
    "teuk_batch_abort": (ctypes.c_int, [_CTX]),
    "teuk_batch_autotune": (ctypes.c_int, [_CTX, ctypes.c_char_p, ctypes.POINTER(TuneEntry), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32)]),
    "teuk_set_kernel_timing": (ctypes.c_int, [_CTX, ctypes.c_int]),
    "teuk_kernel_timing": (ctypes.c_int, [_CTX, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64)]),
    "teuk_flux_workspace_size": (ctypes.c_int, [ctypes.POINTER(FluxDesc), ctypes.POINTER(ctypes.c_size_t)]),
    "teuk_radiated_flux": (ctypes.c_int, [ctypes.POINTER(FluxDesc), _P, _P, ctypes.c_size_t, _P]),
    "teuk_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libteuk.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run python -c 'import __graft_entry__; __graft_entry__.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc):
    if rc != TEUK_OK:
        raise TeukError(rc, load().teuk_last_error().decode())
    return rc
