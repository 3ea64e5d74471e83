"""ctypes binding of ``libtfl.so`` (declared in ``include/tfl.h``).

Argument marshalling only: every function here forwards to the C entry point
of the same name.  The library must be built (``_build.build()``); importing
this module without it raises, so that no code path can run without the HIP
kernels.
"""
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime that the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
# TFL_LIB points the binding at another build of the library (the host-sanitizer test loads one)
LIB_PATH = os.environ.get("TFL_LIB") or os.path.join(HERE, "libtfl.so")

TFL_OK = 0
TFL_E_INVAL = -1
TFL_E_STATE = -2
TFL_E_UNSTABLE = -3
TFL_E_NONFINITE = -4
TFL_E_DEVICE = -5
TFL_E_NOMEM = -6
TFL_E_RANGE = -7
ERROR_NAMES = {
    TFL_E_INVAL: "TFL_E_INVAL",
    TFL_E_STATE: "TFL_E_STATE",
    TFL_E_UNSTABLE: "TFL_E_UNSTABLE",
    TFL_E_NONFINITE: "TFL_E_NONFINITE",
    TFL_E_DEVICE: "TFL_E_DEVICE",
    TFL_E_NOMEM: "TFL_E_NOMEM",
    TFL_E_RANGE: "TFL_E_RANGE",
}

TFL_F64, TFL_F32 = 0, 1
TFL_PERIODIC, TFL_CPML = 0, 1
TFL_SWEEP_AUTO, TFL_SWEEP_TWO_PASS, TFL_SWEEP_FUSED, TFL_SWEEP_TWO_STEP = 0, 1, 2, 3
TFL_WAVE_SIN, TFL_WAVE_GAUSS, TFL_WAVE_MOD_GAUSS = 0, 1, 2
TFL_MAX_SOURCES = 32
TFL_MAX_PROBES = 32
TFL_MAX_FREQS = 16
TFL_MAX_EDGE_CLASSES = 65535


class tfl_config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("dt", ctypes.c_double), ("theta", ctypes.c_double),
        ("dtype", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 3),
        ("pml_lo", ctypes.c_int32 * 3), ("pml_hi", ctypes.c_int32 * 3),
        ("pml_order", ctypes.c_double), ("pml_scale", ctypes.c_double),
        ("kappa_max", ctypes.c_double), ("alpha_max", ctypes.c_double),
    ]


class tfl_source(ctypes.Structure):
    _fields_ = [
        ("comp", ctypes.c_int32), ("box", ctypes.c_int64 * 6), ("amplitude", ctypes.c_double),
        ("waveform", ctypes.c_int32), ("freq", ctypes.c_double), ("t0", ctypes.c_double), ("tw", ctypes.c_double),
    ]


class tfl_probe(ctypes.Structure):
    _fields_ = [
        ("comp", ctypes.c_int32), ("box", ctypes.c_int64 * 6),
        ("series", ctypes.c_void_p), ("capacity", ctypes.c_int64),
        ("nfreq", ctypes.c_int32), ("freqs", ctypes.POINTER(ctypes.c_double)), ("dft", ctypes.c_void_p),
    ]


class tfl_objective(ctypes.Structure):
    _fields_ = [("comp", ctypes.c_int32), ("box", ctypes.c_int64 * 6), ("f0", ctypes.c_double)]


TFL_FIT_MAX_ORDER = 16


class tfl_fit_req(ctypes.Structure):
    _fields_ = [("start", ctypes.c_int64), ("count", ctypes.c_int64), ("decim", ctypes.c_int64),
                ("order", ctypes.c_int32), ("f_hint", ctypes.c_double)]


class tfl_fit_result(ctypes.Structure):
    _fields_ = [("f0", ctypes.c_double), ("alpha", ctypes.c_double), ("Q", ctypes.c_double),
                ("residual", ctypes.c_double), ("order", ctypes.c_int32), ("nmodes", ctypes.c_int32),
                ("modes", ctypes.c_double * (2 * TFL_FIT_MAX_ORDER))]


class TflError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

P = ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)

# name -> argtypes (restype int unless noted)
SIGNATURES = {
    "tfl_create": [ctypes.POINTER(tfl_config), ctypes.POINTER(ctypes.c_void_p)],
    "tfl_destroy": [P],
    "tfl_last_error": [P],
    "tfl_buffer_sizes": [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                         ctypes.POINTER(ctypes.c_size_t)],
    "tfl_bind_state": [P, PP, PP, PP],
    "tfl_bind_workspace": [P, P, P, P],
    "tfl_bind_materials": [P, P, P, P, P],
    "tfl_set_initial_integer_time": [P, P],
    "tfl_add_source": [P, ctypes.POINTER(tfl_source), ctypes.POINTER(ctypes.c_int)],
    "tfl_add_probe": [P, ctypes.POINTER(tfl_probe), ctypes.POINTER(ctypes.c_int)],
    "tfl_clear_sources_probes": [P],
    "tfl_step": [P, ctypes.c_int64, P],
    "tfl_set_nonfinite_check": [P, ctypes.c_int64],
    "tfl_set_sweep": [P, ctypes.c_int32],
    "tfl_sweep_counts": [P, ctypes.POINTER(ctypes.c_int64)],
    "tfl_profile_step": [P, ctypes.c_int64, P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "tfl_sync_integer_time": [P, PP, PP, P],
    "tfl_energy": [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), P],
    "tfl_energy_noalloc": [P, P, P],
    "tfl_get_step": [P, ctypes.POINTER(ctypes.c_int64)],
    "tfl_set_step": [P, ctypes.c_int64],
    "tfl_save_state": [P, P, P],
    "tfl_load_state": [P, P, P],
    "tfl_adjoint_sizes": [P, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t),
                          ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
    "tfl_forward_checkpointed": [P, ctypes.POINTER(tfl_objective), ctypes.c_int64, ctypes.c_int64, P,
                                 ctypes.POINTER(ctypes.c_double), P],
    "tfl_adjoint": [P, ctypes.POINTER(tfl_objective), ctypes.c_int64, ctypes.c_int64, P,
                    ctypes.POINTER(ctypes.c_double), P, P, P, P, P],
    "tfl_ringdown_fit": [P, ctypes.c_int, ctypes.POINTER(tfl_fit_req), ctypes.POINTER(tfl_fit_result), P],
    "tfl_fused_buffer_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
    "tfl_bind_fused_buffer": [P, P],
    "tfl_edge_class_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
    "tfl_bind_edge_classes": [P, P, ctypes.POINTER(ctypes.c_int), P],
    "tfl_esprit_fit": [P, ctypes.c_int, ctypes.POINTER(tfl_fit_req), ctypes.c_int32, ctypes.POINTER(tfl_fit_result),
                       P],
    "tfl_adjoint_nested_sizes": [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t),
                                 ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                 ctypes.POINTER(ctypes.c_size_t)],
    "tfl_adjoint_nested": [P, ctypes.POINTER(tfl_objective), ctypes.c_int64, ctypes.c_int64, P,
                           ctypes.POINTER(ctypes.c_double), ctypes.c_int64, P, P, P, P, P, P],
}
OPTIONAL_SIGNATURES = {}


def lib():
    """Load libtfl.so (after torch, so that both use one HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first (__graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, argt in list(SIGNATURES.items()) + list(OPTIONAL_SIGNATURES.items()):
            fn = getattr(L, name)
            fn.argtypes = argt
            fn.restype = ctypes.c_char_p if name == "tfl_last_error" else ctypes.c_int
        _lib = L
    return _lib


def check(rc, handle=None):
    if rc != TFL_OK:
        msg = lib().tfl_last_error(handle)
        raise TflError(rc, msg.decode() if msg else "")
    return rc


def ptr3(ptrs):
    arr = (ctypes.c_void_p * 3)(*ptrs)
    return ctypes.cast(arr, PP), arr


def call(name, *args, handle=None):
    """Call a C entry point and raise TflError on a negative return code."""
    return check(getattr(lib(), name)(*args), handle)
