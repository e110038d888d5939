"""ctypes binding of libsampx.so (the C ABI of include/sampx.h).

Argument marshalling only.  The library is loaded from the package folder;
if it is missing the import of any compute entry point fails loudly (there
is no CPU fallback).  Build it with ``python -m paper_2301_04835_amd.build``
or ``__graft_entry__.build()``.
"""
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsampx.so")
MEASURE_LIB_PATH = os.path.join(HERE, "libsampx_measure.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sampx.h")
MEASURE_HEADER = os.path.join(os.path.dirname(HERE), "include", "sampx_measure.h")

SX_OK, SX_EINVAL, SX_ENOMEM, SX_ECAPACITY, SX_ENONFINITE, SX_EDEVICE, SX_ESTATE = range(7)
SX_F32, SX_F64 = 0, 1
SX_AOS3, SX_AOS4, SX_SOA = 0, 1, 2
SX_STEP_DEVICE = -1

P = ctypes.c_void_p
i32, i64, f64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
PP = ctypes.POINTER(ctypes.c_void_p)

# name: (restype, argtypes)
SIGNATURES = {
    "sx_create": (i32, [PP, ctypes.c_int, P]),
    "sx_destroy": (None, [P]),
    "sx_last_error": (ctypes.c_char_p, [P]),
    "sx_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sx_set_stream": (i32, [P, P]),
    "sx_add_cv_dihedral": (i32, [P, P]),
    "sx_add_cv_gyration": (i32, [P, P, i32]),
    "sx_add_cv_coordination": (i32, [P, P, i32, P, i32, f64, i32, i32, f64, i32]),
    "sx_set_box": (i32, [P, P]),
    "sx_num_cvs": (i32, [P]),
    "sx_set_walkers": (i32, [P, i32, P, P, i32]),
    "sx_metad_config": (i32, [P, P, f64, f64, f64, i32, i64]),
    "sx_metad_config_dT": (i32, [P, P, f64, f64, i32, i64]),
    "sx_abf_config": (i32, [P, P, P, P, i32]),
    "sx_state_bytes": (sz, [P]),
    "sx_workspace_bytes": (sz, [P]),
    "sx_bind": (i32, [P, P, sz, P, sz]),
    "sx_step": (i32, [P, P, i32, i32, i64, P, P, P, P, P]),
    "sx_check": (i32, [P]),
    "sx_eval_cv": (i32, [P, P, i32, i32, P, P]),
    "sx_jac_slots": (i64, [P]),
    "sx_jac_layout": (i32, [P, P, P]),
    "sx_cv_vjp": (i32, [P, P, i32, i32, P, P]),
    "sx_hillsum": (i32, [P, P, P, P]),
    "sx_deposit": (i32, [P, P]),
    "sx_bias_eval": (i32, [P, i32, P, i64, P, P]),
    "sx_bias_eval_noalloc": (i32, [P, i32, P, i64, P, P]),
    "sx_hills_set": (i32, [P, i32, P, P, i64]),
    "sx_hills_get": (i32, [P, i32, P, P, i64, P]),
    "sx_abf_grid_get": (i32, [P, i32, P, P]),
    "sx_get_step": (i32, [P, P]),
    "sx_checkpoint_bytes": (sz, [P]),
    "sx_state_export": (i32, [P, P, sz]),
    "sx_state_import": (i32, [P, P, sz]),
    "sx_graph_capture": (i32, [P, i32, P, i32, i32, P, P, P, P, P]),
    "sx_graph_launch": (i32, [P]),
    "sx_set_tuning": (i32, [P, i32, i32]),
    "sx_get_tuning": (i32, [P, P, P]),
    "sx_autotune": (i32, [P, P, i32, i32, ctypes.c_char_p]),
    "sx_metad_grid": (i32, [P, P, P, P]),
    "sx_harmonic_config": (i32, [P, P, P, i32]),
    "sx_fes_metad": (i32, [P, i32, P, ctypes.c_int64, f64, P]),
    "sx_fes_metad_grid": (i32, [P, i32, P, P, P, f64, P, P, i64]),
    "sx_abf_fes": (i32, [P, i32, P]),
    "sx_abf_momentum": (i32, [P, f64, P, ctypes.c_int64]),
    "sx_funn_fit": (i32, [P, i32, i32, i32, f64, f64, P, P]),
    "sx_funn_enable": (i32, [P, i32]),
    "sx_umbrella_reset": (i32, [P]),
    "sx_umbrella_stats": (i32, [P, P, P, P]),
    "sx_umbrella_integrate": (i32, [P, P, P]),
    "sx_grid_nodes": (ctypes.c_int64, [P]),
    "sx_grid_eval": (i32, [P, i32, P, ctypes.c_int64, P, P]),
    "sx_grid_get": (i32, [P, i32, P, P, ctypes.c_int64]),
    "sx_set_cell_lists": (i32, [P, i32]),
    "sx_cell_list_cvs": (i32, [P]),
    "sx_surrogate_config": (i32, [P, i32, i64, i32, i32, f64]),
    "sx_surrogate_norm": (i32, [P, P, P]),
    "sx_surrogate_param_count": (i64, [P]),
    "sx_surrogate_params_set": (i32, [P, P, i64]),
    "sx_surrogate_params_get": (i32, [P, P, i64]),
    "sx_surrogate_output": (i32, [P, f64, f64]),
    "sx_surrogate_output_get": (i32, [P, P, P]),
    "sx_surrogate_eval": (i32, [P, P, i64, P, P, P]),
    "sx_surrogate_loss_grad": (i32, [P, P, P, P, i64, f64, f64, P, P]),
    "sx_surrogate_fit": (i32, [P, P, P, P, i64, i32, i32, f64, f64, f64, f64, P]),
    "sx_surrogate_train": (i32, [P, P, i64, i32, i32, f64, f64, P]),
    "sx_surrogate_certify": (i32, [P, P, P, P]),
    "sx_surrogate_tolerance": (i32, [P, f64]),
    "sx_surrogate_enable": (i32, [P, i32]),
    "sx_surrogate_fallback_count": (i32, [P, P]),
}

# the measurement library (include/sampx_measure.h): hooks exported by
# libsampx.so, timing and probes in libsampx_measure.so
MEASURE_HOOKS = {
    "sxm_stream": (P, [P]),
    "sxm_enqueue_hill": (i32, [P, P, P, i32, i32, P, i32]),
    "sxm_enqueue_cell": (i32, [P, P, P, i32, i32, P, i32]),
}
MEASURE_SIGNATURES = {
    "sx_time_hill": (i32, [P, P, i32, i32, P, i32, P, P]),
    "sx_time_cell": (i32, [P, P, i32, i32, P, i32, P, P, P]),
    "sx_time_hill_step": (i32, [P, P, i32, i32, P, i32, P, P]),
    "sx_probe_noop": (i32, [P]),
    "sx_probe_read": (i32, [P, sz, P, i32, i32, P]),
    "sx_probe_copy": (i32, [P, P, sz, i32, P]),
}

_lib = None
_mlib = None


def load_measure(path=MEASURE_LIB_PATH):
    """Load libsampx_measure.so (after libsampx.so, which it links) and
    attach the signatures of the timing and probe calls."""
    global _mlib
    if _mlib is not None:
        return _mlib
    load()
    if not os.path.exists(path):
        raise RuntimeError("libsampx_measure.so not built at %s: run paper_2301_04835_amd/build.py" % path)
    M = ctypes.CDLL(path)
    for name, (res, args) in MEASURE_SIGNATURES.items():
        fn = getattr(M, name)
        fn.restype = res
        fn.argtypes = args
    _mlib = M
    return M


def header_symbols(path=HEADER):
    """Names of the functions include/sampx.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sxm?_[A-Za-z0-9_]+)\s*\(", text)))


def load(path=LIB_PATH):
    """Load libsampx.so and attach the signatures.  Raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libsampx.so not built at %s: run paper_2301_04835_amd/build.py "
                           "(there is no CPU fallback)" % path)
    L = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class SxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("sampx status %d (%s): %s" % (status, _STATUS.get(status, "?"), msg))
        self.status = status


_STATUS = {0: "ok", 1: "invalid argument", 2: "buffer too small", 3: "hill capacity exceeded",
           4: "non-finite value", 5: "device error", 6: "call out of order"}
