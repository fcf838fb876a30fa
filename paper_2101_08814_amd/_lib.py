"""ctypes loader of libsoap_mi355x.so (the C ABI declared in include/soap_mi355x.h).

There is no fallback: if the library is missing, importing the entry points
raises.  Build it with ``python -m paper_2101_08814_amd.build_lib``.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# another build of the same sources (for example one with host-side
# sanitizers) can be named in SOAP_MI355X_LIBRARY
LIB_PATH = os.environ.get("SOAP_MI355X_LIBRARY") or os.path.join(HERE, "libsoap_mi355x.so")

SOAP_OK, SOAP_EINVAL, SOAP_ECAPACITY, SOAP_EDEVICE = 0, -1, -2, -3
SOAP_ENOMEM, SOAP_EUNSUPPORTED, SOAP_EGEOMETRY, SOAP_ESPECIES = -4, -5, -6, -7
SOAP_F64, SOAP_F32, SOAP_BF16_F32ACC = 0, 1, 2
SOAP_RADIAL_GTO, SOAP_RADIAL_DVR = 0, 1

STATUS_NAMES = {0: "SOAP_OK", -1: "SOAP_EINVAL", -2: "SOAP_ECAPACITY", -3: "SOAP_EDEVICE",
                -4: "SOAP_ENOMEM", -5: "SOAP_EUNSUPPORTED", -6: "SOAP_EGEOMETRY", -7: "SOAP_ESPECIES"}

# every symbol the header declares
EXPORTS = [
    "soap_abi_version", "soap_last_error", "soap_calculator_create", "soap_calculator_destroy",
    "soap_calculator_info", "soap_calculator_upload", "soap_radial_integral_host", "soap_radial_integral",
    "soap_neighbors_workspace_size", "soap_compute_neighbors", "soap_compute_neighbors_noalloc",
    "soap_spherical_expansion",
    "soap_power_spectrum", "soap_features", "soap_gradient_rows", "soap_power_spectrum_backward",
    "soap_spherical_expansion_backward", "soap_virial", "soap_power_spectrum_selected",
    "soap_power_spectrum_selected_plan", "soap_power_spectrum_selected_backward", "soap_gpr_workspace_size", "soap_gpr_predict",
    "soap_compress_n_params", "soap_compress_workspace_size", "soap_compress_save", "soap_compress_load",
    "soap_compress_forward_ws",
    "soap_compress_init_pca", "soap_compress_forward", "soap_compress_backward", "soap_spectrum_gram",
    "soap_spectrum_kernel_loss", "soap_adam_step", "soap_read_device_status",
]


class soap_hypers(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("nmax", ctypes.c_int32), ("lmax", ctypes.c_int32),
                ("include_center", ctypes.c_int32), ("rcut", ctypes.c_double), ("cutoff_width", ctypes.c_double),
                ("sigma", ctypes.c_double), ("spline_accuracy", ctypes.c_double), ("radial_basis", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class soap_table_info(ctypes.Structure):
    _fields_ = [("n_intervals", ctypes.c_int64), ("delta", ctypes.c_double), ("max_error", ctypes.c_double),
                ("max_error_deriv", ctypes.c_double), ("overlap_condition", ctypes.c_double),
                ("table_bytes_f64", ctypes.c_int64), ("table_bytes_f32", ctypes.c_int64)]


class soap_exec(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("dev_status", ctypes.c_void_p)]


class SoapError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2101_08814_amd.build_lib`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    st = ctypes.c_int
    L.soap_abi_version.restype = i32
    L.soap_last_error.restype = ctypes.c_char_p
    L.soap_calculator_create.restype = st
    L.soap_calculator_create.argtypes = [P(soap_hypers), P(vp)]
    L.soap_calculator_destroy.restype = st
    L.soap_calculator_destroy.argtypes = [vp]
    L.soap_calculator_info.restype = st
    L.soap_calculator_info.argtypes = [vp, P(soap_table_info)]
    L.soap_calculator_upload.restype = st
    L.soap_calculator_upload.argtypes = [vp]
    L.soap_radial_integral_host.restype = st
    L.soap_radial_integral_host.argtypes = [vp, i32, i64, vp, vp, vp]
    L.soap_radial_integral.restype = st
    L.soap_radial_integral.argtypes = [vp, P(soap_exec), st, i32, i64, vp, vp, vp]
    L.soap_neighbors_workspace_size.restype = st
    L.soap_neighbors_workspace_size.argtypes = [vp, i32, i64, P(ctypes.c_size_t)]
    L.soap_compute_neighbors.restype = st
    L.soap_compute_neighbors.argtypes = [vp, P(soap_exec), i32, i64, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, i64,
                                         st, vp, vp, vp, vp, vp]
    L.soap_compute_neighbors_noalloc.restype = st
    L.soap_compute_neighbors_noalloc.argtypes = [vp, P(soap_exec), i32, i64, vp, vp, vp, vp, vp, i64, st, vp, vp,
                                                 vp, vp, vp]
    L.soap_spherical_expansion.restype = st
    L.soap_spherical_expansion.argtypes = [vp, P(soap_exec), st, i64, vp, vp, vp, vp, i64, vp, vp, vp]
    L.soap_power_spectrum.restype = st
    L.soap_power_spectrum.argtypes = [vp, P(soap_exec), st, i64, vp, vp, vp, vp, vp, i64, vp, vp, vp, vp]
    L.soap_features.restype = st
    L.soap_features.argtypes = [vp, P(soap_exec), st, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp]
    L.soap_gradient_rows.restype = st
    L.soap_gradient_rows.argtypes = [vp, P(soap_exec), st, i64, vp, vp, vp, vp, i64, vp, vp, vp]
    L.soap_power_spectrum_backward.restype = st
    L.soap_power_spectrum_backward.argtypes = [vp, P(soap_exec), st, i64, vp, vp, vp]
    L.soap_spherical_expansion_backward.restype = st
    L.soap_spherical_expansion_backward.argtypes = [vp, P(soap_exec), st, i64, vp, vp, vp, vp, vp, i64, vp, vp, vp]
    L.soap_virial.restype = st
    L.soap_virial.argtypes = [P(soap_exec), st, i32, vp, i64, vp, vp, vp, i64, vp, vp]
    u64, f32, sz = ctypes.c_uint64, ctypes.c_float, ctypes.c_size_t
    L.soap_power_spectrum_selected.restype = st
    L.soap_power_spectrum_selected.argtypes = [P(soap_exec), st, i64, i32, i32, vp, i64, vp, vp]
    L.soap_power_spectrum_selected_plan.restype = st
    L.soap_power_spectrum_selected_plan.argtypes = [i32, i32, i64, vp, vp, vp]
    L.soap_power_spectrum_selected_backward.restype = st
    L.soap_power_spectrum_selected_backward.argtypes = [P(soap_exec), st, i64, i32, i32, vp, i64, vp, vp, vp, vp]
    L.soap_gpr_workspace_size.restype = st
    L.soap_gpr_workspace_size.argtypes = [st, i64, i64, i64, P(sz)]
    L.soap_gpr_predict.restype = st
    L.soap_gpr_predict.argtypes = [P(soap_exec), st, i64, i64, vp, vp, i64, vp, vp, vp, i32, vp, sz, vp, vp]
    L.soap_compress_n_params.restype = st
    L.soap_compress_n_params.argtypes = [vp, i32, i32, P(i64)]
    L.soap_compress_forward_ws.restype = st
    L.soap_compress_forward_ws.argtypes = [vp, vp, ctypes.c_int, i32, i32, i64, vp, vp, vp, vp, vp, ctypes.c_size_t]
    L.soap_compress_save.restype = st
    L.soap_compress_save.argtypes = [vp, i32, i32, i64, vp, vp, vp, ctypes.c_char_p]
    L.soap_compress_load.restype = st
    L.soap_compress_load.argtypes = [vp, i32, i32, ctypes.c_char_p, vp, vp, vp, P(i64)]
    L.soap_compress_workspace_size.restype = st
    L.soap_compress_workspace_size.argtypes = [vp, i32, i32, P(sz)]
    L.soap_compress_init_pca.restype = st
    L.soap_compress_init_pca.argtypes = [vp, P(soap_exec), i32, i32, i64, vp, u64, f32, vp, sz, vp]
    L.soap_compress_forward.restype = st
    L.soap_compress_forward.argtypes = [vp, P(soap_exec), st, i32, i32, i64, vp, vp, vp, vp]
    L.soap_compress_backward.restype = st
    L.soap_compress_backward.argtypes = [vp, P(soap_exec), i32, i32, i64, vp, vp, vp, vp, sz, vp]
    L.soap_spectrum_gram.restype = st
    L.soap_spectrum_gram.argtypes = [P(soap_exec), i32, i32, i32, vp, vp]
    L.soap_spectrum_kernel_loss.restype = st
    L.soap_spectrum_kernel_loss.argtypes = [P(soap_exec), i32, i32, i32, vp, vp, vp, vp, vp]
    L.soap_adam_step.restype = st
    L.soap_adam_step.argtypes = [P(soap_exec), i64, vp, vp, vp, vp, f32, f32, f32, f32, i32]
    L.soap_read_device_status.restype = st
    L.soap_read_device_status.argtypes = [P(soap_exec)]
    _lib = L
    return L


def check(status: int) -> None:
    if status != SOAP_OK:
        msg = lib().soap_last_error().decode(errors="replace")
        raise SoapError(status, msg)
