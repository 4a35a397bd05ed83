"""ctypes declarations of the C ABI in include/litho.h (no torch, no compute)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.environ.get("LITHO_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                            "liblitho.so")

LITHO_OK = 0
LITHO_PENDING = 1
LITHO_E_INVALID = -1
LITHO_E_UNSUPPORTED = -2
LITHO_E_NOMEM = -3
LITHO_E_HIP = -4
LITHO_E_BUSY = -5
LITHO_E_NOTFOUND = -6

LITHO_SRC_ANNULAR = 0
LITHO_SRC_DIPOLE_X = 1
LITHO_SRC_DIPOLE_Y = 2
LITHO_SRC_POINTS = 3
LITHO_PREC_FP32 = 0
LITHO_PREC_F16X3 = 1
LITHO_PREC_BF16X3 = 2
LITHO_PREC_F16 = 3
LITHO_PREC_BF16 = 4
PREC_NAMES = {"fp32": LITHO_PREC_FP32, "f16x3": LITHO_PREC_F16X3, "bf16x3": LITHO_PREC_BF16X3,
              "f16": LITHO_PREC_F16, "bf16": LITHO_PREC_BF16}

ERROR_NAMES = {
    LITHO_E_INVALID: "LITHO_E_INVALID", LITHO_E_UNSUPPORTED: "LITHO_E_UNSUPPORTED",
    LITHO_E_NOMEM: "LITHO_E_NOMEM", LITHO_E_HIP: "LITHO_E_HIP", LITHO_E_BUSY: "LITHO_E_BUSY",
    LITHO_E_NOTFOUND: "LITHO_E_NOTFOUND",
}


class Optics(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("pixel_nm", C.c_double), ("wavelength_nm", C.c_double), ("na", C.c_double),
        ("source_kind", C.c_int), ("source_grid", C.c_int), ("sigma_in", C.c_double),
        ("sigma_out", C.c_double), ("n_focus", C.c_int), ("focus_nm", C.POINTER(C.c_double)),
        ("K", C.c_int), ("dose", C.c_double), ("src_points", C.POINTER(C.c_double)), ("n_src_points", C.c_int),
    ]


class BankInfo(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("b", C.c_int), ("B", C.c_int), ("K", C.c_int), ("n_focus", C.c_int),
        ("n_source", C.c_int), ("inner_grid", C.c_int), ("pupil_radius", C.c_double),
        ("device_bytes", C.c_size_t), ("clear_field", C.c_double), ("degeneracy_gap", C.c_double),
    ]


LITHO_LOSS_L2 = 0
LITHO_LOSS_L1 = 1


class Resist(C.Structure):
    _fields_ = [("slope", C.c_double), ("threshold", C.c_double), ("plane_weight", C.POINTER(C.c_double)),
                ("blur_sigma_px", C.c_double), ("loss", C.c_int)]


class EpeRule(C.Structure):
    _fields_ = [("t_eff", C.c_double), ("tol_neg", C.c_double), ("tol_pos", C.c_double), ("f0", C.c_int)]


class ServeCfg(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_slots", C.c_int), ("max_queue", C.c_int)]


class Request(C.Structure):
    _fields_ = [
        ("bank", C.c_int), ("K_use", C.c_int), ("mode", C.c_int),
        ("h_mask", C.POINTER(C.c_float)), ("h_target", C.POINTER(C.c_float)),
        ("slope", C.c_double), ("threshold", C.c_double), ("prec", C.c_int),
        ("d_mask", C.c_void_p), ("d_target", C.c_void_p), ("d_image", C.c_void_p), ("d_grad", C.c_void_p),
        ("d_loss", C.c_void_p),
    ]


class ResultInfo(C.Structure):
    _fields_ = [
        ("status", C.c_int), ("n", C.c_int), ("n_focus", C.c_int), ("loss", C.c_double),
        ("t_submit_us", C.c_double), ("t_start_us", C.c_double), ("t_done_us", C.c_double),
    ]


VP = C.c_void_p
SIGNATURES = {
    "litho_kernels_build": (C.c_int, [C.POINTER(Optics), C.POINTER(VP)]),
    "litho_kernels_load": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(VP)]),
    "litho_kernels_info": (C.c_int, [VP, C.POINTER(BankInfo)]),
    "litho_kernels_set_inner_grid": (C.c_int, [VP, C.c_int]),
    "litho_kernels_eigenvalues": (C.c_int, [VP, C.POINTER(C.c_double)]),
    "litho_kernels_phi": (C.c_int, [VP, C.c_int, C.c_int, C.POINTER(C.c_double)]),
    "litho_kernels_free": (None, [VP]),
    "litho_socs_host": (C.c_int, [C.POINTER(Optics), C.c_int, C.c_int, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "litho_image": (C.c_int, [VP, VP, C.c_int, C.c_int, VP, C.c_int, VP]),
    "litho_image_grad": (C.c_int, [VP, VP, C.c_int, C.c_int, VP, C.POINTER(Resist), VP, VP, VP, VP,
                                   C.c_int, VP]),
    "litho_lowpass": (C.c_int, [VP, VP, C.c_int, C.c_double, C.c_double, VP, VP]),
    "litho_contours": (C.c_int, [C.c_int, VP, C.c_double, C.c_int, VP, VP, VP, VP, VP, VP]),
    "litho_contours_noalloc": (C.c_int, [C.c_int, VP, C.c_double, C.c_int, VP, VP, VP, VP, VP, VP]),
    "litho_epe": (C.c_int, [C.c_int, VP, VP, C.c_int, C.POINTER(EpeRule), C.c_int, VP, VP, VP, VP, VP]),
    "litho_ai_channels": (C.c_int, [VP, VP, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double), VP, VP]),
    "litho_image_tiled": (C.c_int, [VP, VP, C.c_int, C.c_int, C.c_int, C.c_int, VP, C.c_int, VP]),
    "litho_image_grad_tiled": (C.c_int, [VP, VP, C.c_int, C.c_int, C.c_int, C.c_int, VP, C.POINTER(Resist), VP, VP,
                                         VP, C.c_int, VP]),
    "litho_profile_enable": (C.c_int, [C.c_int]),
    "litho_profile_read": (C.c_int, [C.c_char_p, C.c_size_t]),
    "litho_serve_create": (C.c_int, [C.POINTER(VP), C.c_int, C.POINTER(ServeCfg), C.POINTER(VP)]),
    "litho_serve_submit": (C.c_int, [VP, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "litho_serve_poll": (C.c_int, [VP, C.c_uint64, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                   C.POINTER(ResultInfo), C.c_int64]),
    "litho_serve_destroy": (None, [VP]),
    "litho_last_error": (C.c_char_p, []),
}


def header_symbols(header_path: str) -> list:
    """Names of the functions declared in a litho header (for ABI tests)."""
    import re
    text = open(header_path).read()
    return sorted(set(re.findall(r"\b(litho_[a-z_]+)\s*\(", text)))


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """dlopen liblitho.so and declare every entry point; raises if missing."""
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is not built: run `python -m paper_2602_15036_amd.build` "
            "(the HIP library is required; there is no fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib
