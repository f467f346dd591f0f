"""ctypes binding of libephx.so (the C ABI in include/ephx.h).

Argument marshalling only: device arrays are torch tensors on the current
HIP device, handed over as data pointers together with torch's current
stream.  Every step of the computation runs in the library's kernels; there
is no fallback of any kind -- if the library is missing, importing this module
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libephx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libephx.so is not built (expected at %s); run `python -m paper_2002_02045_amd.build`" % LIB_PATH)

lib = C.CDLL(LIB_PATH)

FP64, FP32, BF16X3, BF16X6, FP16X3 = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "bf16x6": BF16X6, "fp16x3": FP16X3}
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOTHERM", -5: "ENAN", -6: "EUNSUPPORTED"}


class EphxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class ModelDesc(C.Structure):
    _fields_ = [
        ("lattice", C.c_double * 9),
        ("natoms", C.c_int), ("tau", C.c_void_p), ("mass", C.c_void_p),
        ("nw", C.c_int),
        ("n_re", C.c_int), ("re", C.c_void_p), ("w_re", C.c_void_p), ("h", C.c_void_p),
        ("n_rp_ph", C.c_int), ("rp_ph", C.c_void_p), ("w_rp_ph", C.c_void_p), ("ifc", C.c_void_p),
        ("n_re_g", C.c_int), ("re_g", C.c_void_p), ("w_re_g", C.c_void_p),
        ("n_rp_g", C.c_int), ("rp_g", C.c_void_p), ("w_rp_g", C.c_void_p),
        ("g", C.c_void_p),
        ("polar", C.c_int), ("zstar", C.c_void_p), ("eps_inf", C.c_void_p),
        ("alpha_ewald", C.c_double), ("gcut", C.c_double),
        ("g_gen", C.c_int), ("g_seed", C.c_uint64), ("g_env", C.c_void_p),
    ]


class Params(C.Structure):
    _fields_ = [("temp", C.c_double), ("mu", C.c_double), ("sigma", C.c_double),
                ("omega_cut", C.c_double), ("n_q", C.c_double)]


_P = C.c_void_p
_I = C.c_int
_D = C.c_double
_SIGS = {
    "ephx_last_error": ([], C.c_char_p),
    "ephx_version": ([], C.c_char_p),
    "ephx_model_create": ([_P, _P], _I),
    "ephx_model_destroy": ([_P], _I),
    "ephx_bands": ([_P, _I, _P, _P, _P, _P, _P], _I),
    "ephx_phonons": ([_P, _I, _P, _P, _P, _P], _I),
    "ephx_gkq": ([_P, _I, _P, _I, _P, _I, _D, _P, _P], _I),
    "ephx_rates": ([_P, _P, _I, _P, _I, _P, _P, _I, _P, _P, _P], _I),
    "ephx_rates_vjp": ([_P, _P, _I, _P, _I, _P, _P, _P, _P, _P], _I),
    "ephx_rates_part": ([_P, _P, _I, _I, _P, _I, _P, _P, _I, _P, _P, _P], _I),
    "ephx_rates_polar_split": ([_P, _P, _I, _P, _I, _P, _P, _I, _P, _P, _I, _P, _P, _P], _I),
    "ephx_grid_states": ([_P, _P, _I, _I, _I, _D, _D, _I, _I, _P, _P, _P, _P, _P], _I),
    "ephx_table_create": ([_P, _P, _I, _P, _P, _I, _D, _P, _P], _I),
    "ephx_table_destroy": ([_P], _I),
    "ephx_table_g2": ([_P, _P, _P, _P], _I),
    "ephx_collision_setup": ([_P, _P, _P, _P], _I),
    "ephx_collision": ([_P, _P, _P, _P], _I),
    "ephx_collision_noalloc": ([_P, _P, _P, _P], _I),
    "ephx_dynamics": ([_P, _P, _D, _I, _I, _P, _P, _P], _I),
    "ephx_dynamics_field": ([_P, _P, _D, _I, _I, _P, _I, _P, _P, _P], _I),
    "ephx_gkq_pairs": ([_P, _I, _P, _I, _P, _I, _P, _P, _I, _D, _P, _P], _I),
    "ephx_workspace_query": ([_P, _I, _I, _I, _I, _P], _I),
    "ephx_table_stream_info": ([_P, _I, _P, _P, _P, _P], _I),
    "ephx_collision_vjp": ([_P, _P, _P, _P, _P, _P], _I),
    "ephx_dynamics_vjp": ([_P, _P, _D, _I, _I, _P, _P, _P, _P], _I),
    "ephx_mobility": ([_P, _P, _P, _I, _D, _P, _P, _P, _P, _P, _P], _I),
    "ephx_model_set_g": ([_P, _P, _P], _I),
    "ephx_model_g_entries": ([_P, _I, _P, _P], _I),
    "ephx_mobility_vjp": ([_P, _P, _P, _I, _P, _P, _P], _I),
    "ephx_tdf": ([_P, _P, _P, _P, _I, _P, _P, _P, _P, _P], _I),
    "ephx_population": ([_P, _P, _I, _P, _P, _P], _I),
    "ephx_timer_enable": ([_I], _I),
    "ephx_timer_reset": ([], _I),
    "ephx_timer_get": ([C.c_char_p, _P, _P], _I),
}
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


def check(code):
    if code != 0:
        raise EphxError(code, lib.ephx_last_error().decode())


def stream_ptr():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def ptr(t):
    """Device pointer of a contiguous torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("arrays handed to the library must be contiguous")
    return C.c_void_p(t.data_ptr())


def host_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def timer_enable(on=True):
    check(lib.ephx_timer_enable(1 if on else 0))


def timer_reset():
    check(lib.ephx_timer_reset())


def timer_get(stage):
    """(launches, total_ms) of a stage; synchronises its events."""
    n = C.c_int(0)
    ms = C.c_double(0.0)
    check(lib.ephx_timer_get(stage.encode(), C.byref(n), C.byref(ms)))
    return n.value, ms.value
