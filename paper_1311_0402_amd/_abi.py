"""ctypes declarations of the C ABI in include/dpd.h (libdpd.so).

Loading fails loudly when the library has not been built: there is no CPU
fallback for any entry point.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpd.so")
MAX_TYPES = 8

DPD_OK = 0
DPD_EINVAL = -1
DPD_ECAPACITY = -2
DPD_EHIP = -3
DPD_EUNSUPPORTED = -4

STATUS_NLIST_OVERFLOW = 1
STATUS_NONFINITE = 2
STATUS_BAD_BOND = 4
STATUS_HALO_OVERFLOW = 8

FP64 = 0
MIXED = 1

FN_LOG, FN_FASTLOG, FN_COS2PI, FN_FASTCOS2PI, FN_POW, FN_FASTPOW = range(6)


class dpd_params(C.Structure):
    _fields_ = [
        ("box", C.c_double * 3),
        ("r_c", C.c_double),
        ("skin", C.c_double),
        ("dt", C.c_double),
        ("lam", C.c_double),
        ("s", C.c_double),
        ("n_types", C.c_int32),
        ("reserved0", C.c_int32),
        ("a", C.c_double * (MAX_TYPES * MAX_TYPES)),
        ("gamma", C.c_double * (MAX_TYPES * MAX_TYPES)),
        ("sigma", C.c_double * (MAX_TYPES * MAX_TYPES)),
        ("seed", C.c_uint64),
        ("body_g", C.c_double),
        ("body_split", C.c_double),
        ("bond_k", C.c_double),
        ("bond_r0", C.c_double),
        ("bond_partner", C.c_void_p),
    ]


class dpd_state(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("reserved0", C.c_int32),
        ("x", C.c_void_p),
        ("v", C.c_void_p),
        ("f", C.c_void_p),
        ("tag", C.c_void_p),
        ("type", C.c_void_p),
    ]


class dpd_cells(C.Structure):
    _fields_ = [
        ("cell_start", C.c_void_p),
        ("cell_xyz", C.c_void_p),
        ("perm", C.c_void_p),
        ("idx_of_tag", C.c_void_p),
    ]


class dpd_nlist(C.Structure):
    _fields_ = [
        ("capacity", C.c_int64),
        ("offset", C.c_void_p),
        ("index", C.c_void_p),
    ]


class dpd_ghost(C.Structure):
    _fields_ = [
        ("x", C.c_double * 3),
        ("v", C.c_double * 3),
        ("tag", C.c_uint32),
        ("type", C.c_uint32),
    ]


GHOST_BYTES = C.sizeof(dpd_ghost)


class dpd_tiles(C.Structure):
    _fields_ = [
        ("force_grid", C.c_int32),
        ("nlist_waves", C.c_int32),
        ("nlist_kind", C.c_int32),
        ("reserved", C.c_int32),
    ]


P = C.c_void_p
PT = C.POINTER(dpd_tiles)
PP = C.POINTER(dpd_params)
PS = C.POINTER(dpd_state)
PC = C.POINTER(dpd_cells)
PN = C.POINTER(dpd_nlist)

# name -> (restype, argtypes); the exported surface of include/dpd.h
SIGNATURES = {
    "dpd_last_error": (C.c_char_p, []),
    "dpd_version": (C.c_char_p, []),
    "dpd_set_pair_evaluation": (C.c_int, [C.c_int32]),
    "dpd_set_list_builder": (C.c_int, [C.c_int32]),
    "dpd_cell_grid": (C.c_int, [PP, P]),
    "dpd_workspace_bytes": (C.c_size_t, [PP, C.c_int32, C.c_int32]),
    "dpd_bin_reorder": (C.c_int, [PP, PS, PS, PC, P, P, P, C.c_size_t, P]),
    "dpd_build_neighbors": (C.c_int, [PP, PS, PC, P, PN, P, P, C.c_size_t, P]),
    "dpd_forces": (C.c_int, [PP, C.c_int32, PS, PC, P, P, PN, C.c_uint64, P, P, P, P, P, C.c_size_t, P]),
    "dpd_forces_noalloc": (C.c_int, [PP, C.c_int32, PS, PC, P, P, PN, C.c_uint64, P, P, P, P, P]),
    "dpd_step": (C.c_int, [PP, C.c_int32, PS, C.c_int32, P, P, PC, PN, P, P, P, P, P, C.c_size_t, P]),
    "dpd_forces_backward": (C.c_int, [PP, PS, PC, PN, C.c_uint64, P, P, P, P, P, C.c_int32, P, C.c_size_t, P]),
    "dpd_step_backward": (C.c_int, [PP, PS, PC, PN, C.c_uint64, P, P, P, P, P, P, P, P, P, C.c_size_t, P]),
    "dpd_border_workspace_bytes": (C.c_size_t, [C.c_int32]),
    "dpd_border_lists": (C.c_int, [PS, P, P, C.c_double, C.c_int32, P, P, C.c_int64, P, P, C.c_size_t, P]),
    "dpd_border_pack": (C.c_int, [PS, P, P, C.c_int64, P, P, P, P]),
    "dpd_border_unpack": (C.c_int, [P, P, C.c_int64, PS, C.c_int32, P, P]),
    "dpd_math_eval": (C.c_int, [C.c_int32, C.c_int64, P, P, P, P]),
    "dpd_math_latency": (C.c_int, [C.c_int32, C.c_int32, P, P, P]),
    "dpd_tea_signatures": (C.c_int, [C.c_int32, P, P, C.c_uint64, C.c_uint64, P, P]),
    "dpd_tea_gaussians": (C.c_int, [C.c_int64, P, P, C.c_uint64, C.c_uint64, P, P, P]),
    "dpd_gaussian_throughput": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_uint64, P, P, P]),
    "dpd_batch_table_bytes": (C.c_size_t, [C.c_int32, C.c_int64]),
    "dpd_batch_create": (C.c_int, [PP, C.c_int32, P, P, C.c_size_t, P, C.POINTER(C.c_void_p)]),
    "dpd_batch_destroy": (None, [P]),
    "dpd_batch_sizes": (C.c_int, [P, P, P]),
    "dpd_batch_workspace_bytes": (C.c_size_t, [P, C.c_int32]),
    "dpd_batch_set_tiles": (C.c_int, [P, PT]),
    "dpd_batch_get_tiles": (C.c_int, [P, PT]),
    "dpd_batch_bin_reorder": (C.c_int, [P, PS, PS, PC, P, P, P, C.c_size_t, P]),
    "dpd_batch_build_neighbors": (C.c_int, [P, PS, PC, P, PN, P, P, C.c_size_t, P]),
    "dpd_batch_forces": (C.c_int, [P, C.c_int32, PS, PC, P, P, PN, C.c_uint64, P, P, P, P, C.c_size_t, P]),
    "dpd_batch_step": (C.c_int, [P, C.c_int32, PS, C.c_int32, P, P, PC, PN, P, P, P, C.c_int32, P, C.c_size_t,
                                 P]),
}

_lib = None


def lib():
    """The loaded libdpd (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_1311_0402_amd.build)")
        # torch first, so libdpd binds to the HIP runtime torch already loaded
        import torch  # noqa: F401
        handle = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


class DPDError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().dpd_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


def check(code: int, where: str) -> None:
    if code != DPD_OK:
        raise DPDError(code, where)
