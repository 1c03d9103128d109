"""ctypes binding of ``libftlm.so`` (the C ABI in ``include/ftlm.h``).

Argument marshalling only: every step of the path runs inside the library.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libftlm.so")

F64, F32, F16 = 0, 1, 2
RADEMACHER, GAUSSIAN = 0, 1
HV_AUTO, HV_ENTRIES, HV_ONTHEFLY = 0, 1, 2
LAYOUT_AUTO, LAYOUT_BLOCK, LAYOUT_PADDED, LAYOUT_PACKED, LAYOUT_ALIGNED = 0, 1, 2, 3, 4
ENTRIES_AUTO, ENTRIES_WIDE, ENTRIES_COMPACT = 0, 1, 2
ENGINE_AUTO, ENGINE_STEPS, ENGINE_FUSED = 0, 1, 2

STATUS = {
    0: "OK", -1: "INVALID_ARG", -2: "NOT_A_PERMUTATION", -3: "GROUP_TOO_LARGE",
    -4: "BONDS_NOT_INVARIANT", -5: "IRREP_OUT_OF_RANGE", -6: "ROW_OUT_OF_RANGE",
    -7: "DIM_GT_12", -8: "COMPLEX_IRREP_UNSUPPORTED", -9: "OUT_OF_MEMORY", -10: "HIP",
    -11: "BAD_RHO", -12: "UNSUPPORTED", -13: "IRREPS_FAILED", -14: "CANCELLED",
    -15: "QUEUE_FULL",
}


class FtlmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class Cluster(C.Structure):
    _fields_ = [("N", C.c_int32), ("two_s", C.c_int32), ("nbonds", C.c_int32),
                ("bonds", C.POINTER(C.c_int32)), ("J", C.POINTER(C.c_double))]


class Opts(C.Structure):
    _fields_ = [("hv_mode", C.c_int32), ("lanczos_layout", C.c_int32),
                ("user_rho", C.POINTER(C.c_double)), ("user_rho_dim", C.c_int32),
                ("entry_format", C.c_int32), ("hbm_limit_bytes", C.c_int64),
                ("spin_flip", C.c_int32), ("user_rho_weight", C.c_int32), ("reserved", C.c_int64 * 5)]


class SectorInfo(C.Structure):
    _fields_ = [("D_M", C.c_uint64), ("n_reps", C.c_uint64), ("n_entries", C.c_uint64),
                ("n_stab", C.c_int32), ("label_bits", C.c_int32), ("device_bytes", C.c_int64)]


class BlockInfo(C.Structure):
    _fields_ = [("D_M", C.c_uint64), ("n_reps", C.c_uint64), ("n_active", C.c_uint64),
                ("D", C.c_uint64), ("d_gamma", C.c_int32), ("group_order", C.c_int32),
                ("two_M", C.c_int32), ("irrep", C.c_int32), ("row", C.c_int32),
                ("hv_mode", C.c_int32), ("device_bytes", C.c_int64), ("trace_weight", C.c_int32),
                ("reserved", C.c_int32)]


class HvStats(C.Structure):
    _fields_ = [("n_active", C.c_uint64), ("connections", C.c_uint64), ("active_connections", C.c_uint64),
                ("gathered_rows", C.c_uint64), ("nontrivial_targets", C.c_uint64), ("entry_bytes", C.c_int32),
                ("reserved", C.c_int32)]


class HvOpts(C.Structure):
    _fields_ = [("layout", C.c_int32), ("lanes", C.c_int32), ("scale", C.c_void_p), ("dots", C.c_void_p),
                ("shift", C.c_double), ("lanes_used", C.c_int32), ("adjacent_columns", C.c_int32),
                ("reserved", C.c_int64 * 4)]


class CampaignOpts(C.Structure):
    _fields_ = [("R", C.c_int32), ("steps", C.c_int32), ("seed", C.c_uint64), ("storage", C.c_int32),
                ("dist", C.c_int32), ("all_M", C.c_int32), ("two_M", C.c_int32), ("spin_flip", C.c_int32),
                ("chains_per_run", C.c_int32), ("g", C.c_double), ("engine", C.c_int32),
                ("fused_max_rounds", C.c_int32)]


class CampaignStats(C.Structure):
    _fields_ = [("sectors", C.c_int32), ("blocks", C.c_int32), ("empty_blocks", C.c_int32), ("fused_blocks", C.c_int32),
                ("rows", C.c_uint64), ("products", C.c_uint64), ("work", C.c_uint64),
                ("seconds_build", C.c_double), ("seconds_lanczos", C.c_double), ("seconds_thermo", C.c_double),
                ("seconds_total", C.c_double)]


class RunInfo(C.Structure):
    _fields_ = [("layout", C.c_int32), ("hv_launches", C.c_int32), ("rows", C.c_uint64), ("hv_ms", C.c_double)]


class FusedJob(C.Structure):
    _fields_ = [("block", C.c_void_p), ("R", C.c_int32), ("steps", C.c_int32), ("seed", C.c_uint64),
                ("storage", C.c_int32), ("dist", C.c_int32), ("first_chain", C.c_int32), ("reserved", C.c_int32),
                ("alpha", C.POINTER(C.c_double)), ("beta", C.POINTER(C.c_double)), ("nsteps", C.POINTER(C.c_int32))]


class JobDesc(C.Structure):
    _fields_ = [("cluster", Cluster), ("gens", C.POINTER(C.c_int32)), ("ngens", C.c_int32), ("two_M", C.c_int32),
                ("irrep", C.c_int32), ("row", C.c_int32), ("R", C.c_int32), ("steps", C.c_int32),
                ("seed", C.c_uint64), ("storage", C.c_int32), ("dist", C.c_int32), ("engine", C.c_int32),
                ("reserved", C.c_int32)]


class JobResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("R", C.c_int32), ("steps", C.c_int32), ("d_gamma", C.c_int32),
                ("D", C.c_uint64), ("submit_s", C.c_double), ("start_s", C.c_double), ("end_s", C.c_double),
                ("engine", C.c_int32), ("reserved", C.c_int32)]


class Ritz(C.Structure):
    _fields_ = [("two_M", C.c_int32), ("d_gamma", C.c_int32), ("D", C.c_uint64), ("R", C.c_int32),
                ("ld", C.c_int32), ("nsteps", C.POINTER(C.c_int32)),
                ("theta", C.POINTER(C.c_double)), ("weight", C.POINTER(C.c_double))]


class KpmBlock(C.Structure):
    _fields_ = [("two_M", C.c_int32), ("d_gamma", C.c_int32), ("D", C.c_uint64), ("R", C.c_int32),
                ("n_moments", C.c_int32), ("center", C.c_double), ("half_width", C.c_double),
                ("moments", C.POINTER(C.c_double))]


VP = C.c_void_p
I32P = C.POINTER(C.c_int32)
F64P = C.POINTER(C.c_double)

# name -> (restype, argtypes); every symbol declared in include/ftlm.h and include/ftlm_server.h
SIGNATURES = {
    "ftlm_last_error": (C.c_char_p, []),
    "ftlm_group_create": (C.c_int, [C.c_int32, I32P, C.c_int32, C.POINTER(VP)]),
    "ftlm_group_info": (C.c_int, [VP, I32P, I32P, I32P, I32P]),
    "ftlm_group_elements": (C.c_int, [VP, I32P]),
    "ftlm_group_irreps": (C.c_int, [VP, I32P, I32P, I32P, F64P, I32P, F64P]),
    "ftlm_group_rho": (C.c_int, [VP, C.c_int32, F64P]),
    "ftlm_group_free": (None, [VP]),
    "ftlm_sector_create": (C.c_int, [C.POINTER(Cluster), VP, C.c_int32, C.POINTER(Opts), C.POINTER(VP)]),
    "ftlm_sector_info_get": (C.c_int, [VP, C.POINTER(SectorInfo)]),
    "ftlm_sector_export": (C.c_int, [VP, C.POINTER(C.c_uint64), C.POINTER(C.c_uint16), I32P]),
    "ftlm_sector_canonicalize": (C.c_int, [VP, VP, C.c_int64, VP, VP, VP, VP]),
    "ftlm_sector_free": (None, [VP]),
    "ftlm_block_create": (C.c_int, [VP, C.c_int32, C.c_int32, C.POINTER(Opts), C.POINTER(VP)]),
    "ftlm_build_block": (C.c_int, [C.POINTER(Cluster), I32P, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                   C.POINTER(Opts), C.POINTER(VP)]),
    "ftlm_block_info_get": (C.c_int, [VP, C.POINTER(BlockInfo)]),
    "ftlm_block_export": (C.c_int, [VP, C.POINTER(C.c_uint64), C.POINTER(C.c_uint16), C.POINTER(C.c_uint8),
                                    F64P, C.POINTER(C.c_uint64)]),
    "ftlm_block_hv_stats": (C.c_int, [VP, C.POINTER(HvStats)]),
    "ftlm_apply_H": (C.c_int, [VP, VP, VP, C.c_int32, C.c_int64, C.c_int32, VP]),
    "ftlm_apply_H_ex": (C.c_int, [VP, VP, VP, C.c_int32, C.c_int64, C.c_int32, C.POINTER(HvOpts), VP]),
    "ftlm_apply_H_ex_noalloc": (C.c_int, [VP, VP, VP, C.c_int32, C.c_int64, C.c_int32, C.POINTER(HvOpts), VP]),
    "ftlm_block_autotune": (C.c_int, [VP, C.c_int32, C.c_int32, VP, I32P, F64P, I32P, F64P, I32P]),
    "ftlm_device_arch": (C.c_int, [C.c_char_p, C.c_int32]),
    "ftlm_autotune_save": (C.c_int, [C.c_char_p, C.c_char_p, I32P]),
    "ftlm_autotune_load": (C.c_int, [C.c_char_p, C.c_char_p, I32P]),
    "ftlm_autotune_clear": (C.c_int, []),
    "ftlm_run": (C.c_int, [VP, C.c_int32, C.c_int32, C.c_uint64, C.c_int32, C.c_int32, F64P, F64P, I32P, VP]),
    "ftlm_run_ex": (C.c_int, [VP, C.c_int32, C.c_int32, C.c_uint64, C.c_int32, C.c_int32, F64P, F64P, I32P, VP,
                              C.POINTER(RunInfo)]),
    "ftlm_run_fused": (C.c_int, [C.POINTER(FusedJob), C.c_int32, VP]),
    "ftlm_run_begin": (C.c_int, [VP, C.c_int32, C.c_int32, C.c_uint64, C.c_int32, C.c_int32, VP, C.POINTER(VP)]),
    "ftlm_run_advance": (C.c_int, [VP, C.c_int32, I32P]),
    "ftlm_run_save": (C.c_int, [VP, C.c_char_p]),
    "ftlm_run_load": (C.c_int, [VP, C.c_char_p, VP, C.POINTER(VP)]),
    "ftlm_run_finish": (C.c_int, [VP, F64P, F64P, I32P]),
    "ftlm_run_state_free": (None, [VP]),
    "ftlm_kpm": (C.c_int, [VP, C.c_int32, C.c_int32, C.c_uint64, C.c_int32, C.c_int32, C.c_double, C.c_double,
                           F64P, VP]),
    "ftlm_kpm_observables": (C.c_int, [C.POINTER(KpmBlock), C.c_int32, F64P, C.c_int32, C.c_double, C.c_int32,
                                       F64P, F64P, F64P, F64P]),
    "ftlm_tridiag_ritz": (C.c_int, [F64P, F64P, C.c_int32, F64P, F64P]),
    "ftlm_campaign": (C.c_int, [C.POINTER(Cluster), I32P, C.c_int32, C.POINTER(CampaignOpts), F64P, C.c_int32,
                                F64P, F64P, F64P, F64P, C.POINTER(CampaignStats)]),
    "ftlm_observables": (C.c_int, [C.POINTER(Ritz), C.c_int32, F64P, C.c_int32, C.c_double, F64P, F64P, F64P, F64P]),
    "ftlm_block_free": (None, [VP]),
    # include/ftlm_server.h
    "ftlm_server_create": (C.c_int, [C.c_int64, C.c_int32, C.POINTER(VP)]),
    "ftlm_server_submit": (C.c_int, [VP, C.POINTER(JobDesc), C.POINTER(C.c_int64)]),
    "ftlm_server_wait": (C.c_int, [VP, C.c_int64, C.POINTER(JobResult), F64P, F64P, I32P]),
    "ftlm_server_poll": (C.c_int, [VP, C.c_int64, I32P]),
    "ftlm_server_cancel": (C.c_int, [VP, C.c_int64]),
    "ftlm_server_stats": (C.c_int, [VP, C.POINTER(C.c_int64), I32P, I32P]),
    "ftlm_server_free": (None, [VP]),
}

_lib = None


def lib():
    """The library: ``libftlm.so`` of this package, which must export every
    call, or the library named by FTLM_LIBRARY (the sanitizer build of the
    host-only part exports the host calls only; the others stay unbound)."""
    global _lib
    if _lib is None:
        path = os.environ.get("FTLM_LIBRARY") or LIB_PATH
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is None:
                if path != LIB_PATH:
                    continue
                raise ImportError(f"{path} does not export {name}")
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code != 0:
        msg = lib().ftlm_last_error()
        raise FtlmError(code, msg.decode() if msg else "")


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def make_cluster(N, two_s, bonds, J=None):
    bonds = np.ascontiguousarray(np.asarray(bonds, dtype=np.int32).reshape(-1))
    keep = [bonds]
    Jp = None
    if J is not None:
        J = np.ascontiguousarray(np.asarray(J, dtype=np.float64))
        keep.append(J)
        Jp = _ptr(J, C.c_double)
    cl = Cluster(int(N), int(two_s), len(bonds) // 2, _ptr(bonds, C.c_int32), Jp)
    cl._keep = keep
    return cl


def make_opts(hv_mode=HV_AUTO, user_rho=None, hbm_limit=0, layout=0, entry_format=0, spin_flip=False,
              user_rho_weight=0):
    o = Opts()
    o.user_rho_weight = int(user_rho_weight)
    o.spin_flip = 1 if spin_flip else 0
    o.hv_mode = hv_mode
    o.entry_format = int(entry_format)
    o.lanczos_layout = int(layout)
    o.hbm_limit_bytes = int(hbm_limit)
    if user_rho is not None:
        rho = np.ascontiguousarray(np.asarray(user_rho, dtype=np.float64))
        o.user_rho = _ptr(rho, C.c_double)
        o.user_rho_dim = rho.shape[-1]
        o._keep = rho
    return o


def stream_handle(stream=None):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)
