"""MI355X symmetry-adapted finite-temperature Lanczos (FTLM) hot path.

The work runs in ``libftlm.so`` (hand-written HIP for gfx950 + C++ host code)
behind the C ABI of ``include/ftlm.h``; this package only marshals arguments.
"""
from .api import (F32, F64, GAUSSIAN, campaign, HV_AUTO, HV_ENTRIES, HV_ONTHEFLY, RADEMACHER, Block, FtlmError, Group,
                  Sector, LanczosRunState, autotune_clear, autotune_load, autotune_save, device_arch, kpm_observables, observables,
                  ritz_from_run, run_fused, tridiag_ritz)
from ._lib import (ENGINE_AUTO, ENGINE_FUSED, ENGINE_STEPS, ENTRIES_AUTO, ENTRIES_COMPACT, ENTRIES_WIDE, F16,
                   LAYOUT_ALIGNED, LAYOUT_AUTO, LAYOUT_BLOCK, LAYOUT_PACKED, LAYOUT_PADDED, lib)
from .server import Server

__all__ = ["Group", "Sector", "Block", "Server", "campaign", "run_fused", "kpm_observables", "observables", "ritz_from_run",
           "tridiag_ritz", "FtlmError", "lib", "device_arch", "LanczosRunState", "autotune_save", "autotune_load", "autotune_clear",
           "F16", "F32", "F64", "RADEMACHER", "GAUSSIAN", "HV_AUTO", "HV_ENTRIES", "HV_ONTHEFLY",
           "LAYOUT_AUTO", "LAYOUT_BLOCK", "LAYOUT_PADDED", "LAYOUT_PACKED", "LAYOUT_ALIGNED", "ENTRIES_AUTO", "ENTRIES_WIDE", "ENTRIES_COMPACT",
           "ENGINE_AUTO", "ENGINE_STEPS", "ENGINE_FUSED"]
