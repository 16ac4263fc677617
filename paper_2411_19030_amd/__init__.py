"""MI355X (gfx950) hot path of one-shot Parareal topology optimisation for
transient heat conduction: a C-ABI HIP library (libpt.so, include/pt.h) and a
thin Python binding with the same entry-point names.
"""
from ._pt import (EXPORTS, PT_BC, PT_EDOMAIN, PT_EHIP, PT_EINVAL, PT_ENOCONV, PT_ENOMEM, PT_OK,
                  Problem, PtError, load_library, pt_autotune_batched, pt_batch_default_tuning,
                  pt_batched_status, pt_batched_workspace_bytes, pt_parareal_adjoint,
                  pt_parareal_batched, pt_parareal_forward, pt_query_status, pt_sensitivities,
                  pt_validate, pt_workspace_bytes)

__all__ = [
    "EXPORTS", "PT_BC", "PT_EDOMAIN", "PT_EHIP", "PT_EINVAL", "PT_ENOCONV", "PT_ENOMEM", "PT_OK",
    "Problem", "PtError", "load_library", "pt_parareal_adjoint", "pt_parareal_forward",
    "pt_query_status", "pt_sensitivities", "pt_validate", "pt_workspace_bytes",
    "pt_autotune_batched", "pt_batch_default_tuning", "pt_batched_status",
    "pt_batched_workspace_bytes", "pt_parareal_batched",
]
