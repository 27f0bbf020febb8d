"""MI355X (gfx950) implementation of the TCTF2R tensor-completion iteration.

The computation lives in the HIP library ``libtctf2r.so`` (C ABI: include/tctf2r.h);
``binding`` exposes the same functions to Python and a torch-facing ``Completion``.
"""
from .binding import (STAGES, TCTF_FP32, TCTF_MIXED_BF16, Batch, Completion, TctfError, complete, library,
                      make_params, tctf_complete, tctf_create, tctf_default_params, tctf_destroy,
                      tctf_get_result, tctf_get_state, tctf_iterations, tctf_last_error, tctf_objective,
                      tctf_params, tctf_set_state, tctf_state_bytes, tctf_stationarity, tctf_status_string,
                      tctf_profile, tctf_profile_read, tctf_step, tctf_termination, tctf_time_stage,
                      tctf_workspace_bytes)

__all__ = ["STAGES", "TCTF_FP32", "TCTF_MIXED_BF16", "Batch", "Completion", "TctfError", "complete", "library",
           "make_params", "tctf_complete", "tctf_create", "tctf_default_params", "tctf_destroy",
           "tctf_get_result", "tctf_get_state", "tctf_iterations", "tctf_last_error", "tctf_objective",
           "tctf_params", "tctf_set_state", "tctf_state_bytes", "tctf_stationarity", "tctf_status_string",
           "tctf_profile", "tctf_profile_read", "tctf_step", "tctf_termination", "tctf_time_stage",
           "tctf_workspace_bytes"]
