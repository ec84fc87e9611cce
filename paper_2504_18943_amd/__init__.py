"""MI355X-native LTLf synthesiser: bottom-up enumeration of formula semantics.

The compute path is libltlf.so (HIP kernels for gfx950 behind the C ABI in
include/ltlf.h); this package only binds it.
"""
from .ltlf import (Synthesizer, Server, Result, SplitResult, LtlfError, load_library, ltlf_status_str, ltlf_ctx_create,
                   ltlf_ctx_last_error, ltlf_ctx_cancel, FLAG_DIGEST, CANCELLED,
                   ltlf_ctx_set_workspace, ltlf_ctx_set_row_limit, ltlf_ctx_destroy, ltlf_load,
                   ltlf_run, ltlf_solve, ltlf_solve_static, ltlf_solve_batch, ltlf_solve_split, ltlf_autotune, ltlf_ctx_set_tuning,
                   ltlf_server_create, ltlf_server_submit,
                   ltlf_server_step, ltlf_server_poll, ltlf_server_cancel, ltlf_server_load,
                   ltlf_server_destroy, ltlf_export_level, ltlf_formula_of, FLAG_EXHAUST, FLAG_PROFILE,
                   FLAG_KERNEL_LANE, FLAG_KERNEL_GROUP, FLAG_KERNEL_WAVE, FLAG_NO_LOOKAHEAD,
                   FLAG_WEAK_HASH, UNIT_ALL, STATUS_NAMES, LIB_PATH)

__all__ = ["Synthesizer", "Server", "Result", "SplitResult", "LtlfError", "load_library", "ltlf_status_str",
           "ltlf_ctx_create", "ltlf_ctx_last_error", "ltlf_ctx_cancel", "FLAG_DIGEST", "CANCELLED", "ltlf_ctx_set_workspace", "ltlf_ctx_set_row_limit",
           "ltlf_ctx_destroy", "ltlf_load", "ltlf_run", "ltlf_solve", "ltlf_solve_static", "ltlf_solve_batch", "ltlf_solve_split", "ltlf_autotune", "ltlf_ctx_set_tuning", "ltlf_server_create", "ltlf_server_submit", "ltlf_server_step",
           "ltlf_server_poll", "ltlf_server_cancel", "ltlf_server_load", "ltlf_server_destroy", "ltlf_export_level",
           "ltlf_formula_of", "FLAG_EXHAUST", "FLAG_PROFILE", "FLAG_KERNEL_LANE", "FLAG_KERNEL_GROUP", "FLAG_KERNEL_WAVE", "FLAG_NO_LOOKAHEAD", "FLAG_WEAK_HASH", "UNIT_ALL", "STATUS_NAMES",
           "LIB_PATH"]
