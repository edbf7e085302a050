"""ctypes declarations of libba.so (include/ba.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libba.so")

BA_OK, BA_MAXITER = 0, 1
BA_ERR_INVALID_ARG, BA_ERR_NONFINITE, BA_ERR_NOT_SPD, BA_ERR_BREAKDOWN = -1, -2, -3, -4
BA_ERR_WORKSPACE, BA_ERR_HIP, BA_ERR_NOMEM, BA_ERR_UNSUPPORTED = -5, -6, -7, -8
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}


class ProblemDesc(C.Structure):
    _fields_ = [("n_cams", C.c_int32), ("n_lms", C.c_int32), ("n_obs", C.c_int64), ("d_p", C.c_int32),
                ("reserved0", C.c_int32), ("obs_cam", C.c_void_p), ("obs_lm", C.c_void_p),
                ("J_p", C.c_void_p), ("J_l", C.c_void_p), ("r", C.c_void_p), ("lam", C.c_double)]


class BuildOpts(C.Structure):
    _fields_ = [("store_fp32", C.c_int32), ("store_bf16", C.c_int32), ("max_slots", C.c_int32),
                ("max_tiles", C.c_int32), ("explicit_schur", C.c_int32), ("max_tiles_multi", C.c_int32),
                ("ws_groups", C.c_int32), ("ws_max_iter", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("precond", C.c_int32), ("history_mfma", C.c_int32), ("max_history_cols", C.c_int64),
                ("inner_eps", C.c_double), ("max_outer", C.c_int32), ("max_inner", C.c_int32),
                ("history_fp32", C.c_int32), ("reserved", C.c_int32 * 3)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("multi_steps", C.c_int32), ("history_cols", C.c_int32),
                ("refinement_steps", C.c_int32), ("status", C.c_int32), ("trace_cap", C.c_int32),
                ("rel_res_recursive", C.c_double), ("rel_res_true", C.c_double),
                ("t_solve_ms", C.c_double), ("trace_res", C.POINTER(C.c_double)),
                ("trace_t", C.POINTER(C.c_double)), ("trace_k", C.POINTER(C.c_int32))]


class BatchStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("multi_steps", C.c_int32), ("history_cols", C.c_int32),
                ("refinement_steps", C.c_int32), ("status", C.c_int32), ("reserved", C.c_int32),
                ("rel_res_recursive", C.c_double), ("rel_res_true", C.c_double), ("done_ms", C.c_double)]


class SceneDesc(C.Structure):
    _fields_ = [("n_cams", C.c_int32), ("n_lms", C.c_int32), ("n_obs", C.c_int64), ("obs_cam", C.c_void_p),
                ("obs_lm", C.c_void_p), ("u_obs", C.c_void_p)]


class LMOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("solver", C.c_int32), ("n_groups", C.c_int32), ("reserved0", C.c_int32),
                ("tau", C.c_double), ("lambda0", C.c_double), ("ftol", C.c_double), ("lambda_factor", C.c_double),
                ("solve", SolveOpts), ("build", BuildOpts)]


class LMStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("accepted", C.c_int32), ("status", C.c_int32),
                ("solver_iterations", C.c_int32), ("cost0", C.c_double), ("cost", C.c_double),
                ("t_total_ms", C.c_double), ("t_solve_ms", C.c_double), ("t_linearize_ms", C.c_double),
                ("trace_cap", C.c_int32), ("reserved", C.c_int32), ("trace_lambda", C.POINTER(C.c_double)),
                ("trace_cost", C.POINTER(C.c_double)), ("trace_accepted", C.POINTER(C.c_int32)),
                ("trace_solver_iterations", C.POINTER(C.c_int32)), ("trace_solve_ms", C.POINTER(C.c_double))]


# (name, restype, argtypes) for every entry point of include/ba.h
SIGNATURES = [
    ("ba_default_solve_opts", None, [C.POINTER(SolveOpts)]),
    ("ba_build_system", C.c_int, [C.POINTER(ProblemDesc), C.POINTER(BuildOpts), C.c_void_p, C.POINTER(C.c_void_p)]),
    ("ba_build_workspace_bytes", C.c_int, [C.POINTER(ProblemDesc), C.POINTER(BuildOpts), C.POINTER(C.c_size_t)]),
    ("ba_build_system_ws", C.c_int, [C.POINTER(ProblemDesc), C.POINTER(BuildOpts), C.c_void_p, C.c_size_t, C.c_void_p,
                                     C.POINTER(C.c_void_p)]),
    ("ba_system_workspace_used", C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    ("ba_free_system", None, [C.c_void_p]),
    ("ba_schur_matvec", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    ("ba_schur_matvec_noalloc", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    ("ba_schur_matmat_grouped", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]),
    ("ba_precond_apply", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ba_get_rhs", C.c_int, [C.c_void_p, C.c_void_p]),
    ("ba_get_precond_blocks", C.c_int, [C.c_void_p, C.c_void_p]),
    ("ba_pcg_solve", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(SolveOpts), C.POINTER(SolveStats)]),
    ("ba_mcg_solve", C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.c_void_p, C.POINTER(SolveOpts),
                               C.POINTER(SolveStats)]),
    ("ba_back_substitute", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ba_prepare_mcg", C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    ("ba_pinv_sym", C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    ("ba_partition", C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_int32)]),
    ("ba_system_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    ("ba_lowrank_features", C.c_int, [C.c_void_p, C.c_void_p]),
    ("ba_mlp_forward", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p]),
    ("ba_set_lowrank_from_mlp", C.c_int, [C.c_void_p, C.c_void_p]),
    ("ba_set_lowrank_precond", C.c_int, [C.c_void_p, C.c_void_p]),
    ("ba_get_lowrank", C.c_int, [C.c_void_p, C.c_void_p]),
    ("ba_block_scale", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    ("ba_mlp_loss_grad", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                   C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    ("ba_adam_step", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_void_p]),
    ("ba_profile_enable", C.c_int, [C.c_void_p, C.c_int32]),
    ("ba_profile_read", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]),
    ("ba_plan_validate", C.c_int, [C.c_int32, C.c_int32, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int64)]),
    ("ba_plan_validate_error", C.c_char_p, []),
    ("ba_batch_build", C.c_int, [C.POINTER(ProblemDesc), C.c_int32, C.POINTER(C.c_int32), C.POINTER(BuildOpts),
                                 C.c_void_p, C.POINTER(C.c_void_p)]),
    ("ba_batch_free", None, [C.c_void_p]),
    ("ba_batch_system", C.c_void_p, [C.c_void_p]),
    ("ba_batch_mcg_solve", C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.POINTER(SolveOpts), C.c_int32,
                                     C.POINTER(BatchStats), C.POINTER(C.c_double)]),
    ("ba_update_system", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double]),
    ("ba_set_lambda", C.c_int, [C.c_void_p, C.c_double]),
    ("ba_default_lm_opts", None, [C.POINTER(LMOpts)]),
    ("ba_project", C.c_int, [C.POINTER(SceneDesc), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.POINTER(C.c_double), C.c_void_p]),
    ("ba_apply_step", C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p]),
    ("ba_lm_solve", C.c_int, [C.POINTER(SceneDesc), C.c_void_p, C.c_void_p, C.POINTER(LMOpts), C.c_void_p,
                              C.POINTER(LMStats)]),
    ("ba_stream_read_gbs", C.c_int, [C.c_int64, C.c_int32, C.POINTER(C.c_double), C.c_void_p]),
    ("ba_schur_matvec_timed", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                        C.POINTER(C.c_double)]),
    ("ba_explicit_schur_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_double)]),
    ("ba_status_string", C.c_char_p, [C.c_int32]),
    ("ba_last_error", C.c_char_p, []),
]

_lib = None


def load() -> C.CDLL:
    """Load libba.so (built in-tree by build()); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2110_04015_amd.build` "
                           "or __graft_entry__.build() first")
    lib = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
