"""ctypes declarations of the libhmc C ABI (include/hmc.h, include/hmc_testing.h).

Loading fails loudly when the library has not been built: there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhmc.so")

HMC_OK = 0
HMC_ERR_INVALID_ARG = -1
HMC_ERR_NOT_CONVERGED = -2
HMC_ERR_NONFINITE = -3
HMC_ERR_HIP = -4
HMC_ERR_WORKSPACE = -5
HMC_FP64 = 0
HMC_MIXED = 1
HMC_MAX_RHS = 16
HMC_FORCE_PF = 1
HMC_FORCE_BOSON = 2
HMC_PRECOND_NONE = 0
HMC_PRECOND_FOURIER = 1
HMC_NOALLOC_SCRATCH_BYTES = 64 << 20
HMC_PROBE_READ = 0
HMC_PROBE_WRITE = 1
HMC_PROBE_COPY = 2
HMC_PROBE_3R3W = 3
HMC_PROBE_READ_NT = 4

EXPORTED = [
    "hmc_create", "hmc_destroy", "hmc_set_params", "hmc_workspace_bytes", "hmc_set_workspace",
    "hmc_apply_M", "hmc_apply_Mdag", "hmc_apply_MdagM", "hmc_apply_M_f32", "hmc_apply_Mdag_f32",
    "hmc_apply_MdagM_f32", "hmc_apply_MdagM_noalloc", "hmc_cg_solve", "hmc_heatbath", "hmc_force",
    "hmc_force_from_solution", "hmc_pf_action", "hmc_boson_action", "hmc_trajectory",
    "hmc_strerror", "hmc_last_error", "hmc_test_site", "hmc_test_xcd_remap", "hmc_test_tile_span", "hmc_test_fft",
    "hmc_test_fft_freq", "hmc_test_precond", "hmc_test_apply_precond", "hmc_stream_probe",
    "hmc_set_kernel_timing", "hmc_get_kernel_times", "hmc_set_cg_workgroups",
    "hmc_get_cg_workgroups", "hmc_set_mdm_shape", "hmc_get_mdm_shape", "hmc_set_cg_march", "hmc_get_cg_march", "hmc_set_cg_march_step_b", "hmc_get_cg_march_step_b", "hmc_leapfrog", "hmc_autotune", "hmc_set_graphs", "hmc_set_step_graphs",
    "hmc_set_metric", "hmc_metric_momenta", "hmc_metric_kinetic", "hmc_metric_norm2",
    "hmc_metric_accumulate", "hmc_tuner_init", "hmc_tuner_add_step", "hmc_tuner_add_jump",
    "hmc_tuner_best_length", "hmc_jitter", "hmc_warmup_iteration", "hmc_sdw_accumulate",
    "hmc_order_parameter", "hmc_binder",
    "hmc_batch_create", "hmc_batch_destroy", "hmc_batch_workspace_bytes",
    "hmc_batch_set_workspace", "hmc_batch_layout", "hmc_batch_set_cg_workgroups",
    "hmc_batch_get_cg_workgroups", "hmc_batch_set_graphs", "hmc_batch_set_step_graphs", "hmc_batch_set_cg_march", "hmc_batch_get_cg_march", "hmc_batch_set_cg_march_step_b", "hmc_batch_set_params",
    "hmc_batch_apply", "hmc_batch_cg_solve", "hmc_batch_autotune", "hmc_batch_trajectory",
]


class HmcParams(ctypes.Structure):
    _fields_ = [
        ("t", (ctypes.c_double * 2) * 2),
        ("mu", ctypes.c_double * 2),
        ("lambda_", ctypes.c_double),
        ("r", ctypes.c_double),
        ("c", ctypes.c_double),
        ("u", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("n_leap", ctypes.c_int),
        ("n_pf", ctypes.c_int),
        ("cg_tol", ctypes.c_double),
        ("cg_maxit", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("reliable_every", ctypes.c_int),
        ("max_rhs", ctypes.c_int),
        ("precond", ctypes.c_int),
        ("tn", (ctypes.c_double * 2) * 2),
    ]


class HmcCgStats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("status", ctypes.c_int),
        ("iterations", ctypes.c_int * HMC_MAX_RHS),
        ("reliable_updates", ctypes.c_int * HMC_MAX_RHS),
        ("true_resid", ctypes.c_double * HMC_MAX_RHS),
    ]


class HmcTrajStats(ctypes.Structure):
    _fields_ = [
        ("dH", ctypes.c_double),
        ("H0", ctypes.c_double), ("H1", ctypes.c_double),
        ("S_pf0", ctypes.c_double), ("S_pf1", ctypes.c_double),
        ("S_b0", ctypes.c_double), ("S_b1", ctypes.c_double),
        ("K0", ctypes.c_double), ("K1", ctypes.c_double),
        ("accepted", ctypes.c_int),
        ("cg_solves", ctypes.c_int),
        ("cg_iterations", ctypes.c_long),
        ("max_true_resid", ctypes.c_double),
        ("status", ctypes.c_int),
    ]


HMC_TUNE_MAX = 12


HMC_TUNE_MARCH_MAX = 16


class HmcTuneResult(ctypes.Structure):
    _fields_ = [("cg_workgroups", ctypes.c_int * 2), ("us_per_iter", ctypes.c_double * 2),
                ("candidates", ctypes.c_int), ("tried", ctypes.c_int * 2),
                ("tried_workgroups", (ctypes.c_int * HMC_TUNE_MAX) * 2),
                ("tried_us", (ctypes.c_double * HMC_TUNE_MAX) * 2),
                ("march_rows", ctypes.c_int * 2), ("march_slices", ctypes.c_int * 2),
                ("mtried", ctypes.c_int * 2),
                ("mtried_rows", (ctypes.c_int * HMC_TUNE_MARCH_MAX) * 2),
                ("mtried_slices", (ctypes.c_int * HMC_TUNE_MARCH_MAX) * 2),
                ("mtried_us", (ctypes.c_double * HMC_TUNE_MARCH_MAX) * 2),
                ("from_cache", ctypes.c_int), ("march_step_b", ctypes.c_int * 2),
                ("step_b_us", (ctypes.c_double * 2) * 2)]


def tune_dict(r):
    """hmc_tune_result as {"fp64": (workgroups, us), "mixed": ..., "candidates": n,
    "tried": {"fp64": [(workgroups, us), ...], "mixed": [...]}}."""
    names = ("fp64", "mixed")
    out = {names[i]: (r.cg_workgroups[i], r.us_per_iter[i]) for i in range(2)}
    out["candidates"] = r.candidates
    out["tried"] = {names[i]: [(r.tried_workgroups[i][j], r.tried_us[i][j]) for j in range(r.tried[i])]
                    for i in range(2)}
    out["march"] = {names[i]: (r.march_rows[i], r.march_slices[i]) for i in range(2)}
    out["march_tried"] = {names[i]: [(r.mtried_rows[i][j], r.mtried_slices[i][j], r.mtried_us[i][j])
                                     for j in range(r.mtried[i])] for i in range(2)}
    out["from_cache"] = r.from_cache
    out["march_step_b"] = {"fp64": r.march_step_b[0], "mixed": r.march_step_b[1]}
    out["step_b_us"] = {"fp64": tuple(r.step_b_us[0]), "mixed": tuple(r.step_b_us[1])}
    return out


HMC_TUNER_MAX_LEN = 256


class HmcTuner(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("factor", ctypes.c_double), ("window", ctypes.c_int),
                ("n_cap", ctypes.c_int), ("count", ctypes.c_int), ("pad", ctypes.c_int),
                ("sum_alpha_eps", ctypes.c_double), ("sum_alpha_half", ctypes.c_double),
                ("esjd_sum", ctypes.c_double * (HMC_TUNER_MAX_LEN + 1)),
                ("esjd_count", ctypes.c_long * (HMC_TUNER_MAX_LEN + 1))]


class HmcWarmupStats(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("eps_next", ctypes.c_double), ("dH_eps", ctypes.c_double),
                ("dH_half", ctypes.c_double), ("dH", ctypes.c_double), ("sqdist", ctypes.c_double),
                ("n_leap", ctypes.c_int), ("accepted", ctypes.c_int), ("cg_iterations", ctypes.c_long),
                ("max_true_resid", ctypes.c_double)]


class HmcKernelTimes(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 12), ("count", ctypes.c_long * 12)]


KT_NAMES = ("cg_a_f32", "cg_b_f32", "cg_a_f64", "cg_b_f64",
            "pc_xy_fwd_f32", "pc_t_f32", "pc_xy_inv_f32", "pc_xy_fwd_f64", "pc_t_f64", "pc_xy_inv_f64",
            "cg_a_next_f32", "cg_a_next_f64")

_lib = None


def load():
    """Load libhmc.so and declare its signatures.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2204_14241_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    ctx_pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "hmc_create": (I, [I, I, D, ctypes.POINTER(HmcParams), ctx_pp]),
        "hmc_destroy": (I, [P]),
        "hmc_set_params": (I, [P, ctypes.POINTER(HmcParams)]),
        "hmc_workspace_bytes": (S, [P]),
        "hmc_set_workspace": (I, [P, P, S]),
        "hmc_apply_M": (I, [P, P, P, P, I, P]),
        "hmc_apply_Mdag": (I, [P, P, P, P, I, P]),
        "hmc_apply_MdagM": (I, [P, P, P, P, I, P]),
        "hmc_apply_M_f32": (I, [P, P, P, P, I, P]),
        "hmc_apply_Mdag_f32": (I, [P, P, P, P, I, P]),
        "hmc_apply_MdagM_f32": (I, [P, P, P, P, I, P]),
        "hmc_apply_MdagM_noalloc": (I, [P, P, P, P, I, P]),
        "hmc_cg_solve": (I, [P, P, P, P, I, ctypes.POINTER(HmcCgStats), P]),
        "hmc_heatbath": (I, [P, P, P, P, I, P]),
        "hmc_force": (I, [P, P, P, I, P, P, I, ctypes.POINTER(HmcCgStats), P]),
        "hmc_force_from_solution": (I, [P, P, P, I, P, I, P]),
        "hmc_pf_action": (I, [P, P, P, I, P, ctypes.POINTER(D), ctypes.POINTER(HmcCgStats), P]),
        "hmc_boson_action": (I, [P, P, ctypes.POINTER(D), P]),
        "hmc_trajectory": (I, [P, P, P, P, I, D, ctypes.POINTER(HmcTrajStats), P]),
        "hmc_leapfrog": (I, [P, P, P, P, I, ctypes.POINTER(HmcTrajStats), P]),
        "hmc_strerror": (ctypes.c_char_p, [I]),
        "hmc_last_error": (ctypes.c_char_p, []),
        "hmc_test_site": (I, [I, I, I, ctypes.POINTER(ctypes.c_int)]),
        "hmc_test_xcd_remap": (I, [I, I]),
        "hmc_test_tile_span": (I, [I, I, I, ctypes.POINTER(ctypes.c_int)]),
        "hmc_test_fft": (I, [I, I, ctypes.POINTER(D), ctypes.POINTER(D)]),
        "hmc_test_fft_freq": (I, [I, I]),
        "hmc_test_precond": (I, [I, I, D, ctypes.POINTER(HmcParams), ctypes.POINTER(D),
                                 ctypes.POINTER(D), ctypes.POINTER(D)]),
        "hmc_test_apply_precond": (I, [P, I, P, P, I, ctypes.POINTER(D), P]),
        "hmc_stream_probe": (I, [I, P, P, S, I, P]),
        "hmc_set_kernel_timing": (I, [P, I]),
        "hmc_get_kernel_times": (I, [P, ctypes.POINTER(HmcKernelTimes)]),
        "hmc_set_cg_workgroups": (I, [P, I, I]),
        "hmc_get_cg_workgroups": (I, [P, I]),
        "hmc_set_mdm_shape": (I, [P, I, I, I]),
        "hmc_set_cg_march": (I, [P, I, I, I]),
        "hmc_get_cg_march": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "hmc_get_mdm_shape": (I, [P, I, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
        "hmc_autotune": (I, [P, P, P, I, ctypes.POINTER(HmcTuneResult), P]),
        "hmc_set_graphs": (I, [P, I]),
        "hmc_set_step_graphs": (I, [P, I]),
        "hmc_set_metric": (I, [P, P]),
        "hmc_metric_momenta": (I, [P, P, P, P]),
        "hmc_metric_kinetic": (I, [P, P, ctypes.POINTER(D), P]),
        "hmc_metric_norm2": (I, [P, P, ctypes.POINTER(D), P]),
        "hmc_metric_accumulate": (I, [P, P, P, P]),
        "hmc_tuner_init": (I, [ctypes.POINTER(HmcTuner), D, I, D, I]),
        "hmc_tuner_add_step": (I, [ctypes.POINTER(HmcTuner), D, D]),
        "hmc_tuner_add_jump": (I, [ctypes.POINTER(HmcTuner), I, D, D]),
        "hmc_tuner_best_length": (I, [ctypes.POINTER(HmcTuner)]),
        "hmc_jitter": (I, [D, I]),
        "hmc_sdw_accumulate": (I, [P, P, P, P]),
        "hmc_order_parameter": (I, [P, P, ctypes.POINTER(D), P]),
        "hmc_binder": (D, [ctypes.POINTER(D), I]),
        "hmc_warmup_iteration": (I, [P, ctypes.POINTER(HmcTuner), P, P, P, I, D, D,
                                     ctypes.POINTER(HmcWarmupStats), P]),
        "hmc_batch_create": (I, [I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(D), D,
                                 ctypes.POINTER(HmcParams), ctx_pp]),
        "hmc_batch_destroy": (I, [P]),
        "hmc_batch_workspace_bytes": (S, [P]),
        "hmc_batch_set_workspace": (I, [P, P, S]),
        "hmc_batch_layout": (I, [P, ctypes.POINTER(ctypes.c_longlong),
                                 ctypes.POINTER(ctypes.c_longlong)]),
        "hmc_batch_set_cg_workgroups": (I, [P, I, I]),
        "hmc_batch_get_cg_workgroups": (I, [P, I]),
        "hmc_batch_set_graphs": (I, [P, I]),
        "hmc_batch_set_step_graphs": (I, [P, I]),
        "hmc_batch_set_cg_march": (I, [P, I, I, I]),
        "hmc_batch_get_cg_march": (I, [P, I, I, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int)]),
        "hmc_batch_set_cg_march_step_b": (I, [P, I, I]),
        "hmc_set_cg_march_step_b": (I, [P, I, I]),
        "hmc_get_cg_march_step_b": (I, [P, I]),
        "hmc_batch_set_params": (I, [P, ctypes.POINTER(HmcParams)]),
        "hmc_batch_apply": (I, [P, I, I, P, P, P, P]),
        "hmc_batch_cg_solve": (I, [P, P, P, P, ctypes.POINTER(I), ctypes.POINTER(D), P]),
        "hmc_batch_autotune": (I, [P, P, P, ctypes.POINTER(HmcTuneResult), P]),
        "hmc_batch_trajectory": (I, [P, P, P, P, ctypes.POINTER(D), ctypes.POINTER(D),
                                     ctypes.POINTER(I), ctypes.POINTER(HmcTrajStats), P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class HmcError(RuntimeError):
    def __init__(self, code, where):
        lib = load()
        msg = lib.hmc_last_error().decode() or lib.hmc_strerror(code).decode()
        super().__init__(f"{where}: {lib.hmc_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def check(code, where):
    if code != HMC_OK:
        raise HmcError(code, where)
    return code
