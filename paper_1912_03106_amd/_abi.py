"""ctypes mirror of include/mgrit.h and loader of libmgrit.so.

The library is loaded from the package directory only.  There is no fallback:
if libmgrit.so is missing or a symbol is absent, importing this module's
`lib()` raises.
"""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgrit.so")

MAX_LEVELS = 8
MAX_HISTORY = 128

STATUS = {
    0: "OK", -1: "INVALID_ARGUMENT", -2: "NOT_NESTED", -3: "OUT_OF_MEMORY", -4: "HIP_ERROR",
    -5: "PCG_NOT_CONVERGED", -6: "NEWTON_NOT_CONVERGED", -7: "NOT_CONVERGED", -8: "NONFINITE",
    -9: "UNSUPPORTED",
}
FP64, FP32_IR = 0, 1
R_NORMALIZED, R_TRANSPOSE, R_INJECTION = 0, 1, 2

EXPORTS = ("mgrit_default_params", "mgrit_setup", "mgrit_solve", "mgrit_seq_solve", "phi_step",
           "mgrit_level_info", "mgrit_destroy", "mgrit_strerror", "mgrit_last_error",
           "mgrit_train_coarse", "mgrit_coarse_n_params", "mgrit_set_coarse_weights",
           "mgrit_get_coarse_weights", "mgrit_coarse_apply", "mgrit_coarse_gradient",
           "mgrit_coarse_adam", "phi_step_noalloc", "mgrit_joule_losses", "mgrit_circuit_values")


class Mesh(C.Structure):
    _fields_ = [
        ("n_r", C.c_int32), ("n_theta", C.c_int32), ("n_nodes", C.c_int32), ("n_tri", C.c_int32),
        ("xy", C.POINTER(C.c_double)), ("tri", C.POINTER(C.c_int32)),
        ("cell_mat", C.POINTER(C.c_int32)), ("cell_phase", C.POINTER(C.c_int32)),
        ("cell_sign", C.POINTER(C.c_int32)), ("dirichlet", C.POINTER(C.c_uint8)),
        ("cell_bar", C.POINTER(C.c_int32)),
    ]


class Physics(C.Structure):
    _fields_ = [
        ("n_materials", C.c_int32), ("nu", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double)),
        ("iron", C.POINTER(C.c_int32)), ("nonlinear", C.c_int32),
        ("bh_k1", C.c_double), ("bh_k2", C.c_double), ("bh_k3", C.c_double),
        ("J0", C.c_double), ("amplitude", C.c_double), ("freq", C.c_double),
        ("f_carrier", C.c_double), ("phase_offset", C.c_double), ("phases", C.c_double * 3),
        ("carrier", C.c_int32), ("dt", C.c_double), ("n_steps", C.c_int64),
        ("ramp_periods", C.c_double), ("signal", C.c_int32), ("t_start", C.c_double),
        ("circuit", C.c_int32), ("turns_density", C.c_double), ("l_z", C.c_double),
        ("r_phase", C.c_double), ("v0", C.c_double), ("n_bars", C.c_int32), ("ring_r", C.c_double),
    ]


class Problem(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("meshes", C.POINTER(Mesh)), ("phys", Physics)]


class Params(C.Structure):
    _fields_ = [
        ("m", C.c_int32), ("gamma", C.c_int32), ("precision", C.c_int32), ("restriction", C.c_int32),
        ("tol", C.c_double), ("max_iter", C.c_int32), ("pcg_tol", C.c_double),
        ("pcg_max_iter", C.c_int32), ("pcg_check_every", C.c_int32), ("ir_inner_tol", C.c_double),
        ("ir_max_iter", C.c_int32), ("newton_tol", C.c_double), ("newton_max_iter", C.c_int32),
        ("warm_start", C.c_int32), ("device_pointers", C.c_int32), ("profile_kernels", C.c_int32),
        ("autotune", C.c_int32), ("pcg_kernel", C.c_int32), ("coarse_inverse", C.c_int32),
        ("seq_kernel", C.c_int32), ("use_graphs", C.c_int32), ("newton_halvings", C.c_int32),
        ("pcg_tol_eta", C.c_double), ("precision_coarse", C.c_int32), ("coarse_model", C.c_int32),
        ("compact_columns", C.c_int32), ("compact_fraction", C.c_double),
        ("pcg_prefetch", C.c_int32), ("residual_eta", C.c_double), ("pcg_rows_narrow", C.c_int32),
        ("cycle", C.c_int32), ("nested", C.c_int32), ("loss_tol", C.c_double),
        ("m_coarse", C.c_int32), ("coarse_persistent", C.c_int32), ("pcg_check_narrow", C.c_int32),
        ("pcg_rows_per_block", C.c_int32), ("pcg_cols_per_lane", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("iterations", C.c_int32), ("converged", C.c_int32), ("n_history", C.c_int32),
        ("rho", C.c_double * MAX_HISTORY),
        ("phi_columns", C.c_int64 * MAX_LEVELS), ("pcg_sweeps", C.c_int64 * MAX_LEVELS),
        ("newton_sweeps", C.c_int64 * MAX_LEVELS),
        ("kernel_launches", (C.c_int64 * MAX_LEVELS) * 2), ("kernel_columns", C.c_int64 * MAX_LEVELS),
        ("kernel_time_s", (C.c_double * MAX_LEVELS) * 2),
        ("time_relax_s", C.c_double), ("time_total_s", C.c_double),
        ("coarse_fallback", C.c_int32), ("time_nested_s", C.c_double),
        ("loss_change", C.c_double * MAX_HISTORY), ("time_phi_s", C.c_double * MAX_LEVELS),
    ]


class TrainParams(C.Structure):
    _fields_ = [
        ("n_traj", C.c_int32), ("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double),
        ("amp_spread", C.c_double), ("val_fraction", C.c_double), ("seed", C.c_uint64),
        ("perturb", C.c_double),
    ]


class TrainStats(C.Structure):
    _fields_ = [
        ("n_train", C.c_int64), ("n_val", C.c_int64), ("steps", C.c_int64),
        ("loss_first", C.c_double), ("loss_last", C.c_double),
        ("train_err_ie", C.c_double), ("train_err_learned", C.c_double),
        ("val_err_ie", C.c_double), ("val_err_learned", C.c_double),
        ("time_data_s", C.c_double), ("time_train_s", C.c_double),
    ]


_LIB = None


def lib():
    """Load libmgrit.so (raises if it is missing: there is no CPU fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1912_03106_amd.build`")
    L = C.CDLL(LIB_PATH)
    for name in EXPORTS:
        if not hasattr(L, name):
            raise RuntimeError(f"libmgrit.so does not export {name}")
    vp = C.c_void_p
    dp = C.POINTER(C.c_double)
    L.mgrit_default_params.argtypes = [C.POINTER(Params)]
    L.mgrit_default_params.restype = None
    L.mgrit_setup.argtypes = [C.POINTER(Problem), C.POINTER(Params), vp, C.POINTER(vp)]
    L.mgrit_setup.restype = C.c_int
    L.mgrit_solve.argtypes = [vp, vp, vp, vp, C.POINTER(Stats)]
    L.mgrit_solve.restype = C.c_int
    L.mgrit_seq_solve.argtypes = [vp, vp, vp, C.POINTER(Stats)]
    L.mgrit_seq_solve.restype = C.c_int
    L.phi_step.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp]
    L.phi_step.restype = C.c_int
    L.phi_step_noalloc.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp]
    L.phi_step_noalloc.restype = C.c_int
    L.mgrit_joule_losses.argtypes = [vp, vp]
    L.mgrit_joule_losses.restype = C.c_int
    L.mgrit_circuit_values.argtypes = [vp, vp, vp]
    L.mgrit_circuit_values.restype = C.c_int
    L.mgrit_level_info.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64), C.POINTER(C.c_int32 * 5)]
    L.mgrit_level_info.restype = C.c_int
    L.mgrit_destroy.argtypes = [vp]
    L.mgrit_destroy.restype = None
    L.mgrit_strerror.argtypes = [C.c_int]
    L.mgrit_strerror.restype = C.c_char_p
    L.mgrit_last_error.argtypes = [vp]
    L.mgrit_last_error.restype = C.c_char_p
    fp = C.POINTER(C.c_float)
    L.mgrit_train_coarse.argtypes = [vp, C.POINTER(TrainParams), C.POINTER(TrainStats)]
    L.mgrit_train_coarse.restype = C.c_int
    L.mgrit_coarse_n_params.argtypes = [vp]
    L.mgrit_coarse_n_params.restype = C.c_int64
    L.mgrit_set_coarse_weights.argtypes = [vp, fp, C.c_int64]
    L.mgrit_set_coarse_weights.restype = C.c_int
    L.mgrit_get_coarse_weights.argtypes = [vp, fp, C.c_int64]
    L.mgrit_get_coarse_weights.restype = C.c_int
    L.mgrit_coarse_apply.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, vp]
    L.mgrit_coarse_apply.restype = C.c_int
    L.mgrit_coarse_gradient.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, vp, dp, fp]
    L.mgrit_coarse_gradient.restype = C.c_int
    L.mgrit_coarse_adam.argtypes = [vp, fp, C.c_double]
    L.mgrit_coarse_adam.restype = C.c_int
    del dp
    _LIB = L
    return L


class MgritError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name} ({status}): {message}")
