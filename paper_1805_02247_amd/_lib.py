"""ctypes loader for libpmr.so (the HIP library). Argument marshalling only.

The library must have been built (``__graft_entry__.build()`` or ``build.sh``); there is no
fallback: importing the binding without it raises.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmr.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "pmr.h")

PMR_OK = 0
PMR_E_NONFINITE = -5
PMR_E_STATE = -6
PMR_FP32, PMR_MIXED = 0, 1
PMR_LOSS_DENSITY_L2, PMR_LOSS_LOGNORMAL = 0, 1
PMR_HALO_SINGLE, PMR_HALO_TWO = 0, 1
PMR_NNP_FLOATS = 50 * 81 + 50 + 30 * 50 + 30 + 30 + 1
PMR_NNM_FLOATS = 20 * 3 + 20 + 10 * 20 + 10 + 10 + 1
PMR_FFT_YPASS, PMR_FFT_XPASS, PMR_FFT_XPASS_MULTI = 0, 1, 2
DBG = {"x": 1, "force": 2, "sort_ids": 3, "delta_f": 4, "features": 5, "mass_r": 6,
       "res_s": 7, "xbar0": 8, "pbar0": 9, "dbar_f": 10}


class PmrConfig(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int), ("n_part", ctypes.c_int), ("n_mesh", ctypes.c_int),
                ("n_out", ctypes.c_int), ("n_steps", ctypes.c_int), ("mlp_hidden", ctypes.c_int),
                ("precision", ctypes.c_int), ("ckpt_every", ctypes.c_int),
                ("loss_kind", ctypes.c_int), ("box", ctypes.c_double), ("a0", ctypes.c_double),
                ("a1", ctypes.c_double), ("omega_m", ctypes.c_double), ("R1", ctypes.c_double),
                ("R2", ctypes.c_double), ("ic_order", ctypes.c_int),
                ("halo_model", ctypes.c_int)]


class PmrLossParams(ctypes.Structure):
    _fields_ = [("M0", ctypes.c_double), ("mu", ctypes.c_double), ("sigma_N", ctypes.c_double),
                ("R_mass", ctypes.c_double), ("R_sm", ctypes.c_double),
                ("prior_weight", ctypes.c_double), ("logistic_a", ctypes.c_double)]


class PmrLbfgsParams(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("max_iter", ctypes.c_int), ("max_halvings", ctypes.c_int),
                ("c1", ctypes.c_double), ("curvature_eps", ctypes.c_double),
                ("rel_tol", ctypes.c_double), ("stop_below", ctypes.c_double)]


PMR_LBFGS_MAX_M = 64


class PmrLbfgsState(ctypes.Structure):
    """The leading block of the device-driven L-BFGS state (pmr_lbfgs_state)."""
    _fields_ = [("f", ctypes.c_double), ("t", ctypes.c_double), ("gd", ctypes.c_double),
                ("gg", ctypes.c_double), ("rel", ctypes.c_double), ("ft", ctypes.c_double),
                ("ss", ctypes.c_double), ("beta", ctypes.c_double), ("status", ctypes.c_int),
                ("iters", ctypes.c_int), ("evals", ctypes.c_int), ("count", ctypes.c_int),
                ("halvings", ctypes.c_int), ("probe", ctypes.c_int), ("accepted", ctypes.c_int),
                ("slot", ctypes.c_int), ("reset", ctypes.c_int), ("pad", ctypes.c_int),
                ("clock_khz", ctypes.c_longlong), ("p", PmrLbfgsParams),
                ("order", ctypes.c_int * PMR_LBFGS_MAX_M),
                ("alpha", ctypes.c_double * (PMR_LBFGS_MAX_M + 1))]


PMR_LBFGS_STATUS = {0: "idle", 1: "running", 2: "converged", 3: "stationary", 4: "line_search",
                    5: "max_iter", 6: "target_loss"}


class PmrError(RuntimeError):
    def __init__(self, msg, status=None):
        super().__init__(msg)
        self.status = status


_lib = None

vp, sz, ci, cd, cf = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double, ctypes.c_float

SIGNATURES = {
    "pmr_workspace_bytes": (sz, [ctypes.POINTER(PmrConfig)]),
    "pmr_create": (ci, [ctypes.POINTER(PmrConfig), vp, sz, vp, ctypes.POINTER(vp)]),
    "pmr_set_stream": (ci, [vp, vp]),
    "pmr_destroy": (ci, [vp]),
    "pmr_set_prior": (ci, [vp, vp]),
    "pmr_set_mlp": (ci, [vp, vp, vp, vp, vp, vp, vp]),
    "pmr_set_halo_nets": (ci, [vp, vp, vp]),
    "pmr_set_check_finite": (ci, [vp, ci]),
    "pmr_set_target": (ci, [vp, vp]),
    "pmr_set_loss": (ci, [vp, ctypes.POINTER(PmrLossParams)]),
    "pmr_set_loss_device": (ci, [vp, vp]),
    "pmr_forward_count": (ctypes.c_longlong, [vp]),
    "pmr_set_noise_table": (ci, [vp, ci, ctypes.POINTER(cd), ctypes.POINTER(cd),
                                 ctypes.POINTER(cd)]),
    "pmr_forward": (ci, [vp, vp, vp, vp]),
    "pmr_adjoint": (ci, [vp, vp, vp, vp]),
    "pmr_status_string": (ctypes.c_char_p, [ci]),
    "pmr_debug_copy": (ctypes.c_longlong, [vp, ci, ci, vp]),
    "pmr_fft_r2c": (ci, [ci, ci, vp, vp, vp]),
    "pmr_fft_c2r": (ci, [ci, ci, vp, vp, vp]),
    "pmr_sort_scratch_bytes": (sz, [ci, ci, ci]),
    "pmr_cic_sort": (ci, [ci, ci, ci, cd, vp, vp, vp, vp, vp, sz, vp]),
    "pmr_cic_paint": (ci, [ci, ci, ci, cd, vp, vp, vp, vp, cf, cf, vp, vp, sz, vp]),
    "pmr_fft_set_tile": (ci, [ci, ci, ci, ci, ci]),
    "pmr_fft_get_tile": (ci, [ci, ci, ctypes.POINTER(ci), ctypes.POINTER(ci), ctypes.POINTER(ci)]),
    "pmr_fft_set_slab": (ci, [ci, ci]),
    "pmr_paint_set_rows": (ci, [ci, ci, ci]),
    "pmr_paint_get_rows": (ci, [ci, ci, ctypes.POINTER(ci)]),
    "pmr_fft_get_slab": (ci, [ci, ctypes.POINTER(ci)]),
    "pmr_vec_work_bytes": (sz, [sz, ci]),
    "pmr_vec_dot": (ci, [sz, vp, vp, vp, vp, vp]),
    "pmr_vec_axpby": (ci, [sz, cd, vp, cd, vp, vp, vp]),
    "pmr_lbfgs_direction": (ci, [sz, ci, ci, ctypes.POINTER(ci), vp, vp, vp, vp, vp, vp, vp,
                                 vp]),
    "pmr_lbfgs_direction_noalloc": (ci, [sz, ci, ci, ctypes.POINTER(ci), vp, vp, vp, vp, vp,
                                         vp, vp]),
    "pmr_lbfgs_state_bytes": (sz, [ci]),
    "pmr_lbfgs_init": (ci, [sz, ctypes.POINTER(PmrLbfgsParams), vp, vp, vp, vp, vp, vp, vp, vp,
                            vp, vp]),
    "pmr_lbfgs_trial": (ci, [sz, vp, vp, vp, vp, vp]),
    "pmr_lbfgs_update": (ci, [sz, ci, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
    "pmr_power_work_bytes": (sz, [ci]),
    "pmr_power_bins": (ci, [ci, cd, vp, vp, ci, vp, vp, sz, vp]),
    "pmr_profile_begin": (ci, [vp, ci, ci]),
    "pmr_profile_end": (ci, [vp, ctypes.POINTER(cd), ctypes.POINTER(ctypes.c_longlong),
                             ctypes.POINTER(cd)]),
}
PROF = {"paint": 1, "xpass_force": 2, "ypass": 3, "zpass": 4, "kick_drift": 5, "paint3": 6,
        "xpass_force_adj": 7, "adj_gather": 8, "adj_update": 9, "halo2": 10,
        "halo2_stencil": 11, "sort": 13,
        "network": 14}


def lib():
    """Load libpmr.so (once). Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libpmr.so not found at {LIB_PATH}; build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        from . import tune  # applies the autotuned FFT tile shapes, if any
        tune.apply_cache()
    return _lib


def check(status):
    if status != PMR_OK:
        msg = lib().pmr_status_string(int(status)).decode()
        raise PmrError(f"libpmr status {status}: {msg}", int(status))
    return status
