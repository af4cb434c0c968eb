"""ctypes binding of librdbayes.so (the C ABI declared in include/rdbayes.h and
include/rdbayes_growth1d.h).

Argument marshalling only: device arrays are torch tensors on the current
HIP device (passed as raw pointers), host arrays are numpy arrays.  Every
step of the method runs in the library's HIP kernels; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librdbayes.so")

RD_OK, RD_EINVAL, RD_EHIP, RD_ENOMEM, RD_EUNSUPPORTED, RD_ETIMEOUT, RD_EIO = (
    0, -1, -2, -3, -4, -5, -6)
ST_NOT_CONVERGED, ST_BREAKDOWN, ST_NONFINITE, ST_OUT_OF_PRIOR = 1, 2, 4, 8
ST_BAD_GRID, ST_NOT_STEADY, ST_GROUP_TIMEOUT = 16, 32, 64
PRECISION_FP32, PRECISION_FP64 = 0, 1
MODE_PLAIN, MODE_DA = 0, 1
MAX_GRIDS = 8

c_i32, c_u32, c_u64, c_i64, c_d, c_vp = (ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64,
                                         ctypes.c_int64, ctypes.c_double, ctypes.c_void_p)
c_dp = ctypes.POINTER(ctypes.c_double)


class GridDesc(ctypes.Structure):
    _fields_ = [("n", c_i32), ("growth", c_i32), ("growth_rate", c_d),
                ("u0", c_dp), ("v0", c_dp), ("y", c_dp), ("sigma", c_d)]


class ProblemDesc(ctypes.Structure):
    _fields_ = [("n_grids", c_i32), ("grids", ctypes.POINTER(GridDesc)), ("dt", c_d),
                ("n_steps", c_i32), ("cg_rtol", c_d), ("cg_maxit", c_i32), ("precision", c_i32),
                ("free_mask", c_u32), ("lo", c_d * 4), ("hi", c_d * 4), ("step", c_d * 4),
                ("max_batch", c_i32), ("prop_chol", c_d * 16), ("prior_kind", c_i32 * 4),
                ("prior_mean", c_d * 4), ("prior_sd", c_d * 4), ("turing_support", c_i32),
                ("steady_tol", c_d)]


class G1dDesc(ctypes.Structure):
    _fields_ = [("n", c_i32), ("n_steps", c_i32), ("tau", c_d), ("theta", c_d * 4),
                ("law", c_i32), ("rho_T", c_d), ("u0", c_dp), ("v0", c_dp), ("y", c_dp),
                ("obs", c_i32), ("sigma", c_d), ("max_batch", c_i32), ("lo", c_d * 3),
                ("hi", c_d * 3), ("step", c_d * 3), ("prior_kind", c_i32 * 3),
                ("prior_mean", c_d * 3), ("prior_sd", c_d * 3)]


G1D_LAW_POLY, G1D_LAW_EXP, G1D_LAW_LOGISTIC = 0, 1, 2


class Chains(ctypes.Structure):
    _fields_ = [("n_chains", c_i32), ("phi", c_vp), ("loglik", c_vp), ("loglik_sur", c_vp),
                ("grid_id", c_vp), ("n_accept", c_vp), ("n_accept1", c_vp), ("n_solves", c_vp),
                ("cg_iters", c_vp),
                ("trace", c_vp), ("seed", c_u32), ("step", c_u64), ("trace_step0", c_u64),
                ("trace_rows", c_i32), ("imex_steps", c_vp), ("fail_bits", c_vp)]


SYMBOLS = {
    "init_problem": (c_i32, [ctypes.POINTER(ProblemDesc), ctypes.POINTER(c_vp)]),
    "destroy_problem": (c_i32, [c_vp]),
    "forward_solve_batch": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "log_likelihood_batch": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "log_likelihood_batch_noalloc": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "field_misfit_batch": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp]),
    "mcmc_step_batch": (c_i32, [c_vp, ctypes.POINTER(Chains), c_i32, c_i32, c_vp]),
    "propose_batch": (c_i32, [c_vp, ctypes.POINTER(Chains), c_vp, c_vp, c_vp]),
    "accept_batch": (c_i32, [c_vp, ctypes.POINTER(Chains), c_vp, c_vp, c_vp, c_vp]),
    "pmh_step_batch": (c_i32, [c_vp, ctypes.POINTER(Chains), c_i32, c_i32, c_vp]),
    "pmh_propose_batch": (c_i32, [c_vp, ctypes.POINTER(Chains), c_i32, c_vp, c_vp, c_vp]),
    "pmh_resample_batch": (c_i32, [c_vp, ctypes.POINTER(Chains), c_i32, c_vp, c_vp, c_vp, c_vp]),
    "surrogate_create": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_u32]),
    "downsample_batch": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp]),
    "surrogate_set_scaling": (c_i32, [c_vp, c_vp, c_vp, c_d, c_vp]),
    "surrogate_train_step": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_d, c_vp, c_vp]),
    "surrogate_forward": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_i32, c_vp]),
    "surrogate_loglik_batch": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp]),
    "surrogate_params": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_i32, c_vp]),
    "rd_autotune": (c_i32, [c_vp, c_vp]),
    "rd_set_tile": (c_i32, [c_vp, c_i32, c_i32]),
    "forward_solve_steady_batch": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                           c_vp]),
    "rd_set_mixed_threads": (c_i32, [c_vp, c_i32]),
    "rd_set_da_substeps": (c_i32, [c_vp, c_i32]),
    "rd_solver_timing": (c_i32, [c_vp, c_i32, c_dp, ctypes.POINTER(c_i64), c_i32]),
    "rd_mixed_threads": (c_i32, [c_vp, ctypes.POINTER(c_i32)]),
    "rd_captured_graphs": (c_i32, [c_vp, ctypes.POINTER(c_i32)]),
    "surrogate_set_input_box": (c_i32, [c_vp, c_dp, c_dp]),
    "g1d_init": (c_i32, [ctypes.POINTER(G1dDesc), ctypes.POINTER(c_vp)]),
    "g1d_destroy": (c_i32, [c_vp]),
    "g1d_forward_batch": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "g1d_log_likelihood_batch": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp]),
    "g1d_mcmc_step_batch": (c_i32, [c_vp, ctypes.POINTER(Chains), c_i32, c_vp]),
    "rd_check_solves": (c_i32, [c_vp, ctypes.POINTER(c_i64), c_i32]),
    "rd_chains_save": (c_i32, [ctypes.POINTER(Chains), ctypes.c_char_p, c_vp]),
    "rd_chains_load": (c_i32, [ctypes.POINTER(Chains), ctypes.c_char_p, c_vp]),
    "rd_set_coop_wait": (c_i32, [c_vp, c_i64, c_i64]),
    "rd_status_string": (ctypes.c_char_p, [c_i32]),
    "rd_last_error": (ctypes.c_char_p, []),
}


class LibraryMissing(RuntimeError):
    pass


_lib = None


def lib():
    """Loads librdbayes.so (built by paper_1605_04718_amd.build); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} is not built; run `python -m paper_1605_04718_amd.build` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SYMBOLS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class RDError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().rd_last_error().decode(errors="replace")
        super().__init__(f"{where}: error {code} ({lib().rd_status_string(code).decode()}): {msg}")
        self.code = code


def check(code, where):
    if code != RD_OK:
        raise RDError(code, where)
