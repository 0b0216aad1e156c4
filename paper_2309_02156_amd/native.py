"""ctypes view of libsacc.so: the structs and entry points declared in include/sacc.h.

Argument marshalling only.  Loading fails loudly when the library has not been built:
there is no fallback implementation of any step.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsacc.so")

SA_OK, SA_NOTCONV = 0, 1
SA_EINVAL, SA_ENOMEM, SA_EHIP, SA_ESTATE, SA_EBREAKDOWN, SA_ETOOBIG = -1, -2, -3, -4, -5, -6
SA_FP64, SA_MIXED, SA_MIXED_KRYLOV = 0, 1, 2
SA_CG, SA_GMRES = 0, 1
SA_GALERKIN, SA_MINRES = 0, 1
SA_SKETCH_GAUSSIAN, SA_SKETCH_SRHT = 0, 1
SA_GUESS_PROJECTION, SA_GUESS_ZERO, SA_GUESS_PREVIOUS = 0, 1, 2
SA_BASIS_SKETCHED_QR, SA_BASIS_POD = 0, 1
SA_PRECOND_NONE, SA_PRECOND_JACOBI = 0, 1

EXPORTS = ("sa_workspace_bytes", "sa_init_sequence", "sa_push_solution", "sa_initial_guess",
           "sa_solve", "sa_step", "sa_destroy_sequence", "sa_status_string", "sa_spmv", "sa_copy_state",
           "sa_profile_enable", "sa_profile_read", "sa_mlp_create", "sa_mlp_destroy", "sa_mlp_set_scaling",
           "sa_mlp_forward", "sa_mlp_train_step", "sa_mlp_get", "sa_learned_attach", "sa_set_time",
           "sa_batch_create", "sa_batch_destroy", "sa_batch_step", "sa_batch_plan", "sa_batch_set_mode", "sa_batch_solve_stats", "sa_solve_static",
           "sa_static_scratch_bytes", "sa_state_bytes", "sa_export_state", "sa_import_state")


class SaConfig(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("M", ctypes.c_int32), ("s", ctypes.c_int32),
        ("sketch", ctypes.c_int32), ("projection", ctypes.c_int32), ("solver", ctypes.c_int32),
        ("restart", ctypes.c_int32), ("tol", ctypes.c_double), ("maxit", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("inner_tol", ctypes.c_double),
        ("max_refine", ctypes.c_int32), ("guess", ctypes.c_int32),
        ("rank_tol_sketch", ctypes.c_double), ("rank_tol_chol", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("poll", ctypes.c_int32), ("inner_maxit", ctypes.c_int32),
        ("m", ctypes.c_int32), ("refresh", ctypes.c_int32), ("basis", ctypes.c_int32),
        ("precond", ctypes.c_int32),
    ]


class SaCsr(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr_dev", ctypes.c_void_p),
        ("col_dev", ctypes.c_void_p), ("val_dev", ctypes.c_void_p),
        ("val_is_fp32", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class SaInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("refinements", ctypes.c_int32),
        ("k_eff", ctypes.c_int32), ("k_sketch", ctypes.c_int32), ("used_fallback", ctypes.c_int32),
        ("status", ctypes.c_int32), ("history", ctypes.c_int32), ("relres0", ctypes.c_double),
        ("relres", ctypes.c_double), ("ms_guess", ctypes.c_float), ("ms_solve", ctypes.c_float),
        ("used_learned", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class SaMlpConfig(ctypes.Structure):
    _fields_ = [
        ("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_layers", ctypes.c_int32),
        ("n_out", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("lr", ctypes.c_float),
        ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
        ("reserved", ctypes.c_int32),
    ]


class SaKernelProf(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
        ("bytes", ctypes.c_double),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it is missing: build it with paper_2309_02156_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2309_02156_amd.build` "
                           "(or __graft_entry__.build()) first; there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    P = ctypes.POINTER
    L.sa_workspace_bytes.argtypes = [P(SaConfig), P(sz)]
    L.sa_init_sequence.argtypes = [P(SaConfig), vp, sz, vp, P(vp)]
    L.sa_push_solution.argtypes = [vp, vp, vp]
    L.sa_initial_guess.argtypes = [vp, P(SaCsr), vp, vp, P(SaInfo), vp]
    L.sa_solve.argtypes = [vp, P(SaCsr), vp, vp, P(SaInfo), vp]
    L.sa_step.argtypes = [vp, P(SaCsr), vp, vp, P(SaInfo), vp]
    L.sa_destroy_sequence.argtypes = [vp]
    L.sa_status_string.argtypes = [i32]
    L.sa_status_string.restype = ctypes.c_char_p
    L.sa_spmv.argtypes = [P(SaCsr), vp, vp, vp]
    L.sa_copy_state.argtypes = [vp, i32, vp, sz, vp]
    L.sa_profile_enable.argtypes = [vp, i32]
    L.sa_profile_read.argtypes = [vp, P(SaKernelProf), i32, P(i32)]
    fp = ctypes.POINTER(ctypes.c_float)
    L.sa_mlp_create.argtypes = [P(SaMlpConfig), fp, P(vp)]
    L.sa_mlp_destroy.argtypes = [vp]
    L.sa_mlp_set_scaling.argtypes = [vp, fp, fp, fp, fp]
    L.sa_mlp_forward.argtypes = [vp, vp, i32, vp, vp]
    L.sa_mlp_train_step.argtypes = [vp, vp, vp, i32, vp, vp]
    L.sa_mlp_get.argtypes = [vp, i32, fp, sz, vp]
    L.sa_learned_attach.argtypes = [vp, vp, i32]
    L.sa_set_time.argtypes = [vp, ctypes.c_double]
    L.sa_batch_create.argtypes = [P(vp), i32, i32, i32, P(vp)]
    L.sa_batch_destroy.argtypes = [vp]
    L.sa_batch_step.argtypes = [vp, P(vp), P(vp), P(vp), P(SaInfo)]
    L.sa_batch_plan.argtypes = [vp, P(i32), P(i32), P(i32), P(i32)]
    L.sa_batch_set_mode.argtypes = [vp, i32]
    L.sa_batch_solve_stats.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_double)]
    L.sa_solve_static.argtypes = [P(SaConfig), P(SaCsr), vp, vp, P(SaInfo), vp]
    L.sa_static_scratch_bytes.argtypes = [P(SaConfig), P(sz), P(sz)]
    L.sa_state_bytes.argtypes = [vp, P(sz)]
    L.sa_export_state.argtypes = [vp, vp, sz, vp]
    L.sa_import_state.argtypes = [vp, vp, sz, vp]
    for name in EXPORTS:
        if name != "sa_status_string":
            getattr(L, name).restype = i32
    _lib = L
    return L


class SaccError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().sa_status_string(code).decode()
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


def check(code: int, where: str, allow=(SA_OK,)) -> int:
    if code not in allow:
        raise SaccError(code, where)
    return code
