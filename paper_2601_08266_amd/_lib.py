"""ctypes declarations of the C ABI in include/fsi.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsi.so")

FSI_OK = 0
FSI_ERR_ARG = -1
FSI_ERR_HIP = -2
FSI_ERR_WORKSPACE = -3
FSI_ERR_NOT_CONVERGED = -4
FSI_ERR_BREAKDOWN = -5
FSI_ERR_NAN = -6
FSI_ERR_UNSUPPORTED = -7

FSI_F64 = 0
FSI_F32 = 1

FSI_PC_BJACOBI = 0
FSI_PC_SCHUR_DIAG = 1
FSI_PC_SCHUR_TRI = 2


class FsiGrid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("order", ctypes.c_int32),
                ("x0", ctypes.c_double * 3), ("h", ctypes.c_double * 3)]


class FsiVmsParams(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("c_m", ctypes.c_double), ("dt", ctypes.c_double),
                ("C_T", ctypes.c_double), ("C_I", ctypes.c_double),
                ("visc_strong", ctypes.c_int32)]


class FsiProblem(ctypes.Structure):
    _fields_ = [("grid", FsiGrid), ("prm", FsiVmsParams), ("dtype", ctypes.c_int),
                ("a", ctypes.c_void_p), ("s", ctypes.c_void_p), ("dir_mask", ctypes.c_void_p),
                ("m", ctypes.c_int64), ("cell", ctypes.c_void_p), ("xi", ctypes.c_void_p),
                ("perm", ctypes.c_void_p), ("occ_cell", ctypes.c_void_p),
                ("occ_start", ctypes.c_void_p), ("occ_index", ctypes.c_void_p),
                ("n_occ", ctypes.c_int64), ("kappa", ctypes.c_void_p),
                ("dlm_gram", ctypes.c_void_p), ("solid", ctypes.c_void_p), ("solid_U", ctypes.c_void_p),
                ("solid_cM", ctypes.c_double), ("solid_cK", ctypes.c_double), ("solid_cV", ctypes.c_double)]


class FsiSolid(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_elem", ctypes.c_int64), ("X0", ctypes.c_void_p),
                ("conn", ctypes.c_void_p), ("node_start", ctypes.c_void_p),
                ("node_slot", ctypes.c_void_p), ("C0", ctypes.c_double), ("kappa_s", ctypes.c_double),
                ("rho_s0", ctypes.c_double), ("rho_f", ctypes.c_double), ("mu_f", ctypes.c_double)]


class FsiSolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("inner", ctypes.c_int),
                ("inner_reduction", ctypes.c_double), ("precond", ctypes.c_int32),
                ("vel_steps", ctypes.c_int32), ("host_ring", ctypes.c_void_p),
                ("host_ring_len", ctypes.c_int64), ("basis", ctypes.c_int32)]


class FsiSolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("cycles", ctypes.c_int32), ("status", ctypes.c_int32),
                ("bnorm", ctypes.c_double), ("res0", ctypes.c_double),
                ("res_final", ctypes.c_double), ("t_total_ms", ctypes.c_double)]


class FsiNewtonOpts(ctypes.Structure):
    _fields_ = [("max_newton", ctypes.c_int32), ("tol_abs", ctypes.c_double),
                ("eta", ctypes.c_double), ("restart", ctypes.c_int32),
                ("max_krylov", ctypes.c_int32), ("inner", ctypes.c_int),
                ("inner_reduction", ctypes.c_double), ("precond", ctypes.c_int32),
                ("vel_steps", ctypes.c_int32), ("tangent", ctypes.c_int32),
                ("host_ring", ctypes.c_void_p), ("host_ring_len", ctypes.c_int64),
                ("pc_reuse", ctypes.c_int32), ("basis", ctypes.c_int32)]


class FsiNewtonStats(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("krylov_iters", ctypes.c_int32),
                ("status", ctypes.c_int32), ("res_hist", ctypes.c_double * 32),
                ("t_total_ms", ctypes.c_double), ("t_residual_ms", ctypes.c_double),
                ("t_setup_ms", ctypes.c_double), ("t_krylov_ms", ctypes.c_double)]


class FsiNnPackSpec(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p * 32), ("b", ctypes.c_void_p * 32),
                ("c", ctypes.c_void_p * 32), ("ca", ctypes.c_double * 32),
                ("cb", ctypes.c_double * 32), ("cc", ctypes.c_double * 32),
                ("cst", ctypes.c_double * 32), ("shift", ctypes.c_double * 32),
                ("scale", ctypes.c_double * 32), ("nch", ctypes.c_int32)]


class FsiNnUnpackSpec(ctypes.Structure):
    _fields_ = [("shift", ctypes.c_double * 4), ("scale", ctypes.c_double * 4)]


class FsiError(RuntimeError):
    def __init__(self, func, code, msg):
        super().__init__(f"{func} failed with status {code}: {msg}")
        self.code = code


_lib = None

P = ctypes.c_void_p
I64 = ctypes.c_int64
SZ = ctypes.c_size_t

# name -> (restype, argtypes)
SIGNATURES = {
    "fsi_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "fsi_last_error": (ctypes.c_char_p, []),
    "fsi_version": (ctypes.c_char_p, []),
    "fsi_vms_apply_workspace": (SZ, [ctypes.POINTER(FsiGrid), ctypes.c_int]),
    "fsi_vms_apply": (ctypes.c_int, [ctypes.POINTER(FsiGrid), ctypes.POINTER(FsiVmsParams),
                                     ctypes.c_int, P, P, P, P, P, P, SZ, P]),
    "fsi_dlm_locate_workspace": (SZ, [ctypes.POINTER(FsiGrid), I64]),
    "fsi_dlm_locate": (ctypes.c_int, [ctypes.POINTER(FsiGrid), I64, P, ctypes.c_int, P, P, P, P, P,
                                      P, P, ctypes.c_double, ctypes.POINTER(I64),
                                      ctypes.POINTER(I64), P, SZ, P]),
    "fsi_dlm_B": (ctypes.c_int, [ctypes.POINTER(FsiGrid), ctypes.c_int, I64, P, P, P, P, P]),
    "fsi_dlm_B_located": (ctypes.c_int, [ctypes.POINTER(FsiGrid), ctypes.c_int, I64, P, P, I64, P, P, P, P]),
    "fsi_dlm_permute": (ctypes.c_int, [ctypes.c_int, I64, ctypes.c_int32, P, ctypes.c_int32, P, P, P]),
    "fsi_dlm_BT_workspace": (SZ, [ctypes.POINTER(FsiGrid), I64, ctypes.c_int]),
    "fsi_dlm_BT": (ctypes.c_int, [ctypes.POINTER(FsiGrid), ctypes.c_int, I64, P, P, P, P, P, P, I64,
                                  P, P, P, P, SZ, P]),
    "fsi_dlm_gram": (ctypes.c_int, [ctypes.POINTER(FsiGrid), ctypes.c_int, I64, P, P, P, I64, P, P,
                                    P]),
    "fsi_dlm_BT_noalloc_max_bytes": (SZ, []),
    "fsi_dlm_BT_noalloc": (ctypes.c_int, [ctypes.POINTER(FsiGrid), ctypes.c_int, I64, P, P, P, P, P, I64,
                                          P, P, P, P]),
    "fsi_jacobian_workspace": (SZ, [ctypes.POINTER(FsiProblem)]),
    "fsi_jacobian_apply": (ctypes.c_int, [ctypes.POINTER(FsiProblem), P, P, P, SZ, P]),
    "fsi_jacobian_apply_block": (ctypes.c_int, [ctypes.POINTER(FsiProblem), ctypes.c_int32, P, P, P, SZ, P]),
    "fsi_vms_residual": (ctypes.c_int, [ctypes.POINTER(FsiProblem), P, P, P, P, P, P, SZ, P]),
    "fsi_solid_setup": (ctypes.c_int, [I64, I64, P, P, P, P]),
    "fsi_solid_workspace": (SZ, [I64, ctypes.c_int]),
    "fsi_solid_apply": (ctypes.c_int, [ctypes.POINTER(FsiSolid), ctypes.c_int, P, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, P, P, P, SZ, P]),
    "fsi_jacobian_solid_workspace": (SZ, [ctypes.POINTER(FsiProblem), ctypes.POINTER(FsiSolid)]),
    "fsi_solid_residual": (ctypes.c_int, [ctypes.POINTER(FsiSolid), P, P, P, P, P, SZ, P]),
    "fsi_solid_step_workspace": (SZ, [ctypes.POINTER(FsiProblem), ctypes.POINTER(FsiSolid)]),
    "fsi_solid_step_residual": (ctypes.c_int, [ctypes.POINTER(FsiProblem), ctypes.POINTER(FsiSolid), P, P,
                                               ctypes.c_double, ctypes.c_double, P, P, P, P, P, P, P, SZ, P]),
    "fsi_jacobian_solid_apply": (ctypes.c_int, [ctypes.POINTER(FsiProblem), ctypes.POINTER(FsiSolid), P,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P,
                                                P, SZ, P]),
    "fsi_bjacobi_workspace": (SZ, [ctypes.POINTER(FsiGrid)]),
    "fsi_bjacobi_setup": (ctypes.c_int, [ctypes.POINTER(FsiProblem), P, P, P, ctypes.POINTER(I64),
                                         P, SZ, P]),
    "fsi_bjacobi_apply": (ctypes.c_int, [ctypes.POINTER(FsiGrid), ctypes.c_int, P, P, P, P]),
    "fsi_schur_size": (SZ, [ctypes.POINTER(FsiGrid)]),
    "fsi_schur_info": (ctypes.c_int, [ctypes.POINTER(FsiGrid), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(I64)]),
    "fsi_schur_setup": (ctypes.c_int, [ctypes.POINTER(FsiProblem), P, P, SZ, P]),
    "fsi_schur_apply": (ctypes.c_int, [ctypes.POINTER(FsiProblem), ctypes.c_int32, ctypes.c_int32, P, P, P, P,
                                       SZ, P]),
    "fsi_fgmres_workspace": (SZ, [ctypes.POINTER(FsiProblem), ctypes.POINTER(FsiProblem),
                                  ctypes.POINTER(FsiSolveOpts)]),
    "fsi_fgmres_solve": (ctypes.c_int, [ctypes.POINTER(FsiProblem), ctypes.POINTER(FsiProblem), P,
                                        P, P, ctypes.POINTER(FsiSolveOpts),
                                        ctypes.POINTER(FsiSolveStats), P, SZ, P]),
    "fsi_newton_workspace": (SZ, [ctypes.POINTER(FsiProblem), ctypes.POINTER(FsiProblem),
                                  ctypes.POINTER(FsiNewtonOpts)]),
    "fsi_tangent_workspace": (SZ, [ctypes.POINTER(FsiProblem)]),
    "fsi_tangent_apply": (ctypes.c_int, [ctypes.POINTER(FsiProblem), P, P, P, P, P, SZ, P]),
    "fsi_newton_solve": (ctypes.c_int, [ctypes.POINTER(FsiProblem), ctypes.POINTER(FsiProblem), P, P,
                                        P, P, ctypes.POINTER(FsiNewtonOpts),
                                        ctypes.POINTER(FsiNewtonStats), P, SZ, P]),
    "fsi_newton_solid_workspace": (SZ, [ctypes.POINTER(FsiProblem), ctypes.POINTER(FsiProblem),
                                        ctypes.POINTER(FsiSolid), ctypes.POINTER(FsiNewtonOpts)]),
    "fsi_newton_solid_solve": (ctypes.c_int, [ctypes.POINTER(FsiProblem), ctypes.POINTER(FsiProblem),
                                              ctypes.POINTER(FsiSolid), P, P, ctypes.c_double, ctypes.c_double,
                                              P, P, P, P, P,
                                              ctypes.POINTER(FsiNewtonOpts), ctypes.POINTER(FsiNewtonStats), P,
                                              SZ, P]),
    "fsi_conv3d_fwd": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_int32, P,
                                      P, P, P]),
    "fsi_conv3d_wgrad_workspace": (SZ, [P, ctypes.c_int32, ctypes.c_int32]),
    "fsi_conv3d_wgrad": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, SZ, P]),
    "fsi_conv3d_flip_transpose": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, P, P, P]),
    "fsi_mse_workspace": (SZ, []),
    "fsi_mse_loss": (ctypes.c_int, [I64, ctypes.c_int32, ctypes.c_int32, P, P, P,
                                    ctypes.POINTER(ctypes.c_double), P, SZ, P]),
    "fsi_adam_step": (ctypes.c_int, [I64, P, P, P, P, P, ctypes.c_int32, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, ctypes.c_float, P]),
    "fsi_to_bf16": (ctypes.c_int, [I64, P, P, P]),
    "fsi_nn_pack": (ctypes.c_int, [I64, ctypes.c_int32, ctypes.POINTER(FsiNnPackSpec), P, P]),
    "fsi_nn_moments_workspace": (SZ, [ctypes.c_int32]),
    "fsi_nn_moments": (ctypes.c_int, [I64, ctypes.c_int32, P, P, P, SZ, P]),
    "fsi_nn_unpack": (ctypes.c_int, [I64, ctypes.c_int32, P, P, ctypes.POINTER(FsiNnUnpackSpec), P,
                                     P, P, P]),
    "fsi_axpby": (ctypes.c_int, [I64, ctypes.c_double, P, ctypes.c_double, P, P]),
    "fsi_dot": (ctypes.c_int, [I64, P, P, ctypes.POINTER(ctypes.c_double), P, SZ, P]),
    "fsi_dot_workspace": (SZ, []),
    "fsi_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "fsi_profile_read": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(I64)]),
}


def lib():
    """Load libfsi.so (built in-tree by build.py); fail loudly if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} not found: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(func: str, code: int):
    if code != FSI_OK:
        msg = lib().fsi_last_error().decode(errors="replace")
        raise FsiError(func, code, msg)
    return code
