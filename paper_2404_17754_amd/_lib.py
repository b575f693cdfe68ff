"""ctypes declarations of the C-ABI in include/sw.h (argument marshalling
only).  Loading fails loudly when the built library is missing."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsw.so")

SW_OK, SW_EINVAL, SW_ENOWS, SW_EMESH, SW_ENOCONV, SW_EHIP, SW_ESTATE = 0, -1, -2, -3, -4, -5, -6
SW_FLAG_NOCONV, SW_FLAG_NONFINITE, SW_FLAG_GUESS_FALLBACK = 1, 2, 4
SW_FP64, SW_MIXED_FP32, SW_MIXED_FP32_FLEX, SW_MIXED_FP16 = 0, 1, 2, 3
SW_GUESS_ZERO, SW_GUESS_POLY, SW_GUESS_MLP, SW_GUESS_PROJ, SW_GUESS_PROJ_MLP = 0, 1, 2, 3, 4
SW_OP_M, SW_OP_K, SW_OP_CABS, SW_OP_A = 1, 2, 4, 8
MLP_NPARAM, MLP_ROW = 4929, 12
MISFIT_NOALLOC_MAX_REC = 16384
PROF_KINDS = {"tile_f64": 0, "tile_f32": 1, "update_f64": 2, "update_f32": 3, "dir_f64": 4, "dir_f32": 5}

ERRNAMES = {SW_EINVAL: "SW_EINVAL", SW_ENOWS: "SW_ENOWS", SW_EMESH: "SW_EMESH", SW_ENOCONV: "SW_ENOCONV",
            SW_EHIP: "SW_EHIP", SW_ESTATE: "SW_ESTATE"}


class SwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_tets", C.c_int64), ("n_faces", C.c_int64),
                ("xyz", C.c_void_p), ("tet10", C.c_void_p), ("tri6", C.c_void_p),
                ("face_tet", C.c_void_p), ("face_role", C.c_void_p), ("tile_max_nodes", C.c_int32),
                ("tile_max_elems", C.c_int32), ("deterministic", C.c_int32)]


class CaseDesc(C.Structure):
    _fields_ = [("dt", C.c_double), ("ray_alpha", C.c_double), ("ray_beta", C.c_double), ("rtol", C.c_double),
                ("max_iter", C.c_int32), ("precision", C.c_int32), ("guess", C.c_int32), ("poly_order", C.c_int32),
                ("inner_rtol", C.c_double), ("n_mat", C.c_int32), ("mat", C.c_void_p), ("tet_mat", C.c_void_p),
                ("n_rec", C.c_int32), ("rec_node", C.c_void_p), ("n_steps", C.c_int64), ("v_in", C.c_void_p),
                ("proj_dim", C.c_int32), ("deterministic", C.c_int32)]


class CaseStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("cg_iters", C.c_int64), ("ir_outer", C.c_int64),
                ("max_true_rel_res", C.c_double), ("flags", C.c_int32)]


VP = C.c_void_p
PP = C.POINTER(C.c_void_p)
I32, I64, F64, SZ = C.c_int32, C.c_int64, C.c_double, C.c_size_t

# name: (argtypes)
SIGNATURES = {
    "sw_last_error": (),
    "sw_version": (),
    "sw_ctx_create": (C.c_int, VP, PP),
    "sw_ctx_destroy": (VP,),
    "sw_ctx_set_grid_cap": (VP, I32),
    "sw_ctx_set_graphs": (VP, I32),
    "sw_ctx_profile": (VP, I32),
    "sw_ctx_profile_kinds": (VP, C.c_uint32, I32),
    "sw_ctx_profile_read": (VP, I32, C.POINTER(F64), C.POINTER(I64), C.POINTER(F64), C.POINTER(I64)),
    "sw_mesh_workspace_bytes": (C.POINTER(MeshDesc), C.POINTER(SZ)),
    "sw_mesh_create": (VP, C.POINTER(MeshDesc), VP, SZ, PP),
    "sw_mesh_info": (VP, C.POINTER(I32), C.POINTER(I32)),
    "sw_mesh_destroy": (VP,),
    "sw_case_workspace_bytes": (VP, C.POINTER(CaseDesc), C.POINTER(SZ)),
    "sw_case_create": (VP, VP, C.POINTER(CaseDesc), VP, SZ, PP),
    "sw_case_destroy": (VP,),
    "sw_case_set_state": (VP, VP, VP, VP, I64),
    "sw_case_get_state": (VP, VP, VP, VP, C.POINTER(I64)),
    "sw_case_step": (VP, I32),
    "sw_case_stats_get": (VP, C.POINTER(CaseStats)),
    "sw_case_step_log": (VP, I64, I64, VP, VP),
    "sw_case_waveforms": (VP, I64, I64, VP),
    "sw_case_waveform_device": (VP, PP),
    "sw_case_apply": (VP, I32, VP, VP),
    "sw_case_apply_f32": (VP, I32, VP, VP),
    "sw_case_rhs": (VP, VP),
    "sw_case_guess": (VP, VP),
    "sw_case_diag_blocks": (VP, VP),
    "sw_misfit_workspace_bytes": (I32, C.POINTER(SZ)),
    "sw_misfit": (VP, I32, I64, VP, VP, VP, SZ, C.POINTER(F64), C.POINTER(I32)),
    "sw_misfit_noalloc": (VP, I32, I64, VP, VP, C.POINTER(F64), C.POINTER(I32)),
    "sw_case_misfit": (VP, VP, C.POINTER(F64), C.POINTER(I32)),
    "sw_fit_workspace_bytes": (I32, I64, I32, I32, C.POINTER(SZ)),
    "sw_fit_input": (VP, I32, I64, C.POINTER(VP), VP, I32, I32, F64, VP, SZ, VP, C.POINTER(F64), C.POINTER(I32),
                     C.POINTER(I32), VP),
    "sw_fit_events": (VP, I32, I64, C.POINTER(VP), I32, C.POINTER(VP), I32, I32, F64, VP, SZ, VP, VP, VP, VP,
                      C.POINTER(F64), C.POINTER(I32)),
    "sw_mlp_init_params": (C.c_uint64, VP),
    "sw_mlp_workspace_bytes": (C.POINTER(SZ),),
    "sw_mlp_create": (VP, VP, VP, SZ, PP),
    "sw_mlp_destroy": (VP,),
    "sw_mlp_get_params": (VP, VP),
    "sw_mlp_forward": (VP, VP, VP, I64),
    "sw_mlp_gradient": (VP, VP, I64, VP, C.POINTER(F64)),
    "sw_mlp_train": (VP, VP, I64, I32, I32, C.c_float, C.c_uint64, VP),
    "sw_case_attach_mlp": (VP, VP),
    "sw_case_set_sampler": (VP, VP, I64, I32, C.c_uint64),
    "sw_case_samples": (VP, C.POINTER(I64)),
    "sw_batch_workspace_bytes": (C.POINTER(VP), I32, C.POINTER(SZ)),
    "sw_batch_create": (VP, C.POINTER(VP), I32, VP, SZ, PP),
    "sw_batch_step": (VP, I32),
    "sw_batch_stats": (VP, C.POINTER(CaseStats)),
    "sw_batch_autotune": (VP, I32, C.POINTER(I32), VP),
    "sw_case_autotune": (VP, I32, C.POINTER(I32), VP),
    "sw_batch_apply_f32": (VP, C.POINTER(VP), C.POINTER(VP)),
    "sw_batch_destroy": (VP,),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libsw.so and declare every entry point; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = C.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = list(args)
        fn.restype = C.c_char_p if name in ("sw_last_error", "sw_version") else C.c_int
    _lib = lib
    return lib


def check(rc: int):
    if rc != SW_OK:
        raise SwError(rc, _lib.sw_last_error().decode())
    return rc
