"""ctypes binding of the C ABI in include/pff.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpff.so")


class MeshSpec(C.Structure):
    _fields_ = [("n_base", C.c_int32), ("n_local", C.c_int32), ("degree", C.c_int32),
                ("coarse", C.c_int32), ("band_x", C.c_double), ("band_y", C.c_double),
                ("tile_x", C.c_int32), ("tile_y", C.c_int32), ("mg_global", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("Gc", C.c_double),
                ("pressure", C.c_double), ("kappa", C.c_double), ("ell", C.c_double),
                ("cheb_degree", C.c_int32), ("smooth_range", C.c_double),
                ("upper_factor", C.c_double), ("eig_cg_its", C.c_int32),
                ("coarse_mode", C.c_int32), ("coarse_its", C.c_int32),
                ("coarse_eig_its", C.c_int32), ("gmres_restart", C.c_int32),
                ("gmres_max_its", C.c_int32), ("gmres_rtol", C.c_double),
                ("gmres_atol", C.c_double), ("ls_omega", C.c_double), ("ls_max", C.c_int32),
                ("vcycle_fp32", C.c_int32), ("pdas_c", C.c_double), ("mg_kind", C.c_int32),
                ("prec_kind", C.c_int32), ("eig_cg_its_phi", C.c_int32)]


class GmresInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32),
                ("initial_residual", C.c_double), ("final_residual", C.c_double),
                ("tolerance", C.c_double)]


class NewtonInfo(C.Structure):
    _fields_ = [("residual_before", C.c_double), ("residual_after", C.c_double),
                ("rhs_norm", C.c_double), ("gmres_iterations", C.c_int32),
                ("gmres_converged", C.c_int32), ("ls_trials", C.c_int32),
                ("n_active", C.c_int64), ("active_changed", C.c_int64),
                ("setup_seconds", C.c_double), ("solve_seconds", C.c_double),
                ("linesearch_seconds", C.c_double)]


VP = C.c_void_p
_SIGS = {
    "pff_default_params": (C.c_int, [C.POINTER(Params)]),
    "pff_create": (C.c_int, [C.POINTER(MeshSpec), C.POINTER(Params), C.POINTER(VP)]),
    "pff_destroy": (C.c_int, [VP]),
    "pff_set_params": (C.c_int, [VP, C.POINTER(Params)]),
    "pff_sizes": (C.c_int, [VP, C.POINTER(C.c_int64), C.POINTER(C.c_int32), VP]),
    "pff_workspace_bytes": (C.c_int, [VP, C.POINTER(C.c_size_t)]),
    "pff_bind_workspace": (C.c_int, [VP, VP, C.c_size_t]),
    "pff_lattice": (C.c_int, [VP, C.POINTER(C.c_int64)]),
    "pff_node_coords": (C.c_int, [VP, C.c_int32, VP]),
    "pff_node_flags": (C.c_int, [VP, C.c_int32, VP]),
    "pff_tile_stats": (C.c_int, [VP, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int64)]),
    "pff_set_state": (C.c_int, [VP, VP, VP, VP, VP, C.c_int32, VP]),
    "pff_get_active": (C.c_int, [VP, VP, VP]),
    "pff_extrapolate_phi": (C.c_int, [VP, VP, VP, C.c_double, VP, VP]),
    "pff_extrapolate_phi_load": (C.c_int, [VP, VP, VP, C.c_double, C.c_double, C.c_double, VP, VP]),
    "pff_vmult": (C.c_int, [VP, VP, VP, VP]),
    "pff_vmult_T": (C.c_int, [VP, VP, VP, C.c_int32, VP]),
    "pff_vmult_noalloc": (C.c_int, [VP, VP, VP, VP]),
    "pff_inverse_diagonal": (C.c_int, [VP, C.c_int32, VP, C.c_int32, VP]),
    "pff_vcycle": (C.c_int, [VP, VP, VP, C.c_int32, VP]),
    "pff_get_eigen": (C.c_int, [VP, VP, VP]),
    "pff_set_eigen": (C.c_int, [VP, VP, VP]),
    "pff_gmres_solve": (C.c_int, [VP, VP, VP, C.c_int32, C.c_double, C.POINTER(GmresInfo), VP]),
    "pff_newton_step": (C.c_int, [VP, VP, VP, VP, VP, C.POINTER(NewtonInfo), VP]),
    "pff_residual": (C.c_int, [VP, VP, VP, C.c_int32, VP]),
    "pff_tcv": (C.c_int, [VP, VP, C.POINTER(C.c_double), VP, VP]),
    "pff_cod": (C.c_int, [VP, VP, VP, C.c_int32, VP, VP]),
    "pff_param_grad": (C.c_int, [VP, VP, VP, VP]),
    "pff_adjoint_tcv": (C.c_int, [VP, VP, C.POINTER(C.c_double), VP, VP, C.c_double, C.POINTER(GmresInfo), VP]),
    "pff_distribute": (C.c_int, [VP, VP, C.c_int32, VP]),
    "pff_mask_constrained": (C.c_int, [VP, VP, VP]),
    "pff_dot": (C.c_int, [VP, VP, VP, C.c_int64, C.POINTER(C.c_double), VP]),
    "pff_last_error": (C.c_char_p, [VP]),
    # host-only mesh inspection (pff_mesh.h)
    "pff_mesh_build": (C.c_int, [C.POINTER(MeshSpec), C.POINTER(VP)]),
    "pff_mesh_free": (C.c_int, [VP]),
    "pff_mesh_sizes": (C.c_int, [VP, C.POINTER(C.c_int64), C.POINTER(C.c_int32), VP,
                                 C.POINTER(C.c_int64)]),
    "pff_mesh_leaf_cells": (C.c_int, [VP, C.POINTER(C.c_int64)]),
    "pff_mesh_coords": (C.c_int, [VP, C.c_int32, VP]),
    "pff_mesh_flags": (C.c_int, [VP, C.c_int32, VP]),
    "pff_mesh_hanging": (C.c_int, [VP, C.POINTER(C.c_int64), VP, VP, VP]),
    "pff_mesh_prolongation": (C.c_int, [VP, C.c_int32, C.POINTER(C.c_int64), VP, VP, VP]),
    "pff_mesh_leaf_index": (C.c_int, [VP, C.c_int32, VP]),
    "pff_mesh_tile_stats": (C.c_int, [VP, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]),
    "pff_mesh_tile_tables": (C.c_int, [VP, C.c_int32, VP, VP, VP, VP, VP, VP, VP, VP, VP, VP, VP, VP]),
    "pff_mesh_gc_nodes": (C.c_int, [VP, C.c_int32, C.POINTER(C.c_int64)]),
    "pff_mesh_gc_coords": (C.c_int, [VP, C.c_int32, VP]),
    "pff_mesh_gc_flags": (C.c_int, [VP, C.c_int32, VP]),
    "pff_mesh_gc_leaf_index": (C.c_int, [VP, C.c_int32, VP]),
    "pff_mesh_gc_interpolation": (C.c_int, [VP, C.c_int32, C.POINTER(C.c_int64), VP, VP, VP]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
        # PyTorch brings its own HIP runtime: initialise it before the
        # library's first HIP call, or device allocations of a process that
        # loaded the library first (e.g. a host-only caller, then a solver)
        # fail with an out-of-memory error
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        lib = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS)
