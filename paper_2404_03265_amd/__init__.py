"""MI355X-native matrix-free phase-field Jacobian, multigrid and Newton solver.

Thin Python layer over the C ABI of include/pff.h: it only marshals torch
device tensors (memory and streams) into the library, which does all of the
arithmetic in HIP kernels. The library's work buffers live in one torch uint8
tensor bound to the context (pff_bind_workspace), so torch owns the device
memory. There is no CPU fallback: without the built library (libpff.so next
to this file) every call raises.

The drivers above one Newton step (load step, quasi-static load path, adjoint
gradient, torch.autograd forms) are in paper_2404_03265_amd.autograd.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib

__all__ = ["PhaseFieldSolver", "SolverParams", "load_library"]


def load_library():
    return _lib.load()


@dataclass
class SolverParams:
    E: float = 1.0
    nu: float = 0.2
    Gc: float = 1.0
    pressure: float = 1e-3
    kappa: float = 1e-10
    ell: float = 0.1
    cheb_degree: int = 3
    smooth_range: float = 0.08
    upper_factor: float = 1.2
    eig_cg_its: int = 20
    coarse_mode: int = 0
    coarse_its: int = 30
    coarse_eig_its: int = 40
    gmres_restart: int = 30
    gmres_max_its: int = 300
    gmres_rtol: float = 1e-8
    gmres_atol: float = 1e-12
    ls_omega: float = 0.5
    ls_max: int = 10
    vcycle_fp32: int = 0
    pdas_c: float = 0.0
    mg_kind: int = 0   # 0: local smoothing, 1: global coarsening (needs mg_global=True)
    prec_kind: int = 0  # 0: block diagonal, 1: block triangular (keeps the coupling block)
    eig_cg_its_phi: int = 10  # CG steps of the phase-field block's eigenvalue estimate (levels > 0)

    def to_c(self):
        p = _lib.Params()
        for k in self.__dataclass_fields__:
            setattr(p, k, getattr(self, k))
        return p


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class PhaseFieldSolver:
    """One mesh + parameter set on the current HIP device.

    torch_workspace=True: the library's work buffers live in one torch uint8
    tensor bound with pff_bind_workspace (sized for the current
    gmres_restart); False: the library allocates them on first use."""

    def __init__(self, n_base: int, n_local: int, degree: int, coarse: int = 16,
                 band=(2.0, 0.5), tile=(0, 0), params: SolverParams | None = None,
                 torch_workspace: bool = True, mg_global: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("PhaseFieldSolver needs a HIP device")
        self.lib = _lib.load()
        self.params = params or SolverParams()
        spec = _lib.MeshSpec(n_base, n_local, degree, coarse, band[0], band[1], tile[0], tile[1], int(mg_global))
        h = C.c_void_p()
        rc = self.lib.pff_create(C.byref(spec), C.byref(self.params.to_c()), C.byref(h))
        if rc != 0:
            msg = self.lib.pff_last_error(None)
            raise RuntimeError(f"pff_create failed ({rc}): {msg.decode() if msg else ''}")
        self.h = h
        self._sizes()
        M = C.c_int64()
        self._check(self.lib.pff_lattice(self.h, C.byref(M)))
        self.M = M.value
        self.degree = degree
        self._ws = None
        if torch_workspace:
            self._ws = torch.empty(self.workspace_bytes(), dtype=torch.uint8, device="cuda")
            self._check(self.lib.pff_bind_workspace(self.h, _ptr(self._ws), self._ws.numel()))

    def _sizes(self):
        # level sizes of the hierarchy that params.mg_kind selects
        n = C.c_int64()
        nl = C.c_int32()
        self._check(self.lib.pff_sizes(self.h, C.byref(n), C.byref(nl), None))
        self.n = n.value
        self.n_levels = nl.value
        lvl = (C.c_int64 * self.n_levels)()
        self._check(self.lib.pff_sizes(self.h, None, None, C.cast(lvl, C.c_void_p)))
        self.level_nodes = list(lvl)

    def workspace_bytes(self) -> int:
        b = C.c_size_t()
        self._check(self.lib.pff_workspace_bytes(self.h, C.byref(b)))
        return b.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.pff_destroy(self.h)
            self.h = None
        self._ws = None      # the bound workspace outlives the context

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc < 0:
            msg = self.lib.pff_last_error(self.h)
            raise RuntimeError(f"pff error {rc}: {msg.decode() if msg else ''}")
        return rc

    # ---- mesh export -------------------------------------------------------
    def coords(self, level: int = -1) -> np.ndarray:
        nn = self.n if level < 0 else self.level_nodes[level]
        xy = np.zeros(2 * nn, dtype=np.int32)
        self._check(self.lib.pff_node_coords(self.h, level, xy.ctypes.data_as(C.c_void_p)))
        return xy.reshape(2, nn)

    def flags(self, level: int = -1) -> np.ndarray:
        nn = self.n if level < 0 else self.level_nodes[level]
        f = np.zeros(nn, dtype=np.uint8)
        self._check(self.lib.pff_node_flags(self.h, level, f.ctypes.data_as(C.c_void_p)))
        return f

    def tile_stats(self, level: int = -1):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.lib.pff_tile_stats(self.h, level, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def set_params(self, params: SolverParams):
        self._check(self.lib.pff_set_params(self.h, C.byref(params.to_c())))
        self.params = params
        self._sizes()

    # ---- state and operators ---------------------------------------------------
    def set_state(self, U, phi_old, phi_tilde, active=None, setup_mg: bool = True):
        self._check(self.lib.pff_set_state(self.h, _ptr(U), _ptr(phi_old), _ptr(phi_tilde),
                                           _ptr(active), int(setup_mg), _stream()))

    def extrapolate_phi(self, phi_prev, phi_prev2, theta: float = 1.0, out=None):
        import torch
        out = torch.empty_like(phi_prev) if out is None else out
        self._check(self.lib.pff_extrapolate_phi(self.h, _ptr(phi_prev), _ptr(phi_prev2), float(theta), _ptr(out),
                                                 _stream()))
        return out

    def extrapolate_phi_load(self, phi_prev, phi_prev2, t_prev2: float, t_prev: float, t_next: float, out=None):
        import torch
        out = torch.empty_like(phi_prev) if out is None else out
        self._check(self.lib.pff_extrapolate_phi_load(self.h, _ptr(phi_prev), _ptr(phi_prev2), float(t_prev2),
                                                      float(t_prev), float(t_next), _ptr(out), _stream()))
        return out

    def active(self):
        import torch
        a = torch.empty(self.n, dtype=torch.uint8, device="cuda")
        self._check(self.lib.pff_get_active(self.h, _ptr(a), _stream()))
        return a

    def vmult(self, src, out=None):
        import torch
        out = torch.empty_like(src) if out is None else out
        self._check(self.lib.pff_vmult(self.h, _ptr(out), _ptr(src), _stream()))
        return out

    def vmult_noalloc(self, src, out):
        """pff_vmult_noalloc: dst = J~ src with the partial sums in the
        library's static device array (out must be given: nothing is
        allocated)."""
        self._check(self.lib.pff_vmult_noalloc(self.h, _ptr(out), _ptr(src), _stream()))
        return out

    def vmult_T(self, src, batch: int = 1, out=None):
        import torch
        out = torch.empty_like(src) if out is None else out
        self._check(self.lib.pff_vmult_T(self.h, _ptr(out), _ptr(src), batch, _stream()))
        return out

    def inverse_diagonal(self, level: int = -1, fp32: bool = False):
        import torch
        nn = self.n if level < 0 else self.level_nodes[level]
        dt = torch.float32 if (fp32 and level >= 0) else torch.float64
        out = torch.empty(3 * nn, dtype=dt, device="cuda")
        self._check(self.lib.pff_inverse_diagonal(self.h, level, _ptr(out), int(fp32), _stream()))
        return out

    def vcycle(self, src, fp32: bool = False, out=None):
        import torch
        out = torch.empty_like(src) if out is None else out
        self._check(self.lib.pff_vcycle(self.h, _ptr(out), _ptr(src), int(fp32), _stream()))
        return out

    def get_eigen(self):
        lm = np.zeros(2 * self.n_levels)
        l0 = np.zeros(2)
        self._check(self.lib.pff_get_eigen(self.h, lm.ctypes.data_as(C.c_void_p),
                                           l0.ctypes.data_as(C.c_void_p)))
        return lm.reshape(self.n_levels, 2), l0

    def set_eigen(self, lam_max=None, lam_min0=None):
        if lam_max is None:
            self._check(self.lib.pff_set_eigen(self.h, None, None))
            return
        lm = np.ascontiguousarray(np.asarray(lam_max, dtype=np.float64).reshape(-1))
        l0 = np.ascontiguousarray(np.asarray(lam_min0, dtype=np.float64).reshape(-1))
        self._check(self.lib.pff_set_eigen(self.h, lm.ctypes.data_as(C.c_void_p),
                                           l0.ctypes.data_as(C.c_void_p)))

    def gmres(self, b, transpose: bool = False, tol: float = 0.0, out=None):
        import torch
        out = torch.empty_like(b) if out is None else out
        info = _lib.GmresInfo()
        rc = self._check(self.lib.pff_gmres_solve(self.h, _ptr(out), _ptr(b), int(transpose), tol,
                                                  C.byref(info), _stream()))
        return out, {k: getattr(info, k) for k, _ in info._fields_}, rc

    def newton_step(self, U, phi_old, phi_tilde, active=None):
        info = _lib.NewtonInfo()
        rc = self._check(self.lib.pff_newton_step(self.h, _ptr(U), _ptr(phi_old), _ptr(phi_tilde),
                                                  _ptr(active), C.byref(info), _stream()))
        return {k: getattr(info, k) for k, _ in info._fields_}, rc

    def residual(self, U, masked: bool = False, out=None):
        import torch
        out = torch.empty_like(U) if out is None else out
        self._check(self.lib.pff_residual(self.h, _ptr(out), _ptr(U), int(masked), _stream()))
        return out

    def tcv(self, U, grad: bool = False):
        import torch
        v = C.c_double()
        g = torch.empty_like(U) if grad else None
        self._check(self.lib.pff_tcv(self.h, _ptr(U), C.byref(v), _ptr(g), _stream()))
        return (v.value, g) if grad else v.value

    def cod(self, U, xs):
        """Crack opening displacement COD(x) (Sec. 4) at the positions xs."""
        x = np.ascontiguousarray(np.asarray(xs, dtype=np.float64))
        out = np.zeros(x.size)
        self._check(self.lib.pff_cod(self.h, _ptr(U), x.ctypes.data_as(C.c_void_p), int(x.size),
                                     out.ctypes.data_as(C.c_void_p), _stream()))
        return out

    def param_grad(self, z):
        out = np.zeros(3)
        self._check(self.lib.pff_param_grad(self.h, _ptr(z), out.ctypes.data_as(C.c_void_p), _stream()))
        return out

    def adjoint_tcv(self, U, tol: float = 0.0):
        """pff_adjoint_tcv at the loaded state: (TCV, dTCV/d(Gc, E, p) as a
        numpy array, adjoint solution z, GMRES info, return code)."""
        import torch
        v = C.c_double()
        grad = np.zeros(3)
        z = torch.empty_like(U)
        info = _lib.GmresInfo()
        rc = self._check(self.lib.pff_adjoint_tcv(self.h, _ptr(U), C.byref(v), grad.ctypes.data_as(C.c_void_p),
                                                  _ptr(z), float(tol), C.byref(info), _stream()))
        return v.value, grad, z, {k: getattr(info, k) for k, _ in info._fields_}, rc

    def distribute(self, v, ncomp: int):
        self._check(self.lib.pff_distribute(self.h, _ptr(v), ncomp, _stream()))
        return v

    def mask_constrained(self, v):
        self._check(self.lib.pff_mask_constrained(self.h, _ptr(v), _stream()))
        return v

    def dot(self, a, b):
        v = C.c_double()
        self._check(self.lib.pff_dot(self.h, _ptr(a), _ptr(b), a.numel(), C.byref(v), _stream()))
        return v.value
