"""One iteration of the combined Newton / primal-dual active set method
(Alg. 2) and the adjoint crack-volume gradient (oracle). Test infrastructure
only.

Newton iteration (Sec. 3.1, Alg. 2):
 1. R = -F(U) condensed to the unconstrained unknowns.
 2. Active set (eq. AcInS with the constant c of Sec. 2):
    lambda_i = R_i / B_ii with B the lumped phase-field mass,
    c_i = 2 |lambda_i / (phi_i - phi_old_i)| (c_i * 0 taken as 0),
    active <=> lambda_i + c_i (phi_i - phi_old_i) > tau (tau = 1e-12 max |lambda|,
    rounding-level ties count as zero); hanging unknowns never.
 3. Inhomogeneous constraint dphi_i = phi_old_i - phi_i on the active set.
    F is affine in phi at fixed u and dF/dphi does not depend on phi, so
    R~(U_c) with U_c = U + dU_c equals R~(U) - J dU_c exactly.
 4. GMRES on J~ dU_f = R~(U_c) with the block V-cycle as left preconditioner,
    tolerance max(1e-12, 1e-8 |R~|) (Table 1).
 5. dU = dU_c + dU_f, hanging entries distributed from their masters.
 6. Line search: trial U + omega^(l-1) dU, l = 1..l_max; accept the first
    with |R~(trial)| < |R~(U)|, else the last trial.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import LeafProblem
from .krylov import gmres
from .mg import Hierarchy, MGParams, VCycle


@dataclass
class NewtonParams:
    gmres_restart: int = 30
    gmres_maxit: int = 300
    gmres_rtol: float = 1e-8
    gmres_atol: float = 1e-12
    ls_omega: float = 0.5
    ls_max: int = 10
    pdas_c: float = 0.0           # 0: c_i = 2 |lambda_i / (phi_i - phi_old_i)|; > 0: that constant


@dataclass
class NewtonInfo:
    residual_before: float = 0.0
    residual_after: float = 0.0
    rhs_norm: float = 0.0
    gmres_iterations: int = 0
    gmres_converged: bool = False
    ls_trials: int = 0
    n_active: int = 0
    active_changed: int = 0


def active_set(lp: LeafProblem, R, phi, phi_old, c_fixed=0.0):
    """Sec. 2 / Alg. 2 active-set rule, per phase-field unknown: active where
    lambda + c (phi - phi_old) > 0. c_fixed = 0 takes the paper's choice
    c_i = 2 |lambda_i / (phi_i - phi_old_i)|; c_fixed > 0 is one constant for
    every unknown (Sec. 2 leaves c free)."""
    n = lp.n
    B = lp.lumped_phi_mass()
    hang = lp.mesh.hanging
    lam = np.where(hang, 0.0, R[2 * n:] / np.where(hang, 1.0, B))
    diff = phi - phi_old
    if c_fixed > 0.0:
        c = np.full(n, float(c_fixed))
    else:
        nz = diff != 0.0
        c = np.where(nz, 2.0 * np.abs(lam / np.where(nz, diff, 1.0)), 0.0)
    val = lam + c * diff
    # exact ties (lambda = 0 where the state makes the phase-field residual
    # vanish) arrive as rounding noise; values below 1e-12 max|lambda| count
    # as zero, so ties stay inactive as the strict inequality intends
    tau = 1e-12 * np.abs(lam[~hang]).max() if np.any(~hang) else 0.0
    return (val > tau) & ~hang


def extrapolate_phase_field(phi_prev, phi_prev2, theta=1.0):
    """Sec. 2: the linearisation field phi~ of a load step may be extrapolated
    from earlier steps. Linear extrapolation in the load parameter t,
    theta = (t_n - t_{n-1}) / (t_{n-1} - t_{n-2}), kept in the phase field's
    range [0, 1]."""
    return np.clip(phi_prev + theta * (phi_prev - phi_prev2), 0.0, 1.0)


def masked_residual(lp: LeafProblem, U, phit, active):
    return lp.residual(U, phit) * lp.free_mask(active)


def newton_step(lp: LeafProblem, hier: Hierarchy, mgp: MGParams, nwp: NewtonParams,
                U, phi_old, phit, active_prev=None, eigen=None, linear_solver="gmres"):
    n = lp.n
    info = NewtonInfo()
    R = lp.residual(U, phit)
    active = active_set(lp, R, U[2 * n:], phi_old, nwp.pdas_c)
    info.n_active = int(active.sum())
    if active_prev is not None:
        info.active_changed = int(np.sum(active != active_prev))
    free = lp.free_mask(active)
    Uc = U.copy()
    Uc[2 * n:][active] = phi_old[active]
    b = lp.residual(Uc, phit) * free
    info.rhs_norm = float(np.linalg.norm(b))
    base = float(np.linalg.norm(R * free))
    info.residual_before = base
    J = lp.masked_operator(U, phit, active)
    if linear_solver == "gmres":
        # hier: the local-smoothing hierarchy, or a GlobalHierarchy for the
        # global-coarsening cycle (same smoother and coarse solve)
        from .gc import GCVCycle, GlobalHierarchy
        cycle = GCVCycle if isinstance(hier, GlobalHierarchy) else VCycle
        vc = cycle(hier, lp.prm, mgp, U, phit, active, eigen=eigen)
        tol = max(nwp.gmres_atol, nwp.gmres_rtol * info.rhs_norm)
        dUf, ginfo = gmres(lambda v: J @ v, vc.apply, b, tol,
                           restart=nwp.gmres_restart, maxit=nwp.gmres_maxit)
        info.gmres_iterations = ginfo.iterations
        info.gmres_converged = ginfo.converged
    else:
        dUf = spla.spsolve(J.tocsc(), b)
        info.gmres_converged = True
    dU = lp.distribute((Uc - U) + dUf)
    trial = U
    for l in range(1, nwp.ls_max + 1):
        trial = U + nwp.ls_omega ** (l - 1) * dU
        rn = float(np.linalg.norm(masked_residual(lp, trial, phit, active)))
        info.ls_trials = l
        info.residual_after = rn
        if rn < base:
            break
    return trial, active, info


def solve_frozen(lp: LeafProblem, U0, phi_old, phit, active, tol=1e-14, maxit=20):
    """Newton with a fixed active set and exact linear solves (for adjoint
    checks): returns U with R~(U) ~ 0 and phi = phi_old on the active set."""
    n = lp.n
    U = U0.copy()
    U[2 * n:][active] = phi_old[active]
    U = lp.distribute(U)
    for _ in range(maxit):
        b = masked_residual(lp, U, phit, active)
        if np.linalg.norm(b) <= tol:
            break
        J = lp.masked_operator(U, phit, active)
        U = lp.distribute(U + spla.spsolve(J.tocsc(), b))
    return U


def adjoint_gradient(lp: LeafProblem, U, phit, active):
    """dTCV/d(Gc, E, p) = -z^T dF~/dtheta with J~^T z = dTCV/dU on free rows
    (active set, kappa and l frozen)."""
    free = lp.free_mask(active)
    J = lp.masked_operator(U, phit, active)
    gTCV = lp.tcv_gradient(U) * free
    z = spla.spsolve(J.T.tocsc(), gTCV)
    dF = lp.param_derivatives(U, phit)
    return {k: float(-(z * free) @ v) for k, v in dF.items()}, z
