"""Differentiation forms on top of the C ABI (argument marshalling only):

* JacobianApply: torch.autograd.Function whose forward is pff_vmult and whose
  backward is pff_vmult_T, so dst = J~ src can sit inside a torch graph.
* adjoint_tcv_gradient: gradient of the crack volume TCV (Sec. 4) with respect
  to (Gc, E, p) at a converged state with frozen active set:
      J~^T z = dTCV/dU (constrained rows zero),  dTCV/dtheta = -z^T dF~/dtheta.
* TcvOfParams: torch.autograd.Function theta -> TCV(U(theta)) whose forward runs
  Newton / active set iterations (Alg. 2) and whose backward is the adjoint.
* solve_load_step / solve_load_path: one load step, and a sequence of pressure
  increments with the active set carried over (quasi-static loading, Sec. 4).
"""
from __future__ import annotations

import torch


class JacobianApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, src, solver):
        ctx.solver = solver
        return solver.vmult(src.contiguous())

    @staticmethod
    def backward(ctx, grad):
        return ctx.solver.vmult_T(grad.contiguous()), None


class LoadStepNotConverged(RuntimeError):
    """A load step ended without meeting the Newton tolerance (Alg. 2)."""


def solve_load_step(solver, U, phi_old, phi_tilde, active=None, tol=1e-7, max_steps=30, progress=None,
                    strict=False):
    """Alg. 2 loop until the active set repeats and |R~| <= tol. U is updated
    in place; returns (active, list of per-step info dicts). Each info dict
    carries the step's return code under "rc" (PFF_W_NOCONV = 1: GMRES hit
    its iteration limit; PFF_W_LINESEARCH = 2: no trial decreased |R~|), and
    the last one "converged" (tolerance met with an unchanged active set).
    With strict=True a load step that stops at max_steps unconverged raises
    LoadStepNotConverged. progress, if given, is called as
    progress(step_count, info) after every step."""
    if active is None:
        active = torch.zeros(solver.n, dtype=torch.uint8, device=U.device)
    infos = []
    converged = False
    for _ in range(max_steps):
        prev = active.clone()
        info, rc = solver.newton_step(U, phi_old, phi_tilde, active)
        info["rc"] = rc
        infos.append(info)
        if progress is not None:
            progress(len(infos), info)
        if torch.equal(prev, active) and info["residual_before"] <= tol:
            converged = True
            break
    if infos:
        infos[-1]["converged"] = converged
    if strict and not converged:
        codes = sorted({i["rc"] for i in infos if i["rc"]})
        raise LoadStepNotConverged(f"load step not converged in {len(infos)} Newton steps "
                                   f"(last |R~| {infos[-1]['residual_before']:.3e}, warning codes {codes})")
    return active, infos


def solve_load_path(solver, U, phi0, pressures, extrapolate=False, tol=1e-7, max_steps=400, progress=None,
                    done=None):
    """Quasi-static pressure increments: for each p_k in pressures, solve the
    load step (Alg. 2) from the previous solution with the previous active set,
    phi_old = the previous step's phase field (phi0 for the first) and the
    linearisation field phi~ (Sec. 2) either phi_old or, with
    extrapolate=True and two solved steps behind, the linear extrapolation in
    p from the last two (pff_extrapolate_phi, clipped to [0, 1]). U is updated
    in place. progress(k, j, info), if given, is called after Newton step j of
    increment k, done(k, phi~, infos) after increment k. Returns (active,
    per-increment list of (phi~ used, infos, phi_old used))."""
    from dataclasses import replace
    n = solver.n
    active = None
    phi_old = phi0.clone()
    phi_prev2 = None
    out = []
    for k, p in enumerate(pressures):
        solver.set_params(replace(solver.params, pressure=float(p)))
        if extrapolate and phi_prev2 is not None:
            phi_tilde = solver.extrapolate_phi_load(phi_old, phi_prev2, pressures[k - 2], pressures[k - 1], p)
        else:
            phi_tilde = phi_old
        cb = None if progress is None else (lambda j, info, k=k: progress(k, j, info))
        active, infos = solve_load_step(solver, U, phi_old, phi_tilde, active=active, tol=tol,
                                        max_steps=max_steps, progress=cb)
        out.append((phi_tilde, infos, phi_old))
        if done is not None:
            done(k, phi_tilde, infos)
        if k >= 1:
            phi_prev2 = phi_old
        phi_old = U[2 * n:].clone()
    return active, out


def adjoint_tcv_gradient(solver, U, phi_old, phi_tilde, active, tol=0.0):
    """(TCV, dTCV/d(Gc, E, p), adjoint solution z, GMRES info) at U with the
    active set frozen (pff_adjoint_tcv: transposed GMRES and the parameter
    derivatives, sign included, in the library)."""
    solver.set_state(U, phi_old, phi_tilde, active, setup_mg=True)
    tcv, grad, z, info, rc = solver.adjoint_tcv(U, tol=tol)
    info["rc"] = rc
    return tcv, torch.as_tensor(grad, dtype=torch.float64), z, info


class TcvOfParams(torch.autograd.Function):
    """theta = (Gc, E, p) -> TCV of the converged load step."""

    @staticmethod
    def forward(ctx, theta, solver, U0, phi_old, phi_tilde, newton_tol=1e-10):
        p = solver.params
        p.Gc, p.E, p.pressure = (float(x) for x in theta.detach().cpu())
        solver.set_params(p)
        U = U0.clone()
        active, _ = solve_load_step(solver, U, phi_old, phi_tilde, tol=newton_tol)
        tcv, grad, _, _ = adjoint_tcv_gradient(solver, U, phi_old, phi_tilde, active)
        ctx.save_for_backward(grad.to(theta.device))
        ctx.U = U
        return theta.new_tensor(tcv)

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None, None, None
