"""Host logic of the load-step and load-path drivers (no GPU): a stand-in
solver records the calls the drivers make, so the sequence of pressures,
phi_old, phi~ and extrapolation factors can be checked against the rules of
Sec. 2 (phi~ = the previous step's phase field, or from the third increment
the linear extrapolation in the load parameter from the last two steps)."""
from dataclasses import dataclass

import torch

from paper_2404_03265_amd.autograd import solve_load_path, solve_load_step


@dataclass
class _Params:
    pressure: float = 0.0


class _Solver:
    """Newton steps that move the phase field to -pressure (one step each
    converges); extrapolation returns its inputs' linear continuation."""

    def __init__(self, n):
        self.n = n
        self.params = _Params()
        self.calls = []

    def set_params(self, p):
        self.params = p

    def extrapolate_phi_load(self, a, b, t_prev2, t_prev, t_next):
        self.calls.append(("extrapolate", float(a[0]), float(b[0]), (t_prev2, t_prev, t_next)))
        theta = (t_next - t_prev) / (t_prev - t_prev2)
        return a + theta * (a - b)

    def newton_step(self, U, phi_old, phi_tilde, active):
        self.calls.append(("newton", self.params.pressure, float(phi_old[0]), float(phi_tilde[0])))
        U[2 * self.n:] = -self.params.pressure
        return {"residual_before": 0.0, "gmres_iterations": 1}, 0


def test_load_path_phase_fields_and_extrapolation():
    n = 4
    g = _Solver(n)
    U = torch.zeros(3 * n, dtype=torch.float64)
    phi0 = torch.full((n,), 1.0, dtype=torch.float64)
    pressures = [1.0, 2.0, 4.0, 5.0]
    active, out = solve_load_path(g, U, phi0, pressures, extrapolate=True)
    newton = [c for c in g.calls if c[0] == "newton"]
    extra = [c for c in g.calls if c[0] == "extrapolate"]
    # one Newton step per increment (converged at once), pressures in order
    assert [c[1] for c in newton] == pressures
    # phi_old: phi0, then the previous increment's phase field
    assert [c[2] for c in newton] == [1.0, -1.0, -2.0, -4.0]
    # phi~: phi_old for the first two increments, then extrapolated from the
    # last two solved steps with the load parameters (p_{k-2}, p_{k-1}, p_k)
    # (the library forms theta = (p_k - p_{k-1}) / (p_{k-1} - p_{k-2}))
    assert [c[3] for c in newton[:2]] == [1.0, -1.0]
    assert extra == [("extrapolate", -2.0, -1.0, (1.0, 2.0, 4.0)), ("extrapolate", -4.0, -2.0, (2.0, 4.0, 5.0))]
    assert [c[3] for c in newton[2:]] == [-4.0, -5.0]
    assert [float(o[2][0]) for o in out] == [1.0, -1.0, -2.0, -4.0]
    assert float(U[2 * n]) == -5.0


def test_load_path_without_extrapolation_and_step_stop():
    n = 2
    g = _Solver(n)
    U = torch.zeros(3 * n, dtype=torch.float64)
    phi0 = torch.zeros(n, dtype=torch.float64)
    solve_load_path(g, U, phi0, [1.0, 2.0, 3.0], extrapolate=False)
    assert not [c for c in g.calls if c[0] == "extrapolate"]
    newton = [c for c in g.calls if c[0] == "newton"]
    assert [c[3] for c in newton] == [c[2] for c in newton]       # phi~ = phi_old
    # a load step stops when the active set repeats and the residual is small
    g2 = _Solver(n)
    act, infos = solve_load_step(g2, torch.zeros(3 * n, dtype=torch.float64), phi0, phi0, max_steps=7)
    assert len(infos) == 1 and act.dtype == torch.uint8


class _StuckSolver(_Solver):
    """Newton steps that never meet the tolerance and report that GMRES hit
    its iteration limit (return code 1)."""

    def newton_step(self, U, phi_old, phi_tilde, active):
        return {"residual_before": 1.0, "gmres_iterations": 300}, 1


def test_load_step_surfaces_return_codes():
    import pytest
    from paper_2404_03265_amd.autograd import LoadStepNotConverged
    n = 2
    phi0 = torch.zeros(n, dtype=torch.float64)
    act, infos = solve_load_step(_StuckSolver(n), torch.zeros(3 * n, dtype=torch.float64), phi0, phi0, max_steps=3)
    assert len(infos) == 3 and all(i["rc"] == 1 for i in infos)
    assert infos[-1]["converged"] is False
    with pytest.raises(LoadStepNotConverged, match="warning codes \\[1\\]"):
        solve_load_step(_StuckSolver(n), torch.zeros(3 * n, dtype=torch.float64), phi0, phi0, max_steps=3,
                        strict=True)
    act, infos = solve_load_step(_Solver(n), torch.zeros(3 * n, dtype=torch.float64), phi0, phi0, strict=True)
    assert infos[-1]["converged"] is True and infos[-1]["rc"] == 0
