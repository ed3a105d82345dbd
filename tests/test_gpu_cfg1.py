"""The plain FP64 Q1 workload of the benchmark's first configuration, and
its Q2 twin: 128 x 128 base cells plus 2 local levels in the band |x| < 2,
|y| < 0.5 (57 k / 229 k unknowns), state u ~ N(0, 1e-4), phi ~ U[0.5, 1] off
the crack, phi_old = phi~ = phi, active set from the rule of Alg. 2 at that
state (and a Bernoulli(0.1) mask as the second case of the vmult). One vmult,
one V-cycle with Chebyshev degree 3 and one Newton / PDAS step with GMRES,
each against the FP64 oracle on the same seeded inputs."""
import numpy as np
import pytest

import inputs
from oracle.mg import Hierarchy, MGParams, VCycle
from oracle.newton import NewtonParams, newton_step
from tests.gpu_common import Case, rel_err

pytestmark = pytest.mark.gpu

CFG1 = dict(n_base=128, n_local=2, coarse=16, band=(2.0, 0.5))
_cache = {}


def cfg1_case(p, mask):
    key = (p, mask)
    if key not in _cache:
        print(f"[case] cfg1 p={p} mask={mask}", flush=True)
        c = Case(CFG1["n_base"], CFG1["n_local"], p, coarse=CFG1["coarse"], band=CFG1["band"], mask=mask,
                 u_std=1e-4)
        c.load_state(setup_mg=True)
        _cache[key] = c
    return _cache[key]


def hierarchy(c, p):
    if ("hier", p) not in _cache:
        _cache[("hier", p)] = Hierarchy(c.om)
    return _cache[("hier", p)]


@pytest.mark.parametrize("mask", ("rule", "bernoulli"))
@pytest.mark.parametrize("p", (1, 2))
def test_cfg1_vmult(p, mask):
    c = cfg1_case(p, mask)
    J = c.lp.masked_operator(c.U_o, c.phit_o, c.active_o)
    src = inputs.random_vector(c.X, c.Y, 1)
    got = c.g.vmult(c.dev(src)).cpu().numpy()
    ref = c.to_g(J @ c.to_o(src))
    for b in range(3):
        sl = slice(b * c.n, (b + 1) * c.n)
        assert rel_err(got[sl], ref[sl]) <= 1e-12, b
    # the active set of the rule at this state: the oracle's (Alg. 2)
    if mask == "rule":
        assert np.array_equal(c.g.active().cpu().numpy().astype(bool), c.active_o[c.g2o])


@pytest.mark.parametrize("p", (1, 2))
def test_cfg1_vcycle(p):
    """Chebyshev degree 3, coarse Chebyshev 30; the eigenvalue estimates of
    the library are passed to the oracle (they are checked separately)."""
    c = cfg1_case(p, "rule")
    lam_max, lam_min0 = c.g.get_eigen()
    vc = VCycle(hierarchy(c, p), c.prm, MGParams(cheb_degree=3), c.U_o, c.phit_o, c.active_o,
                eigen=([lam_max[l] for l in range(c.g.n_levels)], lam_min0))
    src = inputs.random_vector(c.X, c.Y, 3)
    ref = c.to_g(vc.apply(c.to_o(src)))
    got = c.g.vcycle(c.dev(src)).cpu().numpy()
    assert rel_err(got, ref) <= 1e-12
    got32 = c.g.vcycle(c.dev(src), fp32=True).cpu().numpy()
    assert rel_err(got32, ref) <= 1e-5


@pytest.mark.parametrize("p", (1, 2))
def test_cfg1_newton_step(p):
    """One Alg. 2 iteration from the seeded state: identical active set,
    GMRES iterations within one, update within 1e-6 of the oracle's (same
    eigenvalue estimates), same number of line-search trials."""
    import torch
    c = cfg1_case(p, "rule")
    U = c.dev(c.U_raw)
    ph = c.dev(c.phi_old_raw)
    act = torch.zeros(c.n, dtype=torch.uint8, device="cuda")
    info, rc = c.g.newton_step(U, ph, ph, act)
    assert rc == 0
    lam_max, lam_min0 = c.g.get_eigen()
    Un, act_o, oinfo = newton_step(c.lp, hierarchy(c, p), MGParams(), NewtonParams(), c.U_o, c.phio_o, c.phio_o,
                                   np.zeros(c.n, bool),
                                   eigen=([lam_max[l] for l in range(c.g.n_levels)], lam_min0))
    assert np.array_equal(act.cpu().numpy().astype(bool), act_o[c.g2o])
    assert abs(info["gmres_iterations"] - oinfo.gmres_iterations) <= 1, (info["gmres_iterations"],
                                                                         oinfo.gmres_iterations)
    assert info["ls_trials"] == oinfo.ls_trials
    assert abs(info["residual_before"] - oinfo.residual_before) <= 1e-12 * oinfo.residual_before
    ref = c.to_g(Un)
    assert np.linalg.norm(U.cpu().numpy() - ref) <= 1e-6 * np.linalg.norm(ref)
