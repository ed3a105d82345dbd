"""GPU parity of the block-triangular preconditioner (prec_kind = 1: forward
substitution with the coupling block G_phi,u between the two block V-cycles;
backward substitution for transposed systems) against the oracle's
substitution around its own V-cycle, and GMRES with it against direct solves
of J~ and J~^T."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import inputs
from oracle.mg import Hierarchy, MGParams, VCycle, block_triangular_apply
from tests.gpu_common import Case, rel_err

pytestmark = pytest.mark.gpu

MESHES = {
    "tiny": dict(n_base=16, n_local=2, coarse=4, band=(3.0, 1.0)),
    "small": dict(n_base=32, n_local=2, coarse=16, band=(2.0, 0.5)),
}
_cases = {}


def tri_case(name, p):
    key = (name, p)
    if key not in _cases:
        from paper_2404_03265_amd import SolverParams
        m = MESHES[name]
        print(f"[blocktri] {key}", flush=True)
        c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], u_std=1e-2,
                 solver_params=SolverParams(prec_kind=1), phit="shifted")
        c.load_state(setup_mg=True)
        lam_max, lam_min0 = c.g.get_eigen()
        c.vc = VCycle(Hierarchy(c.om), c.prm, MGParams(), c.U_o, c.phit_o, c.active_o,
                      eigen=([lam_max[l] for l in range(c.g.n_levels)], lam_min0))
        c.J = c.lp.masked_operator(c.U_o, c.phit_o, c.active_o)
        _cases[key] = c
    return _cases[key]


CASES = [(n, p) for n in MESHES for p in (1, 2)]


@pytest.mark.parametrize("name,p", CASES)
def test_block_triangular_preconditioner_matches_oracle(name, p):
    c = tri_case(name, p)
    src = inputs.random_vector(c.X, c.Y, 13)
    got = c.g.vcycle(c.dev(src)).cpu().numpy()
    ref = c.to_g(block_triangular_apply(c.vc.apply, c.J, c.to_o(src), c.n))
    assert rel_err(got, ref) <= 1e-12
    # the coupling matters: the block-diagonal cycle differs
    diag = c.to_g(c.vc.apply(c.to_o(src)))
    assert rel_err(got, diag) > 1e-8


@pytest.mark.parametrize("name,p", CASES)
def test_gmres_with_block_triangular_matches_direct_solve(name, p):
    c = tri_case(name, p)
    b = inputs.random_vector(c.X, c.Y, 14) * c.to_g(c.lp.free_mask(c.active_o)).astype(float)
    x, info, rc = c.g.gmres(c.dev(b), tol=1e-13 * np.linalg.norm(b))
    assert info["converged"] == 1, info
    xd = c.to_g(spla.spsolve(c.J.tocsc(), c.to_o(b)))
    assert np.linalg.norm(x.cpu().numpy() - xd) <= 1e-9 * np.linalg.norm(xd)
    xt, info_t, _ = c.g.gmres(c.dev(b), transpose=True, tol=1e-13 * np.linalg.norm(b))
    xdt = c.to_g(spla.spsolve(c.J.T.tocsc(), c.to_o(b)))
    assert info_t["converged"] == 1
    assert np.linalg.norm(xt.cpu().numpy() - xdt) <= 1e-9 * np.linalg.norm(xdt)
