"""GPU parity of the global-coarsening V-cycle (every level a complete mesh
with its own hanging nodes, the finest being the leaf mesh) against the FP64
oracle cycle: level active sets, level inverse diagonals, eigenvalue
estimates, the cycle in FP64 and FP32, GMRES with it as preconditioner, one
Newton / active-set step, and switching between the two hierarchies on one
context."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import inputs
from oracle.gc import GCVCycle, GlobalHierarchy
from oracle.mg import Hierarchy, MGParams, VCycle, cg_eigs
from oracle.newton import NewtonParams, newton_step
from tests.gpu_common import Case, rel_err

pytestmark = pytest.mark.gpu

MESHES = {
    "tiny": dict(n_base=16, n_local=2, coarse=4, band=(3.0, 1.0)),
    "small": dict(n_base=32, n_local=2, coarse=16, band=(2.0, 0.5)),
    # no locally refined level: the finest level is the uniform base mesh
    "uniform": dict(n_base=16, n_local=0, coarse=4, band=(3.0, 1.0)),
    # three local passes: two own levels between the base mesh and the leaves
    "deep": dict(n_base=16, n_local=3, coarse=4, band=(3.0, 1.0)),
}
_cases = {}


def gc_case(name, p, cheb=3, coarse_its=30, coarse="cheb"):
    key = (name, p, cheb, coarse_its, coarse)
    if key not in _cases:
        from paper_2404_03265_amd import SolverParams
        m = MESHES[name]
        print(f"[gc case] {key}", flush=True)
        sp_ = SolverParams(cheb_degree=cheb, coarse_its=coarse_its, coarse_mode={"cheb": 0, "cg": 1}[coarse],
                           mg_kind=1)
        c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], u_std=1e-2,
                 solver_params=sp_, phit="shifted", mg_global=True)
        c.load_state(setup_mg=True)
        c.gh = GlobalHierarchy(c.om)
        mgp = MGParams(cheb_degree=cheb, coarse_its=coarse_its, coarse_mode=coarse)
        lam_max, lam_min0 = c.g.get_eigen()
        c.vc = GCVCycle(c.gh, c.prm, mgp, c.U_o, c.phit_o, c.active_o,
                        eigen=([lam_max[l] for l in range(c.g.n_levels)], lam_min0))
        c.mgp = mgp
        _cases[key] = c
    return _cases[key]


def gc_level_map(c, l):
    """library level-l node -> oracle level-l node (matched by lattice position)"""
    m = c.gh.meshes[l]
    X, Y = c.g.coords(l)
    pos = {(int(x), int(y)): i for i, (x, y) in enumerate(zip(m.NX, m.NY))}
    return np.array([pos[(int(x), int(y))] for x, y in zip(X, Y)])


def per_level(v, mp):
    nl = mp.size
    return np.concatenate([v[k * nl:(k + 1) * nl][mp] for k in range(3)])


CASES = [(n, p) for n in ("tiny", "small") for p in (1, 2)]


@pytest.mark.parametrize("name,p", CASES + [("uniform", 1), ("deep", 2)])
def test_gc_levels_active_sets_and_inverse_diagonals(name, p):
    """Level sizes are those of the truncated meshes; hanging flags, active
    sets (dilated through the interpolation, no home-level rule) and the
    inverse diagonals of the condensed level operators C^T A C match the
    oracle's; the FP32 copies to FP32 rounding."""
    c = gc_case(name, p)
    assert c.g.n_levels == len(c.gh.meshes)
    assert c.g.level_nodes == [m.n_nodes for m in c.gh.meshes]
    assert c.g.level_nodes[-1] == c.n
    for l in range(c.g.n_levels):
        mp = gc_level_map(c, l)
        f = c.g.flags(l)
        assert np.array_equal((f & 2) != 0, c.gh.meshes[l].hanging[mp]), l
        assert np.array_equal((f & 4) != 0, c.vc.ops[l].extra["active"][mp]), l
        got = c.g.inverse_diagonal(l).cpu().numpy()
        ref_g = per_level(c.vc.ops[l].Dinv, mp)
        assert rel_err(got, ref_g) <= 1e-12, l
        got32 = c.g.inverse_diagonal(l, fp32=True).cpu().numpy().astype(np.float64)
        assert rel_err(got32, ref_g) <= 1e-5, l


@pytest.mark.parametrize("name,p", CASES)
def test_gc_eigenvalue_estimates(name, p):
    """CG-Lanczos estimates of D^-1 A~ per level and block on the condensed
    level operators."""
    c = gc_case(name, p)
    lam_max, lam_min0 = c.g.get_eigen()
    for l, op in enumerate(c.vc.ops):
        nl = c.gh.meshes[l].n_nodes
        bu = np.zeros(3 * nl, bool)
        bu[:2 * nl] = True
        its2 = (c.mgp.coarse_eig_its,) * 2 if l == 0 else (c.mgp.eig_cg_its, c.mgp.eig_cg_its_phi)
        for b, blk in enumerate((bu, ~bu)):
            lo, hi = cg_eigs(op.A, op.Dinv, op.free & blk, its2[b])
            assert abs(lam_max[l, b] - hi) <= 1e-9 * hi, (l, b, lam_max[l, b], hi)
            if l == 0:
                assert abs(lam_min0[b] - lo) <= 1e-9 * hi


@pytest.mark.parametrize("name,p", CASES + [("uniform", 1), ("deep", 1), ("deep", 2)])
def test_gc_vcycle_fp64_matches_oracle(name, p):
    c = gc_case(name, p)
    src = inputs.random_vector(c.X, c.Y, 3)
    got = c.g.vcycle(c.dev(src)).cpu().numpy()
    ref = c.to_g(c.vc.apply(c.to_o(src)))
    assert rel_err(got, ref) <= 1e-12
    # constrained leaf rows pass through
    cons = ~c.to_g(c.lp.free_mask(c.active_o))
    assert np.array_equal(got[cons], src[cons])


@pytest.mark.parametrize("name,p", CASES)
def test_gc_vcycle_fp32_error_bound(name, p):
    c = gc_case(name, p)
    src = inputs.random_vector(c.X, c.Y, 4)
    got = c.g.vcycle(c.dev(src), fp32=True).cpu().numpy()
    ref = c.to_g(c.vc.apply(c.to_o(src)))
    err = rel_err(got, ref)
    print(f"fp32 gc vcycle rel err {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("p", (1, 2))
def test_gc_vcycle_coarse_cg_and_degree4(p):
    c = gc_case("tiny", p, cheb=4, coarse_its=20, coarse="cg")
    src = inputs.random_vector(c.X, c.Y, 8)
    ref = c.to_g(c.vc.apply(c.to_o(src)))
    got = c.g.vcycle(c.dev(src)).cpu().numpy()
    assert rel_err(got, ref) <= 1e-12
    got32 = c.g.vcycle(c.dev(src), fp32=True).cpu().numpy()
    assert rel_err(got32, ref) <= 1e-5


@pytest.mark.parametrize("name,p", CASES)
def test_gc_gmres_matches_direct_solve(name, p):
    c = gc_case(name, p)
    J = c.lp.masked_operator(c.U_o, c.phit_o, c.active_o)
    b = inputs.random_vector(c.X, c.Y, 6) * c.to_g(c.lp.free_mask(c.active_o)).astype(float)
    x, info, rc = c.g.gmres(c.dev(b), tol=1e-13 * np.linalg.norm(b))
    assert info["converged"] == 1, info
    xd = c.to_g(spla.spsolve(J.tocsc(), c.to_o(b)))
    assert np.linalg.norm(x.cpu().numpy() - xd) <= 1e-9 * np.linalg.norm(xd)
    xt, info_t, _ = c.g.gmres(c.dev(b), transpose=True, tol=1e-13 * np.linalg.norm(b))
    xdt = c.to_g(spla.spsolve(J.T.tocsc(), c.to_o(b)))
    assert info_t["converged"] == 1
    assert np.linalg.norm(xt.cpu().numpy() - xdt) <= 1e-9 * np.linalg.norm(xdt)


@pytest.mark.parametrize("p", (1, 2))
def test_gc_newton_step_matches_oracle(p):
    """One Alg. 2 iteration from the load-step start with the global-coarsening
    preconditioner: same active set, GMRES count within one, same update to
    the GMRES tolerance."""
    import torch
    from paper_2404_03265_amd import SolverParams
    m = MESHES["tiny"]
    c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask="rule",
             solver_params=SolverParams(mg_kind=1), mg_global=True)
    n = c.n
    ux, uy, phi = inputs.sneddon_state(c.X, c.Y, c.M, p, random=False)
    U0 = np.concatenate([ux, uy, phi])
    Ud = c.dev(U0)
    ph = c.dev(phi)
    act = torch.zeros(n, dtype=torch.uint8, device="cuda")
    info, rc = c.g.newton_step(Ud, ph, ph, act)
    lam_max, lam_min0 = c.g.get_eigen()
    Uo0 = c.lp.distribute(c.to_o(U0))
    pho = c.to_o(phi)
    Un, act_o, oinfo = newton_step(c.lp, GlobalHierarchy(c.om), MGParams(), NewtonParams(), Uo0, pho, pho,
                                   np.zeros(n, bool),
                                   eigen=([lam_max[l] for l in range(c.g.n_levels)], lam_min0))
    assert np.array_equal(act.cpu().numpy().astype(bool), act_o[c.g2o])
    assert abs(info["gmres_iterations"] - oinfo.gmres_iterations) <= 1
    assert info["ls_trials"] == oinfo.ls_trials
    Ug = Ud.cpu().numpy()
    ref = c.to_g(Un)
    assert np.linalg.norm(Ug - ref) <= 1e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("p", (1, 2))
def test_switch_between_hierarchies_on_one_context(p):
    """The uniform levels are shared by both hierarchies and hold per-kind
    active sets: after each switch (set_params + set_state) the cycle must be
    the oracle cycle of the selected kind."""
    from paper_2404_03265_amd import SolverParams
    c = gc_case("tiny", p)
    src = inputs.random_vector(c.X, c.Y, 11)
    sp_ls = SolverParams(**{**c.sp.__dict__, "mg_kind": 0})
    c.g.set_params(sp_ls)
    c.load_state(setup_mg=True)
    lam_max, lam_min0 = c.g.get_eigen()
    assert c.g.level_nodes[-1] < c.n   # the local-smoothing finest level is a partial level
    vls = VCycle(Hierarchy(c.om), c.prm, c.mgp, c.U_o, c.phit_o, c.active_o,
                 eigen=([lam_max[l] for l in range(c.g.n_levels)], lam_min0))
    got = c.g.vcycle(c.dev(src)).cpu().numpy()
    assert rel_err(got, c.to_g(vls.apply(c.to_o(src)))) <= 1e-12
    c.g.set_params(c.sp)
    c.load_state(setup_mg=True)
    lam_max, lam_min0 = c.g.get_eigen()
    c.vc.set_eigen(([lam_max[l] for l in range(c.g.n_levels)], lam_min0))
    got = c.g.vcycle(c.dev(src)).cpu().numpy()
    assert rel_err(got, c.to_g(c.vc.apply(c.to_o(src)))) <= 1e-12


def test_gc_needs_mg_global():
    """mg_kind = 1 without the global levels is refused at create and at
    set_params."""
    from paper_2404_03265_amd import PhaseFieldSolver, SolverParams
    with pytest.raises(RuntimeError, match="mg_global"):
        PhaseFieldSolver(16, 1, 1, coarse=4, params=SolverParams(mg_kind=1))
    g = PhaseFieldSolver(16, 1, 1, coarse=4)
    with pytest.raises(RuntimeError, match="mg_global"):
        g.set_params(SolverParams(mg_kind=1))
