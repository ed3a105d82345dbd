"""GPU parity of the multigrid preconditioner, GMRES and the Newton / active
set step against the FP64 oracle, plus the FP32 V-cycle error bound."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import inputs
from oracle.mg import Hierarchy, MGParams, VCycle, cg_eigs
from oracle.newton import NewtonParams, newton_step
from tests.gpu_common import Case, rel_err

pytestmark = pytest.mark.gpu

MESHES = {
    "tiny": dict(n_base=16, n_local=2, coarse=4, band=(3.0, 1.0)),
    "small": dict(n_base=32, n_local=2, coarse=16, band=(2.0, 0.5)),
}
_cases = {}


def mg_case(name, p, mask="bernoulli", cheb=3, coarse_its=30, coarse="cheb"):
    key = (name, p, mask, cheb, coarse_its, coarse)
    if key not in _cases:
        from paper_2404_03265_amd import SolverParams
        m = MESHES[name]
        print(f"[case] {key}", flush=True)
        sp_ = SolverParams(cheb_degree=cheb, coarse_its=coarse_its, coarse_mode={"cheb": 0, "cg": 1}[coarse])
        c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask=mask,
                 u_std=1e-2, solver_params=sp_, phit="shifted")
        c.load_state(setup_mg=True)
        c.hier = Hierarchy(c.om)
        mgp = MGParams(cheb_degree=cheb, coarse_its=coarse_its, coarse_mode=coarse)
        lam_max, lam_min0 = c.g.get_eigen()
        c.vc = VCycle(c.hier, c.prm, mgp, c.U_o, c.phit_o, c.active_o,
                      eigen=([lam_max[l] for l in range(c.g.n_levels)], lam_min0))
        c.mgp = mgp
        _cases[key] = c
    return _cases[key]


def level_map(c, l):
    """library level-l node -> oracle level-l node"""
    lv = c.hier.levels[l]
    X, Y = c.g.coords(l)
    pos = {(int(x), int(y)): i for i, (x, y) in enumerate(zip(lv.NX, lv.NY))}
    return np.array([pos[(int(x), int(y))] for x, y in zip(X, Y)])


CASES = [(n, p) for n in MESHES for p in (1, 2)]


@pytest.mark.parametrize("name,p", CASES)
def test_level_active_sets_and_inverse_diagonals(name, p):
    c = mg_case(name, p)
    for l in range(c.g.n_levels):
        mp = level_map(c, l)
        f = c.g.flags(l)
        assert np.array_equal((f & 4) != 0, c.vc.ops[l].extra["active"][mp])
        nl = c.hier.levels[l].n
        got = c.g.inverse_diagonal(l).cpu().numpy()
        ref = c.vc.ops[l].Dinv
        ref_g = np.concatenate([ref[k * nl:(k + 1) * nl][mp] for k in range(3)])
        assert rel_err(got, ref_g) <= 1e-12, l
        # the FP32 copy of the mixed form: the FP64 diagonal to FP32 rounding
        # (entries of the FP32 level operator, summed in FP32)
        got32 = c.g.inverse_diagonal(l, fp32=True).cpu().numpy().astype(np.float64)
        assert rel_err(got32, ref_g) <= 1e-5, l


@pytest.mark.parametrize("name,p", CASES)
def test_eigenvalue_estimates(name, p):
    """CG-Lanczos estimates of D^{-1} A per level and block (Sec. 3.2)."""
    c = mg_case(name, p)
    lam_max, lam_min0 = c.g.get_eigen()
    n = c.hier.levels
    for l, op in enumerate(c.vc.ops):
        nl = n[l].n
        bu = np.zeros(3 * nl, bool)
        bu[:2 * nl] = True
        its2 = (c.mgp.coarse_eig_its,) * 2 if l == 0 else (c.mgp.eig_cg_its, c.mgp.eig_cg_its_phi)
        for b, blk in enumerate((bu, ~bu)):
            lo, hi = cg_eigs(op.A, op.Dinv, op.free & blk, its2[b])
            assert abs(lam_max[l, b] - hi) <= 1e-9 * hi, (l, b, lam_max[l, b], hi)
            if l == 0:
                assert abs(lam_min0[b] - lo) <= 1e-9 * hi


@pytest.mark.parametrize("name,p", CASES)
def test_vcycle_fp64_matches_oracle(name, p):
    c = mg_case(name, p)
    src = inputs.random_vector(c.X, c.Y, 3)
    got = c.g.vcycle(c.dev(src)).cpu().numpy()
    ref = c.to_g(c.vc.apply(c.to_o(src)))
    assert rel_err(got, ref) <= 1e-12


@pytest.mark.parametrize("name,p", CASES)
def test_vcycle_fp32_error_bound(name, p):
    """Mixed precision: the whole V-cycle in FP32 stays within 1e-5 (relative,
    largest entry) of the FP64 oracle V-cycle."""
    c = mg_case(name, p)
    src = inputs.random_vector(c.X, c.Y, 4)
    got = c.g.vcycle(c.dev(src), fp32=True).cpu().numpy()
    ref = c.to_g(c.vc.apply(c.to_o(src)))
    err = rel_err(got, ref)
    print(f"fp32 vcycle rel err {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("name,p", CASES)
def test_vcycle_degree4_and_short_coarse(name, p):
    c = mg_case(name, p, cheb=4, coarse_its=8)
    src = inputs.random_vector(c.X, c.Y, 5)
    got = c.g.vcycle(c.dev(src)).cpu().numpy()
    ref = c.to_g(c.vc.apply(c.to_o(src)))
    assert rel_err(got, ref) <= 1e-12


@pytest.mark.parametrize("cheb", (1, 2))
@pytest.mark.parametrize("p", (1, 2))
def test_vcycle_low_chebyshev_degrees(p, cheb):
    """Chebyshev degree 1 (the first update alone, no operator application
    from x = 0) and 2 (the first two updates in one level pass and nothing
    after): the FP64 V-cycle against the oracle's at 1e-12."""
    c = mg_case("tiny", p, cheb=cheb)
    src = inputs.random_vector(c.X, c.Y, 9)
    got = c.g.vcycle(c.dev(src)).cpu().numpy()
    ref = c.to_g(c.vc.apply(c.to_o(src)))
    assert rel_err(got, ref) <= 1e-12


@pytest.mark.parametrize("name,p", CASES)
def test_vcycle_coarse_cg(name, p):
    """Coarse solve by fixed-step Jacobi-CG (Chebyshev degree 4 smoothing, the
    mixed-precision configuration): FP64 cycle to 1e-12, FP32 cycle to 1e-5,
    both against the oracle cycle with the same coarse CG."""
    c = mg_case(name, p, cheb=4, coarse_its=20, coarse="cg")
    src = inputs.random_vector(c.X, c.Y, 8)
    ref = c.to_g(c.vc.apply(c.to_o(src)))
    got = c.g.vcycle(c.dev(src)).cpu().numpy()
    assert rel_err(got, ref) <= 1e-12
    got32 = c.g.vcycle(c.dev(src), fp32=True).cpu().numpy()
    assert rel_err(got32, ref) <= 1e-5


@pytest.mark.parametrize("coarse", ["cheb", "cg"])
@pytest.mark.parametrize("p", [1, 2])
def test_vcycle_per_step_coarse_path(p, coarse):
    """More coarse steps than the one-kernel coarse solve holds (64): the
    level-0 solve runs step by step (tile kernel, fix-up, CG scalars) and
    must give the oracle cycle as well."""
    c = mg_case("tiny", p, coarse_its=70, coarse=coarse)
    src = inputs.random_vector(c.X, c.Y, 9)
    ref = c.to_g(c.vc.apply(c.to_o(src)))
    got = c.g.vcycle(c.dev(src)).cpu().numpy()
    assert rel_err(got, ref) <= 1e-12
    got32 = c.g.vcycle(c.dev(src), fp32=True).cpu().numpy()
    assert rel_err(got32, ref) <= 1e-5


@pytest.mark.parametrize("name,p", CASES)
def test_gmres_matches_direct_solve(name, p):
    c = mg_case(name, p)
    J = c.lp.masked_operator(c.U_o, c.phit_o, c.active_o)
    b = inputs.random_vector(c.X, c.Y, 6) * c.to_g(c.lp.free_mask(c.active_o)).astype(float)
    x, info, rc = c.g.gmres(c.dev(b), tol=1e-13 * np.linalg.norm(b))
    assert info["converged"] == 1, info
    xd = c.to_g(spla.spsolve(J.tocsc(), c.to_o(b)))
    assert np.linalg.norm(x.cpu().numpy() - xd) <= 1e-9 * np.linalg.norm(xd)
    # transposed system (adjoint solves)
    xt, info_t, _ = c.g.gmres(c.dev(b), transpose=True, tol=1e-13 * np.linalg.norm(b))
    xdt = c.to_g(spla.spsolve(J.T.tocsc(), c.to_o(b)))
    assert info_t["converged"] == 1
    assert np.linalg.norm(xt.cpu().numpy() - xdt) <= 1e-9 * np.linalg.norm(xdt)


@pytest.mark.parametrize("name,p", CASES)
def test_newton_step_matches_oracle(name, p):
    """One Alg. 2 iteration from the load-step start (u = 0, phi = 1 off the
    crack): same active set, same GMRES iteration count within one, and the
    same update to the GMRES tolerance."""
    import torch
    m = MESHES[name]
    c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask="rule")
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
    hier = Hierarchy(c.om)
    Un, act_o, oinfo = newton_step(c.lp, hier, MGParams(), NewtonParams(), Uo0, pho, pho,
                                   np.zeros(n, bool),
                                   eigen=([lam_max[l] for l in range(c.g.n_levels)], lam_min0))
    assert np.array_equal(act.cpu().numpy().astype(bool), act_o[c.g2o])
    assert abs(info["gmres_iterations"] - oinfo.gmres_iterations) <= 1
    assert info["ls_trials"] == oinfo.ls_trials
    assert abs(info["residual_before"] - oinfo.residual_before) <= 1e-12 * oinfo.residual_before
    Ug = Ud.cpu().numpy()
    ref = c.to_g(Un)
    assert np.linalg.norm(Ug - ref) <= 1e-6 * np.linalg.norm(ref)
    assert abs(info["residual_after"] - oinfo.residual_after) <= 1e-6 * oinfo.residual_before + 1e-12


@pytest.mark.parametrize("p", (1, 2))
def test_load_path_with_extrapolated_phi_tilde(p):
    """Three pressure increments with the active set carried over and phi~
    extrapolated from the last two steps in the third (Sec. 2, Sec. 4), against
    the oracle's Newton / PDAS loop with direct solves: the phi~ used, the
    converged states per block and the crack volume agree to the Newton
    tolerance; the active sets agree up to nodes whose decision is a tie."""
    import dataclasses
    from oracle.newton import extrapolate_phase_field
    from paper_2404_03265_amd.autograd import solve_load_path
    m = MESHES["tiny"]
    print(f"[case] load path tiny p={p}", flush=True)
    c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask="rule")
    n = c.n
    lp = c.lp
    ux, uy, phi = inputs.sneddon_state(c.X, c.Y, c.M, p, random=False)
    Uo = lp.distribute(c.to_o(np.concatenate([ux, uy, phi])))
    U = c.dev(c.to_g(Uo))
    pres = [1e-3, 2e-3, 3.5e-3]
    act, out = solve_load_path(c.g, U, U[2 * n:].clone(), pres, extrapolate=True, tol=1e-10)
    phi_old, prev2 = Uo[2 * n:].copy(), None
    act_o = np.zeros(n, bool)
    for k, pk in enumerate(pres):
        lp.prm = dataclasses.replace(lp.prm, pressure=pk)
        if prev2 is not None:
            theta = (pk - pres[k - 1]) / (pres[k - 1] - pres[k - 2])
            phit = lp.distribute(extrapolate_phase_field(phi_old, prev2, theta))
            assert np.abs(phit - phi_old).max() > 1e-9          # the extrapolation changes phi~
        else:
            phit = phi_old
        for _ in range(60):
            Un, an, info = newton_step(lp, None, None, NewtonParams(), Uo, phi_old, phit, act_o,
                                       linear_solver="direct")
            same = np.array_equal(an, act_o)
            Uo, act_o = Un, an
            if same and info.residual_before <= 1e-10:
                break
        phit_g = lp.distribute(c.to_o(out[k][0].cpu().numpy()))
        assert np.abs(phit_g - phit).max() <= 1e-6, k
        assert out[k][1][-1]["residual_before"] <= 1e-10
        phi_prev_o = phi_old
        if k >= 1:
            prev2 = phi_old
        phi_old = Uo[2 * n:].copy()
    Ug = c.to_o(U.cpu().numpy())
    for b in range(3):
        sl = slice(b * n, (b + 1) * n)
        assert rel_err(Ug[sl], Uo[sl]) <= 1e-6, b
    assert abs(c.g.tcv(U) - lp.tcv(Uo)) <= 1e-6 * abs(lp.tcv(Uo))
    # differing flags only where the state sits on the obstacle (a tie)
    diff = np.flatnonzero(act.cpu().numpy().astype(bool)[c.o2g] != act_o)
    assert np.abs(Uo[2 * n:][diff] - phi_prev_o[diff]).max(initial=0.0) <= 1e-8


@pytest.mark.parametrize("p", (1, 2))
def test_mixed_precision_load_step(p):
    """A load step (Alg. 2 to |R~| <= 1e-10) with the FP32 V-cycle inside the
    FP64 GMRES / Newton loop (Chebyshev 4, coarse CG) reaches the state the
    FP64 configuration reaches and the oracle's loop with direct solves: the
    preconditioner's precision changes the iteration counts, not the
    converged residual or the solution."""
    from paper_2404_03265_amd import SolverParams
    from paper_2404_03265_amd.autograd import solve_load_step
    m = MESHES["small"]
    print(f"[case] mixed-precision load step small p={p}", flush=True)
    states = {}
    for label, extra in (("fp64", {}), ("mixed", dict(vcycle_fp32=1, cheb_degree=4, coarse_mode=1))):
        c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask="rule",
                 solver_params=SolverParams(**extra), build_oracle=(label == "fp64"))
        ux, uy, phi = inputs.sneddon_state(c.X, c.Y, c.M, p, random=False)
        U = c.dev(np.concatenate([ux, uy, phi]))
        ph = c.dev(phi)
        act, infos = solve_load_step(c.g, U, ph, ph, tol=1e-10, max_steps=60)
        assert infos[-1]["residual_before"] <= 1e-10, label
        states[label] = (U.cpu().numpy(), act.cpu().numpy().astype(bool), infos)
        if label == "fp64":
            co = c
    n = co.n
    U64, a64, _ = states["fp64"]
    U32, a32, _ = states["mixed"]
    for b in range(3):
        sl = slice(b * n, (b + 1) * n)
        assert rel_err(U32[sl], U64[sl]) <= 1e-8, b
    # nodes whose flag differs sit on the obstacle (phi = phi_old) in both
    # states: active or not, the state is the same there (a tie)
    diff = np.flatnonzero(a32 != a64)
    assert np.abs(U64[2 * n:][diff] - phi[diff]).max(initial=0.0) <= 1e-8
    assert np.abs(U32[2 * n:][diff] - phi[diff]).max(initial=0.0) <= 1e-8
    # oracle: the same loop with direct solves
    lp = co.lp
    Uo = lp.distribute(co.to_o(np.concatenate([ux, uy, phi])))
    pho = Uo[2 * n:].copy()
    act_o = np.zeros(n, bool)
    for _ in range(60):
        Un, an, info = newton_step(lp, None, None, NewtonParams(), Uo, pho, pho, act_o, linear_solver="direct")
        same = np.array_equal(an, act_o)
        Uo, act_o = Un, an
        if same and info.residual_before <= 1e-10:
            break
    Ug = co.to_o(U32)
    for b in range(3):
        sl = slice(b * n, (b + 1) * n)
        assert rel_err(Ug[sl], Uo[sl]) <= 1e-8, b


def test_full_size_vmult_sampled_rows():
    """The benchmark workload (1024 x 1024 base cells + 3 local levels, Q2,
    20.5 M unknowns) in the benchmark's launch configuration: about 600
    sampled nodes (every class of node included) against the oracle row by
    row, for the vmult, its transpose and the residual R = -F(U)."""
    import time
    t0 = time.time()
    c = Case(1024, 3, 2, mask="bernoulli", u_std=1e-4, build_oracle=False, phit="shifted")
    c.load_state()
    src = inputs.random_vector(c.X, c.Y, 1)
    dst = c.g.vmult(c.dev(src)).cpu().numpy()
    dstT = c.g.vmult_T(c.dev(src)).cpu().numpy()
    res = c.g.residual(c.dev(c.U_raw)).cpu().numpy()
    print(f"[full] library side done {time.time() - t0:.1f}s", flush=True)
    c.build_oracle(1024, 3, 2, 16, (2.0, 0.5))
    print(f"[full] oracle mesh built {time.time() - t0:.1f}s", flush=True)
    rng = np.random.default_rng(7)
    n = c.n
    f = c.g.flags()
    pick = []
    for mask in ((f & 2) != 0, (f & 1) != 0, c.active, (f & 7) == 0):
        idx = np.flatnonzero(mask)
        pick.extend(rng.choice(idx, size=min(50, idx.size), replace=False).tolist())
    # masters of sampled hanging nodes, and random nodes
    for h in [k for k in pick if f[k] & 2][:50]:
        pick.extend(int(c.o2g[m]) for m, _ in c.om.hanging_constraints[int(c.g2o[h])])
    pick.extend(rng.choice(n, size=300, replace=False).tolist())
    pick = np.unique(np.array(pick))
    rows_g = np.concatenate([pick + k * n for k in range(3)])
    rows_o = np.concatenate([c.g2o[pick] + k * n for k in range(3)])
    ref = c.lp.masked_rows(rows_o, c.to_o(src), c.U_o, c.phit_o, c.active_o)
    refT = c.lp.masked_rows(rows_o, c.to_o(src), c.U_o, c.phit_o, c.active_o, transpose=True)
    refR = c.lp.residual_rows(rows_o, c.U_o, c.phit_o)
    print(f"[full] oracle rows done {time.time() - t0:.1f}s", flush=True)
    assert np.abs(dst[rows_g] - ref).max() <= 1e-12 * np.abs(dst).max()
    assert np.abs(dstT[rows_g] - refT).max() <= 1e-12 * np.abs(dstT).max()
    # the residual per block: the u rows carry the pressure term, the phase-
    # field rows the much larger Gc / l term
    for b in range(3):
        sel = slice(b * pick.size, (b + 1) * pick.size)
        scale = np.abs(res[b * n:(b + 1) * n]).max()
        assert np.abs(res[rows_g[sel]] - refR[sel]).max() <= 1e-12 * scale, b


def test_full_size_vcycle_properties():
    """The benchmark workload at full size (20.5 M unknowns), where the oracle
    cannot run the cycle: properties that hold at any size. The FP64 V-cycle
    (symmetric smoothing, Chebyshev coarse solve) is a symmetric operator,
    w.(P^-1 v) = v.(P^-1 w); the FP32 V-cycle stays within 1e-5 of it; the
    transposed Jacobian satisfies w.(J v) = (J^T w).v."""
    import time
    import torch
    t0 = time.time()
    c = Case(1024, 3, 2, mask="bernoulli", u_std=1e-4, build_oracle=False)
    c.load_state(setup_mg=True)
    print(f"[full] state and multigrid set up {time.time() - t0:.1f}s", flush=True)
    v = c.dev(inputs.random_vector(c.X, c.Y, 31))
    w = c.dev(inputs.random_vector(c.X, c.Y, 32))
    Pv = c.g.vcycle(v)
    Pw = c.g.vcycle(w)
    a, b = torch.dot(w, Pv).item(), torch.dot(v, Pw).item()
    scale = (torch.linalg.norm(w) * torch.linalg.norm(Pv)).item()
    assert abs(a - b) <= 1e-12 * scale, (a, b, scale)
    Pv32 = c.g.vcycle(v, fp32=True)
    assert rel_err(Pv32.cpu().numpy(), Pv.cpu().numpy()) <= 1e-5
    Jv = c.g.vmult(v)
    JTw = c.g.vmult_T(w)
    a, b = torch.dot(w, Jv).item(), torch.dot(JTw, v).item()
    scale = (torch.linalg.norm(w) * torch.linalg.norm(Jv)).item()
    assert abs(a - b) <= 1e-12 * scale, (a, b, scale)
    print(f"[full] done {time.time() - t0:.1f}s", flush=True)


@pytest.mark.parametrize("name,p", CASES)
def test_adjoint_crack_volume_gradient(name, p):
    """Adjoint gradient of TCV w.r.t. (Gc, E, p) at a converged load step with
    frozen active set: GPU (transposed GMRES + parameter derivatives) against
    the oracle's direct adjoint at the same state; the autograd wrapper returns
    the same gradient; z^T (J~ v) = (J~^T z)^T v."""
    import torch
    from oracle.newton import adjoint_gradient
    from paper_2404_03265_amd import SolverParams
    from paper_2404_03265_amd.autograd import adjoint_tcv_gradient, solve_load_step, JacobianApply
    m = MESHES[name]
    sp_ = SolverParams(gmres_rtol=1e-13, gmres_atol=1e-15)
    c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask="rule",
             solver_params=sp_)
    ux, uy, phi = inputs.sneddon_state(c.X, c.Y, c.M, p, random=False)
    U = c.dev(np.concatenate([ux, uy, phi]))
    ph = c.dev(phi)
    act, infos = solve_load_step(c.g, U, ph, ph, tol=1e-10)
    assert infos[-1]["residual_before"] <= 1e-10
    tcv, grad, z, info = adjoint_tcv_gradient(c.g, U, ph, ph, act, tol=0.0)
    assert info["converged"] == 1
    Uo = c.to_o(U.cpu().numpy())
    act_o = act.cpu().numpy().astype(bool)[c.o2g]
    ref, _ = adjoint_gradient(c.lp, Uo, c.to_o(phi), act_o)
    assert abs(tcv - c.lp.tcv(Uo)) <= 1e-12 * abs(tcv)
    for i, k in enumerate(("Gc", "E", "p")):
        assert abs(grad[i].item() - ref[k]) <= 1e-7 * max(abs(ref[k]), 1e-14 * abs(tcv)), (k, grad[i], ref[k])
    v = c.dev(inputs.random_vector(c.X, c.Y, 21))
    w = c.dev(inputs.random_vector(c.X, c.Y, 22))
    lhs = torch.dot(w, c.g.vmult(v)).item()
    rhs = torch.dot(c.g.vmult_T(w), v).item()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # autograd: backward of JacobianApply is the transpose
    vv = v.clone().requires_grad_(True)
    y = JacobianApply.apply(vv, c.g)
    y.backward(w)
    assert torch.allclose(vv.grad, c.g.vmult_T(w), rtol=0, atol=1e-13 * w.abs().max().item())


@pytest.mark.parametrize("p", (1, 2))
def test_bound_workspace_matches_library_allocation(p):
    """Work buffers carved from a caller-owned torch tensor (pff_bind_workspace)
    give bitwise the results of buffers the library allocates itself: vmult,
    its transpose, both V-cycles, GMRES and a Newton step; binding rules."""
    import ctypes as C
    import torch
    from paper_2404_03265_amd import PhaseFieldSolver, SolverParams
    from paper_2404_03265_amd.autograd import solve_load_step
    m = MESHES["tiny"]
    print(f"[case] workspace tiny p={p}", flush=True)
    ref = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask="rule", build_oracle=False)
    mk = lambda ws: PhaseFieldSolver(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"],
                                     params=ref.sp, torch_workspace=ws)
    solvers = {"library": mk(False), "torch": mk(True)}
    assert solvers["torch"]._ws.numel() == solvers["torch"].workspace_bytes() > 0
    U = ref.dev(ref.U_raw)
    pho = ref.dev(ref.phi_old_raw)
    pht = ref.dev(0.9 * ref.phit_raw + 0.05)
    v = ref.dev(inputs.random_vector(ref.X, ref.Y, 61))
    res = {}
    for name, g in solvers.items():
        g.set_state(U, pho, pht, None, setup_mg=True)
        out = [g.vmult(v), g.vmult_T(v), g.vcycle(v), g.vcycle(v, fp32=True), g.gmres(v)[0]]
        Uw = U.clone()
        act = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
        g.newton_step(Uw, pho, pht, act)
        out += [Uw, act]
        res[name] = [t.cpu().numpy() for t in out]
    for a, b in zip(res["library"], res["torch"]):
        assert np.array_equal(a, b)
    g = solvers["torch"]
    # a second binding, or one after the work vectors exist, is refused
    assert g.lib.pff_bind_workspace(g.h, C.c_void_p(g._ws.data_ptr()), g._ws.numel()) == -2
    assert solvers["library"].lib.pff_bind_workspace(solvers["library"].h, C.c_void_p(g._ws.data_ptr()),
                                                     g._ws.numel()) == -2
    # the bound basis holds the restart it was sized for, not more
    with pytest.raises(RuntimeError):
        g.set_params(SolverParams(**{**ref.sp.__dict__, "gmres_restart": ref.sp.gmres_restart + 1}))
    fresh = mk(False)
    need = fresh.workspace_bytes()
    buf = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    assert fresh.lib.pff_bind_workspace(fresh.h, C.c_void_p(buf.data_ptr() + 8), need) == -1     # misaligned
    assert fresh.lib.pff_bind_workspace(fresh.h, C.c_void_p(buf.data_ptr()), need - 1) == -1     # too small
    assert fresh.lib.pff_bind_workspace(fresh.h, C.c_void_p(buf.data_ptr()), need) == 0
    fresh.close()
    act, infos = solve_load_step(g, U.clone(), pho, pht, tol=1e-9)
    assert infos[-1]["residual_before"] <= 1e-9


@pytest.mark.parametrize("p", (1, 2))
def test_fp32_levels_follow_each_new_state(p):
    """The FP32 copies of the level states and diagonals are rebuilt for every
    multigrid setup, also when the FP32 V-cycle is only requested per call
    (vcycle_fp32 = 0): after a second set_state the FP32 V-cycle equals the one
    of a context that only ever saw the second state."""
    m = MESHES["tiny"]
    print(f"[case] fp32 levels after a new state tiny p={p}", flush=True)
    a = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask="rule", build_oracle=False)
    b = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask="rule", build_oracle=False,
             seed=7, u_std=1e-2)
    v = a.dev(inputs.random_vector(a.X, a.Y, 62))
    a.load_state(setup_mg=True)
    first = a.g.vcycle(v, fp32=True).cpu().numpy()
    a.g.set_state(a.dev(b.U_raw), a.dev(b.phi_old_raw), a.dev(b.phit_raw), None, setup_mg=True)
    second = a.g.vcycle(v, fp32=True).cpu().numpy()
    b.load_state(setup_mg=True)
    lam_max, lam_min0 = b.g.get_eigen()
    a.g.set_eigen(lam_max, lam_min0)
    b.g.set_eigen(lam_max, lam_min0)
    got = a.g.vcycle(v, fp32=True).cpu().numpy()
    ref = b.g.vcycle(v, fp32=True).cpu().numpy()
    assert not np.array_equal(first, second)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("p", (1, 2))
def test_tcv_of_params_autograd(p):
    """theta = (Gc, E, p) -> TCV through torch.autograd: the forward solves the
    load step (Alg. 2) at theta, the backward returns the adjoint gradient
    (bitwise the one of adjoint_tcv_gradient at the same state, which the
    oracle pins), scaled by the incoming gradient; in the linear-elastic
    regime of the Sneddon test u scales with p / E, so dTCV/dp ~ TCV / p and
    dTCV/dE ~ -TCV / E, and a central difference in p agrees."""
    import torch
    from paper_2404_03265_amd import SolverParams
    from paper_2404_03265_amd.autograd import TcvOfParams, adjoint_tcv_gradient, solve_load_step
    m = MESHES["tiny"]
    print(f"[case] TcvOfParams tiny p={p}", flush=True)
    sp_ = SolverParams(gmres_rtol=1e-13, gmres_atol=1e-15)
    c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask="rule",
             solver_params=sp_, build_oracle=False)
    ux, uy, phi = inputs.sneddon_state(c.X, c.Y, c.M, p, random=False)
    U0 = c.dev(np.concatenate([ux, uy, phi]))
    ph = c.dev(phi)
    th0 = [c.prm.Gc, c.prm.E, c.prm.pressure]
    theta = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    tcv = TcvOfParams.apply(theta, c.g, U0, ph, ph)
    (2.0 * tcv).backward()
    U = U0.clone()
    act, _ = solve_load_step(c.g, U, ph, ph, tol=1e-10)
    tcv_ref, grad_ref, _, _ = adjoint_tcv_gradient(c.g, U, ph, ph, act)
    assert tcv.item() == tcv_ref
    assert torch.equal(theta.grad, 2.0 * grad_ref)
    T = tcv.item()
    g = theta.grad.numpy() / 2.0
    assert abs(g[2] - T / th0[2]) <= 1e-2 * T / th0[2]
    assert abs(g[1] + T / th0[1]) <= 1e-2 * T / th0[1]
    h = 1e-3 * th0[2]
    vals = []
    for s in (1.0, -1.0):
        t = torch.tensor([th0[0], th0[1], th0[2] + s * h], dtype=torch.float64)
        vals.append(TcvOfParams.apply(t, c.g, U0, ph, ph).item())
    fd = (vals[0] - vals[1]) / (2 * h)
    print(f"dTCV/dp adjoint {g[2]:.8e} central difference {fd:.8e} TCV/p {T / th0[2]:.8e}", flush=True)
    assert abs(fd - g[2]) <= 1e-4 * abs(g[2])


@pytest.mark.parametrize("p", (1, 2))
def test_gmres_restarts_match_oracle(p):
    """GMRES(4) (Sec. 3.2 with a short restart, so that the solve passes
    through several restarts): the solution matches a direct solve, and the
    iteration count that of the oracle's GMRES(4) with the same V-cycle."""
    from oracle.krylov import gmres
    from paper_2404_03265_amd import SolverParams
    m = MESHES["tiny"]
    print(f"[case] GMRES(4) tiny p={p}", flush=True)
    c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask="bernoulli", u_std=1e-2,
             solver_params=SolverParams(gmres_restart=4), phit="shifted")
    c.load_state(setup_mg=True)
    lam_max, lam_min0 = c.g.get_eigen()
    vc = VCycle(Hierarchy(c.om), c.prm, MGParams(), c.U_o, c.phit_o, c.active_o,
                eigen=([lam_max[l] for l in range(c.g.n_levels)], lam_min0))
    J = c.lp.masked_operator(c.U_o, c.phit_o, c.active_o)
    b = inputs.random_vector(c.X, c.Y, 63) * c.to_g(c.lp.free_mask(c.active_o)).astype(float)
    tol = 1e-11 * np.linalg.norm(b)
    x, info, rc = c.g.gmres(c.dev(b), tol=tol)
    assert info["converged"] == 1 and info["iterations"] > 8, info
    xd = c.to_g(spla.spsolve(J.tocsc(), c.to_o(b)))
    assert np.linalg.norm(x.cpu().numpy() - xd) <= 1e-8 * np.linalg.norm(xd)
    _, oinfo = gmres(lambda v: J @ v, vc.apply, c.to_o(b), tol, restart=4, maxit=300)
    assert oinfo.converged
    assert abs(info["iterations"] - oinfo.iterations) <= 2, (info["iterations"], oinfo.iterations)


@pytest.mark.parametrize("hier", ("local", "global"))
@pytest.mark.parametrize("p", (1, 2))
def test_displacement_estimates_reused_while_phi_tilde_is_unchanged(p, hier):
    """The displacement block's level operators depend on phi~ alone, so a
    set-up at a new U with the same phi~ estimates the phase-field block
    only (its level operator evaluating the phase-field rows alone). Its
    eigenvalues and V-cycle equal those of a fresh context at the second
    state bit for bit; a changed phi~ is estimated again. Both hierarchies
    (the global-coarsening levels carry hanging nodes)."""
    import torch
    from paper_2404_03265_amd import SolverParams
    m = MESHES["tiny"]
    gc = hier == "global"

    def fresh():
        return Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], u_std=1e-2,
                    phit="shifted", build_oracle=False, mg_global=gc,
                    solver_params=SolverParams(mg_kind=1 if gc else 0))
    a = fresh()
    a.load_state(setup_mg=True)
    n = a.n
    act = a.dev(a.active.astype(np.uint8), torch.uint8)
    U2 = a.U_raw.copy()
    U2[:2 * n] *= 1.7
    src = inputs.random_vector(a.X, a.Y, 31)
    for phit in (a.phit_raw, 0.95 * a.phit_raw + 0.01):
        a.g.set_state(a.dev(U2), a.dev(a.phi_old_raw), a.dev(phit), act, setup_mg=True)
        b = fresh()
        b.g.set_state(b.dev(U2), b.dev(b.phi_old_raw), b.dev(phit), act, setup_mg=True)
        la, lb = a.g.get_eigen(), b.g.get_eigen()
        assert np.array_equal(la[0], lb[0]) and np.array_equal(la[1], lb[1])
        assert np.array_equal(a.g.vcycle(a.dev(src)).cpu().numpy(), b.g.vcycle(b.dev(src)).cpu().numpy())
        U2[:2 * n] *= 0.8
