"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(closed forms, exact integrals, invariants, brute force), not against itself."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import inputs
from oracle.assemble import CellSet, LeafProblem, Params, element_jacobian
from oracle.fe import Element
from oracle.mesh import Mesh
from oracle.mg import Hierarchy, MGParams, VCycle, cg_eigs, chebyshev
from oracle.krylov import gmres
from oracle.newton import (NewtonParams, active_set, adjoint_gradient, extrapolate_phase_field,
                           newton_step, solve_frozen)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _state(mesh, lp, seed=0, u_std=0.05):
    n = mesh.n_nodes
    ux, uy, phi = inputs.sneddon_state(mesh.NX, mesh.NY, mesh.M, mesh.p, seed=seed, u_std=u_std)
    U = np.concatenate([ux, uy, phi])
    U[:2 * n][np.concatenate([mesh.dirichlet] * 2)] = 0.0
    U = lp.distribute(U)
    phit = lp.distribute(np.concatenate([0.9 * phi + 0.05]))
    return U, phit


# ---------------------------------------------------------------- paper ---
def test_table1_lame_parameters():
    g = json.load(open(GOLDEN))["table1"]
    prm = Params(E=g["E"], nu=g["nu"])
    assert round(prm.mu, g["printed_decimals"]) == g["mu_printed"]
    assert round(prm.lam, g["printed_decimals"]) == g["lambda_printed"]
    # plane stress would give lambda = E nu / (1 - nu^2) = 0.208, which Table 1 rules out
    assert round(g["E"] * g["nu"] / (1 - g["nu"] ** 2), 2) != g["lambda_printed"]


def test_table2_first_row_mesh():
    """40x40 Q1 cells (a 10x10 grid refined twice): 3 * 41^2 = 5043 DoFs and
    h = diagonal of a 0.5 cell = 0.7071."""
    g = json.load(open(GOLDEN))["table2_row1"]
    m = Mesh(40, 0, 1, coarse=10)
    assert 3 * m.n_nodes == g["dofs"]
    assert abs(m.cell_diameter_min() - g["h"]) < 1e-4


# ----------------------------------------------------------------- mesh ---
@pytest.mark.parametrize("p", [1, 2])
def test_mesh_balance_and_hanging(p, tiny_mesh_factory):
    m = tiny_mesh_factory(p)
    assert m.hanging.sum() > 0
    # 2:1 face balance
    for (l, i, j) in m.leaves:
        n = m.ncells_1d(l)
        for di, dj in Mesh.DIRS:
            ni, nj = i + di, j + dj
            if 0 <= ni < n and 0 <= nj < n:
                f = m.find_leaf(l, ni, nj)
                assert f is None or f[0] >= l - 1
    # hanging interpolation reproduces global polynomials of degree p
    X = -10 + 20 * m.NX / m.M
    Y = -10 + 20 * m.NY / m.M
    lp = LeafProblem(m, Params())
    for f in (X, Y, X * Y) + ((X ** 2, Y ** 2, X ** 2 * Y) if p == 2 else ()):
        v = f.copy()
        v[m.hanging] = 12345.0
        w = lp.distribute(v)
        assert np.allclose(w, f, atol=1e-11)


def test_band_refinement_counts():
    """Refining an a x b block of cells adds 3ab + a + b Q1 vertices."""
    m0 = Mesh(32, 0, 1)
    m1 = Mesh(32, 1, 1)
    refined = [c for c in m0.leaves if m0._in_band(*c)]
    ii = {c[1] for c in refined}
    jj = {c[2] for c in refined}
    a, b = len(ii), len(jj)
    assert a * b == len(refined)
    assert m1.n_nodes - m0.n_nodes == 3 * a * b + a + b


# ----------------------------------------------------- element matrices ---
def _sympy_element(p, H, mu, lam, Gc, ell, pr, phi):
    import sympy as s
    x, y = s.symbols("x y")
    nodes = [s.Rational(k, p) * H for k in range(p + 1)]

    def l1(k, t):
        e = s.Integer(1)
        for m_ in range(p + 1):
            if m_ != k:
                e *= (t - nodes[m_]) / (nodes[k] - nodes[m_])
        return e
    N = [l1(a, x) * l1(b, y) for b in range(p + 1) for a in range(p + 1)]
    nl = len(N)
    K = np.zeros((3 * nl, 3 * nl))

    def integ(e):
        return float(s.integrate(s.integrate(s.expand(e), (x, 0, H)), (y, 0, H)))
    grads = [(s.diff(f, x), s.diff(f, y)) for f in N]
    for k in range(nl):
        for m_ in range(nl):
            gkx, gky = grads[k]
            gmx, gmy = grads[m_]
            # plane-strain elasticity sigma(u):e(v) for u = N_m e_d, v = N_k e_c
            K[k, m_] = integ((2 * mu + lam) * gmx * gkx + mu * gmy * gky)
            K[k, nl + m_] = integ(lam * gmy * gkx + mu * gmx * gky)
            K[nl + k, m_] = integ(lam * gmx * gky + mu * gmy * gkx)
            K[nl + k, nl + m_] = integ((2 * mu + lam) * gmy * gky + mu * gmx * gkx)
            K[2 * nl + k, 2 * nl + m_] = integ(Gc / ell * N[m_] * N[k] + Gc * ell * (gmx * gkx + gmy * gky))
            # coupling at u = 0: 2 p phi div(du) psi
            K[2 * nl + k, m_] = integ(2 * pr * phi * gmx * N[k])
            K[2 * nl + k, nl + m_] = integ(2 * pr * phi * gmy * N[k])
    return K


@pytest.mark.parametrize("p", [1, 2])
def test_single_cell_matches_exact_integrals(p):
    """u = 0, phi~ = 1, kappa = 0: the u block is the plane-strain stiffness,
    the phi block is (Gc/l) M + Gc l K and the coupling block is the pressure
    term 2 p phi (div du, psi); all exact with p+1 Gauss points."""
    H = 0.7
    prm = Params(E=2.5, nu=0.3, Gc=1.7, pressure=0.4, kappa=0.0, ell=0.35)
    el = Element(p)
    cs = CellSet(el, np.array([H]), np.arange(el.nloc)[None, :])
    z = np.zeros((1, el.nloc))
    Ke = element_jacobian(cs, prm, z, z, np.full((1, el.nloc), 0.6), np.ones((1, el.nloc)))[0]
    import sympy as s
    Kx = _sympy_element(p, s.Rational(7, 10), s.nsimplify(prm.mu), s.nsimplify(prm.lam),
                        s.nsimplify(prm.Gc), s.Rational(35, 100), s.Rational(2, 5), s.Rational(3, 5))
    assert np.allclose(Ke, Kx, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------- jacobian ---
@pytest.mark.parametrize("p", [1, 2])
def test_jacobian_is_complex_step_derivative_of_residual(p, tiny_mesh_factory):
    """F is a polynomial in U, so Im F(U + i eps v) / eps = J v to rounding
    (Squire & Trapp 1998)."""
    m = tiny_mesh_factory(p)
    lp = LeafProblem(m, Params(ell=0.3, kappa=1e-3, pressure=0.3))
    U, phit = _state(m, lp)
    v = inputs.random_vector(m.NX, m.NY, 5)
    J = lp.jacobian_raw(U, phit)
    eps = 1e-30
    jv_cs = lp.residual_raw(U + 1j * eps * v, phit).imag / eps
    jv = J @ v
    assert np.abs(jv - jv_cs).max() <= 1e-13 * np.abs(jv).max()
    # central differences as a second opinion
    h = 1e-6
    fd = (lp.residual_raw(U + h * v, phit) - lp.residual_raw(U - h * v, phit)) / (2 * h)
    assert np.abs(jv - fd).max() <= 1e-7 * np.abs(jv).max()


@pytest.mark.parametrize("p", [1, 2])
def test_block_structure_symmetry_and_spd(p, tiny_mesh_factory):
    m = tiny_mesh_factory(p)
    lp = LeafProblem(m, Params(ell=0.3, kappa=1e-3, pressure=0.3))
    U, phit = _state(m, lp)
    n = m.n_nodes
    act = inputs.bernoulli_mask(m.NX, m.NY, 2, 0.1)
    J = lp.masked_operator(U, phit, act).toarray()
    uu, pp = J[:2 * n, :2 * n], J[2 * n:, 2 * n:]
    assert np.abs(J[:2 * n, 2 * n:]).max() == 0.0          # lower block triangular
    assert np.abs(uu - uu.T).max() <= 1e-14 * np.abs(uu).max()
    assert np.abs(pp - pp.T).max() <= 1e-14 * np.abs(pp).max()
    np.linalg.cholesky(uu)
    np.linalg.cholesky(pp)


@pytest.mark.parametrize("p", [1, 2])
def test_rigid_body_modes_annihilated(p, tiny_mesh_factory):
    m = tiny_mesh_factory(p)
    lp = LeafProblem(m, Params(ell=0.3, kappa=1e-3, pressure=0.3))
    U, phit = _state(m, lp)
    J = lp.jacobian_raw(U, phit)
    n = m.n_nodes
    X = -10 + 20 * m.NX / m.M
    Y = -10 + 20 * m.NY / m.M
    for mode in (np.concatenate([np.ones(n), np.zeros(2 * n)]),
                 np.concatenate([np.zeros(n), np.ones(n), np.zeros(n)]),
                 np.concatenate([-Y, X, np.zeros(n)])):
        r = J @ mode
        assert np.abs(r).max() <= 1e-12 * np.abs(J).max() * 20


@pytest.mark.parametrize("p", [1, 2])
def test_patch_test_with_hanging_nodes(p, tiny_mesh_factory):
    """A globally linear displacement with phi~ = 1 and no pressure leaves every
    interior (free) u row of the condensed residual at zero."""
    m = tiny_mesh_factory(p)
    prm = Params(ell=0.3, kappa=0.0, pressure=0.0)
    lp = LeafProblem(m, prm)
    n = m.n_nodes
    X = -10 + 20 * m.NX / m.M
    Y = -10 + 20 * m.NY / m.M
    U = np.concatenate([0.3 * X - 0.2 * Y, 0.1 * X + 0.5 * Y, np.ones(n)])
    R = lp.residual(U, np.ones(n))
    free_u = np.concatenate([~(m.dirichlet | m.hanging)] * 2)
    assert np.abs(R[:2 * n][free_u]).max() < 1e-12


# ----------------------------------------------------------------- TCV ---
@pytest.mark.parametrize("p", [1, 2])
def test_tcv_closed_forms(p, tiny_mesh_factory):
    m = tiny_mesh_factory(p)
    lp = LeafProblem(m, Params())
    n = m.n_nodes
    X = -10 + 20 * m.NX / m.M
    Y = -10 + 20 * m.NY / m.M
    # u = (1, 2), phi = 3x + 5y: u . grad phi = 13 on a 20 x 20 square
    U = np.concatenate([np.ones(n), 2 * np.ones(n), 3 * X + 5 * Y])
    assert abs(lp.tcv(U) - 13 * 400) < 1e-9
    if p == 2:
        # u = (x, 0), phi = x^2 / 2: integral of x^2 = 20 * 2000 / 3
        U = np.concatenate([X, np.zeros(n), 0.5 * X ** 2])
        assert abs(lp.tcv(U) - 40000.0 / 3.0) < 1e-8
    # gradient: TCV is bilinear, complex step is exact
    U, _ = _state(m, lp)
    v = inputs.random_vector(m.NX, m.NY, 9)
    v = lp.distribute(v * np.concatenate([~m.hanging] * 3))
    g = lp.tcv_gradient(U)
    cs = lp.tcv(U + 1e-30j * v) if False else None  # tcv() casts to float; use FD of a bilinear form
    h = 1e-3
    fd = (lp.tcv(U + h * v) - lp.tcv(U - h * v)) / (2 * h)
    assert abs(g @ (v * np.concatenate([~m.hanging] * 3)) - fd) <= 1e-10 * max(1.0, abs(fd))


def test_lumped_mass_sums_to_area(tiny_mesh_factory):
    for p in (1, 2):
        lp = LeafProblem(tiny_mesh_factory(p), Params())
        assert abs(lp.lumped_phi_mass().sum() - 400.0) < 1e-10


# ------------------------------------------------------ param derivatives ---
@pytest.mark.parametrize("p", [1, 2])
def test_parameter_derivatives_complex_step(p, tiny_mesh_factory):
    """mu, lambda are linear in E; p and Gc enter linearly: complex step in each
    parameter of the full residual is exact."""
    m = tiny_mesh_factory(p)
    base = dict(E=1.3, nu=0.2, Gc=0.8, pressure=0.2, kappa=1e-3, ell=0.3)
    lp = LeafProblem(m, Params(**base))
    U, phit = _state(m, lp)
    d = lp.param_derivatives(U, phit)
    for name, key in (("Gc", "Gc"), ("E", "E"), ("p", "pressure")):
        q = dict(base)
        q[key] = base[key] + 1e-30j
        lpc = LeafProblem(m, Params(**q))
        ref = lpc.C3.T @ lpc.residual_raw(U.astype(complex), phit.astype(complex)).imag / 1e-30
        assert np.abs(d[name] - ref).max() <= 1e-12 * np.abs(ref).max()


# ------------------------------------------------------------ transfers ---
@pytest.mark.parametrize("p", [1, 2])
def test_prolongation_reproduces_polynomials(p, tiny_mesh_factory):
    m = tiny_mesh_factory(p)
    h = Hierarchy(m)
    for l in range(1, len(h.levels)):
        f, c = h.levels[l], h.levels[l - 1]
        for fn in (lambda X, Y: 1 + 0 * X, lambda X, Y: X, lambda X, Y: X * Y - 3 * Y) + \
                ((lambda X, Y: X ** 2 * Y + Y ** 2,) if p == 2 else ()):
            vc = fn(c.NX / m.M, c.NY / m.M)
            vf = fn(f.NX / m.M, f.NY / m.M)
            assert np.allclose(h.P[l] @ vc, vf, atol=1e-12)


# ------------------------------------------------------------ Chebyshev ---
def test_chebyshev_matches_closed_form_polynomial():
    """On A = diag(lambda), D = I, b = 0 the error after k updates is
    T_k((theta - lambda)/delta) / T_k(theta/delta) times the start."""
    lam = np.linspace(0.1, 2.0, 40)
    A = sp.diags(lam).tocsr()
    theta, delta = 1.05, 0.95
    for k in (1, 2, 3, 4, 7):
        x0 = np.ones(lam.size)
        x = chebyshev(A, np.ones(lam.size), np.ones(lam.size, bool), np.zeros(lam.size), x0, k,
                      np.full(lam.size, theta), np.full(lam.size, delta))
        T = np.polynomial.chebyshev.Chebyshev.basis(k)
        expect = T((theta - lam) / delta) / T(theta / delta)
        assert np.allclose(x, expect, atol=1e-13)


def test_cg_eigs_exact_with_full_krylov():
    rng = np.random.default_rng(0)
    Q = rng.standard_normal((12, 12))
    A = Q @ Q.T + 12 * np.eye(12)
    d = 1.0 / np.diag(A)
    lo, hi = cg_eigs(sp.csr_matrix(A), d, np.ones(12, bool), 12)
    ev = np.linalg.eigvalsh(np.diag(np.sqrt(d)) @ A @ np.diag(np.sqrt(d)))
    assert abs(hi - ev.max()) < 1e-9 * ev.max()
    assert abs(lo - ev.min()) < 1e-9 * ev.max()


# --------------------------------------------------------------- V-cycle ---
def _embedding(mesh, lv):
    from oracle.fe import basis_1d
    p, S = mesh.p, lv.S
    rows, cols, vals = [], [], []
    for g in range(mesh.n_nodes):
        X, Y = int(mesh.NX[g]), int(mesh.NY[g])
        cands = [(ii, jj) for ii in ([X // S - 1, X // S] if X % S == 0 else [X // S])
                 for jj in ([Y // S - 1, Y // S] if Y % S == 0 else [Y // S])
                 if (ii, jj) in lv.cellset_keys]
        if not cands:
            continue
        ii, jj = cands[0]
        vx, _ = basis_1d(p, [(X - ii * S) / S])
        vy, _ = basis_1d(p, [(Y - jj * S) / S])
        for b in range(p + 1):
            for a in range(p + 1):
                w = vx[0, a] * vy[0, b]
                if w != 0:
                    key = (jj * S + b * S // p) * (mesh.M + 1) + ii * S + a * S // p
                    rows.append(g)
                    cols.append(lv.key_to_node[key])
                    vals.append(w)
    E = sp.csr_matrix((vals, (rows, cols)), shape=(mesh.n_nodes, lv.n))
    return sp.block_diag([E, E, E]).tocsr()


@pytest.mark.parametrize("p", [1, 2])
def test_vcycle_equals_multiplicative_subspace_correction(p, tiny_mesh_factory):
    """With constant coefficients (u = 0, phi~ const, no active set) the
    rediscretised level operators are Galerkin, and the local-smoothing V-cycle
    must equal the literal multiplicative subspace correction
    x += I_l S_l I_l^T (b - A x) over the spaces of level functions that vanish
    on the refinement edge, built here from explicit leaf embeddings."""
    mesh = tiny_mesh_factory(p)
    prm = Params(ell=0.5, kappa=1e-3)
    lp = LeafProblem(mesh, prm)
    n = mesh.n_nodes
    U, phit = np.zeros(3 * n), np.full(n, 0.7)
    active = np.zeros(n, bool)
    h = Hierarchy(mesh)
    vc = VCycle(h, prm, MGParams(cheb_degree=3, coarse_its=5), U, phit, active)
    B = lp.masked_operator(U, phit, active, blocks="diag")
    free = lp.free_mask(active)
    Mf = sp.diags(free.astype(float))
    b = inputs.random_vector(mesh.NX, mesh.NY, 7) * free
    y = vc.apply(b)
    Es = [_embedding(mesh, lv) for lv in h.levels]
    L = len(h.levels) - 1
    x = np.zeros(3 * n)

    def corr(l, x, coarse=False):
        r = (Es[l].T @ (Mf @ (b - B @ x))) * vc.ops[l].free
        s = vc.coarse_solve(r) if coarse else vc.chebyshev(l, r, None, 3)
        return x + Mf @ (Es[l] @ s)
    for l in range(L, 0, -1):
        x = corr(l, x)
    x = corr(0, x, coarse=True)
    for l in range(1, L + 1):
        x = corr(l, x)
    assert np.abs(x - y * free).max() <= 1e-12 * np.abs(y).max()
    # constrained rows pass through
    assert np.array_equal(y[~free], b[~free])


@pytest.mark.parametrize("p", [1, 2])
def test_vcycle_symmetric(p, tiny_mesh_factory):
    """Same smoother before and after a linear coarse correction: P^{-1} is
    symmetric (a fixed number of CG steps would not be linear in the input)."""
    mesh = tiny_mesh_factory(p)
    prm = Params(ell=0.4, kappa=1e-3, pressure=0.2)
    lp = LeafProblem(mesh, prm)
    U, phit = _state(mesh, lp, u_std=0.01)
    act = inputs.bernoulli_mask(mesh.NX, mesh.NY, 2, 0.1) & ~mesh.hanging
    vc = VCycle(Hierarchy(mesh), prm, MGParams(coarse_mode="cheb", coarse_its=8), U, phit, act)
    free = lp.free_mask(act)
    a = inputs.random_vector(mesh.NX, mesh.NY, 11) * free
    c = inputs.random_vector(mesh.NX, mesh.NY, 12) * free
    lhs, rhs = c @ vc.apply(a), a @ vc.apply(c)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ------------------------------------------------------- GMRES / Newton ---
def test_gmres_matches_direct_solve(tiny_mesh_factory):
    mesh = tiny_mesh_factory(1)
    prm = Params(ell=0.4, kappa=1e-3, pressure=0.2)
    lp = LeafProblem(mesh, prm)
    U, phit = _state(mesh, lp, u_std=0.01)
    act = np.zeros(mesh.n_nodes, bool)
    J = lp.masked_operator(U, phit, act)
    b = inputs.random_vector(mesh.NX, mesh.NY, 3) * lp.free_mask(act)
    vc = VCycle(Hierarchy(mesh), prm, MGParams(), U, phit, act)
    x, info = gmres(lambda v: J @ v, vc.apply, b, 1e-13 * np.linalg.norm(b), restart=30, maxit=300)
    xd = spla.spsolve(J.tocsc(), b)
    assert info.converged
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    res = np.array(info.residuals)
    assert np.all(np.diff(res) <= 1e-12 * res[0])


def _sneddon(mesh, prm_kw):
    prm = Params(**prm_kw)
    lp = LeafProblem(mesh, prm)
    n = mesh.n_nodes
    ux, uy, phi = inputs.sneddon_state(mesh.NX, mesh.NY, mesh.M, mesh.p, random=False)
    U = lp.distribute(np.concatenate([ux, uy, phi]))
    return lp, U, U[2 * n:].copy()


def test_newton_u_block_scales_with_p_over_E():
    """The u equation is linear in u with the linearised degradation, so one
    Newton step solves it exactly and u(p, E) = (p/E) u(1, 1)."""
    mesh = Mesh(32, 1, 1)
    n = mesh.n_nodes
    sols = []
    for (pr, E) in ((1e-3, 1.0), (3e-3, 2.0)):
        lp, U, phi_old = _sneddon(mesh, dict(E=E, pressure=pr, ell=0.2, kappa=1e-10))
        Un, act, info = newton_step(lp, Hierarchy(mesh), MGParams(), NewtonParams(), U,
                                    phi_old, phi_old.copy(), linear_solver="direct")
        Rn = lp.residual(Un, phi_old) * lp.free_mask(act)
        assert np.abs(Rn[:2 * n]).max() < 1e-12
        sols.append(Un[:2 * n] * E / pr)
        crack = inputs.crack_mask(mesh.NX, mesh.NY, mesh.M, mesh.p)
        assert np.all(act[crack])                           # active set contains the crack
    assert np.abs(sols[0] - sols[1]).max() <= 1e-10 * np.abs(sols[0]).max()


def test_newton_converges_and_complementarity():
    """Newton / PDAS on a small Sneddon mesh: residual below TOL_N with an
    unchanged active set; at the solution phi <= phi_old off the active set
    and lambda >= 0 on it (Sec. 2, Problem 2)."""
    mesh = Mesh(32, 2, 1)
    n = mesh.n_nodes
    ell = 2 * np.sqrt(2) * 20 / (32 * 4)
    lp, U, phi_old = _sneddon(mesh, dict(ell=ell, kappa=1e-10))
    h = Hierarchy(mesh)
    act = np.zeros(n, bool)
    converged = False
    for _ in range(10):
        Un, act_new, info = newton_step(lp, h, MGParams(), NewtonParams(), U, phi_old, phi_old, act)
        assert info.gmres_converged
        unchanged = np.array_equal(act_new, act)
        U, act = Un, act_new
        if unchanged and info.residual_before <= 1e-7:
            converged = True
            break
    assert converged
    R = lp.residual(U, phi_old)
    lam = R[2 * n:] / np.where(mesh.hanging, 1, lp.lumped_phi_mass())
    assert np.all(U[2 * n:][~act] <= phi_old[~act] + 1e-8)
    assert np.all(lam[act] >= -1e-10)
    assert lp.tcv(U) > 0.0


def test_active_set_rule_cases():
    """Sign rule of the active set with c = 2|lambda/(phi - phi_old)|."""
    m = Mesh(16, 0, 1)
    lp = LeafProblem(m, Params())
    n = m.n_nodes
    B = lp.lumped_phi_mass()
    phi_old = np.full(n, 0.5)
    lamv = np.tile([1.0, -1.0, 0.0], n // 3 + 1)[:n]
    R = np.concatenate([np.zeros(2 * n), lamv * B])
    for shift, expect in ((0.1, lamv != 0), (-0.1, np.zeros(n, bool)), (0.0, lamv > 0)):
        a = active_set(lp, R, phi_old + shift, phi_old)
        assert np.array_equal(a, expect)


def test_active_set_fixed_c_cases():
    """Constant c (Sec. 2 leaves c free): lambda + c (phi - phi_old) > 0 flips
    exactly at c = lambda / |phi - phi_old| when phi < phi_old; c -> 0 leaves
    the sign of lambda, a large c the sign of phi - phi_old."""
    m = Mesh(16, 0, 1)
    lp = LeafProblem(m, Params())
    n = m.n_nodes
    B = lp.lumped_phi_mass()
    phi_old = np.full(n, 0.5)
    lamv = np.tile([1.0, -1.0, 0.0], n // 3 + 1)[:n]
    R = np.concatenate([np.zeros(2 * n), lamv * B])
    down, up = phi_old - 0.1, phi_old + 0.1
    assert np.array_equal(active_set(lp, R, down, phi_old, 9.99), lamv > 0)   # 1 - 0.999 > 0
    assert not active_set(lp, R, down, phi_old, 10.01).any()                 # 1 - 1.001 < 0
    for phi in (down, up, phi_old):
        assert np.array_equal(active_set(lp, R, phi, phi_old, 1e-300), lamv > 0)
    assert np.array_equal(active_set(lp, R, up, phi_old, 1e30), np.ones(n, bool))
    assert not active_set(lp, R, down, phi_old, 1e30).any()
    assert np.array_equal(active_set(lp, R, phi_old, phi_old, 1e30), lamv > 0)


def test_fixed_c_pdas_reaches_the_same_solution():
    """Newton / PDAS with a constant c converges to the solution of the
    complementarity problem (Problem 2) that the per-unknown c reaches: the
    converged states agree up to nodes where lambda is within rounding of zero
    (either set is then consistent), and both satisfy complementarity."""
    mesh = Mesh(32, 2, 1)
    n = mesh.n_nodes
    ell = 2 * np.sqrt(2) * 20 / (32 * 4)
    sols = []
    for c in (0.0, 1.0, 1e4):
        lp, U, phi_old = _sneddon(mesh, dict(ell=ell, kappa=1e-10))
        act = np.zeros(n, bool)
        for _ in range(30):
            Un, act_new, info = newton_step(lp, Hierarchy(mesh), MGParams(), NewtonParams(pdas_c=c), U, phi_old,
                                            phi_old, act, linear_solver="direct")
            unchanged = np.array_equal(act_new, act)
            U, act = Un, act_new
            if unchanged and info.residual_before <= 1e-10:
                break
        else:
            raise AssertionError(f"c = {c}: no convergence")
        R = lp.residual(U, phi_old)
        lam = R[2 * n:] / np.where(mesh.hanging, 1, lp.lumped_phi_mass())
        assert np.all(U[2 * n:][~act] <= phi_old[~act] + 1e-8)
        assert np.all(lam[act] >= -1e-10)
        sols.append(U)
    for U in sols[1:]:
        assert np.abs(U - sols[0]).max() <= 1e-7 * np.abs(sols[0]).max()


def test_phase_field_extrapolation():
    """Linear extrapolation of phi~ in the load parameter (Sec. 2): a field
    affine in t is continued exactly for unequal steps; theta = 0 returns the
    previous step; a continuation outside [0, 1] takes the nearest bound."""
    rng = np.random.default_rng(3)
    a, b = rng.uniform(0.3, 0.7, 64), rng.uniform(-0.05, 0.05, 64)
    t = (0.3, 1.1, 2.0)
    f = [a + b * tk for tk in t]
    theta = (t[2] - t[1]) / (t[1] - t[0])
    assert np.abs(extrapolate_phase_field(f[1], f[0], theta) - f[2]).max() <= 1e-15
    assert np.array_equal(extrapolate_phase_field(f[1], f[0], 0.0), f[1])
    x = rng.uniform(-0.5, 1.5, 1000)
    y = rng.uniform(-0.5, 1.5, 1000)
    e = extrapolate_phase_field(x, y, 0.75)
    assert e.min() >= 0.0 and e.max() <= 1.0
    line = x + 0.75 * (x - y)
    assert np.all(e[line >= 1.0] == 1.0) and np.all(e[line <= 0.0] == 0.0)


# --------------------------------------------------------------- adjoint ---
def test_adjoint_gradient_matches_finite_differences():
    mesh = Mesh(16, 1, 1, coarse=4, band=(3.0, 1.0))
    n = mesh.n_nodes
    base = dict(E=1.0, nu=0.2, Gc=1.0, pressure=1e-3, kappa=1e-10, ell=0.5)
    lp, U0, phi_old = _sneddon(mesh, base)
    R = lp.residual(U0, phi_old)
    act = active_set(lp, R, U0[2 * n:], phi_old)
    U = solve_frozen(lp, U0, phi_old, phi_old, act)
    grad, _ = adjoint_gradient(lp, U, phi_old, act)
    for name, key in (("Gc", "Gc"), ("E", "E"), ("p", "pressure")):
        vals = []
        for sgn in (1, -1):
            q = dict(base)
            q[key] = base[key] * (1 + sgn * 1e-6)
            lq = LeafProblem(mesh, Params(**q))
            vals.append(lq.tcv(solve_frozen(lq, U0, phi_old, phi_old, act)))
        fd = (vals[0] - vals[1]) / (2e-6 * base[key])
        # central differences: truncation ~1e-12 relative, cancellation noise
        # ~ eps * TCV / (h theta) from the 1e-14 solves
        noise = 1e-8 * abs(lp.tcv(U)) / base[key]
        assert abs(grad[name] - fd) <= 1e-6 * abs(fd) + noise


@pytest.mark.parametrize("p", [1, 2])
def test_vcycle_nonsingular_with_scattered_active_set(p, tiny_mesh_factory):
    """With a scattered active set the level sets grow by dilation; every free
    leaf unknown must stay free on its home level, otherwise the V-cycle maps
    it to zero for every input. Checked on the dense matrix of P^{-1} (brute
    force, tiny mesh) and through GMRES against a direct solve."""
    mesh = tiny_mesh_factory(p)
    n = mesh.n_nodes
    prm = Params(ell=0.35, kappa=1e-10, pressure=1e-3)
    lp = LeafProblem(mesh, prm)
    U, phit = _state(mesh, lp, u_std=1e-2)
    act = inputs.bernoulli_mask(mesh.NX, mesh.NY, 2, 0.1) & ~mesh.hanging
    hier = Hierarchy(mesh)
    acts = hier.level_active(act)
    for l, lv in enumerate(hier.levels):
        home = lv.leafcell_node & ~lv.edge
        assert np.array_equal(acts[l][home], act[lv.leaf_index[home]])
    vc = VCycle(hier, prm, MGParams(), U, phit, act)
    free = np.flatnonzero(lp.free_mask(act))
    if free.size <= 1500:
        Pm = np.column_stack([vc.apply(np.eye(3 * n)[:, i])[free] for i in free])
        assert np.linalg.svd(Pm, compute_uv=False).min() > 1e-6
    J = lp.masked_operator(U, phit, act)
    b = inputs.random_vector(mesh.NX, mesh.NY, 6) * lp.free_mask(act)
    x, info = gmres(lambda v: J @ v, vc.apply, b, 1e-13 * np.linalg.norm(b))
    xd = spla.spsolve(J.tocsc(), b)
    assert info.converged and np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_coarse_cg_closed_forms():
    """Coarse-level CG (fixed steps from zero, Jacobi preconditioner, blocks
    separate): one step is the preconditioned steepest-descent step
    x = (r.z / z.Az) z with z = D^{-1} r; with as many steps as free unknowns
    it reproduces the exact solve of each block on its free unknowns."""
    import scipy.sparse.linalg as spla
    from oracle.mg import Hierarchy, MGParams, VCycle, block_masks
    mesh = Mesh(16, 1, 1, coarse=4, band=(3.0, 1.0))
    prm = Params(ell=0.4, kappa=1e-3, pressure=0.2)
    lp = LeafProblem(mesh, prm)
    U, phit = _state(mesh, lp, u_std=0.01)
    rng = np.random.default_rng(3)
    act = inputs.bernoulli_mask(mesh.NX, mesh.NY, 2, 0.1) & ~mesh.hanging
    h = Hierarchy(mesh)
    n0 = h.levels[0].n
    b = rng.standard_normal(3 * n0)
    vc1 = VCycle(h, prm, MGParams(coarse_mode="cg", coarse_its=1), U, phit, act)
    op = vc1.ops[0]
    x1 = vc1.coarse_solve(b)
    for blk in block_masks(n0):
        m = op.free & blk
        r = b * m
        z = op.Dinv * r
        alpha = (r @ z) / (z @ (op.A @ z))
        assert np.allclose(x1[blk], (alpha * z)[blk], rtol=1e-13, atol=1e-15)
    nfree = int(op.free.sum())
    vcn = VCycle(h, prm, MGParams(coarse_mode="cg", coarse_its=nfree + 5), U, phit, act)
    xn = vcn.coarse_solve(b)
    for blk in block_masks(n0):
        idx = np.flatnonzero(op.free & blk)
        xe = spla.spsolve(op.A[idx][:, idx].tocsc(), b[idx])
        assert np.linalg.norm(xn[idx] - xe) <= 1e-8 * np.linalg.norm(xe)
        assert np.all(xn[blk & ~op.free] == 0.0)


# ------------------------------------- energy term at a deformed state ---
def _poly_integral(expr, H, x, y):
    """Exact integral over [0, H]^2 of a polynomial in (x, y), monomial by
    monomial with rational arithmetic."""
    import sympy as s
    P = s.Poly(s.expand(expr), x, y)
    tot = s.Integer(0)
    for (i, j), c in P.terms():
        tot += c * H ** (i + 1) / (i + 1) * H ** (j + 1) / (j + 1)
    return tot


@pytest.mark.parametrize("p", [1, 2])
def test_single_cell_deformed_state_exact_integrals(p):
    """Residual (Problem 2) and Jacobian (Sec. 3.1) on one cell at a state with
    u != 0, so that sigma(u):e(u) != 0 and the degradation-energy terms
    (1-kappa) phi sigma(u):e(u) and their derivatives carry weight; kappa != 0
    and phi~ != 1. The fields are chosen so that p+1 Gauss points integrate
    every term exactly: u affine (constant strain), phi bilinear, phi~
    bilinear in the residual and constant in the u-block of the Jacobian. The
    reference is the weak form integrated exactly in rational arithmetic,
    written from the paper's formulas in terms of the fields themselves (no
    quadrature, no shape-function tables)."""
    import sympy as s
    R_ = s.Rational
    x, y = s.symbols("x y")
    H = R_(7, 10)
    E, nu, Gc, pr, kap, ell = R_(5, 2), R_(3, 10), R_(17, 10), R_(2, 5), R_(1, 20), R_(7, 20)
    mu = E / (2 * (1 + nu))
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    ux = R_(3, 10) + R_(1, 5) * x - R_(1, 2) * y
    uy = -R_(1, 10) + R_(2, 5) * x + R_(1, 4) * y
    phi = R_(3, 5) + R_(1, 5) * x - R_(3, 10) * y + R_(1, 2) * x * y
    phit_res = R_(4, 5) + R_(1, 10) * x + R_(1, 5) * y - R_(3, 10) * x * y
    phit_jac = R_(4, 5)

    def strain(vx, vy):
        return s.diff(vx, x), s.diff(vy, y), (s.diff(vx, y) + s.diff(vy, x)) / 2

    def stress(e):
        exx, eyy, exy = e
        return 2 * mu * exx + lam * (exx + eyy), 2 * mu * eyy + lam * (exx + eyy), 2 * mu * exy

    def ddot(sg, e):
        return sg[0] * e[0] + sg[1] * e[1] + 2 * sg[2] * e[2]

    eu = strain(ux, uy)
    su = stress(eu)
    Sval = ddot(su, eu)
    divu = eu[0] + eu[1]
    # shape functions on [0, H]^2, node (a, b) at (a H / p, b H / p), index a + (p+1) b
    pts = [R_(k, p) * H for k in range(p + 1)]

    def l1(k, t):
        e = s.Integer(1)
        for m_ in range(p + 1):
            if m_ != k:
                e *= (t - pts[m_]) / (pts[k] - pts[m_])
        return e
    N = [l1(a, x) * l1(b, y) for b in range(p + 1) for a in range(p + 1)]
    nl = len(N)
    integ = lambda e: float(_poly_integral(e, H, x, y))   # noqa: E731

    # exact residual
    g_res = (1 - kap) * phit_res ** 2 + kap
    Rx = np.zeros(3 * nl)
    for k, Nk in enumerate(N):
        ex_ = strain(Nk, 0)
        ey_ = strain(0, Nk)
        Rx[k] = integ(g_res * ddot(su, ex_) + pr * phit_res ** 2 * s.diff(Nk, x))
        Rx[nl + k] = integ(g_res * ddot(su, ey_) + pr * phit_res ** 2 * s.diff(Nk, y))
        Rx[2 * nl + k] = integ((1 - kap) * phi * Sval * Nk + 2 * pr * phi * divu * Nk
                               - Gc / ell * (1 - phi) * Nk
                               + Gc * ell * (s.diff(phi, x) * s.diff(Nk, x) + s.diff(phi, y) * s.diff(Nk, y)))
    # exact Jacobian: u-block at constant phi~, full phi rows
    g_jac = (1 - kap) * phit_jac ** 2 + kap
    Kx = np.zeros((3 * nl, 3 * nl))
    trials = [(Nm, 0) for Nm in N] + [(0, Nm) for Nm in N]
    for col, (dx_, dy_) in enumerate(trials):
        ed = strain(dx_, dy_)
        sd = stress(ed)
        for k, Nk in enumerate(N):
            Kx[k, col] = integ(g_jac * ddot(sd, strain(Nk, 0)))
            Kx[nl + k, col] = integ(g_jac * ddot(sd, strain(0, Nk)))
            Kx[2 * nl + k, col] = integ((1 - kap) * 2 * phi * ddot(sd, eu) * Nk
                                        + 2 * pr * phi * (ed[0] + ed[1]) * Nk)
    for m_, Nm in enumerate(N):
        for k, Nk in enumerate(N):
            Kx[2 * nl + k, 2 * nl + m_] = integ(
                (1 - kap) * Nm * Sval * Nk + 2 * pr * Nm * divu * Nk + Gc / ell * Nm * Nk
                + Gc * ell * (s.diff(Nm, x) * s.diff(Nk, x) + s.diff(Nm, y) * s.diff(Nk, y)))

    from oracle.assemble import element_residual
    prm = Params(E=2.5, nu=0.3, Gc=1.7, pressure=0.4, kappa=0.05, ell=0.35)
    el = Element(p)
    cs = CellSet(el, np.array([0.7]), np.arange(nl)[None, :])

    def nodal(f):
        return np.array([[float(f.subs({x: pts[a], y: pts[b]})) for b in range(p + 1)
                          for a in range(p + 1)]])
    vux, vuy, vph = nodal(ux), nodal(uy), nodal(phi)
    Rloc = element_residual(cs, prm, vux, vuy, vph, nodal(phit_res)).reshape(-1)
    Kloc = element_jacobian(cs, prm, vux, vuy, vph, nodal(s.Integer(1) * phit_jac))[0]
    # the energy term is a substantial part of the phase-field rows here
    e_part = np.array([integ((1 - kap) * phi * Sval * Nk) for Nk in N])
    assert np.abs(e_part).max() > 0.05 * np.abs(Rx[2 * nl:]).max()
    assert np.allclose(Rloc, Rx, rtol=1e-13, atol=1e-13 * np.abs(Rx).max())
    assert np.allclose(Kloc, Kx, rtol=1e-13, atol=1e-13 * np.abs(Kx).max())


# ------------------------------------------------ level active sets ---
def _level_sets(hier, mesh, active_xy):
    act = np.zeros(mesh.n_nodes, bool)
    for X, Y in active_xy:
        act[mesh.node_at(X, Y)] = True
    acts = hier.level_active(act)
    return [{(int(lv.NX[i]), int(lv.NY[i])) for i in np.flatnonzero(a)}
            for lv, a in zip(hier.levels, acts)]


def test_level_active_sets_by_hand_q1():
    """Sec. 3.2, last paragraph: a level unknown of the phase field is frozen
    if any finer unknown it interacts with is active. Mesh: 8 x 8 base cells
    (level 1, edge 2 lattice units; level 0 has edge 4) with the central 2 x 2
    block refined once (level 2, edge 1, lattice square [6, 10]^2). The bilinear
    prolongation couples a fine node to the 1, 2 or 4 vertices of its parent
    cell (coinciding node, edge midpoint, cell centre). A level node stays
    free where a leaf cell of that level owns it (its home, reading R19).
    The expected sets below are listed by hand from those stencils."""
    mesh = Mesh(8, 1, 1, coarse=4, band=(3.0, 3.0))
    hier = Hierarchy(mesh)
    assert [lv.S for lv in hier.levels] == [4, 2, 1]
    # (7, 7): interior fine node, home level 2. On level 1 it is the centre of
    # the refined cell [6, 8]^2, whose vertices (6, 6), (8, 6), (6, 8) are nodes
    # of unrefined level-1 leaf cells (home, keep their own inactive flag), and
    # (8, 8), which belongs to refined cells only and is frozen; on level 0 the
    # frozen (8, 8) is a coarse vertex and freezes only itself.
    sets = _level_sets(hier, mesh, [(7, 7)])
    assert sets == [{(8, 8)}, {(8, 8)}, {(7, 7)}]
    # (8, 7): fine edge midpoint between (8, 6) and (8, 8) on level 1; (8, 6)
    # is home on level 1 (cell [6, 8] x [4, 6] is a leaf), (8, 8) is frozen.
    sets = _level_sets(hier, mesh, [(8, 7)])
    assert sets == [{(8, 8)}, {(8, 8)}, {(8, 7)}]
    # (6, 4): a leaf node of the unrefined region, home level 1 (keeps its flag
    # there); it is the midpoint of the level-0 edge from (4, 4) to (8, 4).
    sets = _level_sets(hier, mesh, [(6, 4)])
    assert sets == [{(4, 4), (8, 4)}, {(6, 4)}, set()]
    # (10, 10): corner of the refined square, on level 2 but on its refinement
    # edge; home level 1 (leaf cells there). Level 2 has no finer level and
    # takes the leaf flag at the position; level 0 gets the coarse cell centre
    # stencil of the level-1 node (10, 10) inside [8, 12]^2: the node lies at
    # (1/2, 1/2) of that cell, so all four vertices.
    sets = _level_sets(hier, mesh, [(10, 10)])
    assert sets == [{(8, 8), (12, 8), (8, 12), (12, 12)}, {(10, 10)}, {(10, 10)}]


def test_level_active_sets_by_hand_q2():
    """The same rule for Q2 (lattice doubled: level edges 8, 4, 2; refined
    square [12, 20]^2). A fine node at a quarter point of its parent cell has
    non-zero 1-D Lagrange weights 3/8, 3/4, -1/8 at all three parent nodes, so
    it couples to all nine."""
    mesh = Mesh(8, 1, 2, coarse=4, band=(3.0, 3.0))
    hier = Hierarchy(mesh)
    assert [lv.S for lv in hier.levels] == [8, 4, 2]
    sets = _level_sets(hier, mesh, [(13, 13)])
    # level 1: the nine nodes of the refined cell [12, 16]^2, minus those on
    # x = 12 or y = 12, which belong to unrefined level-1 leaf cells (home)
    lvl1 = {(14, 14), (16, 14), (14, 16), (16, 16)}
    # level 0: (14, 14) sits at (3/4, 3/4) of [8, 16]^2 and couples to all nine
    # of its nodes; (16, 14), (14, 16), (16, 16) couple to subsets of them
    lvl0 = {(a, b) for a in (8, 12, 16) for b in (8, 12, 16)}
    assert sets == [lvl0, lvl1, {(13, 13)}]


@pytest.mark.parametrize("p", [1, 2])
def test_row_sampled_operators_equal_full_assembly(p, tiny_mesh_factory):
    """The row-sampled forms used for spot checks at sizes the full assembly
    cannot reach (rows of J~ src, of J~^T src and of R) equal the same rows
    of the fully assembled definitions, for rows of every node class (free,
    Dirichlet, hanging, active, masters of hanging nodes)."""
    m = tiny_mesh_factory(p)
    lp = LeafProblem(m, Params(ell=0.3, kappa=1e-3, pressure=0.3))
    U, phit = _state(m, lp)
    act = inputs.bernoulli_mask(m.NX, m.NY, 2, 0.2) & ~m.hanging
    n = m.n_nodes
    src = inputs.random_vector(m.NX, m.NY, 5)
    masters = sorted({mm for lst in m.hanging_constraints.values() for mm, _ in lst})
    nodes = np.unique(np.concatenate([np.flatnonzero(m.hanging)[:6], np.flatnonzero(m.dirichlet)[:6],
                                      np.flatnonzero(act)[:6], masters[:6], np.arange(0, n, max(1, n // 25))]))
    rows = np.concatenate([nodes + k * n for k in range(3)])
    Jt = lp.masked_operator(U, phit, act)
    assert np.abs(lp.masked_rows(rows, src, U, phit, act) - (Jt @ src)[rows]).max() <= 1e-13 * np.abs(Jt @ src).max()
    JT = Jt.T.tocsr() @ src
    assert np.abs(lp.masked_rows(rows, src, U, phit, act, transpose=True) - JT[rows]).max() <= 1e-13 * np.abs(JT).max()
    R = lp.residual(U, phit)
    assert np.abs(lp.residual_rows(rows, U, phit) - R[rows]).max() <= 1e-13 * np.abs(R).max()


@pytest.mark.parametrize("p", [1, 2])
def test_block_triangular_with_exact_blocks_inverts_the_jacobian(p, tiny_mesh_factory):
    """The Jacobian is lower block triangular (the u-equation uses phi~), so
    forward substitution with exact diagonal-block solves is its exact
    inverse, and backward substitution that of its transpose; the
    block-diagonal form is not (the coupling block is dropped)."""
    import scipy.sparse.linalg as spla
    from oracle.mg import block_triangular_apply
    mesh = tiny_mesh_factory(p)
    n = mesh.n_nodes
    X = -10 + 20 * mesh.NX / mesh.M
    Y = -10 + 20 * mesh.NY / mesh.M
    prm = Params(pressure=1e-2, kappa=1e-3, ell=0.5)
    lp = LeafProblem(mesh, prm)
    ux, uy, ph = inputs.sneddon_state(mesh.NX, mesh.NY, mesh.M, p, seed=3, u_std=1e-2)
    U = lp.distribute(np.concatenate([ux, uy, ph]))
    phit = lp.distribute(0.9 * ph + 0.05)
    act = inputs.bernoulli_mask(mesh.NX, mesh.NY, 2, 0.1) & ~mesh.hanging
    J = lp.masked_operator(U, phit, act).tocsc()
    Jd = lp.masked_operator(U, phit, act, blocks="diag").tocsc()
    assert abs(J[2 * n:, :2 * n]).max() > 1e-6          # a genuine coupling block
    assert abs(J[:2 * n, 2 * n:]).max() == 0.0           # none above the diagonal
    lu = spla.splu(Jd)
    v = inputs.random_vector(mesh.NX, mesh.NY, 7)
    x = block_triangular_apply(lu.solve, J, J @ v, n)
    assert np.abs(x - v).max() <= 1e-9 * np.abs(v).max()
    xt = block_triangular_apply(lambda w: lu.solve(w, trans="T"), J, J.T @ v, n, transpose=True)
    assert np.abs(xt - v).max() <= 1e-9 * np.abs(v).max()
    xd = lu.solve(J @ v)
    assert np.abs(xd - v).max() > 1e-6 * np.abs(v).max()
