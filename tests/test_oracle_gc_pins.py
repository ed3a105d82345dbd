"""Pins of the global-coarsening multigrid oracle (oracle/gc.py) against
facts fixed by the mathematics: cut meshes are 2:1 balanced with hanging
interpolation exact for Q_p polynomials, interpolation between levels
reproduces global polynomials, the rediscretised level operators equal the
Galerkin products at constant coefficients (nested conforming spaces, exact
quadrature), the V-cycle equals the literal multiplicative subspace
correction there, the cycle is symmetric, GMRES with it reaches the direct
solution, and level active sets listed by hand from the stencils."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import inputs
from oracle.assemble import LeafProblem, Params
from oracle.gc import GCVCycle, GlobalHierarchy, truncated_mesh
from oracle.krylov import gmres
from oracle.mesh import Mesh
from oracle.mg import MGParams

_gh = {}


def hier(tiny_mesh_factory, p):
    if p not in _gh:
        _gh[p] = GlobalHierarchy(tiny_mesh_factory(p))
    return _gh[p]


@pytest.mark.parametrize("p", [1, 2])
def test_cut_meshes(p, tiny_mesh_factory):
    mesh = tiny_mesh_factory(p)
    gh = hier(tiny_mesh_factory, p)
    assert gh.meshes[-1] is mesh
    for k, m in enumerate(gh.meshes):
        assert m.cell_level.max() <= k
        # 2:1 face balance
        for (l, i, j) in m.leaves:
            n = m.ncells_1d(l)
            for di, dj in Mesh.DIRS:
                ni, nj = i + di, j + dj
                if 0 <= ni < n and 0 <= nj < n:
                    f = m.find_leaf(l, ni, nj)
                    assert f is None or f[0] >= l - 1
        # levels up to the base mesh are uniform: (N p + 1)^2 nodes, no hanging
        if k <= m.b:
            N = m.ncells_1d(k)
            assert m.n_nodes == (N * p + 1) ** 2 and not m.hanging.any()
        # hanging interpolation of the cut mesh is exact for Q_p polynomials
        X = -10 + 20 * m.NX / m.M
        Y = -10 + 20 * m.NY / m.M
        lp = LeafProblem(m, Params())
        for f in (X, X * Y) + ((X ** 2 * Y,) if p == 2 else ()):
            v = f.copy()
            v[m.hanging] = 1e3
            assert np.allclose(lp.distribute(v), f, atol=1e-10)
    assert any(m.hanging.any() for m in gh.meshes[:-1])   # some coarser level is locally refined


@pytest.mark.parametrize("p", [1, 2])
def test_interpolation_reproduces_polynomials(p, tiny_mesh_factory):
    gh = hier(tiny_mesh_factory, p)
    for k in range(1, len(gh.meshes)):
        f, c = gh.meshes[k], gh.meshes[k - 1]
        for fn in (lambda X, Y: 1 + 0 * X, lambda X, Y: 2 * X - Y, lambda X, Y: X * Y) + \
                ((lambda X, Y: X ** 2 * Y - Y ** 2,) if p == 2 else ()):
            vc = fn(c.NX / c.M, c.NY / c.M)
            vf = fn(f.NX / f.M, f.NY / f.M)
            assert np.allclose(gh.I[k] @ vc, vf, atol=1e-12)


def _const_cycle(gh, p, mgp):
    mesh = gh.mesh
    n = mesh.n_nodes
    prm = Params(ell=0.5, kappa=1e-3)
    return GCVCycle(gh, prm, mgp, np.zeros(3 * n), np.full(n, 0.7), np.zeros(n, bool)), prm


@pytest.mark.parametrize("p", [1, 2])
def test_level_operators_are_galerkin_at_constant_coefficients(p, tiny_mesh_factory):
    """u = 0, phi~ constant, no active set: the rediscretised operator of every
    level equals P^T A~ P of the next finer one on the free unknowns."""
    gh = hier(tiny_mesh_factory, p)
    vc, _ = _const_cycle(gh, p, MGParams())
    for k in range(1, len(gh.meshes)):
        fine, coarse = vc.ops[k], vc.ops[k - 1]
        G = (vc.P[k].T @ fine.A @ vc.P[k]).toarray()
        Ac = coarse.A.toarray()
        fr = np.flatnonzero(coarse.free)
        sub = Ac[np.ix_(fr, fr)]
        assert np.abs(G[np.ix_(fr, fr)] - sub).max() <= 1e-12 * np.abs(sub).max(), k


@pytest.mark.parametrize("p", [1, 2])
def test_vcycle_equals_multiplicative_subspace_correction(p, tiny_mesh_factory):
    """With Galerkin level operators the V-cycle is the multiplicative
    subspace correction x += E_k S_k E_k^T (b - A x) over the level spaces,
    E_k = P_L ... P_(k+1) the explicit embedding of level k into the leaf."""
    gh = hier(tiny_mesh_factory, p)
    mesh = gh.mesh
    n = mesh.n_nodes
    vc, prm = _const_cycle(gh, p, MGParams(cheb_degree=3, coarse_its=5))
    lp = LeafProblem(mesh, prm)
    B = lp.masked_operator(np.zeros(3 * n), np.full(n, 0.7), np.zeros(n, bool), blocks="diag")
    free = lp.free_mask(np.zeros(n, bool))
    b = inputs.random_vector(mesh.NX, mesh.NY, 7) * free
    y = vc.apply(b)
    L = len(gh.meshes) - 1
    E = [None] * (L + 1)
    E[L] = sp.identity(3 * n, format="csr")
    for k in range(L - 1, -1, -1):
        E[k] = (E[k + 1] @ vc.P[k + 1]).tocsr()
    x = np.zeros(3 * n)

    def corr(k, x, coarse=False):
        r = E[k].T @ (free * (b - B @ x))
        s = vc.coarse_solve(r) if coarse else vc.chebyshev(k, r, None, 3)
        return x + E[k] @ s
    for k in range(L, 0, -1):
        x = corr(k, x)
    x = corr(0, x, coarse=True)
    for k in range(1, L + 1):
        x = corr(k, x)
    assert np.abs(x - y * free).max() <= 1e-12 * np.abs(y).max()
    assert np.array_equal(y[~free], b[~free])


@pytest.mark.parametrize("p", [1, 2])
def test_vcycle_symmetric_and_gmres_direct(p, tiny_mesh_factory):
    gh = hier(tiny_mesh_factory, p)
    mesh = gh.mesh
    n = mesh.n_nodes
    prm = Params(ell=0.4, kappa=1e-3, pressure=0.2)
    lp = LeafProblem(mesh, prm)
    ux, uy, phi = inputs.sneddon_state(mesh.NX, mesh.NY, mesh.M, p, seed=0, u_std=0.01)
    U = np.concatenate([ux, uy, phi])
    U[:2 * n][np.concatenate([mesh.dirichlet] * 2)] = 0.0
    U = lp.distribute(U)
    phit = lp.distribute(0.9 * phi + 0.05)
    act = inputs.bernoulli_mask(mesh.NX, mesh.NY, 2, 0.1) & ~mesh.hanging
    vc = GCVCycle(gh, prm, MGParams(coarse_mode="cheb", coarse_its=8), U, phit, act)
    free = lp.free_mask(act)
    a = inputs.random_vector(mesh.NX, mesh.NY, 11) * free
    c = inputs.random_vector(mesh.NX, mesh.NY, 12) * free
    lhs, rhs = c @ vc.apply(a), a @ vc.apply(c)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    J = lp.masked_operator(U, phit, act)
    b = inputs.random_vector(mesh.NX, mesh.NY, 6) * free
    x, info = gmres(lambda v: J @ v, vc.apply, b, 1e-13 * np.linalg.norm(b))
    xd = spla.spsolve(J.tocsc(), b)
    assert info.converged and np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_level_active_sets_by_hand():
    """Q1, 8 x 8 base cells (level 1, edge 2 lattice units; level 0 edge 4)
    with the central 2 x 2 block refined (level 2, lattice square [6, 10]^2).
    An active leaf unknown at (7, 7) is the centre of the level-1 cell
    [6, 8]^2: its bilinear interpolation reaches the four vertices, all frozen
    on level 1 (no home-level exception: the finest level smooths every free
    leaf unknown); on level 0, (6, 6) is the centre of [4, 8]^2, (8, 6) and
    (6, 8) edge midpoints and (8, 8) a vertex, which together reach the four
    vertices of [4, 8]^2."""
    mesh = Mesh(8, 1, 1, coarse=4, band=(3.0, 3.0))
    gh = GlobalHierarchy(mesh)
    act = np.zeros(mesh.n_nodes, bool)
    act[mesh.node_at(7, 7)] = True
    acts = gh.level_active(act)
    sets = [{(int(m.NX[i]), int(m.NY[i])) for i in np.flatnonzero(a)} for m, a in zip(gh.meshes, acts)]
    assert sets[2] == {(7, 7)}
    assert sets[1] == {(6, 6), (8, 6), (6, 8), (8, 8)}
    assert sets[0] == {(4, 4), (8, 4), (4, 8), (8, 8)}
    # level 1 here is the uniform base mesh, level 0 the coarse grid
    assert not gh.meshes[1].hanging.any() and gh.meshes[1].n_nodes == 81


def test_truncation_of_a_deeper_mesh_has_hanging_nodes():
    """Two local levels: the cut at the first local level is itself locally
    refined and constrained (the level meshes of global coarsening carry
    hanging nodes, unlike the levels of local smoothing)."""
    mesh = Mesh(16, 2, 2, coarse=4, band=(3.0, 1.0))
    m = truncated_mesh(mesh, mesh.lmax - 1)
    assert m.hanging.sum() > 0 and m.n_nodes < mesh.n_nodes


@pytest.mark.parametrize("p", [1, 2])
def test_coarse_hanging_values_reach_only_fine_hanging_rows(p, tiny_mesh_factory):
    """In a 2:1-balanced tree a cell next to a coarser leaf is never refined
    further, so the interpolation reads a coarse hanging node only at fine
    nodes at the same place, which are hanging too: I_k C_(k-1) and I_k agree
    on every free fine row (the transfers need no constraint step)."""
    gh = hier(tiny_mesh_factory, p)
    for k in range(1, len(gh.meshes)):
        D = (gh.I[k] @ gh.C[k - 1] - gh.I[k]).tocsr()
        rows = np.flatnonzero(np.abs(D).sum(axis=1).A.ravel() > 0)
        assert np.all(gh.meshes[k].hanging[rows]), k
        cols = np.flatnonzero(np.abs(gh.I[k]).sum(axis=0).A.ravel() > 0)
        hc = np.flatnonzero(gh.meshes[k - 1].hanging)
        reach = np.flatnonzero(np.abs(gh.I[k][:, hc]).sum(axis=1).A.ravel() > 0)
        assert np.all(gh.meshes[k].hanging[reach]), k
        assert cols.size > 0


@pytest.mark.parametrize("p", [1, 2])
def test_level_state_is_a_level_function(p):
    """The linearisation state of a level is a function of that level's space:
    the leaf values at its regular nodes and the constraint at its own
    hanging nodes. In a 2:1 tree a hanging node of a cut mesh sits between a
    leaf and the finer leaves next to it, so it is a hanging node of the leaf
    mesh with the same masters: for a conforming leaf state the injected value
    already is the constrained one; a leaf field with free values at hanging
    nodes is corrected."""
    mesh = Mesh(16, 2, p, coarse=4, band=(3.0, 1.0))
    gh = GlobalHierarchy(mesh)
    n = mesh.n_nodes
    X = -10 + 20 * mesh.NX / mesh.M
    Y = -10 + 20 * mesh.NY / mesh.M
    lp = LeafProblem(mesh, Params())
    phit_raw = np.cos(0.7 * X) * np.exp(0.3 * Y)
    phit_raw[mesh.hanging] += 0.25     # not a leaf function
    U = np.concatenate([lp.distribute(np.sin(0.5 * X + 0.2 * Y)), lp.distribute(np.cos(0.4 * Y) * X),
                        lp.distribute(phit_raw)])
    vc = GCVCycle(gh, Params(), MGParams(), U, phit_raw, np.zeros(n, bool), eigen=None)
    seen = 0
    for k, m in enumerate(gh.meshes):
        li = gh.leaf_index[k]
        lpk = LeafProblem(m, Params())
        reg = ~m.hanging
        assert np.all(mesh.hanging[li[m.hanging]]), k   # level hanging => leaf hanging
        for comp, (got, leaf) in enumerate(zip(vc.states[k], (U[:n], U[n:2 * n], phit_raw))):
            raw = leaf[li]
            assert np.array_equal(got[reg], raw[reg])
            assert np.allclose(got, lpk.distribute(raw), rtol=0, atol=1e-14)
            if m.hanging.any():
                if comp < 2:
                    assert np.allclose(got[m.hanging], raw[m.hanging], rtol=0, atol=1e-13), k
                else:
                    assert np.abs(got[m.hanging] - raw[m.hanging]).min() > 0.1, k
                    seen += 1
    assert seen >= 2
