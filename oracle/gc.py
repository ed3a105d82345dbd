"""Global-coarsening geometric multigrid for the block-diagonal preconditioner
(oracle). Test infrastructure only.

The alternative to the local smoothing of Sec. 3.2 that Sec. 1 cites from the
matrix-free locally-refined literature: every multigrid level is a complete
mesh of the domain. Level k is the quadtree cut off at depth k (leaves finer
than k are replaced by their level-k ancestor; coarser leaves stay), so it
has hanging nodes of its own wherever it is locally refined, and the finest
level is the leaf mesh itself. There is no refinement edge and no copy
between leaf and levels: the smoother of level k acts on all of level k's
unknowns with that level's hanging-node constraints.

Per level (all assembled here, plainly):
  A_k   the block-diagonal operator diag(G_uu, G_phiphi) of Sec. 3.2 on the
        cells of level k with the injected state (u_x, u_y, phi~ at the same
        lattice point of the leaf mesh, then constrained at the level's own
        hanging nodes so that it is a level function), condensed with the level's hanging
        constraints C_k: A~_k = Mf (C_k^T A_k C_k) Mf + (I - Mf), Mf keeping the
        free unknowns (not Dirichlet for u, not hanging, not level-active for
        phi); the finest level's A~ is the block-diagonal part of J~.
  I_k   interpolation of the level-(k-1) finite-element function at the nodes
        of level k (each fine node evaluated in a coarse cell containing it);
        the prolongation of unknowns is P_k = Mf_k I_k C_(k-1) Mf_(k-1), the
        restriction its transpose.
Level active sets (Sec. 3.2, last paragraph): the finest level takes the
leaf set; a level-(k-1) phase-field unknown is active if the leaf unknown at
its position is or if any level-k unknown its interpolation reaches is. Every
free leaf unknown is smoothed on the finest level, so a coarse level may be
frozen freely (no exception like the home level of local smoothing).

V-cycle (x_k, d_k level vectors, all components):
  d_L = b on free unknowns
  down   k = L..1: x_k = Cheb(d_k, x0 = 0); t = d_k - A~_k x_k on free rows;
         d_(k-1) = P_k^T t
  coarse x_0 = coarse solve of d_0
  up     k = 1..L: x_k += P_k x_(k-1); x_k = Cheb(d_k, x0 = x_k)
  out = x_L on free unknowns, b on constrained ones.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .assemble import Params, assemble_matrix, element_jacobian, kron3
from .fe import Element, basis_1d
from .mesh import Mesh
from .mg import LevelOps, MGParams, block_masks, cg_eigs, chebyshev


def truncated_mesh(mesh: Mesh, k: int) -> Mesh:
    """The quadtree of `mesh` cut off at depth k (same lattice, same band
    parameters): leaves finer than k are replaced by their level-k ancestor.
    A cut of a 2:1-balanced tree is 2:1 balanced."""
    if k >= mesh.lmax:
        return mesh
    m = object.__new__(Mesh)
    for name in ("p", "coarse", "b", "n_local", "lmax", "n_levels", "M", "band"):
        setattr(m, name, getattr(mesh, name))
    leaves = set()
    for (l, i, j) in mesh.leaves:
        leaves.add((l, i, j) if l <= k else (k, i >> (l - k), j >> (l - k)))
    m.leaves = leaves
    m._number_nodes()
    m._find_hanging()
    m.dirichlet = (m.NX == 0) | (m.NX == m.M) | (m.NY == 0) | (m.NY == m.M)
    return m


def interpolation(fine: Mesh, coarse: Mesh) -> sp.csr_matrix:
    """I (n_fine x n_coarse): value of the coarse Q_p function at each fine
    node, evaluated in a coarse leaf cell whose closed box contains the node
    (coarse nodal values with their hanging entries set by the constraints,
    the function is continuous, so any containing cell gives the value)."""
    p = coarse.p
    rows, cols, vals = [], [], []
    for g in range(fine.n_nodes):
        X, Y = int(fine.NX[g]), int(fine.NY[g])
        cell = None
        for l in range(coarse.lmax, -1, -1):
            S = int(coarse.S(l))
            n1 = coarse.ncells_1d(l)
            for i in ([X // S - 1, X // S] if X % S == 0 else [X // S]):
                for j in ([Y // S - 1, Y // S] if Y % S == 0 else [Y // S]):
                    if 0 <= i < n1 and 0 <= j < n1 and (l, i, j) in coarse.leaves:
                        cell = (l, i, j)
                        break
                if cell:
                    break
            if cell:
                break
        assert cell is not None, "fine node outside the coarse mesh"
        l, i, j = cell
        S = int(coarse.S(l))
        vx, _ = basis_1d(p, [(X - i * S) / S])
        vy, _ = basis_1d(p, [(Y - j * S) / S])
        for b in range(p + 1):
            for a in range(p + 1):
                w = vx[0, a] * vy[0, b]
                if w != 0.0:
                    rows.append(g)
                    cols.append(coarse.node_at(i * S + a * S // p, j * S + b * S // p))
                    vals.append(float(w))
    return sp.csr_matrix((vals, (rows, cols)), shape=(fine.n_nodes, coarse.n_nodes))


class GlobalHierarchy:
    """Level meshes 0..L (L = the leaf mesh) and the interpolations between
    consecutive levels."""

    def __init__(self, mesh: Mesh):
        self.mesh = mesh
        self.el = Element(mesh.p)
        L = mesh.lmax
        self.meshes = [truncated_mesh(mesh, k) for k in range(L + 1)]
        self.C = [m.constraint_matrix() for m in self.meshes]
        self.I = [None] + [interpolation(self.meshes[k], self.meshes[k - 1]) for k in range(1, L + 1)]
        # leaf node at each level node's position (every level node is a leaf position)
        self.leaf_index = []
        for m in self.meshes:
            idx = np.array([mesh.node_at(X, Y) for X, Y in zip(m.NX, m.NY)])
            assert np.all(idx != None)  # noqa: E711
            self.leaf_index.append(idx.astype(np.int64))

    def level_active(self, leaf_active):
        """Sec. 3.2: the finest level takes the leaf set; a coarser unknown is
        active if the leaf unknown at its position is, or any unknown of the
        next finer level that its interpolation reaches. Hanging unknowns are
        never active."""
        L = len(self.meshes) - 1
        leaf_active = np.asarray(leaf_active, dtype=bool) & ~self.mesh.hanging
        acts = [None] * (L + 1)
        acts[L] = leaf_active.copy()
        for k in range(L - 1, -1, -1):
            m = self.meshes[k]
            a = leaf_active[self.leaf_index[k]].copy()
            a |= (abs(self.I[k + 1]).T @ acts[k + 1].astype(float)) > 0
            acts[k] = a & ~m.hanging
        return acts


class GCVCycle:
    """Block-diagonal global-coarsening V-cycle for one leaf state and active
    set (same smoother, eigenvalue estimate and coarse solve as the local
    smoothing cycle; level 0 is the same coarse grid)."""

    def __init__(self, gh: GlobalHierarchy, prm: Params, mgp: MGParams, U_leaf, phit_leaf, leaf_active,
                 eigen=None):
        self.gh = gh
        self.prm = prm
        self.mgp = mgp
        n = gh.mesh.n_nodes
        acts = gh.level_active(leaf_active)
        self.ops, self.P = [], [None]
        self.frees = []
        self.states = []
        for k, m in enumerate(gh.meshes):
            li = gh.leaf_index[k]
            # the level's linearisation state is a function of the level's own
            # space: the leaf values at its regular nodes, the constraint at its
            # hanging nodes (C_k on the injected values)
            Ck = gh.C[k]
            ux, uy, pt = Ck @ U_leaf[:n][li], Ck @ U_leaf[n:2 * n][li], Ck @ phit_leaf[li]
            self.states.append((ux, uy, pt))
            from .assemble import leaf_cells
            cs = leaf_cells(m, gh.el)
            g = cs.gather
            Ke = element_jacobian(cs, prm, g(ux), g(uy), np.zeros_like(g(ux)), g(pt), blocks="diag")
            A = assemble_matrix(m.cell_nodes, m.n_nodes, Ke)
            C3 = kron3(gh.C[k])
            fu = ~(m.dirichlet | m.hanging)
            fp = ~(acts[k] | m.hanging)
            free = np.concatenate([fu, fu, fp])
            Mf = sp.diags(free.astype(float))
            At = (Mf @ (C3.T @ A @ C3) @ Mf + sp.diags(1.0 - free.astype(float))).tocsr()
            diag = At.diagonal()
            Dinv = np.where(free, 1.0 / np.where(diag != 0, diag, 1.0), 0.0)
            op = LevelOps(A=At, free=free, Dinv=Dinv)
            op.extra["active"] = acts[k]
            self.ops.append(op)
            self.frees.append(free)
        for k in range(1, len(gh.meshes)):
            Pk = kron3(gh.I[k] @ gh.C[k - 1])
            self.P.append((sp.diags(self.frees[k].astype(float)) @ Pk @
                           sp.diags(self.frees[k - 1].astype(float))).tocsr())
        self.set_eigen(eigen)

    def set_eigen(self, eigen=None):
        """eigen: None (estimate by CG) or (lam_max[levels][2], lam_min0[2])."""
        for k, op in enumerate(self.ops):
            nk = self.gh.meshes[k].n_nodes
            bu, bp = block_masks(nk)
            its_u = self.mgp.coarse_eig_its if k == 0 else self.mgp.eig_cg_its
            its_p = self.mgp.coarse_eig_its if k == 0 else self.mgp.eig_cg_its_phi
            if eigen is None:
                lu = cg_eigs(op.A, op.Dinv, op.free & bu, its_u)
                lp = cg_eigs(op.A, op.Dinv, op.free & bp, its_p)
                op.lam_max = np.array([lu[1], lp[1]])
                op.lam_min = np.array([lu[0], lp[0]])
            else:
                op.lam_max = np.asarray(eigen[0][k], dtype=float)
                op.lam_min = np.asarray(eigen[1], dtype=float) if k == 0 else None

    def eigen(self):
        return ([op.lam_max.copy() for op in self.ops], self.ops[0].lam_min.copy())

    def interval(self, k):
        op = self.ops[k]
        if k == 0 and self.mgp.coarse_mode == "cheb":
            return op.lam_min, self.mgp.upper_factor * op.lam_max
        return self.mgp.smooth_range * op.lam_max, self.mgp.upper_factor * op.lam_max

    def chebyshev(self, k, b, x0, degree):
        op = self.ops[k]
        nk = self.gh.meshes[k].n_nodes
        lo, hi = self.interval(k)
        th, de = 0.5 * (hi + lo), 0.5 * (hi - lo)
        theta = np.concatenate([np.full(2 * nk, th[0]), np.full(nk, th[1])])
        delta = np.concatenate([np.full(2 * nk, de[0]), np.full(nk, de[1])])
        return chebyshev(op.A, op.Dinv, op.free, b, x0, degree, theta, delta)

    def coarse_solve(self, b):
        op = self.ops[0]
        if self.mgp.coarse_mode == "cheb":
            return self.chebyshev(0, b, None, self.mgp.coarse_its)
        if self.mgp.coarse_mode == "exact":
            import scipy.sparse.linalg as spla
            idx = np.flatnonzero(op.free)
            x = np.zeros_like(b)
            x[idx] = spla.spsolve(op.A[idx][:, idx].tocsc(), b[idx])
            return x
        if self.mgp.coarse_mode == "cg":
            n0 = self.gh.meshes[0].n_nodes
            x = np.zeros(3 * n0)
            for blk in block_masks(n0):
                msk = (op.free & blk).astype(float)
                r = b * msk
                z = op.Dinv * r
                pv = z.copy()
                rz = r @ z
                for _ in range(self.mgp.coarse_its):
                    if rz == 0:
                        break
                    q = (op.A @ pv) * msk
                    alpha = rz / (pv @ q)
                    x = x + alpha * pv
                    r = r - alpha * q
                    z = op.Dinv * r
                    rz_new = r @ z
                    pv = z + (rz_new / rz) * pv
                    rz = rz_new
            return x
        raise ValueError(self.mgp.coarse_mode)

    def apply(self, b_leaf):
        L = len(self.ops) - 1
        kdeg = self.mgp.cheb_degree
        d = [None] * (L + 1)
        x = [None] * (L + 1)
        d[L] = np.where(self.frees[L], b_leaf, 0.0)
        for k in range(L, 0, -1):
            x[k] = self.chebyshev(k, d[k], None, kdeg)
            t = np.where(self.frees[k], d[k] - self.ops[k].A @ x[k], 0.0)
            d[k - 1] = self.P[k].T @ t
        x[0] = self.coarse_solve(d[0])
        for k in range(1, L + 1):
            x[k] = x[k] + self.P[k] @ x[k - 1]
            x[k] = self.chebyshev(k, d[k], x[k], kdeg)
        return np.where(self.frees[L], x[L], b_leaf)
