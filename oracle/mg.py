"""Local-smoothing geometric multigrid for the block-diagonal preconditioner
(oracle). Test infrastructure only.

Sec. 3.2: P^{-1} = diag(MG(G_uu), MG(G_phiphi)), one V-cycle per SPD diagonal
block of the Jacobian; Chebyshev-accelerated Jacobi smoothing on levels > 0
over [0.08 lambda_max, 1.2 lambda_max]; on level 0 both extreme eigenvalues
are estimated and the Chebyshev iteration is used as the coarse solver; the
eigenvalues come from a conjugate gradient run. Local smoothing (Janssen &
Kanschat): level l consists of all cells of refinement level l and the smoother
acts only there, with the refinement edge held fixed, so hanging nodes never
appear on a level. Boundary constraints go to every level unchanged; a level
unknown of the phase field is inactive only if all fine unknowns it interacts
with are inactive (Sec. 3.2, last paragraph), except on the home level of a
free leaf unknown (see Hierarchy.level_active).

The two blocks share their level structure, so a level vector holds all three
components: [u_x | u_y | phi]; the u block is the first two components.

V-cycle sequence (all matrices assembled; x_l, d_l are level vectors):
  copy:   d_m[i] = b[g] for each free leaf unknown g, m = coarsest level of
          the leaf cells that own g (g is never on m's refinement edge)
  down:   x_l = Cheb(d_l, x0 = 0) on the free unknowns of level l
          t_l = d_l - A_l x_l on every row (the refinement edge included) except
          Dirichlet and level-active rows, which are zero
          d_{l-1} += P_l^T t_l
  coarse: x_0 = coarse solve of d_0
  up:     x_l += P_l x_{l-1}, then zero on Dirichlet and level-active unknowns
          (edge values of x_l now hold the coarse correction); with the zeroed
          residual rows above, restriction and prolongation stay transposes of
          each other, so the cycle stays symmetric
          x_l = Cheb(d_l, x0 = x_l): residual d_l - A_l x_l over free rows,
          only free entries updated
  back:   out[g] = x_m[i] for free leaf unknowns, out = b on constrained ones.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
from scipy.linalg import eigh_tridiagonal

from .assemble import CellSet, Params, assemble_matrix, element_jacobian, kron3
from .fe import Element
from .mesh import Mesh


@dataclass
class MGParams:
    cheb_degree: int = 3        # number of Chebyshev updates per smoothing
    smooth_range: float = 0.08  # lower end of the interval as a fraction of lambda_max
    upper_factor: float = 1.2   # upper end: factor on lambda_max
    eig_cg_its: int = 20        # CG iterations for the displacement block's estimate (levels > 0)
    eig_cg_its_phi: int = 10    # CG iterations for the phase-field block's estimate (levels > 0)
    coarse_mode: str = "cheb"   # 'cheb' (Sec. 3.2) or 'cg'
    coarse_its: int = 30        # coarse Chebyshev degree or CG iterations
    coarse_eig_its: int = 40    # CG iterations for the coarse eigenvalue estimate


class Level:
    """Mesh of all cells of one refinement level."""

    def __init__(self, mesh: Mesh, level: int, el: Element):
        self.level = level
        p = mesh.p
        cells = np.array(sorted(mesh.level_cells(level)), dtype=np.int64).reshape(-1, 3)
        self.ci, self.cj = cells[:, 1], cells[:, 2]
        self.cellset_keys = {(int(i), int(j)) for i, j in zip(self.ci, self.cj)}
        S = int(mesh.S(level))
        self.S = S
        a = np.tile(np.arange(p + 1), p + 1)
        b = np.repeat(np.arange(p + 1), p + 1)
        X = self.ci[:, None] * S + a[None, :] * (S // p)
        Y = self.cj[:, None] * S + b[None, :] * (S // p)
        keys = Y * (mesh.M + 1) + X
        uniq, inv = np.unique(keys.ravel(), return_inverse=True)
        self.cell_nodes = inv.reshape(keys.shape)
        self.NX = uniq % (mesh.M + 1)
        self.NY = uniq // (mesh.M + 1)
        self.n = uniq.size
        self.key_to_node = {int(k): i for i, k in enumerate(uniq)}
        self.H = np.full(self.ci.size, float(mesh.H(level)))
        self.cells = CellSet(el, self.H, self.cell_nodes)
        M = mesh.M
        self.dirichlet = (self.NX == 0) | (self.NX == M) | (self.NY == 0) | (self.NY == M)
        # refinement edge: a level node next to a region with no level cell
        ncell = mesh.ncells_1d(level)
        edge = np.zeros(self.n, dtype=bool)
        for k in range(self.n):
            X, Y = int(self.NX[k]), int(self.NY[k])
            cand_i = [X // S - 1, X // S] if X % S == 0 else [X // S]
            cand_j = [Y // S - 1, Y // S] if Y % S == 0 else [Y // S]
            for ii in cand_i:
                for jj in cand_j:
                    if 0 <= ii < ncell and 0 <= jj < ncell and (ii, jj) not in self.cellset_keys:
                        edge[k] = True
        self.edge = edge
        # leaf node at the same position (every level node is a leaf position)
        self.leaf_index = np.array([mesh.node_at(X, Y) for X, Y in zip(self.NX, self.NY)])
        assert np.all(self.leaf_index != None)  # noqa: E711
        self.leaf_index = self.leaf_index.astype(np.int64)
        # nodes of level cells that are leaves
        leafcell = np.array([(level, int(i), int(j)) in mesh.leaves for i, j in zip(self.ci, self.cj)])
        self.leafcell_node = np.zeros(self.n, dtype=bool)
        self.leafcell_node[self.cell_nodes[leafcell].ravel()] = True


def prolongation(mesh: Mesh, fine: Level, coarse: Level) -> sp.csr_matrix:
    """P (n_fine x n_coarse): value of the coarse Q_p function at each fine node,
    evaluated in the parent cell (exact interpolation of nested spaces)."""
    from .fe import basis_1d
    p = mesh.p
    Sf, Sc = fine.S, coarse.S
    entries = {}
    for c in range(fine.ci.size):
        pi, pj = int(fine.ci[c]) >> 1, int(fine.cj[c]) >> 1
        # parent's nodes
        pn = [coarse.key_to_node[(pj * Sc + b * Sc // p) * (mesh.M + 1) + pi * Sc + a * Sc // p]
              for b in range(p + 1) for a in range(p + 1)]
        for k, node in enumerate(fine.cell_nodes[c]):
            X, Y = int(fine.NX[node]), int(fine.NY[node])
            sx = (X - pi * Sc) / Sc
            sy = (Y - pj * Sc) / Sc
            vx, _ = basis_1d(p, [sx])
            vy, _ = basis_1d(p, [sy])
            for b in range(p + 1):
                for a in range(p + 1):
                    w = vx[0, a] * vy[0, b]
                    if w != 0.0:
                        entries[(int(node), pn[a + (p + 1) * b])] = float(w)
    rows = [r for r, _ in entries]
    cols = [c for _, c in entries]
    vals = list(entries.values())
    return sp.csr_matrix((vals, (rows, cols)), shape=(fine.n, coarse.n))


@dataclass
class LevelOps:
    A: sp.csr_matrix = None          # full level block operator (all rows/cols)
    free: np.ndarray = None          # free unknowns (3 n_l)
    Dinv: np.ndarray = None          # 1/diag on free unknowns, 0 elsewhere
    lam_max: np.ndarray = None       # per block (u, phi)
    lam_min: np.ndarray = None
    extra: dict = field(default_factory=dict)


class Hierarchy:
    """Levels 0..lmax with transfers and the leaf-to-level copy map."""

    def __init__(self, mesh: Mesh):
        self.mesh = mesh
        self.el = Element(mesh.p)
        self.levels = [Level(mesh, l, self.el) for l in range(mesh.n_levels)]
        self.P = [None] + [prolongation(mesh, self.levels[l], self.levels[l - 1])
                           for l in range(1, mesh.n_levels)]
        self.P3 = [None] + [kron3(P) for P in self.P[1:]]
        # copy map: m0 = min level of leaf cells owning the node
        n = mesh.n_nodes
        m0 = np.full(n, 10 ** 6, dtype=np.int64)
        for c in range(mesh.n_cells):
            lv = int(mesh.cell_level[c])
            nodes = mesh.cell_nodes[c]
            m0[nodes] = np.minimum(m0[nodes], lv)
        self.copy_level = m0
        self.copy_index = np.full(n, -1, dtype=np.int64)
        for g in range(n):
            if mesh.hanging[g]:
                continue
            lvl = self.levels[int(m0[g])]
            key = int(mesh.NY[g]) * (mesh.M + 1) + int(mesh.NX[g])
            i = lvl.key_to_node[key]
            assert not lvl.edge[i]
            self.copy_index[g] = i

    def level_active(self, leaf_active):
        """Level active sets (Sec. 3.2: a level unknown is inactive only if all
        fine unknowns it interacts with are inactive). Reading: on every level a
        node is active if the leaf unknown at its position is active or if any
        finer-level unknown in its prolongation stencil is active, except on the
        one level where a free leaf unknown is copied to and from (its home):
        there it keeps its own flag. Without that exception a free unknown next
        to an active one is frozen on every level that holds it and the
        V-cycle maps it to zero for every input (a singular preconditioner)."""
        L = len(self.levels) - 1
        leaf_active = np.asarray(leaf_active, dtype=bool) & ~self.mesh.hanging
        acts = [None] * (L + 1)
        for l in range(L, -1, -1):
            lv = self.levels[l]
            own = leaf_active[lv.leaf_index]
            a = own.copy()
            if l < L:
                Pabs = abs(self.P[l + 1])
                a |= (Pabs.T @ acts[l + 1].astype(float)) > 0
            home = lv.leafcell_node & ~lv.edge
            a = np.where(home, own, a)
            acts[l] = a
        return acts


def cg_eigs(A, Dinv, free, its):
    """Extreme Ritz values of Dinv A on the free unknowns from `its` Jacobi-
    preconditioned CG steps on A x = 1 (Lanczos tridiagonal from the CG
    coefficients). Returns (lam_min, lam_max)."""
    idx = np.flatnonzero(free)
    if idx.size == 0:
        return 1.0, 1.0
    Af = A[idx][:, idx]
    d = Dinv[idx]
    r = np.ones(idx.size)
    z = d * r
    pvec = z.copy()
    rz = r @ z
    rz0 = rz
    alphas, betas = [], []
    # at most `its` steps and never more than the number of unknowns; stop
    # once the residual has dropped by 1e-12 (later Lanczos steps only add
    # spurious Ritz values)
    for _ in range(min(its, idx.size)):
        q = Af @ pvec
        pq = pvec @ q
        if pq <= 0 or rz == 0:
            break
        alpha = rz / pq
        r = r - alpha * q
        z = d * r
        rz_new = r @ z
        beta = rz_new / rz
        alphas.append(alpha)
        betas.append(beta)
        pvec = z + beta * pvec
        rz = rz_new
        if rz <= 1e-24 * rz0:
            break
    k = len(alphas)
    diag = np.array([1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
                     for j in range(k)])
    off = np.array([np.sqrt(betas[j]) / alphas[j] for j in range(k - 1)])
    ev = eigh_tridiagonal(diag, off, eigvals_only=True) if k > 1 else diag
    return float(ev.min()), float(ev.max())


def block_masks(n):
    u = np.zeros(3 * n, dtype=bool)
    u[:2 * n] = True
    return u, ~u


def chebyshev(A, Dinv, free, b, x0, degree, theta, delta):
    """Chebyshev acceleration of Jacobi (Saad, Iterative Methods for Sparse
    Linear Systems, 2nd ed., Alg. 12.1, applied to D^{-1} A) on the free
    unknowns. theta, delta: centre and half-width of the eigenvalue interval
    (arrays per unknown so that each block has its own). `degree` updates of x;
    the residual is formed from its definition b - A x before every update
    after the first, and only free entries of x change."""
    f = free
    if x0 is None:
        x = np.zeros(b.size)
        r = np.where(f, b, 0.0)
    else:
        x = x0.copy()
        r = np.where(f, b - A @ x, 0.0)
    d = Dinv * r / theta
    rho_prev = delta / theta
    x = x + d
    for _ in range(1, degree):
        r = np.where(f, b - A @ x, 0.0)
        rho = 1.0 / (2.0 * theta / delta - rho_prev)
        d = rho * rho_prev * d + (2.0 * rho / delta) * Dinv * r
        x = x + d
        rho_prev = rho
    return x


class VCycle:
    """Block-diagonal local-smoothing V-cycle for one leaf state and active set."""

    def __init__(self, hier: Hierarchy, prm: Params, mgp: MGParams, U_leaf, phit_leaf,
                 leaf_active, eigen=None):
        self.h = hier
        self.prm = prm
        self.mgp = mgp
        mesh = hier.mesh
        n = mesh.n_nodes
        self.leaf_free = np.concatenate([~(mesh.dirichlet | mesh.hanging)] * 2 +
                                        [~(np.asarray(leaf_active, bool) | mesh.hanging)])
        acts = hier.level_active(leaf_active)
        self.ops = []
        for l, lv in enumerate(hier.levels):
            ux = U_leaf[:n][lv.leaf_index]
            uy = U_leaf[n:2 * n][lv.leaf_index]
            pt = phit_leaf[lv.leaf_index]
            cs = lv.cells
            g = cs.gather
            Ke = element_jacobian(cs, prm, g(ux), g(uy), np.zeros_like(g(ux)), g(pt), blocks="diag")
            A = assemble_matrix(lv.cell_nodes, lv.n, Ke)
            fu = ~(lv.dirichlet | lv.edge)
            fp = ~(acts[l] | lv.edge)
            free = np.concatenate([fu, fu, fp])
            diag = A.diagonal()
            Dinv = np.where(free, 1.0 / np.where(diag != 0, diag, 1.0), 0.0)
            op = LevelOps(A=A, free=free, Dinv=Dinv)
            op.extra["active"] = acts[l]
            # unknowns held at zero on this level (the edge is not: it carries
            # the coarse correction)
            op.extra["held"] = np.concatenate([lv.dirichlet, lv.dirichlet, acts[l]])
            self.ops.append(op)
        self.set_eigen(eigen)

    def set_eigen(self, eigen=None):
        """eigen: None (estimate by CG) or (lam_max[levels][2], lam_min0[2])."""
        for l, op in enumerate(self.ops):
            n = self.h.levels[l].n
            bu, bp = block_masks(n)
            its_u = self.mgp.coarse_eig_its if l == 0 else self.mgp.eig_cg_its
            its_p = self.mgp.coarse_eig_its if l == 0 else self.mgp.eig_cg_its_phi
            if eigen is None:
                lu = cg_eigs(op.A, op.Dinv, op.free & bu, its_u)
                lp = cg_eigs(op.A, op.Dinv, op.free & bp, its_p)
                op.lam_max = np.array([lu[1], lp[1]])
                op.lam_min = np.array([lu[0], lp[0]])
            else:
                op.lam_max = np.asarray(eigen[0][l], dtype=float)
                op.lam_min = np.asarray(eigen[1], dtype=float) if l == 0 else None

    def eigen(self):
        return ([op.lam_max.copy() for op in self.ops], self.ops[0].lam_min.copy())

    # -- smoother ---------------------------------------------------------
    def interval(self, l):
        op = self.ops[l]
        if l == 0 and self.mgp.coarse_mode == "cheb":
            lo, hi = op.lam_min, self.mgp.upper_factor * op.lam_max
        else:
            lo, hi = self.mgp.smooth_range * op.lam_max, self.mgp.upper_factor * op.lam_max
        return lo, hi

    def chebyshev(self, l, b, x0, degree):
        """Chebyshev-Jacobi smoothing on the free unknowns of level l."""
        op = self.ops[l]
        n = self.h.levels[l].n
        lo, hi = self.interval(l)
        theta_b = 0.5 * (hi + lo)
        delta_b = 0.5 * (hi - lo)
        theta = np.concatenate([np.full(2 * n, theta_b[0]), np.full(n, theta_b[1])])
        delta = np.concatenate([np.full(2 * n, delta_b[0]), np.full(n, delta_b[1])])
        return chebyshev(op.A, op.Dinv, op.free, b, x0, degree, theta, delta)

    def coarse_solve(self, b):
        op = self.ops[0]
        if self.mgp.coarse_mode == "cheb":
            return self.chebyshev(0, b, None, self.mgp.coarse_its)
        if self.mgp.coarse_mode == "cg":
            return self.coarse_cg(b)
        if self.mgp.coarse_mode == "exact":
            import scipy.sparse.linalg as spla
            idx = np.flatnonzero(op.free)
            x = np.zeros_like(b)
            x[idx] = spla.spsolve(op.A[idx][:, idx].tocsc(), b[idx])
            return x
        raise ValueError(self.mgp.coarse_mode)

    def coarse_cg(self, b):
        """Fixed number of Jacobi-preconditioned CG steps from x = 0, each block
        with its own inner products (the blocks are independent systems)."""
        op = self.ops[0]
        n = self.h.levels[0].n
        x = np.zeros(3 * n)
        for blk in block_masks(n):
            m = (op.free & blk).astype(float)
            r = b * m
            z = op.Dinv * r
            pv = z.copy()
            rz = r @ z
            for _ in range(self.mgp.coarse_its):
                if rz == 0:
                    break
                q = (op.A @ pv) * m
                alpha = rz / (pv @ q)
                x = x + alpha * pv
                r = r - alpha * q
                z = op.Dinv * r
                rz_new = r @ z
                pv = z + (rz_new / rz) * pv
                rz = rz_new
        return x

    # -- cycle ------------------------------------------------------------
    def apply(self, b_leaf):
        h = self.h
        mesh = h.mesh
        n = mesh.n_nodes
        L = len(h.levels) - 1
        k = self.mgp.cheb_degree
        d = [np.zeros(3 * lv.n) for lv in h.levels]
        for c in range(3):
            for g in range(n):
                if self.leaf_free[c * n + g]:
                    lv = h.levels[int(h.copy_level[g])]
                    d[int(h.copy_level[g])][c * lv.n + h.copy_index[g]] = b_leaf[c * n + g]
        x = [None] * (L + 1)
        for l in range(L, 0, -1):
            x[l] = self.chebyshev(l, d[l], None, k)
            t = np.where(self.ops[l].extra["held"], 0.0, d[l] - self.ops[l].A @ x[l])
            d[l - 1] = d[l - 1] + h.P3[l].T @ t
        x[0] = self.coarse_solve(d[0])
        for l in range(1, L + 1):
            x[l] = x[l] + h.P3[l] @ x[l - 1]
            x[l] = np.where(self.ops[l].extra["held"], 0.0, x[l])
            x[l] = self.chebyshev(l, d[l], x[l], k)
        out = np.array(b_leaf, dtype=float, copy=True)
        for c in range(3):
            for g in range(n):
                if self.leaf_free[c * n + g]:
                    lv = h.levels[int(h.copy_level[g])]
                    out[c * n + g] = x[int(h.copy_level[g])][c * lv.n + h.copy_index[g]]
        return out


def block_triangular_apply(block_solve, J, b, n, transpose=False):
    """Block-triangular preconditioner (the alternative to the block-diagonal
    P of Sec. 3.2 that keeps the coupling block G_phi,u of the linearised
    Jacobian, which is lower block triangular since the u-equation uses phi~,
    Sec. 2 after Problem 1). block_solve(v) applies the diagonal blocks'
    approximate inverses to both blocks of v at once (the V-cycle of either
    hierarchy); J is the masked Jacobian. Forward substitution:
        x_u   = M_uu^-1 b_u,
        x_phi = M_phiphi^-1 (b_phi - G_phi,u x_u),
    with G_phi,u x_u read off the phi rows of J (x_u, 0). transpose=True gives
    the upper-triangular form for systems with J^T: x_phi first, then x_u with
    b_u - G_phi,u^T x_phi from the u rows of J^T (0, x_phi). Constrained rows
    pass through as in block_solve."""
    b = np.asarray(b, dtype=float)
    first = np.zeros_like(b)
    if not transpose:
        first[:2 * n] = b[:2 * n]
        y1 = block_solve(first)
        r = np.zeros_like(b)
        r[2 * n:] = b[2 * n:] - (J @ y1)[2 * n:]
    else:
        first[2 * n:] = b[2 * n:]
        y1 = block_solve(first)
        r = np.zeros_like(b)
        r[:2 * n] = b[:2 * n] - (J.T @ y1)[:2 * n]
    return y1 + block_solve(r)
