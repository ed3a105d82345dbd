"""Residual, Jacobian and derived operators of the phase-field system (oracle).

Test infrastructure only.

Unknowns per node: (u_x, u_y, phi). Global vectors are blocked:
[u_x(n) | u_y(n) | phi(n)]. Element arrays are (cells, 3, nloc) with the
component first.

Material law (Sec. 2, Problem 1): e(u) = sym grad u, sigma(u) = 2 mu e +
lambda tr(e) I, degradation g(phi) = (1 - kappa) phi^2 + kappa. The Lame
parameters come from (E, nu) in plane strain (Table 1's rounded values 0.42 and
0.28 are mu = 5/12 and lambda = 5/18 at E = 1, nu = 0.2).

Residual F(U)(Psi) (Problem 2, with phi in g and in the u-equation pressure
replaced by the linearisation point phi~, Sec. 2 after Problem 1):
  u rows:   (g(phi~) sigma(u), e(psi_u)) + (p phi~^2, div psi_u)
  phi rows: (1-kappa)(phi sigma(u):e(u), psi) + 2 p (phi div u, psi)
            - (Gc/l)(1 - phi, psi) + Gc l (grad phi, grad psi)
Jacobian A'(U)(dU, Psi) (Sec. 3.1):
  (g(phi~) sigma(du), e(psi_u))
  + (1-kappa)(dphi sigma(u):e(u) + 2 phi sigma(du):e(u), psi)
  + 2 p (dphi div u + phi div du, psi)
  + Gc ((1/l)(dphi, psi) + l (grad dphi, grad psi))

Constrained operator (Sec. 3.3 applies the Jacobian with constraints): with C
the hanging-node interpolation, J~ = Mf C^T J C Mf + (I - Mf), where Mf keeps
the free unknowns (not Dirichlet for u, not hanging, not active for phi).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .fe import Element, basis_1d, gauss_01
from .mesh import Mesh


@dataclass
class Params:
    E: float = 1.0
    nu: float = 0.2
    Gc: float = 1.0
    pressure: float = 1e-3
    kappa: float = 1e-10
    ell: float = 0.1

    @property
    def mu(self):
        return self.E / (2.0 * (1.0 + self.nu))

    @property
    def lam(self):
        return self.E * self.nu / ((1.0 + self.nu) * (1.0 - 2.0 * self.nu))


# ---------------------------------------------------------------- helpers --
def at_points(el: Element, H, loc):
    """Value and physical gradient at Gauss points of nodal cell values loc (nc, nloc)."""
    val = loc @ el.N.T
    gx = (loc @ el.dNx.T) / H[:, None]
    gy = (loc @ el.dNy.T) / H[:, None]
    return val, gx, gy


def strain_stress(prm: Params, gxx, gxy, gyx, gyy):
    """e(u) and sigma(u) components from the displacement gradient
    (gab = d u_a / d x_b)."""
    exx, eyy, exy = gxx, gyy, 0.5 * (gxy + gyx)
    tr = exx + eyy
    sxx = 2 * prm.mu * exx + prm.lam * tr
    syy = 2 * prm.mu * eyy + prm.lam * tr
    sxy = 2 * prm.mu * exy
    return (exx, eyy, exy), (sxx, syy, sxy), tr


def test_integrate(el: Element, H, JxW, fval, fx, fy):
    """Local vector sum_q JxW (fval N_k + fx dN_k/dx + fy dN_k/dy)."""
    out = (JxW * fval) @ el.N
    out = out + ((JxW * fx) / H[:, None]) @ el.dNx
    out = out + ((JxW * fy) / H[:, None]) @ el.dNy
    return out


class CellSet:
    """Cells to integrate over: edge H per cell and the node index map."""

    def __init__(self, el: Element, H, nodes):
        self.el = el
        self.H = np.asarray(H, dtype=float)
        self.nodes = np.asarray(nodes)
        self.JxW = (self.H ** 2)[:, None] * el.w[None, :]

    def gather(self, v):
        return v[self.nodes]


def leaf_cells(mesh: Mesh, el: Element) -> CellSet:
    return CellSet(el, mesh.H(mesh.cell_level), mesh.cell_nodes)


# --------------------------------------------------------------- residual --
def element_residual(cs: CellSet, prm: Params, ux, uy, phi, phit, terms="all"):
    """Local residual (nc, 3, nloc) for nodal fields given as cell arrays.

    terms selects pieces for parameter derivatives: 'all', 'sigma' (terms
    linear in E), 'pressure' (terms linear in p, divided by p), 'gc' (terms
    linear in Gc, divided by Gc)."""
    el, H, JxW = cs.el, cs.H, cs.JxW
    _, uxx, uxy = at_points(el, H, ux)
    _, uyx, uyy = at_points(el, H, uy)
    ph, phx, phy = at_points(el, H, phi)
    pt, _, _ = at_points(el, H, phit)
    (exx, eyy, exy), (sxx, syy, sxy), tr = strain_stress(prm, uxx, uxy, uyx, uyy)
    g = (1 - prm.kappa) * pt ** 2 + prm.kappa
    S = sxx * exx + syy * eyy + 2 * sxy * exy
    zero = np.zeros_like(ph)
    if terms == "all":
        cs_sig, cs_p, cs_gc = 1.0, prm.pressure, prm.Gc
    elif terms == "sigma":
        cs_sig, cs_p, cs_gc = 1.0, 0.0, 0.0
    elif terms == "pressure":
        cs_sig, cs_p, cs_gc = 0.0, 1.0, 0.0
    elif terms == "gc":
        cs_sig, cs_p, cs_gc = 0.0, 0.0, 1.0
    else:
        raise ValueError(terms)
    # u rows: (g sigma, e(psi)) + (p phi~^2, div psi)
    rx = test_integrate(el, H, JxW, zero, cs_sig * g * sxx + cs_p * pt ** 2, cs_sig * g * sxy)
    ry = test_integrate(el, H, JxW, zero, cs_sig * g * sxy, cs_sig * g * syy + cs_p * pt ** 2)
    # phi rows
    fval = (cs_sig * (1 - prm.kappa) * ph * S + cs_p * 2 * ph * tr
            - cs_gc * (1.0 / prm.ell) * (1 - ph))
    rphi = test_integrate(el, H, JxW, fval, cs_gc * prm.ell * phx, cs_gc * prm.ell * phy)
    return np.stack([rx, ry, rphi], axis=1)


# --------------------------------------------------------------- jacobian --
def element_jacobian(cs: CellSet, prm: Params, ux, uy, phi, phit, blocks="full"):
    """Element matrices (nc, 3 nloc, 3 nloc) of the Jacobian, rows (comp, k),
    columns (comp, m), from the Sec. 3.1 formula with one trial function at a
    time. blocks='diag' drops the coupling block (phi rows, u columns)."""
    el, H, JxW = cs.el, cs.H, cs.JxW
    nc, nl = ux.shape[0], el.nloc
    _, uxx, uxy = at_points(el, H, ux)
    _, uyx, uyy = at_points(el, H, uy)
    ph, _, _ = at_points(el, H, phi)
    pt, _, _ = at_points(el, H, phit)
    (exx, eyy, exy), (sxx, syy, sxy), tr = strain_stress(prm, uxx, uxy, uyx, uyy)
    g = (1 - prm.kappa) * pt ** 2 + prm.kappa
    S = sxx * exx + syy * eyy + 2 * sxy * exy
    K = np.zeros((nc, 3 * nl, 3 * nl), dtype=np.result_type(ux, phi, phit, float))
    mu, lam = prm.mu, prm.lam
    zero = np.zeros_like(ph)
    for m in range(nl):
        Nm = el.N[:, m][None, :]
        dx = (el.dNx[:, m][None, :]) / H[:, None]
        dy = (el.dNy[:, m][None, :]) / H[:, None]
        dx = np.broadcast_to(dx, ph.shape)
        dy = np.broadcast_to(dy, ph.shape)
        Nm = np.broadcast_to(Nm, ph.shape)
        for comp in (0, 1):
            if comp == 0:   # trial (N_m, 0)
                dsxx, dsyy, dsxy, ddiv = (2 * mu + lam) * dx, lam * dx, mu * dy, dx
            else:           # trial (0, N_m)
                dsxx, dsyy, dsxy, ddiv = lam * dy, (2 * mu + lam) * dy, mu * dx, dy
            col = comp * nl + m
            K[:, 0 * nl:1 * nl, col] = test_integrate(el, H, JxW, zero, g * dsxx, g * dsxy)
            K[:, 1 * nl:2 * nl, col] = test_integrate(el, H, JxW, zero, g * dsxy, g * dsyy)
            if blocks == "full":
                sde = dsxx * exx + dsyy * eyy + 2 * dsxy * exy
                fval = (1 - prm.kappa) * 2 * ph * sde + 2 * prm.pressure * ph * ddiv
                K[:, 2 * nl:3 * nl, col] = test_integrate(el, H, JxW, fval, zero, zero)
        col = 2 * nl + m
        fval = ((1 - prm.kappa) * Nm * S + 2 * prm.pressure * Nm * tr
                + (prm.Gc / prm.ell) * Nm)
        K[:, 2 * nl:3 * nl, col] = test_integrate(el, H, JxW, fval, prm.Gc * prm.ell * dx,
                                                  prm.Gc * prm.ell * dy)
    return K


# ------------------------------------------------------------- assembling --
def dof_map(nodes, n):
    """(nc, 3 nloc) global blocked dof indices of a cell node map."""
    return np.concatenate([nodes + c * n for c in range(3)], axis=1)


def assemble_vector(nodes, n, local):
    nc, ncomp, nl = local.shape
    dofs = dof_map(nodes, n)
    out = np.zeros(3 * n, dtype=local.dtype)
    np.add.at(out, dofs.ravel(), local.reshape(nc, -1).ravel())
    return out


def assemble_matrix(nodes, n, Ke):
    dofs = dof_map(nodes, n)
    nd = dofs.shape[1]
    rows = np.repeat(dofs, nd, axis=1).ravel()
    cols = np.tile(dofs, (1, nd)).ravel()
    return sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(3 * n, 3 * n))


def kron3(C):
    return sp.block_diag([C, C, C], format="csr")


# ------------------------------------------------------------------ model --
class LeafProblem:
    """Leaf-mesh operators for one mesh, parameter set and state.

    State vectors are nodal arrays of length n (hanging entries are expected
    to hold their interpolated values; `distribute` provides them)."""

    def __init__(self, mesh: Mesh, prm: Params):
        self.mesh = mesh
        self.prm = prm
        self.el = Element(mesh.p)
        self.cells = leaf_cells(mesh, self.el)
        self.n = mesh.n_nodes
        self.C = mesh.constraint_matrix()
        self.C3 = kron3(self.C)

    # constraints
    def distribute(self, v):
        """Set hanging-node entries from their masters (per component block)."""
        n = self.n
        v = np.array(v, copy=True)
        for c in range(v.size // n):
            blk = v[c * n:(c + 1) * n].copy()
            blk[self.mesh.hanging] = 0.0
            v[c * n:(c + 1) * n] = self.C @ blk
        return v

    def free_mask(self, active):
        m = self.mesh
        fu = ~(m.dirichlet | m.hanging)
        fphi = ~(np.asarray(active, dtype=bool) | m.hanging)
        return np.concatenate([fu, fu, fphi])

    def state_cells(self, U, phit):
        n = self.n
        g = self.cells.gather
        return g(U[:n]), g(U[n:2 * n]), g(U[2 * n:]), g(phit)

    # residual
    def residual_raw(self, U, phit, terms="all"):
        ux, uy, ph, pt = self.state_cells(U, phit)
        loc = element_residual(self.cells, self.prm, ux, uy, ph, pt, terms)
        return assemble_vector(self.cells.nodes, self.n, loc)

    def residual(self, U, phit):
        """R = -C^T F(U): the Newton right-hand side before masking."""
        return -(self.C3.T @ self.residual_raw(U, phit))

    # jacobian
    def jacobian_raw(self, U, phit, blocks="full"):
        ux, uy, ph, pt = self.state_cells(U, phit)
        Ke = element_jacobian(self.cells, self.prm, ux, uy, ph, pt, blocks)
        return assemble_matrix(self.cells.nodes, self.n, Ke)

    def masked_operator(self, U, phit, active, blocks="full"):
        """J~ = Mf C^T J C Mf + (I - Mf) (identity on constrained rows/cols)."""
        J = self.jacobian_raw(U, phit, blocks)
        f = self.free_mask(active).astype(float)
        Mf = sp.diags(f)
        Jc = self.C3.T @ J @ self.C3
        return (Mf @ Jc @ Mf + sp.diags(1.0 - f)).tocsr()

    def _cells_for_rows(self, rows):
        """Cells whose element arrays reach the given blocked rows of a
        condensed (C^T ... C) operator: cells with the row's node or with a
        hanging node that has the row's node among its masters."""
        n = self.n
        mesh = self.mesh
        nodes = np.unique(np.asarray(rows) % n)
        need = set(int(k) for k in nodes)
        for h, lst in mesh.hanging_constraints.items():
            if any(m in need for m, _ in lst):
                need.add(int(h))
        need = np.array(sorted(need))
        sel = np.isin(mesh.cell_nodes, need).any(axis=1)
        return CellSet(self.el, self.cells.H[sel], self.cells.nodes[sel])

    def masked_rows(self, rows, src, U, phit, active, transpose=False):
        """Selected rows of J~ src (or of J~^T src), assembling only the cells
        that touch those rows. For spot checks on large meshes: the
        row of J~^T at node k needs column k of J, which only cells holding k
        (or a hanging node mastered by k) reach, the same cells as row k."""
        n = self.n
        rows = np.asarray(rows)
        cs = self._cells_for_rows(rows)
        g = cs.gather
        Ke = element_jacobian(cs, self.prm, g(U[:n]), g(U[n:2 * n]), g(U[2 * n:]), g(phit))
        J = assemble_matrix(cs.nodes, n, Ke)
        if transpose:
            J = J.T.tocsr()
        f = self.free_mask(active)
        x = self.C3 @ (src * f)
        y = (self.C3.T @ (J @ x))[rows]
        return np.where(f[rows], y, src[rows])

    def residual_rows(self, rows, U, phit):
        """Selected rows of R = -C^T F(U), assembling only the cells that
        touch those rows."""
        n = self.n
        rows = np.asarray(rows)
        cs = self._cells_for_rows(rows)
        g = cs.gather
        loc = element_residual(cs, self.prm, g(U[:n]), g(U[n:2 * n]), g(U[2 * n:]), g(phit))
        raw = assemble_vector(cs.nodes, n, loc)
        return -(self.C3.T @ raw)[rows]

    # crack volume (Sec. 4) and its derivative
    def tcv(self, U):
        n = self.n
        cs = self.cells
        ux, uy, ph = cs.gather(U[:n]), cs.gather(U[n:2 * n]), cs.gather(U[2 * n:])
        vx, _, _ = at_points(cs.el, cs.H, ux)
        vy, _, _ = at_points(cs.el, cs.H, uy)
        _, px, py = at_points(cs.el, cs.H, ph)
        return float(np.sum(cs.JxW * (vx * px + vy * py)))

    def cod(self, U, xs):
        """Crack opening displacement (Sec. 4): COD(x) = the integral over y of
        u . grad phi along the vertical line at x, for each x in xs. Summed
        over the leaf cells whose x-range [x_c, x_c + H) holds x (a line on a
        cell boundary belongs to the cell on its right; x = 10 lies in none),
        each by p + 1 Gauss points in y, which is exact for the degree-2p
        integrand. U: nodal values with hanging entries set (as in tcv)."""
        m = self.mesh
        n = self.n
        p = m.p
        t, wt = gauss_01(p + 1)
        vt, dt = basis_1d(p, t)                       # (p+1 points) x (p+1 functions)
        H = m.H(m.cell_level)
        xc = -10.0 + m.cell_i * H
        out = np.zeros(len(xs))
        comps = [U[:n], U[n:2 * n], U[2 * n:3 * n]]
        for j, x in enumerate(xs):
            sel = np.flatnonzero((xc <= x) & (x < xc + H))
            total = 0.0
            for c in sel:
                s = (x - xc[c]) / H[c]
                vs, ds = basis_1d(p, [s])
                vs, ds = vs[0], ds[0]
                # nodal values as (b, a) arrays: node k = a + (p + 1) b
                ux, uy, ph = (v[m.cell_nodes[c]].reshape(p + 1, p + 1) for v in comps)
                # along the line: f(t_q) = sum_ab f_ab l_a(s) l_b(t_q); reference
                # derivatives, since dy = H dt cancels the 1 / H of the gradient
                uxq = vt @ ux @ vs
                uyq = vt @ uy @ vs
                psq = vt @ ph @ ds
                ptq = dt @ ph @ vs
                total += float(np.sum(wt * (uxq * psq + uyq * ptq)))
            out[j] = total
        return out

    def tcv_gradient(self, U):
        """d TCV / d(master values), blocked, as C^T of the nodal gradient."""
        n = self.n
        cs = self.cells
        el = cs.el
        ux, uy, ph = cs.gather(U[:n]), cs.gather(U[n:2 * n]), cs.gather(U[2 * n:])
        vx, _, _ = at_points(el, cs.H, ux)
        vy, _, _ = at_points(el, cs.H, uy)
        _, px, py = at_points(el, cs.H, ph)
        zero = np.zeros_like(vx)
        gx = test_integrate(el, cs.H, cs.JxW, px, zero, zero)
        gy = test_integrate(el, cs.H, cs.JxW, py, zero, zero)
        gp = test_integrate(el, cs.H, cs.JxW, zero, vx, vy)
        raw = assemble_vector(cs.nodes, n, np.stack([gx, gy, gp], axis=1))
        return self.C3.T @ raw

    def param_derivatives(self, U, phit):
        """dF/d(Gc, E, p) as condensed vectors C^T dF_raw/dtheta.

        sigma is linear in E at fixed nu; p and Gc enter linearly."""
        out = {}
        out["Gc"] = self.C3.T @ self.residual_raw(U, phit, terms="gc")
        out["E"] = self.C3.T @ self.residual_raw(U, phit, terms="sigma") / self.prm.E
        out["p"] = self.C3.T @ self.residual_raw(U, phit, terms="pressure")
        return out

    def lumped_phi_mass(self):
        """Row sums of the condensed phase-field mass matrix (the B of Alg. 2)."""
        cs = self.cells
        loc = (cs.JxW @ cs.el.N)                       # sum_q JxW N_k
        raw = np.zeros(self.n)
        np.add.at(raw, cs.nodes.ravel(), loc.ravel())
        return self.C.T @ raw
