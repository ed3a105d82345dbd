"""Quadtree mesh of Omega = (-10, 10)^2 with local refinement (oracle).

Test infrastructure only (see the package docstring).

Geometry and refinement follow the Sneddon setting of Sec. 4 (Fig. 1, Table 1):
a uniform base mesh of n_base x n_base squares (reached from a coarse grid of
`coarse` x `coarse` squares by global refinement), then `n_local` passes of
local refinement of every leaf whose centre lies strictly inside the band
|x| < bx, |y| < by, then 2:1 face balancing (at most one hanging node per face,
which the hanging-node treatment of conforming Q_p elements on locally refined
meshes requires, Sec. 3.2). Displacements are in H^1_0 (Sec. 2, Problem 1), so
u is fixed to zero on the whole boundary; the phase field has natural boundary
conditions.

Positions are integers on a lattice of M units across the domain, with
M = coarse * 2^lmax * p, so that every Q_p node of every level is a lattice
point: x = -10 + 20 X / M.

Cell (l, i, j): refinement level l (l = 0 is the coarse grid), column i and
row j on that level; its edge is S_l = p * 2^(lmax - l) lattice units.
Local Q_p node (a, b), a, b in 0..p, has local index a + (p + 1) b.
"""
from __future__ import annotations

import numpy as np


def lagrange_1d(p: int, s: float) -> np.ndarray:
    """Values of the equispaced 1-D Lagrange basis of degree p at s in [0, 1]."""
    nodes = np.arange(p + 1) / p
    out = np.ones(p + 1)
    for k in range(p + 1):
        for m in range(p + 1):
            if m != k:
                out[k] *= (s - nodes[m]) / (nodes[k] - nodes[m])
    return out


class Mesh:
    """Leaf mesh, nodes and constraints. Plain Python sets and loops."""

    DIRS = ((-1, 0), (1, 0), (0, -1), (0, 1))

    def __init__(self, n_base: int, n_local: int, degree: int, coarse: int = 16,
                 band=(2.0, 0.5)):
        ratio = n_base // coarse
        assert ratio * coarse == n_base and ratio & (ratio - 1) == 0, "n_base = coarse * 2^b"
        self.p = degree
        self.coarse = coarse
        self.b = ratio.bit_length() - 1
        self.n_local = n_local
        self.lmax = self.b + n_local
        self.n_levels = self.lmax + 1
        self.M = coarse * 2 ** self.lmax * degree
        self.band = band
        self.leaves = self._refine()
        self._balance()
        self._number_nodes()
        self._find_hanging()
        self.dirichlet = ((self.NX == 0) | (self.NX == self.M) |
                          (self.NY == 0) | (self.NY == self.M))

    # -- geometry ---------------------------------------------------------
    def S(self, level):
        """Cell edge in lattice units at a refinement level."""
        return self.p * 2 ** (self.lmax - np.asarray(level))

    def H(self, level):
        """Physical cell edge at a refinement level."""
        return 20.0 / (self.coarse * 2.0 ** np.asarray(level))

    def ncells_1d(self, level: int) -> int:
        return self.coarse * 2 ** level

    def _in_band(self, l, i, j) -> bool:
        # centre x = 10 ((2i+1) S - M) / M; |x| < bx  <=>  10^4 |(2i+1)S - M| < 1000 bx M
        S = int(self.S(l))
        bx = int(round(self.band[0] * 1000))
        by = int(round(self.band[1] * 1000))
        return (10000 * abs((2 * i + 1) * S - self.M) < bx * self.M and
                10000 * abs((2 * j + 1) * S - self.M) < by * self.M)

    # -- refinement -------------------------------------------------------
    def _refine(self):
        n = self.ncells_1d(self.b)
        leaves = {(self.b, i, j) for i in range(n) for j in range(n)}
        for _ in range(self.n_local):
            new = set()
            for (l, i, j) in leaves:
                if self._in_band(l, i, j):
                    new.update(((l + 1, 2 * i + a, 2 * j + c) for a in (0, 1) for c in (0, 1)))
                else:
                    new.add((l, i, j))
            leaves = new
        return leaves

    def find_leaf(self, l, i, j):
        """Leaf whose closure contains level-l cell (i, j), searching level l
        and coarser; None if that region is refined beyond level l."""
        for k in range(l, -1, -1):
            key = (k, i >> (l - k), j >> (l - k))
            if key in self.leaves:
                return key
        return None

    def _balance(self):
        """2:1 face balance: refine any leaf with a face neighbour two levels finer."""
        while True:
            marks = set()
            for (l, i, j) in self.leaves:
                if l < self.b + 2:
                    continue
                n = self.ncells_1d(l)
                for di, dj in self.DIRS:
                    ni, nj = i + di, j + dj
                    if not (0 <= ni < n and 0 <= nj < n):
                        continue
                    f = self.find_leaf(l, ni, nj)
                    if f is not None and f[0] < l - 1:
                        marks.add(f)
            if not marks:
                return
            for (l, i, j) in marks:
                self.leaves.discard((l, i, j))
                self.leaves.update(((l + 1, 2 * i + a, 2 * j + c) for a in (0, 1) for c in (0, 1)))

    # -- nodes ------------------------------------------------------------
    def _number_nodes(self):
        cells = np.array(sorted(self.leaves), dtype=np.int64).reshape(-1, 3)
        self.cell_level, self.cell_i, self.cell_j = cells[:, 0], cells[:, 1], cells[:, 2]
        p = self.p
        S = self.S(self.cell_level)
        a = np.tile(np.arange(p + 1), p + 1)          # local x index
        b = np.repeat(np.arange(p + 1), p + 1)        # local y index
        X = self.cell_i[:, None] * S[:, None] + a[None, :] * (S[:, None] // p)
        Y = self.cell_j[:, None] * S[:, None] + b[None, :] * (S[:, None] // p)
        keys = Y * (self.M + 1) + X
        uniq, inv = np.unique(keys.ravel(), return_inverse=True)
        self.cell_nodes = inv.reshape(keys.shape)
        self.NX = uniq % (self.M + 1)
        self.NY = uniq // (self.M + 1)
        self.n_nodes = uniq.size
        self._key_to_node = {int(k): n for n, k in enumerate(uniq)}

    def node_at(self, X, Y):
        return self._key_to_node.get(int(Y) * (self.M + 1) + int(X))

    @property
    def n_cells(self):
        return self.cell_level.size

    # -- hanging nodes ----------------------------------------------------
    def _find_hanging(self):
        """Hanging nodes: nodes of a fine cell on a face whose neighbour is one
        level coarser and that are not nodes of that coarse face. Their value
        is the coarse face's Q_p trace: sum_k L_k(s) * master_k."""
        p = self.p
        cons = {}
        for c in range(self.n_cells):
            l, i, j = int(self.cell_level[c]), int(self.cell_i[c]), int(self.cell_j[c])
            n = self.ncells_1d(l)
            S = int(self.S(l))
            for di, dj in self.DIRS:
                ni, nj = i + di, j + dj
                if not (0 <= ni < n and 0 <= nj < n):
                    continue
                if (l, ni, nj) in self.leaves:
                    continue
                coarse = (l - 1, ni >> 1, nj >> 1)
                if coarse not in self.leaves:
                    continue
                Sc = 2 * S
                I, J = coarse[1], coarse[2]
                if di != 0:   # vertical face x = const
                    Xf = (i + (1 if di > 0 else 0)) * S
                    pts = [(Xf, j * S + t * S // p) for t in range(p + 1)]
                    par = [(Y - J * Sc) for (_, Y) in pts]
                    mast = [(Xf, J * Sc + k * Sc // p) for k in range(p + 1)]
                else:         # horizontal face y = const
                    Yf = (j + (1 if dj > 0 else 0)) * S
                    pts = [(i * S + t * S // p, Yf) for t in range(p + 1)]
                    par = [(X - I * Sc) for (X, _) in pts]
                    mast = [(X, Yf) for X in (I * Sc + k * Sc // p for k in range(p + 1))]
                mids = [self.node_at(*m) for m in mast]
                for (pt, d) in zip(pts, par):
                    if (d * p) % Sc == 0:
                        continue   # coincides with a coarse face node
                    node = self.node_at(*pt)
                    w = lagrange_1d(p, d / Sc)
                    cons[node] = [(mids[k], float(w[k])) for k in range(p + 1) if w[k] != 0.0]
        # masters are never hanging themselves on 2:1 meshes; resolve chains anyway
        changed = True
        while changed:
            changed = False
            for h, lst in cons.items():
                if any(m in cons for m, _ in lst):
                    new = {}
                    for m, w in lst:
                        if m in cons:
                            for m2, w2 in cons[m]:
                                new[m2] = new.get(m2, 0.0) + w * w2
                        else:
                            new[m] = new.get(m, 0.0) + w
                    cons[h] = sorted(new.items())
                    changed = True
        self.hanging_constraints = cons
        self.hanging = np.zeros(self.n_nodes, dtype=bool)
        self.hanging[list(cons.keys())] = True

    def constraint_matrix(self):
        """C (n x n, scipy CSR): maps master values to all nodal values.

        Row of a regular node = unit row; row of a hanging node = its weights;
        column of a hanging node is empty."""
        import scipy.sparse as sp
        rows, cols, vals = [], [], []
        for k in range(self.n_nodes):
            if self.hanging[k]:
                for m, w in self.hanging_constraints[k]:
                    rows.append(k)
                    cols.append(m)
                    vals.append(w)
            else:
                rows.append(k)
                cols.append(k)
                vals.append(1.0)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.n_nodes, self.n_nodes))

    # -- levels -----------------------------------------------------------
    def level_cells(self, level: int):
        """All tree cells on a level (leaves on it and ancestors of finer leaves)."""
        out = set()
        for (l, i, j) in self.leaves:
            if l >= level:
                out.add((level, i >> (l - level), j >> (l - level)))
        return out

    def cell_diameter_min(self) -> float:
        return float(np.sqrt(2.0) * self.H(self.cell_level.max()))
