"""The library's host mesh builder against the oracle's mesh (CPU only).

Both build the quadtree, nodes, hanging constraints and multigrid levels from
the same geometric rules in independent code; nodes are matched by their
integer lattice coordinates. Integer and index data must agree exactly."""
import numpy as np
import pytest

from oracle.mesh import Mesh
from oracle.mg import Hierarchy

lib_mod = pytest.importorskip("paper_2404_03265_amd.meshinfo")

CASES = [
    dict(n_base=16, n_local=2, coarse=4, band=(3.0, 1.0)),
    dict(n_base=32, n_local=2, coarse=16, band=(2.0, 0.5)),
    dict(n_base=32, n_local=3, coarse=8, band=(2.0, 0.5)),
    dict(n_base=32, n_local=0, coarse=8, band=(2.0, 0.5)),     # uniform
    dict(n_base=40, n_local=2, coarse=10, band=(3.0, 1.0)),    # the paper's mesh family
]


def _key(X, Y, M):
    return np.asarray(Y, dtype=np.int64) * (M + 1) + np.asarray(X, dtype=np.int64)


def _built():
    try:
        from paper_2404_03265_amd import _lib
        _lib.load()
        return True
    except Exception:
        return False


pytestmark = pytest.mark.skipif(not _built(), reason="libpff.so not built")


@pytest.fixture(scope="module", params=[(c, p) for c in range(len(CASES)) for p in (1, 2)],
                ids=lambda x: f"case{x[0]}-Q{x[1]}")
def pair(request):
    ci, p = request.param
    c = CASES[ci]
    om = Mesh(c["n_base"], c["n_local"], p, coarse=c["coarse"], band=c["band"])
    hm = lib_mod.HostMesh(c["n_base"], c["n_local"], p, coarse=c["coarse"], band=c["band"])
    return om, Hierarchy(om), hm


def test_leaf_nodes_and_flags(pair):
    om, _, hm = pair
    assert hm.M == om.M and hm.n == om.n_nodes and hm.n_levels == om.n_levels
    X, Y = hm.coords()
    kh = _key(X, Y, hm.M)
    ko = _key(om.NX, om.NY, om.M)
    order_h, order_o = np.argsort(kh), np.argsort(ko)
    assert np.array_equal(kh[order_h], ko[order_o])
    f = hm.flags()
    assert np.array_equal((f[order_h] & 1) != 0, om.dirichlet[order_o])
    assert np.array_equal((f[order_h] & 2) != 0, om.hanging[order_o])


def test_hanging_constraints(pair):
    om, _, hm = pair
    X, Y = hm.coords()
    node, mast, w = hm.hanging()
    assert node.size == int(om.hanging.sum())
    for i in range(node.size):
        h = om.node_at(X[node[i]], Y[node[i]])
        ref = {(int(om.NX[m]), int(om.NY[m])): wt for m, wt in om.hanging_constraints[h]}
        got = {(int(X[m]), int(Y[m])): wt for m, wt in zip(mast[i], w[i]) if m >= 0 and wt != 0.0}
        assert got == ref


def test_levels_transfers_and_flags(pair):
    om, hier, hm = pair
    X, Y = hm.coords()
    for l, lv in enumerate(hier.levels):
        assert hm.level_nodes[l] == lv.n
        lx, ly = hm.coords(l)
        kh = _key(lx, ly, hm.M)
        ko = _key(lv.NX, lv.NY, om.M)
        perm_o = {int(k): i for i, k in enumerate(ko)}
        assert set(perm_o) == set(int(k) for k in kh)
        to_o = np.array([perm_o[int(k)] for k in kh])
        f = hm.flags(l)
        assert np.array_equal((f & 1) != 0, lv.dirichlet[to_o])
        assert np.array_equal((f & 8) != 0, lv.edge[to_o])
        assert np.array_equal((f & 16) != 0, lv.leafcell_node[to_o])
        assert np.array_equal((f & 32) != 0, lv.leafcell_node[to_o] & ~lv.edge[to_o])
        li = hm.leaf_index(l)
        assert np.array_equal(X[li], lx) and np.array_equal(Y[li], ly)
        if l == 0:
            continue
        ptr, col, val = hm.prolongation(l)
        cx, cy = hm.coords(l - 1)
        got = {}
        for r in range(lv.n):
            for e in range(ptr[r], ptr[r + 1]):
                got[(int(kh[r]), int(_key(cx[col[e]], cy[col[e]], hm.M)))] = val[e]
        P = hier.P[l].tocoo()
        cl = hier.levels[l - 1]
        ref = {(int(ko[r]), int(_key(cl.NX[c], cl.NY[c], om.M))): v for r, c, v in zip(P.row, P.col, P.data)}
        assert got == ref


def test_every_free_leaf_node_copied_once(pair):
    om, hier, hm = pair
    X, Y = hm.coords()
    hits = np.zeros(hm.n, dtype=int)
    for l in range(hm.n_levels):
        f = hm.flags(l)
        li = hm.leaf_index(l)
        np.add.at(hits, li[(f & 32) != 0], 1)
    hang = (hm.flags() & 2) != 0
    assert np.all(hits[~hang] == 1) and np.all(hits[hang] == 0)


# ---- global-coarsening levels ---------------------------------------------
GC_CASES = [CASES[0], CASES[2], CASES[3], CASES[4]]


@pytest.mark.parametrize("ci", range(len(GC_CASES)))
@pytest.mark.parametrize("p", (1, 2))
def test_global_coarsening_levels_match_oracle(ci, p):
    """Every global-coarsening level of the library (node positions, Dirichlet
    and hanging flags, leaf position of each node, interpolation from the
    level below) against the oracle's cut meshes, matched by lattice
    coordinates; the interpolation weights are exact dyadic values."""
    import scipy.sparse as sp
    from oracle.gc import GlobalHierarchy
    c = GC_CASES[ci]
    om = Mesh(c["n_base"], c["n_local"], p, coarse=c["coarse"], band=c["band"])
    gh = GlobalHierarchy(om)
    hm = lib_mod.HostMesh(c["n_base"], c["n_local"], p, coarse=c["coarse"], band=c["band"], mg_global=True)
    assert len(gh.meshes) == hm.n_levels
    maps = []
    for k, m in enumerate(gh.meshes):
        X, Y = hm.gc_coords(k)
        assert X.size == m.n_nodes
        kh = _key(X, Y, hm.M)
        ko = _key(m.NX, m.NY, m.M)
        pos = {int(v): i for i, v in enumerate(ko)}
        h2o = np.array([pos[int(v)] for v in kh])
        maps.append(h2o)
        f = hm.gc_flags(k)
        assert np.array_equal((f & 1) != 0, m.dirichlet[h2o])
        assert np.array_equal((f & 2) != 0, m.hanging[h2o])
        li = hm.gc_leaf_index(k)
        lX, lY = hm.coords()
        assert np.array_equal(lX[li], X) and np.array_equal(lY[li], Y)
    for k in range(1, len(gh.meshes)):
        ptr, col, val = hm.gc_interpolation(k)
        n_f, n_c = maps[k].size, maps[k - 1].size
        Ph = sp.csr_matrix((val, col, ptr), shape=(n_f, n_c))
        # oracle interpolation in library numbering
        Po = gh.I[k][maps[k]][:, maps[k - 1]]
        assert abs(Ph - Po).max() == 0.0, k
