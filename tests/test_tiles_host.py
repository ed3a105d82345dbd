"""Tile tables of the cell-partition kernels, checked on the CPU.

The device kernels stage a tile's local nodes, let every cell of the tile add
its contribution to them in colour phases, write private nodes directly and
leave partial sums of shared nodes in per-tile slots that a fix-up pass adds.
Hanging nodes are interpolated from their masters after staging and their
sums distributed back to the masters after accumulation. Here that data flow
is replayed in numpy with a random dense matrix per cell and compared with
the product through the constraint matrix, and the structural invariants the
kernels rely on are checked (partition of cells and nodes, slot lists,
colourings of cells and of hanging-node records, constraint records)."""
import numpy as np
import pytest

from oracle.mesh import Mesh

lib_mod = pytest.importorskip("paper_2404_03265_amd.meshinfo")


def _built():
    try:
        from paper_2404_03265_amd import _lib
        _lib.load()
        return True
    except Exception:
        return False


pytestmark = pytest.mark.skipif(not _built(), reason="libpff.so not built")

CASES = [
    dict(n_base=16, n_local=2, coarse=4, band=(3.0, 1.0)),
    dict(n_base=32, n_local=2, coarse=16, band=(2.0, 0.5)),
    dict(n_base=32, n_local=0, coarse=8, band=(2.0, 0.5)),     # uniform: no hanging nodes
    dict(n_base=40, n_local=2, coarse=10, band=(3.0, 1.0)),    # the paper's mesh family
]
TILES = [(0, 0), (1, 1), (3, 5), (8, 8), (16, 16)]


def _global_ids(t, tile):
    o0, no, s0, ns = (int(v) for v in t["tile_info"][tile, :4])
    return np.concatenate([np.arange(o0, o0 + no), t["shared"][s0:s0 + ns].astype(np.int64)])


def _replay(t, n, A, x, sub):
    """The kernels' data flow: stage, interpolate hanging nodes from their
    masters, per-cell product over the cells' own nodes, colour phases,
    distribute hanging-node sums to the masters, private epilogue, shared
    slots, fix-up in ascending slot-list order. With sub=True: the per-cell
    form over the substituted footprints and no node-level constraints."""
    y = np.full(n, np.nan)
    part = np.full(t["n_slots"], np.nan)
    loc_all = t["cell_loc_sub"] if sub else t["cell_loc"]
    for tile in range(t["n_tiles"]):
        o0, no, s0, ns, c0, nc, ncol, slot0, h0, nh, nhcol = (int(v) for v in t["tile_info"][tile, :11])
        g = _global_ids(t, tile)
        xl = x[g].copy()
        recs = t["hang_rec"][h0:h0 + nh].astype(np.int64)
        ws = t["hang_w"][h0:h0 + nh]
        if not sub:
            for r in range(nh):
                xl[recs[r, 0]] = ws[r] @ xl[recs[r, 1:]]
        acc = np.zeros(no + ns)
        for col in range(ncol):
            for r in range(c0, c0 + nc):
                if (int(t["cell_info"][r]) >> 11) & 15 != col:
                    continue
                loc = loc_all[r].astype(np.int64)
                np.add.at(acc, loc, A[r] @ xl[loc])
        if not sub:
            for col in range(nhcol):
                for r in range(nh):
                    if t["hang_col"][h0 + r] == col:
                        np.add.at(acc, recs[r, 1:], ws[r] * acc[recs[r, 0]])
        y[o0:o0 + no] = acc[:no]
        part[slot0:slot0 + ns] = acc[no:]
    for s in range(t["n_shared"]):
        v = 0.0
        for j in t["shared_slot"][t["shared_ptr"][s]:t["shared_ptr"][s + 1]]:
            v += part[j]
        y[t["n_private"] + s] = v
    return y


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("tile", TILES, ids=lambda v: f"{v[0]}x{v[1]}")
def test_tile_tables(case, p, tile):
    c = CASES[case]
    hm = lib_mod.HostMesh(c["n_base"], c["n_local"], p, coarse=c["coarse"], band=c["band"], tile=tile)
    om = Mesh(c["n_base"], c["n_local"], p, coarse=c["coarse"], band=c["band"])
    nl = (p + 1) ** 2
    rng = np.random.default_rng(100 * case + 10 * p + tile[0])
    hnode, hmast, hw = hm.hanging()
    for level in [-1] + list(range(hm.n_levels)):
        t = hm.tile_tables(level)
        n = hm.n if level < 0 else hm.level_nodes[level]
        n_cells = om.cell_level.size if level < 0 else len(om.level_cells(level))
        ti = t["tile_info"]
        hanging = (hm.flags(level) & 2) != 0
        # cells: one record per cell, records of a tile consecutive
        assert t["cell_loc"].shape[0] == n_cells == int(ti[:, 5].sum())
        assert np.array_equal(ti[:, 4], np.concatenate([[0], np.cumsum(ti[:-1, 5])]))
        tx, ty = tile if tile[0] > 0 else ((16, 16) if p == 1 else (8, 8))
        assert ti[:, 5].max() <= tx * ty
        # nodes: private ranges partition [0, n_private), shared nodes follow
        assert t["n_private"] + t["n_shared"] == n
        assert np.array_equal(ti[:, 0], np.concatenate([[0], np.cumsum(ti[:-1, 1])]))
        assert int(ti[:, 1].sum()) == t["n_private"]
        # slots: tile-major, one per entry of the tiles' shared lists, each
        # listed by exactly one shared node
        assert np.array_equal(ti[:, 7], np.concatenate([[0], np.cumsum(ti[:-1, 3])]))
        assert int(ti[:, 3].sum()) == t["n_slots"] == t["shared_ptr"][-1]
        assert np.array_equal(np.sort(t["shared_slot"]), np.arange(t["n_slots"]))
        assert np.all(np.diff(t["shared_ptr"]) >= 2)
        # hanging records: consecutive per tile
        assert np.array_equal(ti[:, 8], np.concatenate([[0], np.cumsum(ti[:-1, 9])]))
        if level >= 0:
            assert t["hang_rec"].shape[0] == 0
        slot_tile = np.repeat(np.arange(t["n_tiles"]), ti[:, 3])
        slot_node = t["shared"].astype(np.int64)
        touched = [set() for _ in range(n)]
        for tile_id in range(t["n_tiles"]):
            o0, no, s0, ns, c0, nc, ncol, slot0, h0, nh, nhcol = (int(v) for v in ti[tile_id, :11])
            sh = t["shared"][s0:s0 + ns]
            assert np.all(sh >= t["n_private"]) and np.all(np.diff(sh) > 0)
            # runs of consecutive ids in the header reproduce the list
            nrun = int(ti[tile_id, 11])
            if ns and nrun:
                starts, offs = ti[tile_id, 16:16 + nrun], ti[tile_id, 24:24 + nrun]
                assert offs[0] == 0 and np.all(np.diff(offs) > 0)
                r = np.arange(ns)
                k = np.searchsorted(offs, r, side="right") - 1
                assert np.array_equal(starts[k] + (r - offs[k]), sh)
            elif ns:
                assert 1 + np.sum(np.diff(sh) != 1) > 8
            g = _global_ids(t, tile_id)
            assert no + ns <= t["max_local"]
            locs = t["cell_loc"][c0:c0 + nc].astype(np.int64)
            lsub = t["cell_loc_sub"][c0:c0 + nc].astype(np.int64)
            both = np.concatenate([locs, lsub], axis=1)
            assert both.max(initial=0) < no + ns
            for gi in np.unique(g[both.reshape(-1)]):
                touched[gi].add(tile_id)
            # every shared local node is touched by this tile's cells
            assert set(np.unique(both[both >= no])) == set(range(no, no + ns))
            # cells of one colour share no local node of either footprint
            cols = (t["cell_info"][c0:c0 + nc].astype(np.int64) >> 11) & 15
            assert cols.max(initial=0) < max(ncol, 1)
            for col in range(ncol):
                for r1 in np.flatnonzero(cols == col):
                    for r2 in np.flatnonzero(cols == col):
                        if r1 < r2:
                            assert not (set(both[r1]) & set(both[r2]))
            # non-hanging cells: both footprints agree
            plain = (t["cell_info"][c0:c0 + nc] & 15) == 0
            assert np.array_equal(locs[plain], lsub[plain])
            # hanging records: exactly the hanging nodes among the cells' own
            # nodes, masters and weights as in the mesh's constraint list
            recs = t["hang_rec"][h0:h0 + nh].astype(np.int64)
            hgl = g[recs[:, 0]] if nh else np.zeros(0, dtype=np.int64)
            own = np.unique(g[locs.reshape(-1)])
            assert set(hgl.tolist()) == set(own[hanging[own]].tolist())
            for r in range(nh):
                k = int(np.flatnonzero(hnode == hgl[r])[0])
                npm = p + 1
                assert np.array_equal(g[recs[r, 1:1 + npm]], hmast[k, :npm])
                assert np.allclose(t["hang_w"][h0 + r, :npm], hw[k, :npm], rtol=0, atol=0)
                assert np.all(t["hang_w"][h0 + r, npm:] == 0.0)
            hcol = t["hang_col"][h0:h0 + nh]
            assert hcol.max(initial=0) < max(nhcol, 1)
            for col in range(nhcol):
                m = recs[hcol == col][:, 1:1 + p + 1].reshape(-1)
                assert np.unique(m).size == m.size
        for gi in range(t["n_private"]):
            assert len(touched[gi]) <= 1
        for s in range(t["n_shared"]):
            sl = t["shared_slot"][t["shared_ptr"][s]:t["shared_ptr"][s + 1]]
            assert np.all(slot_node[sl] == t["n_private"] + s)
            tiles_s = slot_tile[sl]
            assert np.all(np.diff(tiles_s) > 0)           # ascending tile order
            assert set(tiles_s.tolist()) == touched[t["n_private"] + s]
        assert np.array_equal(t["order"], np.arange(t["n_tiles"]))
        # replay of the data flow against a direct product with the
        # constraint matrix C: y = C^T sum_cells A_c (C x)|_c on unconstrained rows
        A = rng.standard_normal((n_cells, nl, nl))
        x = rng.standard_normal(n)
        Cx = x.copy()
        if level < 0:
            for k in range(hnode.size):
                Cx[hnode[k]] = hw[k, :p + 1] @ x[hmast[k, :p + 1]]
        rec_tile = np.repeat(np.arange(t["n_tiles"]), ti[:, 5])
        gids = [_global_ids(t, k) for k in range(t["n_tiles"])]
        z = np.zeros(n)
        y_sub = np.zeros(n)
        for r in range(n_cells):
            g = gids[rec_tile[r]][t["cell_loc"][r].astype(np.int64)]
            np.add.at(z, g, A[r] @ Cx[g])
            gs = gids[rec_tile[r]][t["cell_loc_sub"][r].astype(np.int64)]
            np.add.at(y_sub, gs, A[r] @ x[gs])
        y_ref = z.copy()
        if level < 0:
            for k in range(hnode.size):
                np.add.at(y_ref, hmast[k, :p + 1], hw[k, :p + 1] * z[hnode[k]])
        y = _replay(t, n, A, x, sub=False)
        free = ~hanging
        assert np.allclose(y[free], y_ref[free], rtol=1e-12, atol=1e-12)
        y2 = _replay(t, n, A, x, sub=True)
        assert np.allclose(y2, y_sub, rtol=1e-12, atol=1e-12)


def test_tile_shape_limit():
    with pytest.raises(RuntimeError):
        lib_mod.HostMesh(32, 1, 1, tile=(32, 16))
