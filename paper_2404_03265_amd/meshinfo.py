"""Host-only view of the library's mesh (pff_mesh.h): no GPU needed."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib


def _np(a):
    return a.ctypes.data_as(C.c_void_p)


class HostMesh:
    def __init__(self, n_base, n_local, degree, coarse=16, band=(2.0, 0.5), tile=(0, 0), mg_global=False):
        self.lib = _lib.load()
        spec = _lib.MeshSpec(n_base, n_local, degree, coarse, band[0], band[1], tile[0], tile[1], int(mg_global))
        h = C.c_void_p()
        rc = self.lib.pff_mesh_build(C.byref(spec), C.byref(h))
        if rc != 0:
            raise RuntimeError(f"pff_mesh_build failed ({rc})")
        self.h = h
        n, nl, M = C.c_int64(), C.c_int32(), C.c_int64()
        self.lib.pff_mesh_sizes(self.h, C.byref(n), C.byref(nl), None, C.byref(M))
        self.n, self.n_levels, self.M = n.value, nl.value, M.value
        lv = np.zeros(self.n_levels, dtype=np.int64)
        self.lib.pff_mesh_sizes(self.h, None, None, _np(lv), None)
        self.level_nodes = [int(x) for x in lv]
        self.degree = degree

    def __del__(self):
        try:
            self.lib.pff_mesh_free(self.h)
        except Exception:
            pass

    def _nn(self, level):
        return self.n if level < 0 else self.level_nodes[level]

    def leaf_cells(self):
        c = C.c_int64()
        assert self.lib.pff_mesh_leaf_cells(self.h, C.byref(c)) == 0
        return c.value

    def coords(self, level=-1):
        xy = np.zeros(2 * self._nn(level), dtype=np.int32)
        assert self.lib.pff_mesh_coords(self.h, level, _np(xy)) == 0
        return xy.reshape(2, -1)

    def flags(self, level=-1):
        f = np.zeros(self._nn(level), dtype=np.uint8)
        assert self.lib.pff_mesh_flags(self.h, level, _np(f)) == 0
        return f

    def hanging(self):
        cnt = C.c_int64()
        self.lib.pff_mesh_hanging(self.h, C.byref(cnt), None, None, None)
        node = np.zeros(cnt.value, dtype=np.int32)
        mast = np.zeros(3 * cnt.value, dtype=np.int32)
        w = np.zeros(3 * cnt.value)
        self.lib.pff_mesh_hanging(self.h, C.byref(cnt), _np(node), _np(mast), _np(w))
        return node, mast.reshape(-1, 3), w.reshape(-1, 3)

    def prolongation(self, level):
        nnz = C.c_int64()
        assert self.lib.pff_mesh_prolongation(self.h, level, C.byref(nnz), None, None, None) == 0
        ptr = np.zeros(self.level_nodes[level] + 1, dtype=np.int64)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value)
        self.lib.pff_mesh_prolongation(self.h, level, C.byref(nnz), _np(ptr), _np(col), _np(val))
        return ptr, col, val

    def leaf_index(self, level):
        idx = np.zeros(self.level_nodes[level], dtype=np.int32)
        assert self.lib.pff_mesh_leaf_index(self.h, level, _np(idx)) == 0
        return idx

    def tile_stats(self, level=-1):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self.lib.pff_mesh_tile_stats(self.h, level, C.byref(a), C.byref(b), C.byref(c))
        return a.value, b.value, c.value

    def tile_tables(self, level=-1):
        """Tile tables as the device kernels read them (see pff_mesh_tile_tables)."""
        sz = np.zeros(10, dtype=np.int64)
        assert self.lib.pff_mesh_tile_tables(self.h, level, _np(sz), *([None] * 12)) == 0
        n_tiles, n_sh_list, n_priv, n_sh, n_slots, n_rec, n_reg, max_local, n_hang, max_hcol = (int(v) for v in sz)
        nl = (self.degree + 1) ** 2
        t = dict(n_tiles=n_tiles, n_private=n_priv, n_shared=n_sh, n_slots=n_slots, n_regular=n_reg,
                 max_local=max_local, max_hang_colors=max_hcol,
                 tile_info=np.zeros((n_tiles, 32), dtype=np.int32),
                 shared=np.zeros(n_sh_list, dtype=np.int32),
                 shared_ptr=np.zeros(n_sh + 1, dtype=np.int32),
                 shared_slot=np.zeros(n_slots, dtype=np.int32),
                 cell_loc=np.zeros((n_rec, nl), dtype=np.uint16),
                 cell_loc_sub=np.zeros((n_rec, nl), dtype=np.uint16),
                 cell_info=np.zeros(n_rec, dtype=np.uint16),
                 order=np.zeros(n_tiles, dtype=np.int32),
                 hang_rec=np.zeros((n_hang, 4), dtype=np.uint16),
                 hang_w=np.zeros((n_hang, 3)),
                 hang_col=np.zeros(n_hang, dtype=np.uint8))
        keys = ("tile_info", "shared", "shared_ptr", "shared_slot", "cell_loc", "cell_loc_sub", "cell_info",
                "order", "hang_rec", "hang_w", "hang_col")
        assert self.lib.pff_mesh_tile_tables(self.h, level, _np(sz), *[_np(t[k]) for k in keys]) == 0
        return t

    # ---- global-coarsening levels (mg_global=True) -----------------------
    def gc_nodes(self, level):
        n = C.c_int64()
        assert self.lib.pff_mesh_gc_nodes(self.h, level, C.byref(n)) == 0
        return n.value

    def gc_coords(self, level):
        xy = np.zeros(2 * self.gc_nodes(level), dtype=np.int32)
        assert self.lib.pff_mesh_gc_coords(self.h, level, _np(xy)) == 0
        return xy.reshape(2, -1)

    def gc_flags(self, level):
        f = np.zeros(self.gc_nodes(level), dtype=np.uint8)
        assert self.lib.pff_mesh_gc_flags(self.h, level, _np(f)) == 0
        return f

    def gc_leaf_index(self, level):
        idx = np.zeros(self.gc_nodes(level), dtype=np.int32)
        assert self.lib.pff_mesh_gc_leaf_index(self.h, level, _np(idx)) == 0
        return idx

    def gc_interpolation(self, level):
        """CSR (ptr, col, val) of the interpolation from level - 1."""
        nnz = C.c_int64()
        assert self.lib.pff_mesh_gc_interpolation(self.h, level, C.byref(nnz), None, None, None) == 0
        n = self.gc_nodes(level)
        ptr = np.zeros(n + 1, dtype=np.int64)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value, dtype=np.float64)
        assert self.lib.pff_mesh_gc_interpolation(self.h, level, C.byref(nnz), _np(ptr), _np(col), _np(val)) == 0
        return ptr, col, val
