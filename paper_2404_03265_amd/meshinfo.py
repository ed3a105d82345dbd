"""Host-only view of the library's mesh (pff_mesh.h): no GPU needed."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib


def _np(a):
    return a.ctypes.data_as(C.c_void_p)


class HostMesh:
    def __init__(self, n_base, n_local, degree, coarse=16, band=(2.0, 0.5), tile=(0, 0)):
        self.lib = _lib.load()
        spec = _lib.MeshSpec(n_base, n_local, degree, coarse, band[0], band[1], tile[0], tile[1])
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
