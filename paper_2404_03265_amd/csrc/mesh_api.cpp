// Host-only C ABI over the mesh builder (declared in pff_mesh.h).
#include <cstring>

#include "../../include/pff_mesh.h"
#include "mesh.hpp"

struct pff_mesh {
  pff::Mesh m;
};

namespace {
pff::MeshSpec to_spec(const pff_mesh_spec* s) {
  pff::MeshSpec ms;
  ms.n_base = s->n_base;
  ms.n_local = s->n_local;
  ms.degree = s->degree;
  ms.coarse = s->coarse > 0 ? s->coarse : 16;
  ms.band_x = s->band_x;
  ms.band_y = s->band_y;
  ms.tile_x = s->tile_x;
  ms.tile_y = s->tile_y;
  ms.mg_global = s->mg_global != 0;
  return ms;
}
bool bad_gc(const pff_mesh* m, int32_t level) {
  return !m || m->m.gc.empty() || level < 0 || level >= int32_t(m->m.gc.size());
}
// coordinates, flags and leaf positions of a global-coarsening level: its own
// tables, the shared local-smoothing level, or the leaf mesh
const std::vector<int32_t>& gc_x(const pff::Mesh& M, int k) {
  const pff::GcLevel& G = M.gc[k];
  return G.own ? G.NX : (k == M.lmax ? M.NX : M.levels[k].NX);
}
const std::vector<int32_t>& gc_y(const pff::Mesh& M, int k) {
  const pff::GcLevel& G = M.gc[k];
  return G.own ? G.NY : (k == M.lmax ? M.NY : M.levels[k].NY);
}
bool bad_level(const pff_mesh* m, int32_t level) {
  return !m || level < -1 || level >= int32_t(m->m.levels.size());
}
}  // namespace

extern "C" {

int pff_mesh_build(const pff_mesh_spec* spec, pff_mesh** out) {
  if (!spec || !out) return PFF_E_ARG;
  *out = nullptr;
  pff_mesh* m = new pff_mesh();
  try {
    if (!m->m.build(to_spec(spec))) {
      delete m;
      return PFF_E_MESH;
    }
  } catch (...) {
    delete m;
    return PFF_E_MESH;
  }
  *out = m;
  return PFF_OK;
}

int pff_mesh_free(pff_mesh* m) {
  delete m;
  return PFF_OK;
}

int pff_mesh_sizes(const pff_mesh* m, int64_t* n_nodes, int32_t* n_levels, int64_t* level_nodes, int64_t* M) {
  if (!m) return PFF_E_ARG;
  if (n_nodes) *n_nodes = m->m.n_nodes;
  if (n_levels) *n_levels = int32_t(m->m.levels.size());
  if (level_nodes)
    for (size_t l = 0; l < m->m.levels.size(); ++l) level_nodes[l] = m->m.levels[l].n;
  if (M) *M = m->m.M;
  return PFF_OK;
}

int pff_mesh_leaf_cells(const pff_mesh* m, int64_t* n_cells) {
  if (!m || !n_cells) return PFF_E_ARG;
  *n_cells = m->m.n_leaf_cells;
  return PFF_OK;
}

int pff_mesh_coords(const pff_mesh* m, int32_t level, int32_t* xy) {
  if (bad_level(m, level) || !xy) return PFF_E_ARG;
  const auto& X = level < 0 ? m->m.NX : m->m.levels[level].NX;
  const auto& Y = level < 0 ? m->m.NY : m->m.levels[level].NY;
  std::memcpy(xy, X.data(), X.size() * sizeof(int32_t));
  std::memcpy(xy + X.size(), Y.data(), Y.size() * sizeof(int32_t));
  return PFF_OK;
}

int pff_mesh_flags(const pff_mesh* m, int32_t level, uint8_t* flags) {
  if (bad_level(m, level) || !flags) return PFF_E_ARG;
  const auto& F = level < 0 ? m->m.flags : m->m.levels[level].flags;
  std::memcpy(flags, F.data(), F.size());
  return PFF_OK;
}

int pff_mesh_hanging(const pff_mesh* m, int64_t* count, int32_t* node, int32_t* masters, double* weights) {
  if (!m || !count) return PFF_E_ARG;
  *count = int64_t(m->m.hanging.size());
  for (size_t i = 0; i < m->m.hanging.size(); ++i) {
    const pff::Hanging& h = m->m.hanging[i];
    if (node) node[i] = h.node;
    for (int k = 0; k < 3; ++k) {
      if (masters) masters[3 * i + k] = h.master[k];
      if (weights) weights[3 * i + k] = h.weight[k];
    }
  }
  return PFF_OK;
}

int pff_mesh_prolongation(const pff_mesh* m, int32_t level, int64_t* nnz, int64_t* ptr, int32_t* col, double* val) {
  if (!m || !nnz || level < 1 || level >= int32_t(m->m.levels.size())) return PFF_E_ARG;
  const pff::Csr& P = m->m.levels[level].P;
  *nnz = int64_t(P.col.size());
  if (ptr) std::memcpy(ptr, P.ptr.data(), P.ptr.size() * sizeof(int64_t));
  if (col) std::memcpy(col, P.col.data(), P.col.size() * sizeof(int32_t));
  if (val) std::memcpy(val, P.val.data(), P.val.size() * sizeof(double));
  return PFF_OK;
}

int pff_mesh_leaf_index(const pff_mesh* m, int32_t level, int32_t* idx) {
  if (!m || !idx || level < 0 || level >= int32_t(m->m.levels.size())) return PFF_E_ARG;
  const auto& L = m->m.levels[level].leaf_index;
  std::memcpy(idx, L.data(), L.size() * sizeof(int32_t));
  return PFF_OK;
}

int pff_mesh_tile_stats(const pff_mesh* m, int32_t level, int64_t* n_tiles, int64_t* n_records, int64_t* max_cells) {
  if (bad_level(m, level)) return PFF_E_ARG;
  const pff::TileSet& t = level < 0 ? m->m.tiles : m->m.levels[level].tiles;
  if (n_tiles) *n_tiles = t.n_tiles;
  if (n_records) *n_records = t.n_cell_records;
  if (max_cells) *max_cells = t.max_cells;
  return PFF_OK;
}

int pff_mesh_tile_tables(const pff_mesh* m, int32_t level, int64_t* sizes, int32_t* tile_info, int32_t* shared,
                         int32_t* shared_ptr, int32_t* shared_slot, uint16_t* cell_loc, uint16_t* cell_loc_sub,
                         uint16_t* cell_info, int32_t* order, uint16_t* hang_rec, double* hang_w, uint8_t* hang_col) {
  if (bad_level(m, level) || !sizes) return PFF_E_ARG;
  const pff::TileSet& t = level < 0 ? m->m.tiles : m->m.levels[level].tiles;
  sizes[0] = t.n_tiles;
  sizes[1] = int64_t(t.shared.size());
  sizes[2] = t.n_private;
  sizes[3] = t.n_shared;
  sizes[4] = t.n_slots;
  sizes[5] = t.n_cell_records;
  sizes[6] = t.n_regular;
  sizes[7] = t.max_local;
  sizes[8] = int64_t(t.hang_col.size());
  sizes[9] = t.max_hang_colors;
  auto put = [](auto* dst, const auto& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
  };
  put(tile_info, t.tile_info);
  put(shared, t.shared);
  put(shared_ptr, t.shared_ptr);
  put(shared_slot, t.shared_slot);
  put(cell_loc, t.cell_loc);
  put(cell_loc_sub, t.cell_loc_sub);
  put(cell_info, t.cell_info);
  put(order, t.order);
  put(hang_rec, t.hang_rec);
  put(hang_w, t.hang_w);
  put(hang_col, t.hang_col);
  return PFF_OK;
}

int pff_mesh_gc_nodes(const pff_mesh* m, int32_t level, int64_t* n) {
  if (bad_gc(m, level) || !n) return PFF_E_ARG;
  *n = m->m.gc[level].n;
  return PFF_OK;
}

int pff_mesh_gc_coords(const pff_mesh* m, int32_t level, int32_t* xy) {
  if (bad_gc(m, level) || !xy) return PFF_E_ARG;
  const auto& X = gc_x(m->m, level);
  const auto& Y = gc_y(m->m, level);
  std::memcpy(xy, X.data(), X.size() * sizeof(int32_t));
  std::memcpy(xy + X.size(), Y.data(), Y.size() * sizeof(int32_t));
  return PFF_OK;
}

int pff_mesh_gc_flags(const pff_mesh* m, int32_t level, uint8_t* flags) {
  if (bad_gc(m, level) || !flags) return PFF_E_ARG;
  const pff::Mesh& M = m->m;
  const pff::GcLevel& G = M.gc[level];
  const int64_t n = G.n;
  for (int64_t i = 0; i < n; ++i) {
    uint8_t f;
    if (G.own) f = G.flags[i];
    else if (level == M.lmax) f = M.flags[i];
    else f = M.levels[level].flags[i];
    flags[i] = uint8_t(f & (pff::NODE_DIRICHLET | pff::NODE_HANGING));
  }
  return PFF_OK;
}

int pff_mesh_gc_leaf_index(const pff_mesh* m, int32_t level, int32_t* idx) {
  if (bad_gc(m, level) || !idx) return PFF_E_ARG;
  const pff::Mesh& M = m->m;
  const pff::GcLevel& G = M.gc[level];
  for (int64_t i = 0; i < G.n; ++i)
    idx[i] = G.own ? G.leaf_index[i] : (level == M.lmax ? int32_t(i) : M.levels[level].leaf_index[i]);
  return PFF_OK;
}

int pff_mesh_gc_interpolation(const pff_mesh* m, int32_t level, int64_t* nnz, int64_t* ptr, int32_t* col,
                              double* val) {
  if (bad_gc(m, level) || level < 1 || !nnz) return PFF_E_ARG;
  const pff::Mesh& M = m->m;
  const pff::Csr& P = (level <= M.b && level < M.lmax) ? M.levels[level].P : M.gc[level].P;
  *nnz = int64_t(P.col.size());
  if (ptr) std::memcpy(ptr, P.ptr.data(), P.ptr.size() * sizeof(int64_t));
  if (col) std::memcpy(col, P.col.data(), P.col.size() * sizeof(int32_t));
  if (val) std::memcpy(val, P.val.data(), P.val.size() * sizeof(double));
  return PFF_OK;
}

}  // extern "C"
