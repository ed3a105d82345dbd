// Host-side quadtree mesh, tile decomposition and multigrid level tables for
// the matrix-free phase-field operator (Kolditz & Wick, Sec. 3.2-3.3 and
// Sec. 4). Everything here runs once at context creation; device kernels
// only read the flat tables it produces.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace pff {

// Bits of a per-cell info word (uint16).
enum : uint16_t {
  CELL_HANG_L = 1u << 0,   // left face lies on a coarser neighbour's face
  CELL_HANG_R = 1u << 1,
  CELL_HANG_B = 1u << 2,
  CELL_HANG_T = 1u << 3,
  CELL_CX = 1u << 4,       // child position inside the parent (x)
  CELL_CY = 1u << 5,       // child position inside the parent (y)
  CELL_LEVEL_SHIFT = 6,    // 5 bits: refinement level
  CELL_COLOR_SHIFT = 11,   // 5 bits: colour inside its tile
};

// Bits of a per-node flag byte.
enum : uint8_t {
  NODE_DIRICHLET = 1u << 0,  // u fixed to zero (boundary of the domain)
  NODE_HANGING = 1u << 1,    // constrained to the coarse face trace
  NODE_ACTIVE = 1u << 2,     // phase field fixed (set per state)
  NODE_EDGE = 1u << 3,       // level node on the refinement edge
  NODE_LEAFCELL = 1u << 4,   // level node belongs to a level cell that is a leaf
  NODE_COPY = 1u << 5,       // level node receives/returns a leaf value
};

// One set of cells processed by tiles: each tile owns a contiguous range of
// nodes and lists every cell contributing to them (own and halo cells).
struct TileSet {
  int p = 1;
  int n_tiles = 0;
  int max_cells = 0;        // largest cell count of a tile
  int max_local = 0;        // largest local node count of a tile
  int max_owned = 0;
  int typ_cells = 0;        // median cell count of a tile
  int n_regular = 0;        // tiles without hanging-face cells (listed first in `order`)
  std::vector<int32_t> order;       // tile ids: regular tiles, then tiles with hanging cells
  std::vector<int32_t> tile_info;   // 8 ints per tile, see TILE_* below
  std::vector<int32_t> halo;        // global node ids of halo nodes, per tile
  std::vector<uint16_t> cell_loc;   // (p+1)^2 local node ids per cell record
  std::vector<uint16_t> cell_info;  // info word per cell record
  int64_t n_cell_records = 0;
};
enum { TILE_OWNED0 = 0, TILE_NOWNED, TILE_HALO0, TILE_NHALO, TILE_CELL0, TILE_NCELL, TILE_NCOLOR, TILE_PAD };

// A CSR matrix with double weights (exact dyadic values).
struct Csr {
  int64_t rows = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

struct Level {
  int level = 0;
  int64_t n = 0;                 // level nodes
  int64_t n_cells = 0;
  std::vector<int32_t> NX, NY;   // lattice coordinates
  std::vector<uint8_t> flags;    // NODE_DIRICHLET | NODE_EDGE | NODE_LEAFCELL | NODE_COPY
  std::vector<int32_t> leaf_index;  // leaf node at the same position
  TileSet tiles;
  Csr P;    // prolongation from level-1 (rows: this level's nodes)
  Csr PT;   // its transpose (rows: level-1 nodes)
};

struct Hanging {
  int32_t node;
  int32_t master[3];
  double weight[3];
};

struct MeshSpec {
  int n_base = 128;
  int n_local = 2;
  int degree = 1;
  int coarse = 16;
  double band_x = 2.0;
  double band_y = 0.5;
  int tile_x = 0;  // owned cells per tile (0 = default for the degree)
  int tile_y = 0;
};

struct Mesh {
  MeshSpec spec;
  int p = 1, b = 0, lmax = 0, n_levels = 0;
  int64_t M = 0;                 // lattice units across the domain
  int64_t n_nodes = 0;
  int64_t n_leaf_cells = 0;
  std::vector<int32_t> NX, NY;
  std::vector<uint8_t> flags;    // NODE_DIRICHLET | NODE_HANGING
  std::vector<Hanging> hanging;
  std::vector<double> level_H;   // physical cell edge per level
  TileSet tiles;                 // leaf operator tiles
  std::vector<Level> levels;
  std::string error;

  bool build(const MeshSpec& s);
};

}  // namespace pff
