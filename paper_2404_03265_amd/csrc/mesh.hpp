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

// One set of cells processed by tiles. The tiles partition the cells; the
// local nodes of a tile are the nodes its cells touch. A node touched by the
// cells of one tile only (or by none, like a hanging node, which then belongs
// to the tile of the cell holding it) is private to that tile; a node touched
// by several tiles is shared. Numbering: private nodes grouped by tile, then
// shared nodes. Every tile writes a partial sum per shared local node into a
// slot of its own; a fix-up pass adds the slots of each shared node in
// ascending tile order, so results do not depend on scheduling.
struct TileSet {
  int p = 1;
  int n_tiles = 0;
  int max_cells = 0;        // largest cell count of a tile
  int max_local = 0;        // largest local node count of a tile
  int max_owned = 0;        // largest private node count of a tile
  int n_regular = 0;        // tiles without hanging-face cells (listed first in `order`)
  int64_t n_private = 0;    // nodes [0, n_private) are private
  int64_t n_shared = 0;     // nodes [n_private, n_private + n_shared) are shared
  int64_t n_slots = 0;      // partial-sum slots
  std::vector<int32_t> order;        // tile ids: regular tiles, then tiles with hanging cells
  std::vector<int32_t> tile_info;    // TILE_STRIDE ints per tile, see TILE_* below
  std::vector<int32_t> shared;       // global ids of each tile's shared local nodes
  std::vector<int32_t> shared_ptr;   // n_shared + 1 offsets into shared_slot
  std::vector<int32_t> shared_slot;  // slots of a shared node, ascending tile order
  // cell footprints in local ids, (p+1)^2 per cell record: the cell's own
  // nodes (hanging nodes included), and the same with the slots of a hanging
  // face replaced by the nodes of the coarse face (per-cell constraint form)
  std::vector<uint16_t> cell_loc;
  std::vector<uint16_t> cell_loc_sub;
  std::vector<uint16_t> cell_info;   // info word per cell record
  int64_t n_cell_records = 0;
  // hanging nodes of a tile, one record each: local id of the hanging node
  // and of its p+1 masters (unused slots repeat master 0 with weight 0),
  // weights, and a colour such that records of one colour share no master
  std::vector<uint16_t> hang_rec;    // 4 per record
  std::vector<double> hang_w;        // 3 per record
  std::vector<uint8_t> hang_col;     // 1 per record
  int max_hang_colors = 0;
};
// Per tile: private node range, shared local node list, cell records, number
// of cell colours, first partial-sum slot (slots are consecutive per tile:
// entry r of the tile's shared list writes slot TILE_SLOT0 + r), hanging-node
// records and their number of colours, and the shared list as at most
// TILE_MAX_RUNS runs of consecutive node ids (TILE_NRUN = 0: read the list):
// entry r lies in the last run k with TILE_RUN_OFF + k <= r and has id
// TILE_RUN_START + k's value + (r - offset).
constexpr int TILE_MAX_RUNS = 8;
// slots per shared node in the fix-up table: a node of a conforming corner
// touches 2 x 2 tiles; tables of meshes with more use a wider row
constexpr int SHARED_SLOTS = 4;
enum {
  TILE_OWNED0 = 0, TILE_NOWNED, TILE_SHARED0, TILE_NSHARED, TILE_CELL0, TILE_NCELL, TILE_NCOLOR, TILE_SLOT0,
  TILE_HANG0, TILE_NHANG, TILE_NHCOLOR, TILE_NRUN,
  TILE_RUN_START = 16, TILE_RUN_OFF = TILE_RUN_START + TILE_MAX_RUNS,
  TILE_STRIDE = TILE_RUN_OFF + TILE_MAX_RUNS
};

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

// A level of global-coarsening multigrid: the quadtree cut off at depth
// `level` (leaves finer than that replaced by their ancestor), a complete
// mesh of the domain with its own hanging nodes. Levels up to the base mesh
// are uniform and identical to the local-smoothing levels (own = false: the
// tables of Mesh::levels serve both); the last level is the leaf mesh itself
// (own = false as well). P interpolates the previous level's finite-element
// function at this level's nodes (rows: this level's nodes); PT is its
// transpose.
struct GcLevel {
  int level = 0;
  bool own = false;
  int64_t n = 0;
  std::vector<int32_t> NX, NY;
  std::vector<uint8_t> flags;       // NODE_DIRICHLET | NODE_HANGING
  std::vector<int32_t> leaf_index;  // leaf node at the same position
  TileSet tiles;
  Csr P, PT;
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
  int tile_x = 0;  // cells per tile in x (0 = default for the degree)
  int tile_y = 0;
  bool mg_global = false;  // also build the global-coarsening levels
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
  std::vector<GcLevel> gc;       // global-coarsening levels (spec.mg_global)
  std::string error;

  bool build(const MeshSpec& s);
};

}  // namespace pff
