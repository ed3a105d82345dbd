/*
 * pff_mesh.h - host-only inspection of the mesh the library builds (no GPU
 * needed). Same geometry rules as pff_create (pff.h): quadtree of
 * (-10,10)^2 with band refinement and 2:1 face balancing (Kolditz & Wick,
 * Sec. 4, Table 1), Q_p nodes on an integer lattice, hanging-node constraints
 * and the local-smoothing level hierarchy of Sec. 3.2.
 *
 * All pointers are HOST pointers owned by the caller; sizes come from
 * pff_mesh_sizes. Return 0 on success, PFF_E_ARG / PFF_E_MESH otherwise.
 */
#ifndef PFF_MESH_H_
#define PFF_MESH_H_

#include "pff.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pff_mesh pff_mesh;

/* Build the mesh on the host. */
int pff_mesh_build(const pff_mesh_spec* spec, pff_mesh** out);
int pff_mesh_free(pff_mesh* m);
/* n_nodes: leaf nodes; n_levels; level_nodes (n_levels entries, nullable);
 * M: lattice units across the domain (x = -10 + 20 X / M). */
int pff_mesh_sizes(const pff_mesh* m, int64_t* n_nodes, int32_t* n_levels, int64_t* level_nodes, int64_t* M);
/* Number of leaf cells. */
int pff_mesh_leaf_cells(const pff_mesh* m, int64_t* n_cells);
/* xy: 2 n int32 (all X, then all Y) of the leaf (level = -1) or a level. */
int pff_mesh_coords(const pff_mesh* m, int32_t level, int32_t* xy);
/* flags: n bytes, bits as in pff_node_flags (active bits are never set here). */
int pff_mesh_flags(const pff_mesh* m, int32_t level, uint8_t* flags);
/* Hanging constraints: *count entries; node (count), masters and weights
 * (3 per entry, unused slots -1 / 0). Pass NULL arrays to query the count. */
int pff_mesh_hanging(const pff_mesh* m, int64_t* count, int32_t* node, int32_t* masters, double* weights);
/* Prolongation from level-1 to level (level >= 1) in CSR form over the level's
 * nodes: ptr (n_level + 1), col and val (nnz). NULL arrays query nnz. */
int pff_mesh_prolongation(const pff_mesh* m, int32_t level, int64_t* nnz, int64_t* ptr, int32_t* col, double* val);
/* Leaf node at the position of every node of a level (n_level int32). */
int pff_mesh_leaf_index(const pff_mesh* m, int32_t level, int32_t* idx);
/* Tile statistics: tiles, cell records (one per cell), largest tile. */
int pff_mesh_tile_stats(const pff_mesh* m, int32_t level, int64_t* n_tiles, int64_t* n_records, int64_t* max_cells);
/* Tile tables of the leaf (level = -1) or a level operator, as the device
 * kernels read them. sizes (10 int64, required): n_tiles, length of the
 * shared list, n_private, n_shared, n_slots, cell records, regular tiles,
 * largest local node count, hanging-node records, largest number of
 * hanging-node colours of a tile. Arrays are optional (NULL skips):
 * tile_info (32 per tile: private start, private count, shared-list start,
 * shared count, first cell record, cell count, cell colours, first slot,
 * first hanging record, hanging records, hanging colours, number of runs of
 * consecutive ids in the shared list (0 = more than 8), 4 unused, 8 run start
 * ids, 8 run offsets into the shared list), shared
 * (global ids), shared_ptr (n_shared + 1), shared_slot (n_slots: slots of each
 * shared node in ascending tile order; slots are tile-major), cell_loc and
 * cell_loc_sub ((p+1)^2 per record, local ids: private nodes first, then the
 * tile's shared list; own nodes, and with hanging faces replaced by the coarse
 * face's nodes), cell_info (per record), order (n_tiles: tiles without
 * hanging-face cells first), hang_rec (4 per record: hanging node, masters),
 * hang_w (3 per record), hang_col (per record). */
int pff_mesh_tile_tables(const pff_mesh* m, int32_t level, int64_t* sizes, int32_t* tile_info, int32_t* shared,
                         int32_t* shared_ptr, int32_t* shared_slot, uint16_t* cell_loc, uint16_t* cell_loc_sub,
                         uint16_t* cell_info, int32_t* order, uint16_t* hang_rec, double* hang_w, uint8_t* hang_col);

/* Global-coarsening levels (spec.mg_global != 0; PFF_E_ARG otherwise), level
 * 0 .. n_levels - 1, the last one being the leaf mesh: node count, lattice
 * coordinates (2 n int32), flags (n bytes: 1 Dirichlet, 2 hanging), leaf node
 * at each node's position (n int32), and the interpolation from level - 1
 * (level >= 1; CSR over this level's nodes: ptr n + 1, col and val nnz; NULL
 * arrays query nnz). */
int pff_mesh_gc_nodes(const pff_mesh* m, int32_t level, int64_t* n);
int pff_mesh_gc_coords(const pff_mesh* m, int32_t level, int32_t* xy);
int pff_mesh_gc_flags(const pff_mesh* m, int32_t level, uint8_t* flags);
int pff_mesh_gc_leaf_index(const pff_mesh* m, int32_t level, int32_t* idx);
int pff_mesh_gc_interpolation(const pff_mesh* m, int32_t level, int64_t* nnz, int64_t* ptr, int32_t* col,
                              double* val);

#ifdef __cplusplus
}
#endif
#endif /* PFF_MESH_H_ */
