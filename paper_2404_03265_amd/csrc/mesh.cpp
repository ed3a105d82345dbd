// Quadtree mesh of (-10,10)^2 with band refinement and 2:1 face balance,
// Q_p nodes on an integer lattice, hanging-node constraints, tile tables for
// the cell-partition operator kernels and the local-smoothing level hierarchy.
//
// Geometry (Sec. 4, Fig. 1, Table 1): uniform base mesh reached from a coarse
// grid by global refinement, then local refinement of cells whose centre is
// strictly inside |x| < band_x, |y| < band_y. u is in H^1_0 (Sec. 2), so
// boundary nodes carry the Dirichlet flag.
//
// Lattice: M = coarse * 2^lmax * p units across the domain; a cell of level l
// has edge S_l = p * 2^(lmax - l) units; its Q_p node (a, b) sits at
// (i S_l + a S_l / p, j S_l + b S_l / p).
#include "mesh.hpp"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <numeric>
#include <stdexcept>
#include <unordered_map>
#include <unordered_set>

namespace pff {
namespace {

inline uint64_t ckey(int l, int64_t i, int64_t j) {
  return (uint64_t(l) << 58) | (uint64_t(i) << 29) | uint64_t(j);
}

struct Cell {
  int l;
  int32_t i, j;
};

// 1-D Lagrange basis on equispaced nodes k/p, evaluated at s.
double lagrange(int p, int k, double s) {
  double v = 1.0;
  for (int m = 0; m <= p; ++m)
    if (m != k) v *= (s - double(m) / p) / (double(k - m) / p);
  return v;
}

struct PosIndex {
  std::vector<uint64_t> keys;  // sorted position keys
  uint64_t W = 0;
  void build(std::vector<uint64_t>&& k, uint64_t w) {
    keys = std::move(k);
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    W = w;
  }
  int64_t find(int64_t X, int64_t Y) const {
    uint64_t k = uint64_t(Y) * W + uint64_t(X);
    auto it = std::lower_bound(keys.begin(), keys.end(), k);
    if (it == keys.end() || *it != k) return -1;
    return int64_t(it - keys.begin());
  }
  int64_t size() const { return int64_t(keys.size()); }
  int64_t X(int64_t n) const { return int64_t(keys[n] % W); }
  int64_t Y(int64_t n) const { return int64_t(keys[n] / W); }
};

// Generic tile builder. cell_tile partitions the cells into tiles; node_home
// names the tile of a cell holding each node (used for nodes no footprint
// touches). fp holds the substituted footprints, fp_raw the cells' own nodes
// (the same arrays where there are no hanging nodes); hang lists the hanging
// constraints by temporary node id. Produces the node renumbering and the
// tile tables (see TileSet).
void build_tiles(int p, int n_tiles, const std::vector<int32_t>& fp, const std::vector<int32_t>& fp_raw,
                 const std::unordered_map<int64_t, Hanging>& hang,
                 const std::vector<uint16_t>& info, const std::vector<int32_t>& cell_tile,
                 const std::vector<int32_t>& node_home,
                 const std::vector<int32_t>& NXt, const std::vector<int32_t>& NYt,
                 TileSet& T, std::vector<int32_t>& new_id) {
  const int NL = (p + 1) * (p + 1);
  const int64_t n_nodes = int64_t(node_home.size());
  const int64_t n_cells = int64_t(info.size());
  T.p = p;
  T.n_tiles = n_tiles;
  // first and last tile touching every node (through either footprint: a
  // tile writes the masters of its hanging nodes)
  std::vector<int32_t> tmin(n_nodes, INT32_MAX), tmax(n_nodes, -1);
  for (int64_t c = 0; c < n_cells; ++c) {
    const int32_t t = cell_tile[c];
    for (int k = 0; k < 2 * NL; ++k) {
      const int32_t nd = k < NL ? fp[c * NL + k] : fp_raw[c * NL + k - NL];
      tmin[nd] = std::min(tmin[nd], t);
      tmax[nd] = std::max(tmax[nd], t);
    }
  }
  // private nodes by (tile, Y, X), then shared nodes by (first tile, Y, X)
  std::vector<int32_t> key_tile(n_nodes);
  std::vector<char> is_shared(n_nodes, 0);
  for (int64_t nd = 0; nd < n_nodes; ++nd) {
    if (tmax[nd] < 0) {
      key_tile[nd] = node_home[nd];
    } else {
      key_tile[nd] = tmin[nd];
      is_shared[nd] = tmin[nd] != tmax[nd];
    }
  }
  std::vector<int32_t> order(n_nodes);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    if (is_shared[a] != is_shared[b]) return is_shared[a] < is_shared[b];
    if (key_tile[a] != key_tile[b]) return key_tile[a] < key_tile[b];
    if (NYt[a] != NYt[b]) return NYt[a] < NYt[b];
    return NXt[a] < NXt[b];
  });
  new_id.assign(n_nodes, -1);
  std::vector<int32_t> owned0(n_tiles + 1, 0);
  T.n_private = 0;
  for (int64_t r = 0; r < n_nodes; ++r) {
    new_id[order[r]] = int32_t(r);
    if (!is_shared[order[r]]) {
      owned0[key_tile[order[r]] + 1]++;
      T.n_private++;
    }
  }
  for (int t = 0; t < n_tiles; ++t) owned0[t + 1] += owned0[t];
  T.n_shared = n_nodes - T.n_private;
  // hanging constraints by new id
  std::unordered_map<int32_t, const Hanging*> hang_new;
  for (const auto& kv : hang) hang_new[new_id[kv.first]] = &kv.second;
  // cells of each tile, in cell order
  std::vector<int32_t> cell0(n_tiles + 1, 0), cells(n_cells);
  for (int64_t c = 0; c < n_cells; ++c) cell0[cell_tile[c] + 1]++;
  for (int t = 0; t < n_tiles; ++t) cell0[t + 1] += cell0[t];
  {
    std::vector<int32_t> fill(cell0.begin(), cell0.end() - 1);
    for (int64_t c = 0; c < n_cells; ++c) cells[fill[cell_tile[c]]++] = int32_t(c);
  }
  T.tile_info.assign(size_t(n_tiles) * TILE_STRIDE, 0);
  T.shared.clear();
  T.cell_loc.clear();
  T.cell_loc_sub.clear();
  T.cell_info.clear();
  T.hang_rec.clear();
  T.hang_w.clear();
  T.hang_col.clear();
  T.max_cells = T.max_local = T.max_owned = T.max_hang_colors = 0;
  std::vector<std::vector<std::pair<int32_t, int32_t>>> slots_of(T.n_shared);  // (tile, slot)
  std::vector<int32_t> sh, hn;
  int64_t slot0 = 0;
  for (int t = 0; t < n_tiles; ++t) {
    const int32_t o0 = owned0[t], no = owned0[t + 1] - owned0[t];
    sh.clear();
    hn.clear();
    for (int32_t r = cell0[t]; r < cell0[t + 1]; ++r)
      for (int k = 0; k < 2 * NL; ++k) {
        const int64_t c = cells[r];
        const int32_t g = new_id[k < NL ? fp[c * NL + k] : fp_raw[c * NL + k - NL]];
        if (g >= T.n_private) sh.push_back(g);
        else if (g < o0 || g >= o0 + no) throw std::runtime_error("private node of another tile");
        if (k >= NL && hang_new.count(g)) hn.push_back(g);
      }
    std::sort(sh.begin(), sh.end());
    sh.erase(std::unique(sh.begin(), sh.end()), sh.end());
    std::sort(hn.begin(), hn.end());
    hn.erase(std::unique(hn.begin(), hn.end()), hn.end());
    int32_t* ti = &T.tile_info[size_t(t) * TILE_STRIDE];
    ti[TILE_OWNED0] = o0;
    ti[TILE_NOWNED] = no;
    ti[TILE_SHARED0] = int32_t(T.shared.size());
    ti[TILE_NSHARED] = int32_t(sh.size());
    ti[TILE_CELL0] = int32_t(T.cell_info.size());
    ti[TILE_NCELL] = cell0[t + 1] - cell0[t];
    ti[TILE_SLOT0] = int32_t(slot0);
    for (size_t r = 0; r < sh.size(); ++r)
      slots_of[sh[r] - T.n_private].push_back({t, int32_t(slot0 + int64_t(r))});
    slot0 += int64_t(sh.size());
    if (slot0 > INT32_MAX) throw std::runtime_error("too many partial-sum slots");
    T.shared.insert(T.shared.end(), sh.begin(), sh.end());
    {
      int nrun = 0;
      bool fits = true;
      for (size_t r = 0; r < sh.size() && fits; ++r) {
        if (r > 0 && sh[r] == sh[r - 1] + 1) continue;
        if (nrun == TILE_MAX_RUNS) { fits = false; break; }
        ti[TILE_RUN_START + nrun] = sh[r];
        ti[TILE_RUN_OFF + nrun] = int32_t(r);
        ++nrun;
      }
      ti[TILE_NRUN] = fits ? nrun : 0;
    }
    const int nloc = no + int(sh.size());
    if (nloc > 65535) throw std::runtime_error("tile has more than 65535 local nodes");
    auto local = [&](int32_t g) -> uint16_t {
      return uint16_t(g < T.n_private ? g - o0
                                      : no + int32_t(std::lower_bound(sh.begin(), sh.end(), g) - sh.begin()));
    };
    // cells: local ids of both footprints; greedy colouring so that cells of
    // one colour share no node of either footprint
    std::vector<uint32_t> used(nloc, 0u);
    int ncol = 0;
    for (int32_t r = cell0[t]; r < cell0[t + 1]; ++r) {
      const int64_t c = cells[r];
      uint16_t loc[9], lsub[9];
      uint32_t busy = 0;
      for (int k = 0; k < NL; ++k) {
        loc[k] = local(new_id[fp_raw[c * NL + k]]);
        lsub[k] = local(new_id[fp[c * NL + k]]);
        busy |= used[loc[k]] | used[lsub[k]];
      }
      int col = 0;
      while (busy & (1u << col)) ++col;
      for (int k = 0; k < NL; ++k) {
        used[loc[k]] |= (1u << col);
        used[lsub[k]] |= (1u << col);
      }
      ncol = std::max(ncol, col + 1);
      for (int k = 0; k < NL; ++k) {
        T.cell_loc.push_back(loc[k]);
        T.cell_loc_sub.push_back(lsub[k]);
      }
      T.cell_info.push_back(uint16_t((info[c] & ~(uint16_t(31) << CELL_COLOR_SHIFT)) |
                                     (uint16_t(col) << CELL_COLOR_SHIFT)));
    }
    ti[TILE_NCOLOR] = ncol;
    if (ncol > 16) throw std::runtime_error("more than 16 colours in a tile");
    // hanging nodes touched by the tile's cells; colours over masters
    ti[TILE_HANG0] = int32_t(T.hang_col.size());
    ti[TILE_NHANG] = int32_t(hn.size());
    std::fill(used.begin(), used.end(), 0u);
    int nhcol = 0;
    for (int32_t g : hn) {
      const Hanging& h = *hang_new[g];
      uint16_t rec[4];
      double w[3] = {0.0, 0.0, 0.0};
      rec[0] = local(g);
      uint32_t busy = 0;
      for (int k = 0; k < 3; ++k) {
        const bool on = k <= p;
        rec[1 + k] = local(new_id[h.master[on ? k : 0]]);
        w[k] = on ? h.weight[k] : 0.0;
        busy |= used[rec[1 + k]];
      }
      int col = 0;
      while (busy & (1u << col)) ++col;
      if (col > 15) throw std::runtime_error("more than 16 hanging-node colours in a tile");
      for (int k = 0; k <= p; ++k) used[rec[1 + k]] |= (1u << col);
      nhcol = std::max(nhcol, col + 1);
      for (int k = 0; k < 4; ++k) T.hang_rec.push_back(rec[k]);
      for (int k = 0; k < 3; ++k) T.hang_w.push_back(w[k]);
      T.hang_col.push_back(uint8_t(col));
    }
    ti[TILE_NHCOLOR] = nhcol;
    T.max_hang_colors = std::max(T.max_hang_colors, nhcol);
    T.max_cells = std::max<int>(T.max_cells, ti[TILE_NCELL]);
    T.max_owned = std::max<int>(T.max_owned, no);
    T.max_local = std::max<int>(T.max_local, nloc);
  }
  // slots are tile-major (a tile writes its partial sums contiguously); the
  // fix-up reads the slots of shared node s from shared_slot in ascending
  // tile order
  T.n_slots = slot0;
  T.shared_ptr.assign(size_t(T.n_shared) + 1, 0);
  T.shared_slot.clear();
  T.shared_slot.reserve(size_t(slot0));
  for (int64_t s = 0; s < T.n_shared; ++s) {
    auto& v = slots_of[s];
    std::sort(v.begin(), v.end());
    if (v.size() < 2) throw std::runtime_error("shared node with fewer than two tiles");
    for (auto& e : v) T.shared_slot.push_back(e.second);
    T.shared_ptr[s + 1] = int32_t(T.shared_slot.size());
  }
  T.n_cell_records = int64_t(T.cell_info.size());
  // launch order: tiles in (level, row, column) order, so that a contiguous
  // chunk of the list covers neighbouring tiles; n_regular counts the tiles
  // without hanging-face cells
  T.order.resize(n_tiles);
  std::iota(T.order.begin(), T.order.end(), 0);
  T.n_regular = 0;
  for (int t = 0; t < n_tiles; ++t) {
    const int32_t* ti = &T.tile_info[size_t(t) * TILE_STRIDE];
    bool h = false;
    for (int c = 0; c < ti[TILE_NCELL]; ++c)
      if (T.cell_info[size_t(ti[TILE_CELL0]) + c] & 15u) h = true;
    if (!h) T.n_regular++;
  }
}

// Nodes, hanging-node constraints and tiles of the mesh made of `cells`
// (2:1-balanced quadtree leaves covering the domain): the leaf mesh, and the
// cut meshes of global-coarsening multigrid.
struct Part {
  int64_t n = 0;
  int64_t n_cells = 0;
  std::vector<int32_t> NX, NY;     // by final node id
  std::vector<uint8_t> flags;      // NODE_DIRICHLET | NODE_HANGING
  std::vector<Hanging> hanging;    // final ids
  TileSet tiles;
  PosIndex pos;                    // temporary ids by position
  std::vector<int32_t> new_id;     // temporary -> final id
  int32_t at(int64_t X, int64_t Y) const {
    int64_t t = pos.find(X, Y);
    return t < 0 ? -1 : new_id[t];
  }
};

bool build_part(int p, int lmax, int64_t coarse, int64_t M, int TX, int TY, std::vector<Cell> cells, Part& out,
                std::string& error) {
  auto S = [&](int l) { return int64_t(p) << (lmax - l); };
  auto ncell = [&](int l) { return int64_t(coarse) << l; };
  std::unordered_set<uint64_t> leaves;
  leaves.reserve(cells.size() * 2);
  for (const Cell& c : cells) leaves.insert(ckey(c.l, c.i, c.j));
  auto is_leaf = [&](int l, int64_t i, int64_t j) { return leaves.count(ckey(l, i, j)) > 0; };
  static const int DI[4] = {-1, 1, 0, 0}, DJ[4] = {0, 0, -1, 1};
  std::sort(cells.begin(), cells.end(), [](const Cell& a, const Cell& c) {
    if (a.l != c.l) return a.l < c.l;
    if (a.j != c.j) return a.j < c.j;
    return a.i < c.i;
  });
  out.n_cells = int64_t(cells.size());
  const int NL = (p + 1) * (p + 1);

  // ---- nodes (temporary numbering by position) ----------------------------
  const uint64_t W = uint64_t(M) + 1;
  {
    std::vector<uint64_t> k;
    k.reserve(cells.size() * NL);
    for (const Cell& c : cells) {
      int64_t Sl = S(c.l), h = Sl / p;
      for (int bb = 0; bb <= p; ++bb)
        for (int a = 0; a <= p; ++a) k.push_back(uint64_t(c.j * Sl + bb * h) * W + uint64_t(c.i * Sl + a * h));
    }
    out.pos.build(std::move(k), W);
  }
  const int64_t nn = out.pos.size();
  std::vector<int32_t> NXt(nn), NYt(nn);
  for (int64_t n = 0; n < nn; ++n) { NXt[n] = int32_t(out.pos.X(n)); NYt[n] = int32_t(out.pos.Y(n)); }

  // footprints with hanging substitution
  std::vector<int32_t> fp(cells.size() * NL), fp_raw(cells.size() * NL);
  std::vector<uint16_t> info(cells.size());
  std::unordered_map<int64_t, Hanging> hang_tmp;
  for (size_t c = 0; c < cells.size(); ++c) {
    const Cell& C = cells[c];
    const int64_t Sl = S(C.l), h = Sl / p;
    uint16_t inf = uint16_t(C.l << CELL_LEVEL_SHIFT);
    if (C.i & 1) inf |= CELL_CX;
    if (C.j & 1) inf |= CELL_CY;
    for (int bb = 0; bb <= p; ++bb)
      for (int a = 0; a <= p; ++a) fp[c * NL + bb * (p + 1) + a] = int32_t(out.pos.find(C.i * Sl + a * h, C.j * Sl + bb * h));
    for (int k = 0; k < NL; ++k) fp_raw[c * NL + k] = fp[c * NL + k];
    for (int d = 0; d < 4; ++d) {
      int64_t ni = C.i + DI[d], nj = C.j + DJ[d];
      if (ni < 0 || nj < 0 || ni >= ncell(C.l) || nj >= ncell(C.l)) continue;
      if (is_leaf(C.l, ni, nj) || C.l == 0 || !is_leaf(C.l - 1, ni >> 1, nj >> 1)) continue;
      // coarse neighbour: this face is half of the coarse face
      const int64_t Sc = 2 * Sl, hc = Sc / p;
      const int sub = (d < 2) ? (C.j & 1) : (C.i & 1);
      int32_t mast[3];
      int slot[3];
      for (int k = 0; k <= p; ++k) {
        int64_t X, Y;
        if (d < 2) {  // vertical face
          X = (C.i + (d == 1 ? 1 : 0)) * Sl;
          Y = (nj >> 1) * Sc + k * hc;
          slot[k] = k * (p + 1) + (d == 1 ? p : 0);
        } else {
          X = (ni >> 1) * Sc + k * hc;
          Y = (C.j + (d == 3 ? 1 : 0)) * Sl;
          slot[k] = (d == 3 ? p : 0) * (p + 1) + k;
        }
        mast[k] = int32_t(out.pos.find(X, Y));
        if (mast[k] < 0) { error = "coarse face node missing"; return false; }
      }
      inf |= uint16_t(1u << d);
      // fine nodes of the face not on a coarse node are hanging
      for (int t = 0; t <= p; ++t) {
        int32_t node = fp[c * NL + slot[t]];
        int num = sub * p + t;  // position along the coarse face in units of S/p ... over 2p
        if (num % 2 == 0) continue;
        double sfr = double(num) / double(2 * p);
        Hanging hg{};
        hg.node = node;
        for (int k = 0; k < 3; ++k) { hg.master[k] = -1; hg.weight[k] = 0.0; }
        for (int k = 0; k <= p; ++k) { hg.master[k] = mast[k]; hg.weight[k] = lagrange(p, k, sfr); }
        hang_tmp[node] = hg;
      }
      for (int k = 0; k <= p; ++k) fp[c * NL + slot[k]] = mast[k];
    }
    info[c] = inf;
  }
  std::vector<uint8_t> flags_t(nn, 0);
  for (int64_t n = 0; n < nn; ++n)
    if (NXt[n] == 0 || NXt[n] == M || NYt[n] == 0 || NYt[n] == M) flags_t[n] |= NODE_DIRICHLET;
  for (auto& kv : hang_tmp) {
    flags_t[kv.first] |= NODE_HANGING;
    for (int k = 0; k <= p; ++k)
      if (hang_tmp.count(kv.second.master[k])) { error = "chained hanging constraint"; return false; }
  }

  // ---- tiles -------------------------------------------------------------
  std::unordered_map<uint64_t, int32_t> tile_of;
  std::vector<int32_t> cell_tile(cells.size());
  {
    std::vector<uint64_t> tkeys;
    for (const Cell& C : cells) tkeys.push_back(ckey(C.l, C.j / TY, C.i / TX));  // (level, by, bx)
    std::vector<uint64_t> u = tkeys;
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    for (size_t t = 0; t < u.size(); ++t) tile_of[u[t]] = int32_t(t);
    for (size_t c = 0; c < cells.size(); ++c) cell_tile[c] = tile_of[tkeys[c]];
  }
  const int n_leaf_tiles = int(tile_of.size());
  std::unordered_map<uint64_t, int32_t> leaf_cell_id;
  leaf_cell_id.reserve(cells.size() * 2);
  for (size_t c = 0; c < cells.size(); ++c) leaf_cell_id[ckey(cells[c].l, cells[c].i, cells[c].j)] = int32_t(c);
  std::vector<int32_t> node_tile(nn, -1);
  for (int64_t n = 0; n < nn; ++n) {
    // leaf cell whose half-open box holds the node
    for (int l = lmax; l >= 0; --l) {
      int64_t ci = std::min<int64_t>(NXt[n] / S(l), ncell(l) - 1);
      int64_t cj = std::min<int64_t>(NYt[n] / S(l), ncell(l) - 1);
      auto it = leaf_cell_id.find(ckey(l, ci, cj));
      if (it != leaf_cell_id.end()) { node_tile[n] = cell_tile[it->second]; break; }
    }
    if (node_tile[n] < 0) { error = "node without owner cell"; return false; }
  }
  std::vector<int32_t>& new_id = out.new_id;
  build_tiles(p, n_leaf_tiles, fp, fp_raw, hang_tmp, info, cell_tile, node_tile, NXt, NYt, out.tiles, new_id);
  out.n = nn;
  out.NX.assign(nn, 0);
  out.NY.assign(nn, 0);
  out.flags.assign(nn, 0);
  for (int64_t n = 0; n < nn; ++n) {
    out.NX[new_id[n]] = NXt[n];
    out.NY[new_id[n]] = NYt[n];
    out.flags[new_id[n]] = flags_t[n];
  }
  out.hanging.clear();
  for (auto& kv : hang_tmp) {
    Hanging hg = kv.second;
    hg.node = new_id[hg.node];
    for (int k = 0; k <= p; ++k) hg.master[k] = new_id[hg.master[k]];
    out.hanging.push_back(hg);
  }
  std::sort(out.hanging.begin(), out.hanging.end(), [](const Hanging& a, const Hanging& c) { return a.node < c.node; });
  return true;
}

}  // namespace

bool Mesh::build(const MeshSpec& s) {
  spec = s;
  p = s.degree;
  if (p != 1 && p != 2) { error = "degree must be 1 or 2"; return false; }
  if (s.coarse <= 0 || s.n_base % s.coarse != 0) { error = "n_base must be a multiple of coarse"; return false; }
  int ratio = s.n_base / s.coarse;
  if (ratio & (ratio - 1)) { error = "n_base / coarse must be a power of two"; return false; }
  b = 0;
  while ((1 << b) < ratio) ++b;
  if (s.n_local < 0 || b + s.n_local > 14) { error = "too many levels"; return false; }
  lmax = b + s.n_local;
  n_levels = lmax + 1;
  M = int64_t(s.coarse) << lmax;
  M *= p;
  const int TX = s.tile_x > 0 ? s.tile_x : (p == 1 ? 16 : 8);
  const int TY = s.tile_y > 0 ? s.tile_y : (p == 1 ? 16 : 8);
  if (TX * TY > 256) { error = "a tile holds at most 256 cells"; return false; }
  auto S = [&](int l) { return int64_t(p) << (lmax - l); };
  auto ncell = [&](int l) { return int64_t(s.coarse) << l; };
  level_H.assign(n_levels, 0.0);
  for (int l = 0; l < n_levels; ++l) level_H[l] = 20.0 / double(int64_t(s.coarse) << l);
  const int64_t bx = std::llround(s.band_x * 1000.0), by = std::llround(s.band_y * 1000.0);
  auto in_band = [&](int l, int64_t i, int64_t j) {
    // centre x = 10 ((2i+1) S - M) / M; |x| < band_x  <=>  10^4 |(2i+1) S - M| < 1000 band_x M
    int64_t Sl = S(l);
    return 10000 * std::llabs((2 * i + 1) * Sl - M) < bx * M &&
           10000 * std::llabs((2 * j + 1) * Sl - M) < by * M;
  };

  // ---- leaves ------------------------------------------------------------
  std::unordered_set<uint64_t> leaves;
  leaves.reserve(size_t(ncell(b) * ncell(b) * 2));
  std::vector<Cell> list;
  for (int64_t j = 0; j < ncell(b); ++j)
    for (int64_t i = 0; i < ncell(b); ++i) list.push_back({b, int32_t(i), int32_t(j)});
  for (int pass = 0; pass < s.n_local; ++pass) {
    std::vector<Cell> next;
    next.reserve(list.size());
    for (const Cell& c : list) {
      if (in_band(c.l, c.i, c.j)) {
        for (int dj = 0; dj < 2; ++dj)
          for (int di = 0; di < 2; ++di) next.push_back({c.l + 1, 2 * c.i + di, 2 * c.j + dj});
      } else {
        next.push_back(c);
      }
    }
    list.swap(next);
  }
  for (const Cell& c : list) leaves.insert(ckey(c.l, c.i, c.j));
  auto is_leaf = [&](int l, int64_t i, int64_t j) { return leaves.count(ckey(l, i, j)) > 0; };
  auto find_leaf_level = [&](int l, int64_t i, int64_t j) -> int {
    for (int k = l; k >= 0; --k)
      if (is_leaf(k, i >> (l - k), j >> (l - k))) return k;
    return -1;
  };
  static const int DI[4] = {-1, 1, 0, 0}, DJ[4] = {0, 0, -1, 1};
  for (;;) {  // 2:1 face balance
    std::vector<Cell> marks;
    for (uint64_t key : leaves) {
      int l = int(key >> 58);
      if (l < b + 2) continue;
      int64_t i = int64_t((key >> 29) & ((1u << 29) - 1)), j = int64_t(key & ((1u << 29) - 1));
      for (int d = 0; d < 4; ++d) {
        int64_t ni = i + DI[d], nj = j + DJ[d];
        if (ni < 0 || nj < 0 || ni >= ncell(l) || nj >= ncell(l)) continue;
        int k = find_leaf_level(l, ni, nj);
        if (k >= 0 && k < l - 1) marks.push_back({k, int32_t(ni >> (l - k)), int32_t(nj >> (l - k))});
      }
    }
    if (marks.empty()) break;
    for (const Cell& c : marks) {
      if (!leaves.erase(ckey(c.l, c.i, c.j))) continue;
      for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) leaves.insert(ckey(c.l + 1, 2 * c.i + di, 2 * c.j + dj));
    }
  }
  std::vector<Cell> cells;
  cells.reserve(leaves.size());
  for (uint64_t key : leaves)
    cells.push_back({int(key >> 58), int32_t((key >> 29) & ((1u << 29) - 1)), int32_t(key & ((1u << 29) - 1))});
  Part leaf;
  if (!build_part(p, lmax, s.coarse, M, TX, TY, cells, leaf, error)) return false;
  n_leaf_cells = leaf.n_cells;
  n_nodes = leaf.n;
  NX = leaf.NX;
  NY = leaf.NY;
  flags = leaf.flags;
  hanging = leaf.hanging;
  tiles = std::move(leaf.tiles);
  const int NL = (p + 1) * (p + 1);
  const uint64_t W = uint64_t(M) + 1;
  auto leaf_node_at = [&](int64_t X, int64_t Y) -> int32_t { return leaf.at(X, Y); };

  // ---- levels ------------------------------------------------------------
  levels.assign(n_levels, Level());
  std::vector<std::vector<int32_t>> lev_fp(n_levels);
  std::vector<std::vector<Cell>> lev_cells(n_levels);
  std::vector<std::unordered_map<uint64_t, int32_t>> lev_cell_id(n_levels);
  std::vector<PosIndex> lev_pos(n_levels);
  std::vector<std::vector<int32_t>> lev_new(n_levels);
  for (int l = 0; l < n_levels; ++l) {
    Level& L = levels[l];
    L.level = l;
    std::vector<uint64_t> keys;
    for (const Cell& C : cells)
      if (C.l >= l) keys.push_back(ckey(l, C.j >> (C.l - l), C.i >> (C.l - l)));
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    auto& lc = lev_cells[l];
    lc.reserve(keys.size());
    for (uint64_t k : keys) lc.push_back({l, int32_t(k & ((1u << 29) - 1)), int32_t((k >> 29) & ((1u << 29) - 1))});
    for (size_t c = 0; c < lc.size(); ++c) lev_cell_id[l][ckey(l, lc[c].i, lc[c].j)] = int32_t(c);
    L.n_cells = int64_t(lc.size());
    const int64_t Sl = S(l), h = Sl / p;
    std::vector<uint64_t> pk;
    pk.reserve(lc.size() * NL);
    for (const Cell& C : lc)
      for (int bb = 0; bb <= p; ++bb)
        for (int a = 0; a <= p; ++a) pk.push_back(uint64_t(C.j * Sl + bb * h) * W + uint64_t(C.i * Sl + a * h));
    lev_pos[l].build(std::move(pk), W);
    const int64_t n = lev_pos[l].size();
    auto& lfp = lev_fp[l];
    lfp.resize(lc.size() * NL);
    std::vector<uint16_t> linfo(lc.size());
    for (size_t c = 0; c < lc.size(); ++c) {
      for (int bb = 0; bb <= p; ++bb)
        for (int a = 0; a <= p; ++a)
          lfp[c * NL + bb * (p + 1) + a] = int32_t(lev_pos[l].find(lc[c].i * Sl + a * h, lc[c].j * Sl + bb * h));
      linfo[c] = uint16_t(l << CELL_LEVEL_SHIFT);
    }
    auto has = [&](int64_t i, int64_t j) { return lev_cell_id[l].count(ckey(l, i, j)) > 0; };
    // tiles and owners
    std::unordered_map<uint64_t, int32_t> ltile;
    std::vector<int32_t> lcell_tile(lc.size());
    {
      std::vector<uint64_t> tk;
      for (const Cell& C : lc) tk.push_back(ckey(l, C.j / TY, C.i / TX));
      std::vector<uint64_t> u = tk;
      std::sort(u.begin(), u.end());
      u.erase(std::unique(u.begin(), u.end()), u.end());
      for (size_t t = 0; t < u.size(); ++t) ltile[u[t]] = int32_t(t);
      for (size_t c = 0; c < lc.size(); ++c) lcell_tile[c] = ltile[tk[c]];
    }
    std::vector<int32_t> NXl(n), NYl(n), ntile(n, -1);
    std::vector<uint8_t> fl(n, 0);
    for (int64_t k = 0; k < n; ++k) {
      int64_t X = lev_pos[l].X(k), Y = lev_pos[l].Y(k);
      NXl[k] = int32_t(X);
      NYl[k] = int32_t(Y);
      if (X == 0 || X == M || Y == 0 || Y == M) fl[k] |= NODE_DIRICHLET;
      int64_t ci[2], cj[2];
      int ni = 0, nj = 0;
      ci[ni++] = X / Sl;
      if (X % Sl == 0) ci[ni++] = X / Sl - 1;
      cj[nj++] = Y / Sl;
      if (Y % Sl == 0) cj[nj++] = Y / Sl - 1;
      for (int a = 0; a < ni; ++a)
        for (int c2 = 0; c2 < nj; ++c2) {
          int64_t ii = ci[a], jj = cj[c2];
          if (ii < 0 || jj < 0 || ii >= ncell(l) || jj >= ncell(l)) continue;
          auto it = lev_cell_id[l].find(ckey(l, ii, jj));
          if (it == lev_cell_id[l].end()) {
            fl[k] |= NODE_EDGE;
          } else if (ntile[k] < 0) {
            ntile[k] = lcell_tile[it->second];
          }
        }
      if (ntile[k] < 0) { error = "level node without cell"; return false; }
    }
    (void)has;
    // nodes of level cells that are leaves
    for (size_t c = 0; c < lc.size(); ++c)
      if (is_leaf(l, lc[c].i, lc[c].j))
        for (int k = 0; k < NL; ++k) fl[lfp[c * NL + k]] |= NODE_LEAFCELL;
    build_tiles(p, int(ltile.size()), lfp, lfp, {}, linfo, lcell_tile, ntile, NXl, NYl, L.tiles, lev_new[l]);
    L.n = n;
    L.NX.assign(n, 0);
    L.NY.assign(n, 0);
    L.flags.assign(n, 0);
    L.leaf_index.assign(n, -1);
    for (int64_t k = 0; k < n; ++k) {
      int32_t id = lev_new[l][k];
      L.NX[id] = NXl[k];
      L.NY[id] = NYl[k];
      uint8_t f = fl[k];
      if ((f & NODE_LEAFCELL) && !(f & NODE_EDGE)) f |= NODE_COPY;
      L.flags[id] = f;
      L.leaf_index[id] = leaf_node_at(NXl[k], NYl[k]);
      if (L.leaf_index[id] < 0) { error = "level node is not a leaf position"; return false; }
    }
  }
  // prolongation l-1 -> l
  for (int l = 1; l < n_levels; ++l) {
    Level& L = levels[l];
    const int64_t Sf = S(l), hf = Sf / p;
    std::vector<std::vector<std::pair<int32_t, double>>> rows(L.n);
    std::vector<char> done(L.n, 0);
    const auto& lc = lev_cells[l];
    for (size_t c = 0; c < lc.size(); ++c) {
      int64_t pi = lc[c].i >> 1, pj = lc[c].j >> 1;
      auto it = lev_cell_id[l - 1].find(ckey(l - 1, pi, pj));
      if (it == lev_cell_id[l - 1].end()) { error = "missing parent cell"; return false; }
      const int32_t* pfp = &lev_fp[l - 1][size_t(it->second) * NL];
      for (int bb = 0; bb <= p; ++bb)
        for (int a = 0; a <= p; ++a) {
          int32_t fn = lev_new[l][lev_fp[l][c * NL + bb * (p + 1) + a]];
          if (done[fn]) continue;
          done[fn] = 1;
          int64_t tx = (lc[c].i & 1) * p + a, ty = (lc[c].j & 1) * p + bb;  // in units of hf within parent
          (void)hf;
          for (int cb = 0; cb <= p; ++cb)
            for (int ca = 0; ca <= p; ++ca) {
              double w = lagrange(p, ca, double(tx) / (2 * p)) * lagrange(p, cb, double(ty) / (2 * p));
              if (w != 0.0) rows[fn].push_back({lev_new[l - 1][pfp[cb * (p + 1) + ca]], w});
            }
        }
    }
    L.P.rows = L.n;
    L.P.ptr.assign(L.n + 1, 0);
    for (int64_t r = 0; r < L.n; ++r) {
      std::sort(rows[r].begin(), rows[r].end());
      L.P.ptr[r + 1] = L.P.ptr[r] + int64_t(rows[r].size());
      for (auto& e : rows[r]) { L.P.col.push_back(e.first); L.P.val.push_back(e.second); }
    }
    // transpose
    const int64_t nc = levels[l - 1].n;
    L.PT.rows = nc;
    L.PT.ptr.assign(nc + 1, 0);
    for (int32_t cidx : L.P.col) L.PT.ptr[cidx + 1]++;
    for (int64_t r = 0; r < nc; ++r) L.PT.ptr[r + 1] += L.PT.ptr[r];
    L.PT.col.assign(L.P.col.size(), 0);
    L.PT.val.assign(L.P.col.size(), 0.0);
    std::vector<int64_t> fill(L.PT.ptr.begin(), L.PT.ptr.end() - 1);
    for (int64_t r = 0; r < L.n; ++r)
      for (int64_t e = L.P.ptr[r]; e < L.P.ptr[r + 1]; ++e) {
        int64_t q = fill[L.P.col[e]]++;
        L.PT.col[q] = int32_t(r);
        L.PT.val[q] = L.P.val[e];
      }
  }
  if (!s.mg_global) return true;

  // ---- global-coarsening levels ------------------------------------------
  // level k: the leaves cut off at depth k; k <= b: the uniform level-k mesh
  // (shared with the local-smoothing level), k = lmax: the leaf mesh
  gc.assign(n_levels, GcLevel());
  std::vector<Part> parts(n_levels);
  std::vector<std::unordered_set<uint64_t>> cut(n_levels);
  for (int k = 0; k < n_levels; ++k) {
    GcLevel& G = gc[k];
    G.level = k;
    if (k == lmax) {
      G.n = n_nodes;
      continue;
    }
    if (k <= b) {
      G.n = levels[k].n;
      continue;
    }
    for (const Cell& C : cells) {
      const int l = std::min(C.l, k);
      cut[k].insert(ckey(l, C.i >> (C.l - l), C.j >> (C.l - l)));
    }
    std::vector<Cell> ck;
    ck.reserve(cut[k].size());
    for (uint64_t key : cut[k])
      ck.push_back({int(key >> 58), int32_t((key >> 29) & ((1u << 29) - 1)), int32_t(key & ((1u << 29) - 1))});
    if (!build_part(p, lmax, s.coarse, M, TX, TY, ck, parts[k], error)) return false;
    Part& P = parts[k];
    G.own = true;
    G.n = P.n;
    G.NX = P.NX;
    G.NY = P.NY;
    G.flags = P.flags;
    G.tiles = std::move(P.tiles);
    G.leaf_index.assign(P.n, -1);
    for (int64_t g = 0; g < P.n; ++g) {
      G.leaf_index[g] = leaf_node_at(P.NX[g], P.NY[g]);
      if (G.leaf_index[g] < 0) { error = "global-coarsening node is not a leaf position"; return false; }
    }
  }
  // interpolation k-1 -> k for the levels above the base mesh and for the
  // leaf level (the uniform levels below use levels[k].P)
  for (int k = std::min(b + 1, lmax); k < n_levels; ++k) {
    if (k == 0) continue;
    GcLevel& G = gc[k];
    const int kc = k - 1;
    // coarse level: cell set and node id by position
    auto coarse_has = [&](int l, int64_t i, int64_t j) {
      if (i < 0 || j < 0 || i >= ncell(l) || j >= ncell(l)) return false;
      if (kc <= b) return l == kc;
      return cut[kc].count(ckey(l, i, j)) > 0;
    };
    auto coarse_node = [&](int64_t X, int64_t Y) -> int32_t {
      if (kc <= b) {
        const int64_t t = lev_pos[kc].find(X, Y);
        return t < 0 ? -1 : lev_new[kc][t];
      }
      return parts[kc].at(X, Y);
    };
    const std::vector<int32_t>& FX = k == lmax ? NX : G.NX;
    const std::vector<int32_t>& FY = k == lmax ? NY : G.NY;
    G.P.rows = G.n;
    G.P.ptr.assign(G.n + 1, 0);
    G.P.col.clear();
    G.P.val.clear();
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t g = 0; g < G.n; ++g) {
      const int64_t X = FX[g], Y = FY[g];
      int cl = -1;
      int64_t ci = 0, cj = 0;
      for (int l = kc; l >= 0 && cl < 0; --l) {
        const int64_t Sl = S(l);
        int64_t is[2], js[2];
        int ni = 0, nj = 0;
        is[ni++] = X / Sl;
        if (X % Sl == 0) is[ni++] = X / Sl - 1;
        js[nj++] = Y / Sl;
        if (Y % Sl == 0) js[nj++] = Y / Sl - 1;
        for (int a = 0; a < ni && cl < 0; ++a)
          for (int c2 = 0; c2 < nj && cl < 0; ++c2)
            if (coarse_has(l, is[a], js[c2])) { cl = l; ci = is[a]; cj = js[c2]; }
      }
      if (cl < 0) { error = "global-coarsening node outside the coarse level"; return false; }
      const int64_t Sc = S(cl), hc = Sc / p;
      row.clear();
      for (int cb = 0; cb <= p; ++cb)
        for (int ca = 0; ca <= p; ++ca) {
          const double w = lagrange(p, ca, double(X - ci * Sc) / double(Sc)) *
                           lagrange(p, cb, double(Y - cj * Sc) / double(Sc));
          if (w == 0.0) continue;
          const int32_t cn = coarse_node(ci * Sc + ca * hc, cj * Sc + cb * hc);
          if (cn < 0) { error = "global-coarsening coarse node missing"; return false; }
          row.push_back({cn, w});
        }
      std::sort(row.begin(), row.end());
      G.P.ptr[g + 1] = G.P.ptr[g] + int64_t(row.size());
      for (auto& e : row) { G.P.col.push_back(e.first); G.P.val.push_back(e.second); }
    }
    const int64_t nc = gc[kc].n;
    G.PT.rows = nc;
    G.PT.ptr.assign(nc + 1, 0);
    for (int32_t cidx : G.P.col) G.PT.ptr[cidx + 1]++;
    for (int64_t r = 0; r < nc; ++r) G.PT.ptr[r + 1] += G.PT.ptr[r];
    G.PT.col.assign(G.P.col.size(), 0);
    G.PT.val.assign(G.P.col.size(), 0.0);
    std::vector<int64_t> fill(G.PT.ptr.begin(), G.PT.ptr.end() - 1);
    for (int64_t r = 0; r < G.n; ++r)
      for (int64_t e = G.P.ptr[r]; e < G.P.ptr[r + 1]; ++e) {
        int64_t q = fill[G.P.col[e]]++;
        G.PT.col[q] = int32_t(r);
        G.PT.val[q] = G.P.val[e];
      }
  }
  return true;
}

}  // namespace pff
