// C ABI of the matrix-free phase-field solver library (declared in pff.h).
// Host orchestration: device tables, state setup, operator launches, the
// local-smoothing V-cycle, GMRES and the Newton / active set iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/pff.h"
#include "mesh.hpp"
#include "tile_kernel.hpp"
#include "tile_batch.hpp"
#include "util_kernels.hpp"
#include "coarse_kernel.hpp"
#include "cod_kernel.hpp"

using namespace pff;

namespace {

// a reduction or norm that came out NaN or infinite (reported as PFF_E_NONFINITE)
struct nonfinite_error : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIPCHK(expr)                                                            \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      throw std::runtime_error(std::string("HIP error ") + hipGetErrorString(e_) + " at " #expr); \
    }                                                                           \
  } while (0)

struct DevTiles {
  int n_regular = 0;
  int32_t* info = nullptr;
  int32_t* shared = nullptr;
  int32_t* sh_tab = nullptr;    // [n_shared][sh_w] slots, -1 padded
  int sh_w = SHARED_SLOTS;
  uint16_t* loc = nullptr;
  uint16_t* loc_sub = nullptr;
  uint16_t* cinfo = nullptr;
  uint16_t* hang_rec = nullptr;
  double* hang_w = nullptr;
  uint8_t* hang_col = nullptr;
  int n_tiles = 0, max_local = 0, max_cells = 0;
  int64_t n_rec = 0, n_private = 0, n_shared = 0, n_slots = 0;
};

template <typename T>
struct LevelWork {
  bool ready = false;
  T* state = nullptr;  // (u_x, u_y, phit): 3 n
  T* d = nullptr;      // right-hand side / defect
  T* x[2] = {nullptr, nullptr};
  T* dir[2] = {nullptr, nullptr};
  T* dinv = nullptr;
  T* coef = nullptr;   // operator state coefficients: [2 (p+1)^2][cell records]
};

struct DevLevel {
  int64_t n = 0;
  DevTiles tiles;
  uint8_t* flags = nullptr;
  int32_t* leaf_index = nullptr;
  int64_t* PT_ptr = nullptr;   // restriction stencils (CSR), for the level active sets
  int32_t* PT_col = nullptr;
  // transfers in ELL form: P over all nodes of this level, P^T over the
  // coarse rows that receive contributions
  uint32_t* P_ell = nullptr;
  int P_width = 0;
  uint32_t* PT_ell = nullptr;
  float* P_wtab = nullptr;      // distinct weights of P (index 0: 0)
  int32_t* PT_rows = nullptr;
  int64_t PT_nrows = 0;
  int PT_width = 0;
  int PT_group = 1;   // lanes per P^T row (ell_from_csr)
  LevelWork<double> w64;
  LevelWork<float> w32;
  double lam_max[2] = {1, 1}, lam_min[2] = {1, 1};
  bool shares_leaf = false;   // tiles and flags are the leaf operator's (not freed with the level)
  // the level's own scratch for its eigenvalue estimate, so that the levels'
  // estimates run concurrently: partial sums of the level operator's shared
  // nodes, CG scalars, Lanczos coefficients, reduction partials
  double* epart = nullptr;
  size_t epart_bytes = 0;
  double* esc = nullptr;
  double* eal = nullptr;
  double* ebe = nullptr;
  double* ered = nullptr;
};

template <typename T>
T* dalloc(int64_t count) {
  if (count <= 0) count = 1;
  void* p = nullptr;
  if (hipMalloc(&p, size_t(count) * sizeof(T)) != hipSuccess) throw std::bad_alloc();
  return static_cast<T*>(p);
}

template <typename T>
T* upload(const std::vector<T>& v) {
  T* d = dalloc<T>(int64_t(v.size()));
  if (!v.empty()) HIPCHK(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

DevTiles upload_tiles(const TileSet& t) {
  DevTiles d;
  d.info = upload(t.tile_info);
  d.n_regular = t.n_regular;
  d.shared = upload(t.shared);
  {
    int w = SHARED_SLOTS;
    for (int64_t sn = 0; sn < t.n_shared; ++sn)
      w = std::max(w, t.shared_ptr[size_t(sn) + 1] - t.shared_ptr[size_t(sn)]);
    std::vector<int32_t> tab(size_t(std::max<int64_t>(t.n_shared, 1)) * size_t(w), -1);
    for (int64_t sn = 0; sn < t.n_shared; ++sn) {
      const int j0 = t.shared_ptr[size_t(sn)], j1 = t.shared_ptr[size_t(sn) + 1];
      for (int j = j0; j < j1; ++j) tab[size_t(sn) * size_t(w) + size_t(j - j0)] = t.shared_slot[size_t(j)];
    }
    d.sh_tab = upload(tab);
    d.sh_w = w;
  }
  d.loc = upload(t.cell_loc);
  d.loc_sub = upload(t.cell_loc_sub);
  d.cinfo = upload(t.cell_info);
  d.hang_rec = upload(t.hang_rec);
  d.hang_w = upload(t.hang_w);
  d.hang_col = upload(t.hang_col);
  d.n_tiles = t.n_tiles;
  d.max_local = t.max_local;
  d.max_cells = t.max_cells;
  d.n_rec = t.n_cell_records;
  d.n_private = t.n_private;
  d.n_shared = t.n_shared;
  d.n_slots = t.n_slots;
  return d;
}

// Column-major ELL copies of P (all fine rows) and P^T (the coarse rows with
// entries) with packed (column, weight index) entries; the weights must be
// exact in float (dyadic values) and shared through one table per level.
// grouped (P^T): width G^2 (25, 9 or 4) with the rows on average at least
// half full gives group = G, the rows stored for k_restrict_add_grouped
// (entry j G + g of row k at (j nr + k) G + g); else group = 1.
void ell_from_csr(const Csr& A, const std::vector<int64_t>& rows, std::vector<double>& wtab,
                  std::vector<uint32_t>& E, int& width, bool grouped, int& group) {
  width = 0;
  int64_t nnz = 0;
  for (int64_t r : rows) {
    width = std::max<int>(width, int(A.ptr[r + 1] - A.ptr[r]));
    nnz += A.ptr[r + 1] - A.ptr[r];
  }
  const int64_t nr = int64_t(rows.size());
  const int g2 = width == 25 ? 5 : width == 9 ? 3 : width == 4 ? 2 : 1;
  group = (grouped && g2 > 1 && 2 * nnz >= int64_t(width) * nr) ? g2 : 1;
  const size_t G = size_t(group);
  E.assign(size_t(std::max(width, 1)) * size_t(std::max<int64_t>(nr, 1)), 0u);
  for (int64_t k = 0; k < nr; ++k) {
    const int64_t r = rows[k];
    for (int64_t e = A.ptr[r]; e < A.ptr[r + 1]; ++e) {
      const double v = A.val[e];
      if (double(float(v)) != v) throw std::runtime_error("transfer weight not exact in float");
      size_t wi = size_t(std::find(wtab.begin(), wtab.end(), v) - wtab.begin());
      if (wi == wtab.size()) wtab.push_back(v);
      if (wi >= size_t(TRANSFER_WEIGHTS)) throw std::runtime_error("too many distinct transfer weights");
      if (uint32_t(A.col[e]) > TRANSFER_COL_MASK) throw std::runtime_error("level too large for packed transfers");
      const size_t j = size_t(e - A.ptr[r]) / G, g = size_t(e - A.ptr[r]) % G;
      E[(j * size_t(nr) + size_t(k)) * G + g] = uint32_t(A.col[e]) | (uint32_t(wi) << TRANSFER_COL_BITS);
    }
  }
}

void upload_transfers(const Csr& P, const Csr& PT, DevLevel& D) {
  std::vector<uint32_t> E;
  std::vector<double> wtab(1, 0.0);   // index 0: padding
  std::vector<int64_t> rows(size_t(P.rows));
  std::iota(rows.begin(), rows.end(), 0);
  int group = 1;
  ell_from_csr(P, rows, wtab, E, D.P_width, false, group);
  D.P_ell = upload(E);
  rows.clear();
  for (int64_t r = 0; r < PT.rows; ++r)
    if (PT.ptr[r + 1] > PT.ptr[r]) rows.push_back(r);
  ell_from_csr(PT, rows, wtab, E, D.PT_width, true, D.PT_group);
  D.PT_ell = upload(E);
  std::vector<int32_t> r32(rows.begin(), rows.end());
  D.PT_rows = upload(r32);
  D.PT_nrows = int64_t(rows.size());
  std::vector<float> wf(size_t(TRANSFER_WEIGHTS), 0.0f);
  for (size_t i = 0; i < wtab.size(); ++i) wf[i] = float(wtab[i]);
  D.P_wtab = upload(wf);
}

inline int grid_for(int64_t n, int threads = 256) {
  int64_t b = (n + threads - 1) / threads;
  return int(std::max<int64_t>(1, std::min<int64_t>(b, 65536)));
}

// Partial sums of shared nodes for pff_vmult_noalloc: a file-scope device
// array, one copy per GPU, held until the process ends. Host code never
// passes `scratch` itself to a kernel (in host code the name is a host-side
// stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns on each device, resolved once per device with
// that device current (pff_create).
__device__ __align__(256) double scratch[PFF_NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// device address of `scratch` on the current device (resolved on first use)
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

}  // namespace

struct pff_ctx {
  Mesh mesh;
  pff_params prm{};
  int p = 1;
  int64_t n = 0;
  DevTiles tiles;
  uint8_t* flags = nullptr;
  Hanging* hang = nullptr;
  int n_hang = 0;
  std::vector<DevLevel> lv;      // local-smoothing levels (Sec. 3.2)
  // global-coarsening levels above the base mesh and the leaf level (the
  // uniform levels up to the base mesh are lv's); H: the hierarchy in use
  // (prm.mg_kind), level 0 = the coarse grid
  std::vector<DevLevel> gcown;
  std::vector<DevLevel*> H_ls, H_gc, H;
  bool has_gc = false;
  // the displacement block's eigenvalue estimates belong to the current phi~,
  // hierarchy and parameters (cleared when any of them changes)
  bool ucache = false;
  // side streams (default priority) for the levels' concurrent eigenvalue
  // estimates, forked from and joined into the caller's stream by events
  static constexpr int EIG_STREAMS = 4;
  hipStream_t es[EIG_STREAMS] = {};
  hipEvent_t efork = nullptr;
  hipEvent_t ejoin[EIG_STREAMS] = {};
  double* U = nullptr;
  double* phio = nullptr;
  double* phit = nullptr;
  double* mass = nullptr;
  static constexpr int N_WORK = 10;   // leaf work vectors
  double* wv[N_WORK] = {};
  double* red_part = nullptr;
  double* red_out = nullptr;
  double* host_red = nullptr;   // pinned
  double* eig_host = nullptr;   // pinned: per level 2 EIG_SC + 4 EIG_MAX_ITS doubles of estimate output
  double* V = nullptr;          // GMRES basis
  double* ccg_s = nullptr;      // coarse CG scalars
  // level-0 cells for the one-kernel coarse solve: node ids sorted by colour
  int32_t* coarse_nodes = nullptr;
  int coarse_ncell = 0, coarse_ncolor = 0;
  int coarse_cstart[COARSE_MAX_COLORS + 1] = {};
  bool coarse_fusable = false;
  void* part = nullptr;         // partial sums of shared nodes (largest tile set)
  size_t part_bytes = 0;
  double* part_jt = nullptr;    // leaf partial sums of JT_BATCH_MAX right-hand sides (vmult_T)
  int32_t* nodeX = nullptr;     // lattice x coordinate of every leaf node (COD lines)
  void* scratch_dev = nullptr;  // device address of `scratch` on this context's GPU
  int V_cap = 0;
  // caller-bound workspace (pff_bind_workspace): the work vectors, level
  // vectors and GMRES basis are carved from it instead of allocated
  char* ws = nullptr;
  size_t ws_size = 0;
  int ws_restart = 0;           // GMRES restart the bound basis holds
  bool work_ready = false;      // leaf work vectors exist and the lumped mass is computed
  bool has_state = false;
  bool mg_ready = false;
  bool fp32_ready = false;      // FP32 level states and diagonals belong to the current setup
  bool eig_fixed = false;
  std::string err;
  hipStream_t s = nullptr;

  DevLevel& lev(int l) { return *H[size_t(l)]; }
  const DevLevel& lev(int l) const { return *H[size_t(l)]; }
  int nlev() const { return int(H.size()); }
  void select_hierarchy() { H = (prm.mg_kind == 1 && has_gc) ? H_gc : H_ls; }

  Material mat() const {
    Material m;
    m.E = prm.E;
    m.mu = prm.E / (2.0 * (1.0 + prm.nu));
    m.lam = prm.E * prm.nu / ((1.0 + prm.nu) * (1.0 - 2.0 * prm.nu));
    m.kappa = prm.kappa;
    m.pressure = prm.pressure;
    m.Gc = prm.Gc;
    m.ell = prm.ell;
    return m;
  }

  // ---------------------------------------------------------------- tiles --
  // part_buf / part_cap: partial-sum buffer and its size in bytes (nullptr:
  // the context's own)

  template <typename T, int MODE, int EPI>
  void launch_tile(const DevTiles& t, const uint8_t* fl, int64_t nn, TileArgs<T>& a, void* part_buf = nullptr,
                   size_t part_cap = 0) {
    if (!part_buf) {
      part_buf = part;
      part_cap = part_bytes;
    }
    tile_args(t, fl, nn, a, part_buf);
    using TR = ModeTraits<MODE>;
    constexpr int NF = TR::n_src + TR::n_state;
    // staged fields (the accumulators reuse the first three), node flags
    const size_t lds = size_t((NF > 3 ? NF : 3) * t.max_local) * sizeof(double) + size_t(t.max_local);
    // one thread per cell of the largest tile
    const int threads = std::max(64, ((t.max_cells + 63) / 64) * 64);
    if (threads > 256) throw std::runtime_error("a tile holds at most 256 cells");
    if (size_t(3 * t.n_slots) * sizeof(T) > part_cap) throw std::runtime_error("partial-sum buffer too small");
    if (lds > size_t(160 * 1024)) throw std::runtime_error("tile needs more LDS than a CU has; use smaller tiles");
    // hanging nodes are handled on the tile's nodes; only the inverse
    // diagonal runs the per-cell constraint form
    constexpr bool HANG = (MODE == MODE_DIAG_LEAF || MODE == MODE_DIAG_LEVEL);
    // the default tiles' block size (Q1 256, Q2 64 threads) is compiled in
    const bool fixed = threads == (p == 1 ? 256 : 64);
    const void* kfn =
        p == 1 ? (fixed ? reinterpret_cast<const void*>(&tile_kernel<1, T, MODE, EPI, HANG, true>)
                        : reinterpret_cast<const void*>(&tile_kernel<1, T, MODE, EPI, HANG, false>))
               : (fixed ? reinterpret_cast<const void*>(&tile_kernel<2, T, MODE, EPI, HANG, true>)
                        : reinterpret_cast<const void*>(&tile_kernel<2, T, MODE, EPI, HANG, false>));
    if (lds > size_t(64 * 1024))
      HIPCHK(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    a.tile_base = 0;
    a.n_grid = int(t.n_tiles);
    if (t.n_tiles > 0) {
      if (p == 1 && fixed)
        hipLaunchKernelGGL((tile_kernel<1, T, MODE, EPI, HANG, true>), dim3(t.n_tiles), dim3(threads), lds, s, a);
      else if (p == 1)
        hipLaunchKernelGGL((tile_kernel<1, T, MODE, EPI, HANG, false>), dim3(t.n_tiles), dim3(threads), lds, s, a);
      else if (fixed)
        hipLaunchKernelGGL((tile_kernel<2, T, MODE, EPI, HANG, true>), dim3(t.n_tiles), dim3(threads), lds, s, a);
      else
        hipLaunchKernelGGL((tile_kernel<2, T, MODE, EPI, HANG, false>), dim3(t.n_tiles), dim3(threads), lds, s, a);
    }
    if (MODE != MODE_LEVEL_COEF && t.n_shared > 0)
      hipLaunchKernelGGL((shared_fixup<T, MODE, EPI>), dim3(grid_for(t.n_shared)), dim3(256), 0, s, a);
    HIPCHK(hipGetLastError());
  }

  // the tables, sizes and constants of a tile set in TileArgs
  template <typename T>
  void tile_args(const DevTiles& t, const uint8_t* fl, int64_t nn, TileArgs<T>& a, void* part_buf) {
    a.tile_info = t.info;
    a.shared = t.shared;
    a.cell_loc = t.loc;
    a.cell_loc_sub = t.loc_sub;
    a.cell_info = t.cinfo;
    a.hang_rec = t.hang_rec;
    a.hang_w = t.hang_w;
    a.hang_col = t.hang_col;
    a.flags = fl;
    a.n = nn;
    a.max_local = t.max_local;
    a.part = reinterpret_cast<T*>(part_buf);
    a.n_slots = t.n_slots;
    a.n_private = t.n_private;
    a.n_shared = t.n_shared;
    a.sh_tab = t.sh_tab;
    a.sh_w = t.sh_w;
    a.H0 = T(mesh.level_H[0]);
    a.mat = mat();
  }

  // dst = J~^T src for nb <= JT_BATCH_MAX right-hand sides (3n each), the
  // leaf state read once per tile
  void leaf_jt_batch(double* dst, const double* src, int nb) {
    const DevTiles& t = tiles;
    TileArgs<double> a{};
    tile_args(t, flags, n, a, part_jt);
    a.src = src;
    a.dst = dst;
    const double* st[4];
    leaf_state4(st);
    for (int i = 0; i < 4; ++i) a.st[i] = st[i];
    const size_t lds = size_t(7 * t.max_local) * sizeof(double) + size_t(t.max_local);
    const int threads = std::max(64, ((t.max_cells + 63) / 64) * 64);
    if (threads > 256) throw std::runtime_error("a tile holds at most 256 cells");
    if (nb < 1 || nb > JT_BATCH_MAX) throw std::runtime_error("vmult_T batch chunk out of range");
    if (lds > size_t(160 * 1024)) throw std::runtime_error("tile needs more LDS than a CU has; use smaller tiles");
    const void* kfn = p == 1 ? reinterpret_cast<const void*>(&tile_kernel_jt_batch<1>)
                             : reinterpret_cast<const void*>(&tile_kernel_jt_batch<2>);
    if (lds > size_t(64 * 1024))
      HIPCHK(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    a.tile_base = 0;
    if (t.n_tiles > 0) {
      if (p == 1)
        hipLaunchKernelGGL(tile_kernel_jt_batch<1>, dim3(t.n_tiles), dim3(threads), lds, s, a, nb);
      else
        hipLaunchKernelGGL(tile_kernel_jt_batch<2>, dim3(t.n_tiles), dim3(threads), lds, s, a, nb);
    }
    if (t.n_shared > 0)
      hipLaunchKernelGGL(shared_fixup_jt_batch, dim3(grid_for(t.n_shared * nb)), dim3(256), 0, s, a, nb);
    HIPCHK(hipGetLastError());
  }

  template <int MODE>
  void leaf_op(double* dst, const double* src, const double* const* st) {
    TileArgs<double> a{};
    a.src = src;
    a.dst = dst;
    for (int i = 0; i < 4; ++i) a.st[i] = st ? st[i] : nullptr;
    launch_tile<double, MODE, EPI_PLAIN>(tiles, flags, n, a);
  }

  const double* const* leaf_state4(const double** buf) {
    buf[0] = U;
    buf[1] = U + n;
    buf[2] = U + 2 * n;
    buf[3] = phit;
    return buf;
  }

  // ------------------------------------------------------------ reductions --
  double dot(const double* a, const double* b, int64_t len) {
    hipLaunchKernelGGL((k_dot_partial<double>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, a, b, len, red_part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, s, red_part, RED_BLOCKS, 1, red_out);
    HIPCHK(hipMemcpyAsync(host_red, red_out, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return host_red[0];
  }
  template <typename T>
  void dot2_async(const T* a, const T* b, int64_t len, double* out_dev, double* partials = nullptr) {
    if (!partials) partials = red_part;
    hipLaunchKernelGGL((k_dot_partial<T>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, a, b, len, partials);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, s, partials, RED_BLOCKS, 1, out_dev);
  }
  // the k <= 64 running sums of the orthogonalisation kernels are held in
  // registers: instantiate for the smallest bound that covers k
  template <template <int> class F, typename... A>
  void launch_k(int k, A... args) {
    if (k <= 8)
      F<8>::run(s, args...);
    else if (k <= 16)
      F<16>::run(s, args...);
    else if (k <= 32)
      F<32>::run(s, args...);
    else if (k <= 64)
      F<64>::run(s, args...);
    else
      throw std::runtime_error("more than 64 Krylov vectors");
  }
  template <int K>
  struct MdotL {
    static void run(hipStream_t st, const double* V, const double* w, int k, int64_t len, double* part) {
      hipLaunchKernelGGL(k_mdot_partial<K>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, V, w, k, len, part);
    }
  };
  template <int K>
  struct DcgsL {
    static void run(hipStream_t st, double* V, const double* w, DcgsCoef cf, int64_t len, double* part) {
      hipLaunchKernelGGL(k_dcgs2_partial<K>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, V, w, cf, len, part);
    }
  };
  // out = sums of the k partial columns left in red_part, copied to the host
  void reduce_to_host(int k, double* host_out) {
    hipLaunchKernelGGL(k_reduce_final, dim3(k), dim3(RED_THREADS), 0, s, red_part, RED_BLOCKS, k, red_out);
    HIPCHK(hipMemcpyAsync(host_out, red_out, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  void mdot(const double* Vb, int k, const double* w, int64_t len, double* host_out) {
    launch_k<MdotL>(k, Vb, w, k, len, red_part);
    reduce_to_host(k, host_out);
  }
  double norm(const double* a, int64_t len) { return std::sqrt(dot(a, a, len)); }

  // -------------------------------------------------------- workspace -----
  // The work buffers in a fixed order, each rounded up to 256 bytes. With
  // carve == false only their sizes are summed (restart m for the basis);
  // with carve == true they are placed in the bound workspace.
  size_t layout_work(bool carve, int m) {
    size_t off = 0;
    auto take = [&](auto*& ptr, int64_t count) {
      using E = std::remove_pointer_t<std::remove_reference_t<decltype(ptr)>>;
      const size_t b = (size_t(std::max<int64_t>(count, 1)) * sizeof(E) + 255) & ~size_t(255);
      if (carve) ptr = reinterpret_cast<E*>(ws + off);
      off += b;
    };
    const int64_t N = 3 * n;
    double* dummy = nullptr;
    take(carve ? U : dummy, N);
    take(carve ? phio : dummy, n);
    take(carve ? phit : dummy, n);
    take(carve ? mass : dummy, N);
    for (int i = 0; i < N_WORK; ++i) take(carve ? wv[i] : dummy, N);
    double* pp = nullptr;
    take(pp, int64_t(part_bytes / sizeof(double)));
    if (carve) part = pp;
    take(carve ? part_jt : dummy, int64_t(JT_BATCH_MAX) * 3 * tiles.n_slots);
    std::vector<DevLevel*> all;
    for (DevLevel& L : lv) all.push_back(&L);
    for (DevLevel& L : gcown) all.push_back(&L);
    for (DevLevel* Lp : all) {
      DevLevel& L = *Lp;
      const int64_t nl = 3 * L.n;
      LevelWork<double>& a = L.w64;
      LevelWork<float>& b = L.w32;
      double* d64 = nullptr;
      float* d32 = nullptr;
      take(carve ? a.state : d64, nl); take(carve ? a.d : d64, nl); take(carve ? a.x[0] : d64, nl);
      take(carve ? a.x[1] : d64, nl); take(carve ? a.dir[0] : d64, nl); take(carve ? a.dir[1] : d64, nl);
      take(carve ? a.dinv : d64, nl);
      take(carve ? a.coef : d64, int64_t(2 * (p + 1) * (p + 1)) * L.tiles.n_rec);
      take(carve ? b.state : d32, nl); take(carve ? b.d : d32, nl); take(carve ? b.x[0] : d32, nl);
      take(carve ? b.x[1] : d32, nl); take(carve ? b.dir[0] : d32, nl); take(carve ? b.dir[1] : d32, nl);
      take(carve ? b.dinv : d32, nl);
      take(carve ? b.coef : d32, int64_t(2 * (p + 1) * (p + 1)) * L.tiles.n_rec);
      if (carve) a.ready = b.ready = true;
    }
    take(carve ? V : dummy, int64_t(m + 1) * N);
    if (carve) V_cap = m + 1;
    return off;
  }
  size_t workspace_bytes() { return layout_work(false, std::max(1, prm.gmres_restart)); }

  // leaf work vectors (from the workspace if one is bound) and the lumped
  // phase-field mass; called by every entry point that uses them
  void ensure_work() {
    if (work_ready) return;
    if (!ws) {
      U = dalloc<double>(3 * n);
      phio = dalloc<double>(n);
      phit = dalloc<double>(n);
      mass = dalloc<double>(3 * n);
      for (int i = 0; i < N_WORK; ++i) wv[i] = dalloc<double>(3 * n);
      part = dalloc<double>(int64_t(part_bytes / sizeof(double)));
      part_jt = dalloc<double>(int64_t(JT_BATCH_MAX) * 3 * tiles.n_slots);
    }
    // lumped phase-field mass (the B of Alg. 2)
    leaf_op<MODE_MASS>(mass, nullptr, nullptr);
    HIPCHK(hipStreamSynchronize(s));
    work_ready = true;
  }

  // ------------------------------------------------------------ levels -----
  template <typename T>
  LevelWork<T>& work(DevLevel& L);

  template <typename T>
  void ensure_level_work(DevLevel& L) {
    LevelWork<T>& w = work<T>(L);
    if (w.ready) return;
    const int64_t nl = L.n;
    w.state = dalloc<T>(3 * nl);
    w.d = dalloc<T>(3 * nl);
    for (int i = 0; i < 2; ++i) { w.x[i] = dalloc<T>(3 * nl); w.dir[i] = dalloc<T>(3 * nl); }
    w.dinv = dalloc<T>(3 * nl);
    w.coef = dalloc<T>(int64_t(2 * (p + 1) * (p + 1)) * L.tiles.n_rec);
    w.ready = true;
  }

  template <typename T>
  void level_apply(int l, const T* x, T* dst, int epi, const T* b, const T* dold, T* xnew, const T c1[2],
                   const T c2[2], const T* c0 = nullptr, void* part_buf = nullptr, size_t part_cap = 0) {
    DevLevel& L = lev(l);
    LevelWork<T>& w = work<T>(L);
    TileArgs<T> a{};
    a.src = x;
    a.dst = dst;
    a.coef = w.coef;
    a.n_coef = L.tiles.n_rec;
    a.b = b;
    a.dold = dold;
    a.dinv = w.dinv;
    a.xnew = xnew;
    for (int i = 0; i < 2; ++i) {
      a.c1[i] = c1 ? c1[i] : T(0);
      a.c2[i] = c2 ? c2[i] : T(0);
      a.c0[i] = c0 ? c0[i] : T(0);
    }
    if (epi == EPI_PLAIN) launch_tile<T, MODE_LEVEL, EPI_PLAIN>(L.tiles, L.flags, L.n, a, part_buf, part_cap);
    else if (epi == EPI_PHI) launch_tile<T, MODE_LEVEL, EPI_PHI>(L.tiles, L.flags, L.n, a, part_buf, part_cap);
    else if (epi == EPI_RESID) launch_tile<T, MODE_LEVEL, EPI_RESID>(L.tiles, L.flags, L.n, a);
    else if (epi == EPI_CHEB_FIRST) launch_tile<T, MODE_LEVEL, EPI_CHEB_FIRST>(L.tiles, L.flags, L.n, a);
    else launch_tile<T, MODE_LEVEL, EPI_CHEB>(L.tiles, L.flags, L.n, a);
  }

  // the level operator's state coefficients per cell (from the level state)
  template <typename T>
  void level_coef(int l) {
    DevLevel& L = lev(l);
    LevelWork<T>& w = work<T>(L);
    TileArgs<T> a{};
    a.st[0] = w.state;
    a.st[1] = w.state + L.n;
    a.st[2] = w.state + 2 * L.n;
    a.coef = w.coef;
    a.n_coef = L.tiles.n_rec;
    launch_tile<T, MODE_LEVEL_COEF, EPI_PLAIN>(L.tiles, L.flags, L.n, a);
  }

  template <typename T>
  void level_diag(int l) {
    DevLevel& L = lev(l);
    LevelWork<T>& w = work<T>(L);
    TileArgs<T> a{};
    a.dst = w.dinv;
    a.st[0] = w.state;
    a.st[1] = w.state + L.n;
    a.st[2] = w.state + 2 * L.n;
    launch_tile<T, MODE_DIAG_LEVEL, EPI_PLAIN>(L.tiles, L.flags, L.n, a);
  }

  // smoothing interval per block on level l
  void interval(int l, double lo[2], double hi[2]) const {
    const DevLevel& L = lev(l);
    for (int b = 0; b < 2; ++b) {
      if (l == 0 && prm.coarse_mode == 0) {
        lo[b] = L.lam_min[b];
        hi[b] = prm.upper_factor * L.lam_max[b];
      } else {
        lo[b] = prm.smooth_range * L.lam_max[b];
        hi[b] = prm.upper_factor * L.lam_max[b];
      }
    }
  }

  // Chebyshev-Jacobi smoothing (Saad, Alg. 12.1 on D^{-1}A; residual from its
  // definition at every update). x_in = nullptr: start from x = 0. Result in
  // w.x[*out_idx].
  template <typename T>
  int chebyshev(int l, const T* b, int x_in_idx, int degree) {
    DevLevel& L = lev(l);
    LevelWork<T>& w = work<T>(L);
    double lo[2], hi[2];
    interval(l, lo, hi);
    double theta[2], delta[2], rho_prev[2];
    for (int k = 0; k < 2; ++k) {
      theta[k] = 0.5 * (hi[k] + lo[k]);
      delta[k] = 0.5 * (hi[k] - lo[k]);
      rho_prev[k] = delta[k] / theta[k];
    }
    const int64_t nl = L.n;
    int xi, di = 0, j0 = 1;
    T c1[2], c2[2];
    if (x_in_idx < 0 && degree >= 2) {
      // first update (d_0 = D^-1 b / theta, x_1 = d_0) and the second in one
      // pass: d_0 is formed inside the level kernel
      const T c0[2] = {T(1.0 / theta[0]), T(1.0 / theta[1])};
      for (int k = 0; k < 2; ++k) {
        const double rho = 1.0 / (2.0 * theta[k] / delta[k] - rho_prev[k]);
        c1[k] = T(rho * rho_prev[k]);
        c2[k] = T(2.0 * rho / delta[k]);
        rho_prev[k] = rho;
      }
      level_apply<T>(l, nullptr, w.dir[1], EPI_CHEB_FIRST, b, nullptr, w.x[1], c1, c2, c0);
      xi = 1;
      di = 1;
      j0 = 2;
    } else if (x_in_idx < 0) {
      xi = 0;
      hipLaunchKernelGGL((k_cheb_first<T>), dim3(grid_for(3 * nl)), dim3(256), 0, s, w.x[0], w.dir[0], b, w.dinv,
                         nl, T(1.0 / theta[0]), T(1.0 / theta[1]));
    } else {
      xi = x_in_idx;
      for (int k = 0; k < 2; ++k) { c1[k] = T(0); c2[k] = T(1.0 / theta[k]); }
      level_apply<T>(l, w.x[xi], w.dir[0], EPI_CHEB, b, nullptr, w.x[1 - xi], c1, c2);
      xi = 1 - xi;
    }
    for (int j = j0; j < degree; ++j) {
      for (int k = 0; k < 2; ++k) {
        const double rho = 1.0 / (2.0 * theta[k] / delta[k] - rho_prev[k]);
        c1[k] = T(rho * rho_prev[k]);
        c2[k] = T(2.0 * rho / delta[k]);
        rho_prev[k] = rho;
      }
      level_apply<T>(l, w.x[xi], w.dir[1 - di], EPI_CHEB, b, w.dir[di], w.x[1 - xi], c1, c2);
      xi = 1 - xi;
      di = 1 - di;
    }
    return xi;
  }

  // Level-0 cells for the one-kernel coarse solve: global node ids of every
  // cell, cells coloured greedily so that cells of one colour share no node
  // and sorted by colour. The solve runs in one kernel when the level fits
  // one workgroup (at most COARSE_THREADS cells, level-0 cells only, five
  // vectors in LDS); otherwise the per-step launches are used.
  void setup_coarse_cells() {
    const Level& HL = mesh.levels[0];
    const TileSet& t = HL.tiles;
    const int NL = (p + 1) * (p + 1);
    std::vector<std::vector<int32_t>> cells;
    bool ok = true;
    for (int tile = 0; tile < t.n_tiles; ++tile) {
      const int32_t* ti = t.tile_info.data() + TILE_STRIDE * tile;
      const int o0 = ti[TILE_OWNED0], no = ti[TILE_NOWNED], s0 = ti[TILE_SHARED0];
      for (int r = ti[TILE_CELL0]; r < ti[TILE_CELL0] + ti[TILE_NCELL]; ++r) {
        if (((t.cell_info[size_t(r)] >> CELL_LEVEL_SHIFT) & 31u) != 0u || (t.cell_info[size_t(r)] & 15u)) ok = false;
        std::vector<int32_t> g(static_cast<size_t>(NL), 0);
        for (int k = 0; k < NL; ++k) {
          const int l = t.cell_loc[size_t(r) * size_t(NL) + size_t(k)];
          g[size_t(k)] = l < no ? o0 + l : t.shared[size_t(s0 + l - no)];
        }
        cells.push_back(std::move(g));
      }
    }
    const int ncell = int(cells.size());
    std::vector<int> color(size_t(ncell), 0);
    std::vector<uint32_t> used(size_t(HL.n), 0u);   // colour bit mask per node
    int ncolor = 0;
    for (int c = 0; c < ncell; ++c) {
      uint32_t m = 0;
      for (int32_t g : cells[size_t(c)]) m |= used[size_t(g)];
      int col = 0;
      while (col < 32 && (m >> col) & 1u) ++col;
      color[size_t(c)] = col;
      for (int32_t g : cells[size_t(c)]) used[size_t(g)] |= 1u << col;
      ncolor = std::max(ncolor, col + 1);
    }
    const size_t lds = size_t(15 * HL.n) * sizeof(double) + size_t(HL.n);
    coarse_fusable = ok && ncell > 0 && ncell <= COARSE_THREADS && ncolor <= COARSE_MAX_COLORS &&
                     lds <= size_t(160 * 1024) && 3 * HL.n <= int64_t(COARSE_THREADS) * COARSE_PER_THREAD;
    if (!coarse_fusable) return;
    std::vector<int32_t> flat;
    flat.reserve(size_t(ncell) * size_t(NL));
    coarse_cstart[0] = 0;
    for (int col = 0; col < ncolor; ++col) {
      for (int c = 0; c < ncell; ++c)
        if (color[size_t(c)] == col) flat.insert(flat.end(), cells[size_t(c)].begin(), cells[size_t(c)].end());
      coarse_cstart[col + 1] = int(flat.size() / size_t(NL));
    }
    coarse_nodes = upload(flat);
    coarse_ncell = ncell;
    coarse_ncolor = ncolor;
  }

  // the whole level-0 solve in one kernel (Chebyshev or CG, as the
  // per-step path); result in w.x[0]
  template <typename T>
  int coarse_fused() {
    DevLevel& L = lev(0);
    LevelWork<T>& w = work<T>(L);
    CoarseArgs<T> a{};
    a.n0 = int(L.n);
    a.ncell = coarse_ncell;
    a.ncolor = coarse_ncolor;
    for (int c = 0; c <= coarse_ncolor; ++c) a.cstart[c] = coarse_cstart[c];
    a.steps = prm.coarse_its;
    a.cg = prm.coarse_mode == 1 ? 1 : 0;
    a.cell_nodes = coarse_nodes;
    a.flags = L.flags;
    a.state = w.state;
    a.b = w.d;
    a.dinv = w.dinv;
    a.x = w.x[0];
    a.H = T(mesh.level_H[0]);
    a.mat = mat();
    if (!a.cg) {
      // the coefficients of chebyshev(0, b, start from zero, coarse_its)
      double lo[2], hi[2], theta[2], delta[2], rho_prev[2];
      interval(0, lo, hi);
      for (int k = 0; k < 2; ++k) {
        theta[k] = 0.5 * (hi[k] + lo[k]);
        delta[k] = 0.5 * (hi[k] - lo[k]);
        rho_prev[k] = delta[k] / theta[k];
        a.c1[0][k] = T(0);
        a.c2[0][k] = T(1.0 / theta[k]);
      }
      for (int j = 1; j < a.steps; ++j)
        for (int k = 0; k < 2; ++k) {
          const double rho = 1.0 / (2.0 * theta[k] / delta[k] - rho_prev[k]);
          a.c1[j][k] = T(rho * rho_prev[k]);
          a.c2[j][k] = T(2.0 * rho / delta[k]);
          rho_prev[k] = rho;
        }
    }
    const size_t lds = size_t(15 * L.n) * sizeof(double) + size_t(L.n);
    const void* kfn = p == 1 ? reinterpret_cast<const void*>(&coarse_kernel<1, T>)
                             : reinterpret_cast<const void*>(&coarse_kernel<2, T>);
    if (lds > size_t(64 * 1024)) HIPCHK(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    if (p == 1)
      hipLaunchKernelGGL((coarse_kernel<1, T>), dim3(2), dim3(COARSE_THREADS), lds, s, a);
    else
      hipLaunchKernelGGL((coarse_kernel<2, T>), dim3(2), dim3(COARSE_THREADS), lds, s, a);
    HIPCHK(hipGetLastError());
    return 0;
  }

  // Coarse solve by a fixed number of Jacobi-preconditioned CG steps from
  // x = 0 (both blocks, each with its own scalars) on level 0's right-hand
  // side; the result is left in w.x[0].
  template <typename T>
  int coarse_cg() {
    DevLevel& L = lev(0);
    LevelWork<T>& w = work<T>(L);
    T* x = w.x[0];
    T* r = w.x[1];
    T* pv = w.dir[0];
    T* q = w.dir[1];
    hipLaunchKernelGGL((k_ccg_init<T>), dim3(1), dim3(CCG_THREADS), 0, s, x, r, pv, w.d, w.dinv, L.n, ccg_s);
    for (int it = 0; it < prm.coarse_its; ++it) {
      level_apply<T>(0, pv, q, EPI_PLAIN, nullptr, nullptr, nullptr, nullptr, nullptr);
      hipLaunchKernelGGL((k_ccg_step<T>), dim3(1), dim3(CCG_THREADS), 0, s, x, r, pv, q, w.dinv, L.n, ccg_s);
    }
    return 0;
  }

  // transfers of level D (to and from level D - 1): prolongation with the
  // row width as a compile-time constant for the widths of Q1 and Q2 (4 and
  // 9); restriction with PT_group = G > 1 (widths 9 and 25 with Q1 and Q2,
  // rows at least half full) by the grouped kernel, 64 / G rows per wave and
  // four waves a block, the layout of ell_from_csr; otherwise one lane per
  // row, the widths 9 and 25 as compile-time constants
  static dim3 grouped_grid(int64_t rows, int G) { return dim3(grid_for((rows + 64 / G - 1) / (64 / G) * 64)); }
  template <typename T>
  void prolong_add(T* xf, const T* xc, int64_t nc, const DevLevel& D) {
    const dim3 g(grid_for(D.n)), b(256);
    switch (D.P_width) {
      case 4: hipLaunchKernelGGL((k_prolong_add<T, 4>), g, b, 0, s, xf, xc, D.n, nc, 4, D.P_ell, D.P_wtab, D.flags); break;
      case 9: hipLaunchKernelGGL((k_prolong_add<T, 9>), g, b, 0, s, xf, xc, D.n, nc, 9, D.P_ell, D.P_wtab, D.flags); break;
      default:
        hipLaunchKernelGGL((k_prolong_add<T, 0>), g, b, 0, s, xf, xc, D.n, nc, D.P_width, D.P_ell, D.P_wtab, D.flags);
    }
  }
  template <typename T>
  void restrict_add(T* dc, const T* tf, int64_t nc, const DevLevel& D) {
    const dim3 b(256);
    const int64_t nr = D.PT_nrows;
    switch (D.PT_group) {
      case 2:
        hipLaunchKernelGGL((k_restrict_add_grouped<T, 2>), grouped_grid(nr, 2), b, 0, s, dc, tf, nc, D.n, nr,
                           D.PT_rows, D.PT_ell, D.P_wtab);
        break;
      case 3:
        hipLaunchKernelGGL((k_restrict_add_grouped<T, 3>), grouped_grid(nr, 3), b, 0, s, dc, tf, nc, D.n, nr,
                           D.PT_rows, D.PT_ell, D.P_wtab);
        break;
      case 5:
        hipLaunchKernelGGL((k_restrict_add_grouped<T, 5>), grouped_grid(nr, 5), b, 0, s, dc, tf, nc, D.n, nr,
                           D.PT_rows, D.PT_ell, D.P_wtab);
        break;
      default: {
        const dim3 g(grid_for(nr));
        switch (D.PT_width) {
          case 9:
            hipLaunchKernelGGL((k_restrict_add<T, 9>), g, b, 0, s, dc, tf, nc, D.n, nr, D.PT_rows, 9, D.PT_ell,
                               D.P_wtab);
            break;
          case 25:
            hipLaunchKernelGGL((k_restrict_add<T, 25>), g, b, 0, s, dc, tf, nc, D.n, nr, D.PT_rows, 25, D.PT_ell,
                               D.P_wtab);
            break;
          default:
            hipLaunchKernelGGL((k_restrict_add<T, 0>), g, b, 0, s, dc, tf, nc, D.n, nr, D.PT_rows, D.PT_width,
                               D.PT_ell, D.P_wtab);
        }
      }
    }
  }

  template <typename T>
  void vcycle_impl(double* dst, const double* src) {
    const int L = int(lv.size()) - 1;
    const int k = prm.cheb_degree;
    std::vector<int> xi(L + 1, 0);
    LevelCopyArgs<T> ca{};
    ca.nlev = L + 1;
    for (int l = 0; l <= L; ++l) {
      ca.start[l + 1] = ca.start[l] + lv[l].n;
      ca.bstart[l + 1] = ca.bstart[l] + int((lv[l].n + 255) / 256);
      ca.vec[l] = work<T>(lv[l]).d;
      ca.fl[l] = lv[l].flags;
      ca.leaf_index[l] = lv[l].leaf_index;
    }
    hipLaunchKernelGGL((k_copy_to_levels<T>), dim3(ca.bstart[L + 1]), dim3(256), 0, s, ca, src, flags, n);
    for (int l = L; l >= 1; --l) {
      DevLevel& D = lv[l];
      LevelWork<T>& w = work<T>(D);
      xi[l] = chebyshev<T>(l, w.d, -1, k);
      // t = d - A x (all rows) into the free direction buffer
      T* t = w.dir[0];
      level_apply<T>(l, w.x[xi[l]], t, EPI_RESID, w.d, nullptr, nullptr, nullptr, nullptr);
      DevLevel& C = lv[l - 1];
      LevelWork<T>& wc = work<T>(C);
      if (D.PT_nrows > 0)
        restrict_add<T>(wc.d, t, C.n, D);
    }
    {
      LevelWork<T>& w0 = work<T>(lv[0]);
      if (coarse_fusable && prm.coarse_its <= COARSE_MAX_STEPS)
        xi[0] = coarse_fused<T>();
      else
        xi[0] = prm.coarse_mode == 1 ? coarse_cg<T>() : chebyshev<T>(0, w0.d, -1, prm.coarse_its);
    }
    for (int l = 1; l <= L; ++l) {
      DevLevel& D = lv[l];
      LevelWork<T>& w = work<T>(D);
      LevelWork<T>& wc = work<T>(lv[l - 1]);
      prolong_add<T>(w.x[xi[l]], wc.x[xi[l - 1]], lv[l - 1].n, D);
      xi[l] = chebyshev<T>(l, w.d, xi[l], k);
    }
    for (int l = 0; l <= L; ++l) ca.vec[l] = work<T>(lv[l]).x[xi[l]];
    hipLaunchKernelGGL((k_copy_from_levels<T>), dim3(ca.bstart[L + 1]), dim3(256), 0, s, dst, ca, src, flags,
                       n);
    if (n_hang)
      hipLaunchKernelGGL(k_copy_hanging, dim3(grid_for(3 * n_hang)), dim3(256), 0, s, dst, src, n, hang, n_hang);
    HIPCHK(hipGetLastError());
  }

  // Global-coarsening V-cycle (the level sequence of the design notes): the
  // finest level is the leaf mesh; every level is smoothed over all of its
  // free unknowns with its hanging-node constraints, restriction is the
  // transpose of the interpolation, no refinement edge and no copies.
  template <typename T>
  void vcycle_gc_impl(double* dst, const double* src) {
    const int L = nlev() - 1;
    const int k = prm.cheb_degree;
    std::vector<int> xi(L + 1, 0);
    hipLaunchKernelGGL((k_leaf_to_level<T>), dim3(grid_for(n)), dim3(256), 0, s, work<T>(lev(L)).d, src, flags, n);
    for (int l = L; l >= 1; --l) {
      DevLevel& D = lev(l);
      LevelWork<T>& w = work<T>(D);
      xi[l] = chebyshev<T>(l, w.d, -1, k);
      T* t = w.dir[0];
      level_apply<T>(l, w.x[xi[l]], t, EPI_RESID, w.d, nullptr, nullptr, nullptr, nullptr);
      DevLevel& C = lev(l - 1);
      LevelWork<T>& wc = work<T>(C);
      hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(3 * C.n)), dim3(256), 0, s, wc.d, T(0), 3 * C.n);
      if (D.PT_nrows > 0) restrict_add<T>(wc.d, t, C.n, D);
    }
    {
      LevelWork<T>& w0 = work<T>(lev(0));
      if (coarse_fusable && prm.coarse_its <= COARSE_MAX_STEPS)
        xi[0] = coarse_fused<T>();
      else
        xi[0] = prm.coarse_mode == 1 ? coarse_cg<T>() : chebyshev<T>(0, w0.d, -1, prm.coarse_its);
    }
    for (int l = 1; l <= L; ++l) {
      DevLevel& D = lev(l);
      LevelWork<T>& w = work<T>(D);
      LevelWork<T>& wc = work<T>(lev(l - 1));
      prolong_add<T>(w.x[xi[l]], wc.x[xi[l - 1]], lev(l - 1).n, D);
      xi[l] = chebyshev<T>(l, w.d, xi[l], k);
    }
    hipLaunchKernelGGL((k_level_to_leaf<T>), dim3(grid_for(n)), dim3(256), 0, s, dst, work<T>(lev(L)).x[xi[L]], src,
                       flags, n);
    HIPCHK(hipGetLastError());
  }

  // Extreme Ritz values of D^{-1} A (free unknowns of one block) from
  // `its` Jacobi-preconditioned CG steps on A x = 1.
  // Extreme eigenvalues of D^-1 A on each block of level l by `its` steps of
  // Jacobi-preconditioned CG from r = 1 on the free unknowns, through the
  // Lanczos tridiagonal of its coefficients. The level operator is block
  // diagonal, so both blocks run at once (one operator application per step);
  // their scalars stay on the device and are read back once at the end.
  // Eigenvalue estimate of level l, enqueued without a host wait: the CG
  // runs `its` steps (the device scalars stop a block earlier), and its
  // scalars and Lanczos coefficients are copied to the pinned area `out`
  // (2 EIG_SC + 4 EIG_MAX_ITS doubles). eig_finish turns them into the
  // extreme Ritz values once the stream has been synchronised.
  // skip_u: the displacement block keeps its estimate and the vector passes
  // cover the phase-field rows only (the level operator is block diagonal,
  // so the phase-field rows of q do not depend on the other rows of p)
  void eig_launch(int l, int its, int its_phi, double* out, bool skip_u = false) {
    DevLevel& L = lev(l);
    LevelWork<double>& w = w64of(L);
    const int64_t nl = L.n;
    double* r = w.x[0];
    double* z = w.x[1];
    double* pv = w.dir[0];
    double* q = w.dir[1];
    const int64_t off[2] = {0, 2 * nl}, len[2] = {2 * nl, nl};
    const int64_t begin = skip_u ? 2 * nl : 0, span = 3 * nl - begin;
    // r = 1 on free unknowns (dinv != 0 exactly there), z = D^-1 r, p = z
    hipLaunchKernelGGL(k_free_ones, dim3(grid_for(span)), dim3(256), 0, s, r + begin, w.dinv + begin, span);
    hipLaunchKernelGGL(k_mul, dim3(grid_for(span)), dim3(256), 0, s, z + begin, w.dinv + begin, r + begin, span);
    HIPCHK(hipMemcpyAsync(pv + begin, z + begin, sizeof(double) * span, hipMemcpyDeviceToDevice, s));
    // the level's own scratch (the levels' estimates run concurrently)
    double* sc = L.esc;
    double* rp = L.ered;
    for (int b = skip_u ? 1 : 0; b < 2; ++b) {
      dot2_async(r + off[b], r + off[b], len[b], sc + EIG_SC * b + EIG_PQ, rp);   // n_free (scratch slot)
      dot2_async(r + off[b], z + off[b], len[b], sc + EIG_SC * b + EIG_RZ, rp);
    }
    hipLaunchKernelGGL(k_eig_init, dim3(1), dim3(64), 0, s, sc, its, its_phi, skip_u ? 1 : 0);
    const int stride = EIG_MAX_ITS;
    // steps of the longer of the estimated blocks (a block past its own count
    // takes no step)
    const int max_it = std::min(skip_u ? its_phi : std::max(its, its_phi), stride);
    // per step: operator, p.q partials, alpha, update fused with the r.z
    // partials, beta, direction update (both blocks in every launch)
    // the same partition of the rows with and without the displacement block
    const int nb = std::min(RED_BLOCKS, grid_for(2 * nl));
    for (int it = 0; it < max_it; ++it) {
      // the phase-field block alone: its rows of the block operator
      level_apply<double>(l, pv, q, skip_u ? EPI_PHI : EPI_PLAIN, nullptr, nullptr, nullptr, nullptr, nullptr,
                          nullptr, L.epart, L.epart_bytes);
      hipLaunchKernelGGL(k_eig_pq_partial, dim3(nb), dim3(RED_THREADS), 0, s, pv, q, nl, begin, rp);
      hipLaunchKernelGGL(k_eig_alpha_reduce, dim3(1), dim3(RED_THREADS), 0, s, rp, nb, sc, L.eal, stride, it);
      hipLaunchKernelGGL(k_eig_update_partial, dim3(nb), dim3(RED_THREADS), 0, s, r, z, q, w.dinv, sc, nl, begin,
                         rp);
      hipLaunchKernelGGL(k_eig_beta_reduce, dim3(1), dim3(RED_THREADS), 0, s, rp, nb, sc, L.ebe, stride, it);
      hipLaunchKernelGGL(k_eig_waxpy, dim3(grid_for(span)), dim3(256), 0, s, pv, z, sc, nl, begin);
    }
    HIPCHK(hipMemcpyAsync(out, sc, sizeof(double) * 2 * EIG_SC, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(out + 2 * EIG_SC, L.eal, sizeof(double) * 2 * stride, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(out + 2 * EIG_SC + 2 * stride, L.ebe, sizeof(double) * 2 * stride,
                          hipMemcpyDeviceToHost, s));
  }
  void eig_finish(int l, const double* in, bool skip_u = false) {
    DevLevel& L = lev(l);
    const int stride = EIG_MAX_ITS;
    const double* h = in;
    const double* al = in + 2 * EIG_SC;
    const double* be = in + 2 * EIG_SC + 2 * stride;
    for (int b = skip_u ? 1 : 0; b < 2; ++b) {
      const int m = int(h[EIG_SC * b + EIG_STEPS]);
      double lo = 1.0, hi = 1.0;
      if (m > 0) {
        const double* A = al + b * stride;
        const double* B = be + b * stride;
        std::vector<double> dg(m), of(m > 1 ? m - 1 : 0);
        for (int j = 0; j < m; ++j) dg[j] = 1.0 / A[j] + (j > 0 ? B[j - 1] / A[j - 1] : 0.0);
        for (int j = 0; j + 1 < m; ++j) of[j] = std::sqrt(B[j]) / A[j];
        tridiag_extremes(dg, of, &lo, &hi);
      }
      L.lam_max[b] = hi;
      L.lam_min[b] = lo;
    }
  }
  // every level's estimate with one host wait. The levels are independent
  // (own vectors and scratch): they run on the side streams, largest level
  // first and round-robin, forked from and joined into the caller's stream;
  // each level's arithmetic is the same on any stream.
  void eig_estimate_all(bool skip_u = false) {
    const size_t per = size_t(2 * EIG_SC + 4 * EIG_MAX_ITS);
    const int nl = nlev();
    std::vector<int> order(static_cast<size_t>(nl));
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lev(a).n > lev(b).n; });
    hipStream_t main = s;
    HIPCHK(hipEventRecord(efork, main));
    for (int k = 0; k < EIG_STREAMS; ++k) HIPCHK(hipStreamWaitEvent(es[k], efork, 0));
    for (int i = 0; i < nl; ++i) {
      const int l = order[size_t(i)];
      s = es[i % EIG_STREAMS];
      eig_launch(l, l == 0 ? prm.coarse_eig_its : prm.eig_cg_its, l == 0 ? prm.coarse_eig_its : prm.eig_cg_its_phi,
                 eig_host + per * size_t(l), skip_u);
    }
    s = main;
    for (int k = 0; k < EIG_STREAMS; ++k) {
      HIPCHK(hipEventRecord(ejoin[k], es[k]));
      HIPCHK(hipStreamWaitEvent(main, ejoin[k], 0));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(main));
    for (int l = 0; l < nl; ++l) eig_finish(l, eig_host + per * size_t(l), skip_u);
  }

  // Smallest and largest eigenvalue of a symmetric tridiagonal matrix by
  // bisection on the Sturm sequence count.
  static void tridiag_extremes(const std::vector<double>& d, const std::vector<double>& e, double* lo, double* hi) {
    const int m = int(d.size());
    double a = d[0], b = d[0];
    for (int i = 0; i < m; ++i) {
      double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
      a = std::min(a, d[i] - r);
      b = std::max(b, d[i] + r);
    }
    auto count_below = [&](double x) {
      int c = 0;
      double q = d[0] - x;
      if (q < 0) ++c;
      for (int i = 1; i < m; ++i) {
        const double qq = (q == 0.0) ? 1e-300 : q;
        q = d[i] - x - e[i - 1] * e[i - 1] / qq;
        if (q < 0) ++c;
      }
      return c;
    };
    auto kth = [&](int k) {  // k-th smallest (0-based)
      double l = a, u = b;
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (l + u);
        if (mid == l || mid == u) break;
        if (count_below(mid) > k) u = mid; else l = mid;
      }
      return 0.5 * (l + u);
    };
    *lo = kth(0);
    *hi = kth(m - 1);
  }

  LevelWork<double>& w64of(DevLevel& L) { return L.w64; }

  template <typename T>
  void setup_levels() {
    for (int l = 0; l < nlev(); ++l) {
      DevLevel& L = lev(l);
      ensure_level_work<T>(L);
      LevelWork<T>& w = work<T>(L);
      hipLaunchKernelGGL((k_inject<T>), dim3(grid_for(L.n)), dim3(256), 0, s, w.state, L.n, L.leaf_index, U, phit,
                         n);
    }
    for (int l = 0; l < nlev(); ++l) {
      level_coef<T>(l);
      level_diag<T>(l);
    }
    HIPCHK(hipGetLastError());
  }

  void level_active_sets() {
    const int L = int(lv.size()) - 1;
    for (int l = L; l >= 0; --l) {
      const int64_t* ptp = l < L ? lv[l + 1].PT_ptr : nullptr;
      const int32_t* ptc = l < L ? lv[l + 1].PT_col : nullptr;
      const uint8_t* ff = l < L ? lv[l + 1].flags : nullptr;
      hipLaunchKernelGGL(k_level_active, dim3(grid_for(lv[l].n)), dim3(256), 0, s, lv[l].flags, lv[l].n,
                         lv[l].leaf_index, flags, ptp, ptc, ff, 1);
    }
    HIPCHK(hipGetLastError());
  }
  // global coarsening: the finest level is the leaf mesh and shares the leaf
  // flags (the leaf active set); a coarser unknown is active if the leaf
  // unknown at its position is or any finer unknown its interpolation
  // reaches (no home-level rule: every free leaf unknown is smoothed on the
  // finest level)
  void gc_level_active_sets() {
    const int L = nlev() - 1;
    for (int l = L - 1; l >= 0; --l) {
      DevLevel& D = lev(l);
      DevLevel& F = lev(l + 1);
      hipLaunchKernelGGL(k_level_active, dim3(grid_for(D.n)), dim3(256), 0, s, D.flags, D.n, D.leaf_index, flags,
                         F.PT_ptr, F.PT_col, F.flags, 0);
    }
    HIPCHK(hipGetLastError());
  }

  void setup_mg() {
    fp32_ready = false;
    select_hierarchy();
    if (H == H_gc && has_gc) gc_level_active_sets();
    else level_active_sets();
    setup_levels<double>();
    if (!eig_fixed) {
      // the displacement block's level operators depend on phi~ alone (the
      // degradation g(phi~) times elasticity, Dirichlet and edge rows fixed):
      // while phi~ is unchanged their diagonals and estimates repeat bit for
      // bit, so only the phase-field block is estimated again
      eig_estimate_all(ucache);
      ucache = true;
    }
    if (prm.vcycle_fp32) setup_fp32();
    mg_ready = true;
  }
  // FP32 copies of the level states and diagonals, made once per setup
  void setup_fp32() {
    setup_levels<float>();
    fp32_ready = true;
  }

  void residual(double* R, const double* Ust) {
    const double* st[4] = {phit, nullptr, nullptr, nullptr};
    leaf_op<MODE_RESID>(R, Ust, st);
  }

  // ---------------------------------------------------------------- GMRES --
  void apply_A(double* dst, const double* src, bool transpose) {
    const double* st[4];
    leaf_state4(st);
    if (transpose) leaf_op<MODE_JT>(dst, src, st);
    else leaf_op<MODE_J>(dst, src, st);
  }
  // P^-1 src: the block-diagonal V-cycle (Sec. 3.2), or with prec_kind = 1
  // the block-triangular form that keeps the coupling block: forward
  // substitution x_u = M_u^-1 b_u, x_phi = M_phi^-1 (b_phi - G_phi,u x_u)
  // (G_phi,u x_u from the phi rows of J~ (x_u, 0)); for systems with J~^T the
  // backward form, phi block first. Work vectors wv[8], wv[9].
  void apply_Minv(double* dst, const double* src, bool fp32, bool transpose = false) {
    if (prm.prec_kind != 1) {
      apply_block(dst, src, fp32);
      return;
    }
    double* t1 = wv[8];
    double* t2 = wv[9];
    const int first = transpose ? 1 : 0;
    hipLaunchKernelGGL(k_block_select, dim3(grid_for(3 * n)), dim3(256), 0, s, t1, src, n, first);
    apply_block(dst, t1, fp32);
    apply_A(t1, dst, transpose);
    hipLaunchKernelGGL(k_block_rhs, dim3(grid_for(3 * n)), dim3(256), 0, s, t1, src, n, 1 - first);
    apply_block(t2, t1, fp32);
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(3 * n)), dim3(256), 0, s, dst, t2, 1.0, 3 * n);
    HIPCHK(hipGetLastError());
  }
  void apply_block(double* dst, const double* src, bool fp32) {
    const bool gc = H == H_gc && has_gc;
    if (fp32) {
      if (!fp32_ready) setup_fp32();
      if (gc) vcycle_gc_impl<float>(dst, src);
      else vcycle_impl<float>(dst, src);
    } else {
      if (gc) vcycle_gc_impl<double>(dst, src);
      else vcycle_impl<double>(dst, src);
    }
  }

  // GMRES(m) with left preconditioning (Sec. 3.2, Table 1). Arnoldi by
  // classical Gram-Schmidt twice with the second projection delayed by one
  // step (DCGS2: Swirydowicz, Langou, Ananthan, Yang, Thomas, Numer. Linear
  // Algebra Appl. 2021; Bielich et al., Parallel Comput. 2022). Column j of V
  // holds q_j, the candidate for v_j after one projection, with its pending
  // coefficients cq = V_j^T q_j and |q_j|^2; the operator is applied to q_j,
  // and since the preconditioned operator is linear,
  //   M^-1 A v_j = (M^-1 A q_j - V_(j+1) Hbar_j cq) / rho_j,
  //   rho_j = (|q_j|^2 - |cq|^2)^(1/2),
  // so the correction happens in coefficient space. Per step two sweeps over
  // the basis: V_(j+1)^T w, then one pass writing v_j and q_(j+1) with the
  // products V_(j+2)^T q_(j+1) and |q_(j+1)|^2 (the second projection of the
  // next column and its norm). Where |cq|^2 would cancel more than a quarter
  // of |q|^2, the second projection is applied explicitly instead.
  int gmres(double* x, const double* b, bool transpose, double tol, pff_gmres_info* info, bool fp32) {
    const int64_t N = 3 * n;
    const int m = std::max(1, prm.gmres_restart);
    if (m + 2 > DCGS_MAX) throw std::runtime_error("gmres_restart too large");
    if (V_cap < m + 1) {
      if (ws) throw std::runtime_error("gmres_restart exceeds the bound workspace");
      if (V) hipFree(V);
      V = dalloc<double>(int64_t(m + 1) * N);
      V_cap = m + 1;
    }
    double* w = wv[0];
    double* t = wv[1];
    HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * N, s));
    apply_Minv(V, b, fp32, transpose);
    double beta = norm(V, N);
    if (!std::isfinite(beta)) throw nonfinite_error("GMRES: |P^-1 b| is not finite");
    pff_gmres_info inf{};
    inf.initial_residual = beta;
    inf.final_residual = beta;
    inf.tolerance = tol;
    int its = 0;
    bool conv = beta <= tol;
    // H: the Arnoldi Hessenberg matrix (for the coefficient-space
    // correction), R: its rotated upper-triangular factor
    std::vector<double> H(size_t(m + 1) * m), R(size_t(m) * m), cs(m), sn(m), g(m + 1);
    double* hdev = red_out + 64;
    auto sumsq = [](const std::vector<double>& v) {
      double r = 0.0;
      for (double e : v) r += e * e;
      return r;
    };
    while (!conv && its < prm.gmres_max_its) {
      // q_0 = the preconditioned residual, unnormalised (rho_0 = beta)
      std::vector<double> cq;
      double nq2 = beta * beta;
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int jdone = 0;
      double resid = beta;
      for (int j = 0; j < m; ++j) {
        double* qj = V + int64_t(j) * N;
        double* qn = V + int64_t(j + 1) * N;
        apply_A(t, qj, transpose);
        apply_Minv(w, t, fp32, transpose);
        const double rho = std::sqrt(nq2 - sumsq(cq));
        // sweep 1: a_i = v_i . w (i < j), a_j = q_j . w
        launch_k<MdotL>(j + 1, (const double*)V, (const double*)w, j + 1, N, red_part);
        reduce_to_host(j + 1, host_red);
        std::vector<double> a(host_red, host_red + j + 1);
        bool finite = std::isfinite(rho) && rho > 0.0;
        for (double e : a) finite = finite && std::isfinite(e);
        if (!finite) throw nonfinite_error("GMRES: a Gram-Schmidt coefficient or norm is not finite");
        // e = Hbar_j cq (rows 0..j), h1 = V_(j+1)^T M^-1 A v_j
        std::vector<double> e(j + 1, 0.0), h1(j + 1);
        for (int i = 0; i < j; ++i)
          for (int l = 0; l <= i + 1; ++l) e[l] += H[size_t(l) * m + i] * cq[i];
        double ca = 0.0;
        for (int i = 0; i < j; ++i) ca += cq[i] * a[i];
        const double vjw = (a[j] - ca) / rho;
        for (int i = 0; i < j; ++i) h1[i] = (a[i] - e[i]) / rho;
        h1[j] = (vjw - e[j]) / rho;
        // sweep 2: v_j in place, q_(j+1), V_(j+2)^T q_(j+1) and |q_(j+1)|^2
        DcgsCoef cf{};
        for (int i = 0; i < j; ++i) {
          cf.c[i] = cq[i];
          cf.d[i] = e[i] / rho + h1[i];
        }
        cf.gamma = e[j] / rho + h1[j];
        cf.inv_rho = 1.0 / rho;
        cf.j = j;
        launch_k<DcgsL>(j + 2, V, (const double*)w, cf, N, red_part);
        reduce_to_host(j + 2, host_red);
        std::vector<double> cn(host_red, host_red + j + 1);
        double nn2 = host_red[j + 1];
        finite = std::isfinite(nn2);
        for (double v : cn) finite = finite && std::isfinite(v);
        if (!finite) throw nonfinite_error("GMRES: a Gram-Schmidt coefficient or norm is not finite");
        if (sumsq(cn) > 0.25 * nn2) {
          // the delayed norm would cancel: project q_(j+1) now
          HIPCHK(hipMemcpyAsync(hdev, cn.data(), sizeof(double) * (j + 1), hipMemcpyHostToDevice, s));
          hipLaunchKernelGGL(k_mcombine_sq_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, (const double*)V, qn,
                             (const double*)hdev, j + 1, N, red_part);
          reduce_to_host(1, host_red);
          nn2 = host_red[0];
          if (!std::isfinite(nn2)) throw nonfinite_error("GMRES: a Gram-Schmidt norm is not finite");
          cq.assign(size_t(j + 1), 0.0);
        } else {
          cq = cn;
        }
        nq2 = nn2;
        const double hn = std::sqrt(std::max(nq2 - sumsq(cq), 0.0));
        std::vector<double> h(j + 2);
        for (int i = 0; i <= j; ++i) h[i] = h1[i] + cn[i];
        for (int i = 0; i < j; ++i) {
          const double tt = cs[i] * h[i] + sn[i] * h[i + 1];
          h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
          h[i] = tt;
        }
        for (int i = 0; i <= j; ++i) H[size_t(i) * m + j] = h1[i] + cn[i];
        H[size_t(j + 1) * m + j] = hn;
        const double den = std::hypot(h[j], hn);
        cs[j] = h[j] / den;
        sn[j] = hn / den;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        // the triangular factor R (rotated columns) for the back substitution
        for (int i = 0; i < j; ++i) R[size_t(i) * m + j] = h[i];
        R[size_t(j) * m + j] = den;
        resid = std::fabs(g[j + 1]);
        ++its;
        jdone = j + 1;
        if (resid <= tol || its >= prm.gmres_max_its || hn == 0.0) break;
      }
      std::vector<double> y(jdone);
      for (int i = jdone - 1; i >= 0; --i) {
        double sum = g[i];
        for (int k = i + 1; k < jdone; ++k) sum -= R[size_t(i) * m + k] * y[k];
        y[i] = sum / R[size_t(i) * m + i];
      }
      HIPCHK(hipMemcpyAsync(hdev, y.data(), sizeof(double) * jdone, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_mcombine, dim3(grid_for(N)), dim3(256), 0, s, x, V, hdev, jdone, N, 1.0);
      inf.final_residual = resid;
      if (resid <= tol) { conv = true; break; }
      if (its >= prm.gmres_max_its) break;
      // restart: V_0 = Minv (b - A x)
      apply_A(t, x, transpose);
      hipLaunchKernelGGL(k_sub, dim3(grid_for(N)), dim3(256), 0, s, w, b, t, N);
      apply_Minv(V, w, fp32, transpose);
      beta = norm(V, N);
      if (!std::isfinite(beta)) throw nonfinite_error("GMRES: restart residual is not finite");
      inf.final_residual = beta;
      if (beta <= tol) { conv = true; break; }
    }
    HIPCHK(hipStreamSynchronize(s));
    inf.iterations = its;
    inf.converged = conv ? 1 : 0;
    if (info) *info = inf;
    return conv ? PFF_OK : PFF_W_NOCONV;
  }
};

template <>
LevelWork<double>& pff_ctx::work<double>(DevLevel& L) { return L.w64; }
template <>
LevelWork<float>& pff_ctx::work<float>(DevLevel& L) { return L.w32; }

// ------------------------------------------------------------------ C ABI --
#define GUARD_BEGIN try {
#define GUARD_END(ctx)                                      \
  }                                                         \
  catch (const nonfinite_error& e) {                        \
    if (ctx) (ctx)->err = e.what();                         \
    return PFF_E_NONFINITE;                                 \
  }                                                         \
  catch (const std::bad_alloc&) {                           \
    if (ctx) (ctx)->err = "device allocation failed";       \
    return PFF_E_NOMEM;                                     \
  }                                                         \
  catch (const std::exception& e) {                         \
    if (ctx) (ctx)->err = e.what();                         \
    return PFF_E_HIP;                                       \
  }

static bool params_valid(const pff_params& p) {
  return p.cheb_degree >= 1 && p.coarse_its >= 1 && p.gmres_restart >= 1 && p.gmres_restart <= 60 &&
         p.gmres_max_its >= 1 && p.ls_max >= 1 && p.ls_omega > 0.0 && p.ls_omega <= 1.0 &&
         p.coarse_mode >= 0 && p.coarse_mode <= 1 && p.eig_cg_its >= 1 && p.eig_cg_its <= EIG_MAX_ITS &&
         p.coarse_eig_its >= 1 && p.coarse_eig_its <= EIG_MAX_ITS && std::isfinite(p.pdas_c) && p.pdas_c >= 0.0 &&
         p.mg_kind >= 0 && p.mg_kind <= 1 && p.prec_kind >= 0 && p.prec_kind <= 1 && p.eig_cg_its_phi >= 1 &&
         p.eig_cg_its_phi <= EIG_MAX_ITS;
}

extern "C" {

int pff_default_params(pff_params* p) {
  if (!p) return PFF_E_ARG;
  std::memset(p, 0, sizeof(*p));
  p->E = 1.0;
  p->nu = 0.2;
  p->Gc = 1.0;
  p->pressure = 1e-3;
  p->kappa = 1e-10;
  p->ell = 0.1;
  p->cheb_degree = 3;
  p->smooth_range = 0.08;
  p->upper_factor = 1.2;
  p->eig_cg_its = 20;
  p->coarse_mode = 0;
  p->coarse_its = 30;
  p->coarse_eig_its = 40;
  p->gmres_restart = 30;
  p->gmres_max_its = 300;
  p->gmres_rtol = 1e-8;
  p->gmres_atol = 1e-12;
  p->ls_omega = 0.5;
  p->ls_max = 10;
  p->vcycle_fp32 = 0;
  p->pdas_c = 0.0;
  p->eig_cg_its_phi = 10;
  return PFF_OK;
}

// text of the last failed pff_create on this thread (pff_last_error(NULL))
static thread_local std::string g_create_err = "null context";

static int create_failed(pff_ctx* c, int rc, const std::string& why) {
  g_create_err = why;
  if (c) pff_destroy(c);   // frees whatever was uploaded before the failure
  return rc;
}

int pff_create(const pff_mesh_spec* spec, const pff_params* params, pff_ctx** out) {
  if (!spec || !params || !out) return create_failed(nullptr, PFF_E_ARG, "pff_create: null argument");
  *out = nullptr;
  std::unique_ptr<pff_ctx> c(new pff_ctx());
  MeshSpec ms;
  ms.n_base = spec->n_base;
  ms.n_local = spec->n_local;
  ms.degree = spec->degree;
  ms.coarse = spec->coarse > 0 ? spec->coarse : 16;
  ms.band_x = spec->band_x;
  ms.band_y = spec->band_y;
  ms.tile_x = spec->tile_x;
  ms.tile_y = spec->tile_y;
  ms.mg_global = spec->mg_global != 0;
  if (!params_valid(*params)) return create_failed(nullptr, PFF_E_ARG, "pff_create: invalid parameters");
  if (params->mg_kind == 1 && !ms.mg_global)
    return create_failed(nullptr, PFF_E_ARG, "pff_create: mg_kind = 1 needs a mesh spec with mg_global");
  try {
    bool built = false;
    try {
      built = c->mesh.build(ms);
    } catch (const std::runtime_error& e) {
      c->mesh.error = e.what();
    }
    if (!built) return create_failed(nullptr, PFF_E_MESH, "pff_create: mesh: " + c->mesh.error);
    if (c->mesh.n_levels > COPY_MAX_LEVELS)
      return create_failed(nullptr, PFF_E_ARG, "pff_create: more multigrid levels than the library holds (" +
                                                   std::to_string(COPY_MAX_LEVELS) + ")");
    bool too_big = c->mesh.tiles.max_local > 65535;
    for (const Level& L : c->mesh.levels) too_big = too_big || L.tiles.max_local > 65535;
    for (const GcLevel& G : c->mesh.gc) too_big = too_big || G.tiles.max_local > 65535;
    if (too_big) return create_failed(nullptr, PFF_E_MESH, "pff_create: a tile has more than 65535 local nodes");
    // the tile kernels address node arrays and partial sums with 32-bit byte
    // offsets per component (8-byte elements)
    bool too_many = c->mesh.n_nodes >= (int64_t(1) << 29) || c->mesh.tiles.n_slots >= (int64_t(1) << 29);
    for (const GcLevel& G : c->mesh.gc) too_many = too_many || G.tiles.n_slots >= (int64_t(1) << 29);
    for (const Level& L : c->mesh.levels) too_many = too_many || L.tiles.n_slots >= (int64_t(1) << 29);
    if (too_many) return create_failed(nullptr, PFF_E_MESH, "pff_create: more than 2^29 nodes or partial-sum slots");
    c->prm = *params;
    c->p = ms.degree;
    c->n = c->mesh.n_nodes;
    const int64_t n = c->n;
    c->tiles = upload_tiles(c->mesh.tiles);
    c->flags = upload(c->mesh.flags);
    c->nodeX = upload(c->mesh.NX);
    c->hang = upload(c->mesh.hanging);
    c->n_hang = int(c->mesh.hanging.size());
    c->lv.resize(c->mesh.levels.size());
    for (size_t l = 0; l < c->lv.size(); ++l) {
      const Level& HL = c->mesh.levels[l];
      DevLevel& D = c->lv[l];
      D.n = HL.n;
      D.tiles = upload_tiles(HL.tiles);
      D.flags = upload(HL.flags);
      D.leaf_index = upload(HL.leaf_index);
      if (l > 0) {
        D.PT_ptr = upload(HL.PT.ptr);
        D.PT_col = upload(HL.PT.col);
        upload_transfers(HL.P, HL.PT, D);
      }
    }
    for (size_t l = 0; l < c->lv.size(); ++l) c->H_ls.push_back(&c->lv[l]);
    if (!c->mesh.gc.empty()) {
      // global-coarsening levels: k <= b shared with local smoothing, own
      // levels above the base mesh, the leaf level last
      const int nl = int(c->mesh.gc.size());
      c->gcown.reserve(size_t(nl));
      for (int k = 0; k < nl; ++k) {
        const GcLevel& G = c->mesh.gc[size_t(k)];
        if (k < nl - 1 && !G.own) {
          c->H_gc.push_back(&c->lv[size_t(k)]);
          continue;
        }
        c->gcown.emplace_back();
        DevLevel& D = c->gcown.back();
        D.n = G.n;
        if (k == nl - 1) {
          D.tiles = c->tiles;
          D.flags = c->flags;
          D.shares_leaf = true;
          std::vector<int32_t> id(size_t(G.n));
          std::iota(id.begin(), id.end(), 0);
          D.leaf_index = upload(id);
        } else {
          D.tiles = upload_tiles(G.tiles);
          D.flags = upload(G.flags);
          D.leaf_index = upload(G.leaf_index);
        }
        if (k > 0) {
          const Csr& P = G.P.rows > 0 ? G.P : c->mesh.levels[size_t(k)].P;
          const Csr& PT = G.P.rows > 0 ? G.PT : c->mesh.levels[size_t(k)].PT;
          D.PT_ptr = upload(PT.ptr);
          D.PT_col = upload(PT.col);
          upload_transfers(P, PT, D);
        }
        c->H_gc.push_back(&D);
      }
      c->has_gc = true;
    }
    c->select_hierarchy();
    c->setup_coarse_cells();
    int64_t slots = c->mesh.tiles.n_slots;
    for (const Level& L : c->mesh.levels) slots = std::max(slots, L.tiles.n_slots);
    for (const GcLevel& G : c->mesh.gc) slots = std::max(slots, G.tiles.n_slots);
    c->part_bytes = size_t(3 * std::max<int64_t>(slots, 1)) * sizeof(double);
    {
      // per-level scratch of the concurrent eigenvalue estimates
      std::vector<DevLevel*> all;
      for (DevLevel& D : c->lv) all.push_back(&D);
      for (DevLevel& D : c->gcown) all.push_back(&D);
      for (DevLevel* D : all) {
        D->epart_bytes = size_t(3 * std::max<int64_t>(D->tiles.n_slots, 1)) * sizeof(double);
        D->epart = dalloc<double>(int64_t(D->epart_bytes / sizeof(double)));
        D->esc = dalloc<double>(2 * EIG_SC);
        D->eal = dalloc<double>(2 * EIG_MAX_ITS);
        D->ebe = dalloc<double>(2 * EIG_MAX_ITS);
        D->ered = dalloc<double>(2 * RED_BLOCKS);
      }
      for (int k = 0; k < pff_ctx::EIG_STREAMS; ++k) HIPCHK(hipStreamCreateWithFlags(&c->es[k], hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&c->efork, hipEventDisableTiming));
      for (int k = 0; k < pff_ctx::EIG_STREAMS; ++k)
        HIPCHK(hipEventCreateWithFlags(&c->ejoin[k], hipEventDisableTiming));
    }
    c->red_part = dalloc<double>(RED_BLOCKS * 64);
    c->red_out = dalloc<double>(256);
    c->ccg_s = dalloc<double>(8);
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&c->host_red), 256 * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&c->eig_host),
                         size_t(COPY_MAX_LEVELS) * size_t(2 * EIG_SC + 4 * EIG_MAX_ITS) * sizeof(double),
                         hipHostMallocDefault));
    HIPCHK(scratch_address(&c->scratch_dev));
    (void)n;
  } catch (const std::bad_alloc&) {
    return create_failed(c.release(), PFF_E_NOMEM, "pff_create: device allocation failed");
  } catch (const std::exception& e) {
    return create_failed(c.release(), PFF_E_HIP, std::string("pff_create: ") + e.what());
  }
  *out = c.release();
  return PFF_OK;
}

int pff_destroy(pff_ctx* c) {
  if (!c) return PFF_E_ARG;
  auto f = [](void* p) { if (p) hipFree(p); };
  auto ft = [&](DevTiles& t) {
    f(t.info); f(t.shared); f(t.sh_tab); f(t.loc); f(t.loc_sub); f(t.cinfo);
    f(t.hang_rec); f(t.hang_w); f(t.hang_col);
  };
  ft(c->tiles);
  f(c->flags);
  f(c->nodeX);
  f(c->hang);
  std::vector<DevLevel*> all;
  for (DevLevel& D : c->lv) all.push_back(&D);
  for (DevLevel& D : c->gcown) all.push_back(&D);
  for (DevLevel* Dp : all) {
    DevLevel& D = *Dp;
    if (!D.shares_leaf) {
      ft(D.tiles);
      f(D.flags);
    }
    f(D.epart); f(D.esc); f(D.eal); f(D.ebe); f(D.ered);
    f(D.leaf_index); f(D.PT_ptr); f(D.PT_col); f(D.P_ell); f(D.PT_ell); f(D.PT_rows); f(D.P_wtab);
    if (!c->ws) {   // a bound workspace belongs to the caller
      LevelWork<double>& a = D.w64;
      f(a.state); f(a.d); f(a.x[0]); f(a.x[1]); f(a.dir[0]); f(a.dir[1]); f(a.dinv); f(a.coef);
      LevelWork<float>& b = D.w32;
      f(b.state); f(b.d); f(b.x[0]); f(b.x[1]); f(b.dir[0]); f(b.dir[1]); f(b.dinv); f(b.coef);
    }
  }
  if (!c->ws) {
    f(c->U); f(c->phio); f(c->phit); f(c->mass);
    for (int i = 0; i < pff_ctx::N_WORK; ++i) f(c->wv[i]);
    f(c->V); f(c->part); f(c->part_jt);
  }
  for (int k = 0; k < pff_ctx::EIG_STREAMS; ++k) {
    if (c->es[k]) hipStreamDestroy(c->es[k]);
    if (c->ejoin[k]) hipEventDestroy(c->ejoin[k]);
  }
  if (c->efork) hipEventDestroy(c->efork);
  f(c->red_part); f(c->red_out); f(c->ccg_s); f(c->coarse_nodes); 
  if (c->host_red) hipHostFree(c->host_red);
  if (c->eig_host) hipHostFree(c->eig_host);
  delete c;
  return PFF_OK;
}

int pff_set_params(pff_ctx* c, const pff_params* p) {
  if (!c || !p) return PFF_E_ARG;
  if (!params_valid(*p)) return PFF_E_ARG;
  if (c->ws && p->gmres_restart > c->ws_restart) {
    c->err = "gmres_restart exceeds the restart the bound workspace was sized for";
    return PFF_E_ARG;
  }
  if (p->mg_kind == 1 && !c->has_gc) {
    c->err = "mg_kind = 1 needs a context created with mg_global";
    return PFF_E_ARG;
  }
  c->prm = *p;
  c->mg_ready = false;
  c->fp32_ready = false;
  c->ucache = false;
  c->select_hierarchy();
  return PFF_OK;
}

int pff_workspace_bytes(const pff_ctx* c, size_t* bytes) {
  if (!c || !bytes) return PFF_E_ARG;
  *bytes = const_cast<pff_ctx*>(c)->workspace_bytes();   // sizes only: nothing is modified
  return PFF_OK;
}

int pff_bind_workspace(pff_ctx* c, void* ptr, size_t bytes) {
  if (!c || !ptr || (reinterpret_cast<uintptr_t>(ptr) & 255) != 0) return PFF_E_ARG;
  if (c->ws || c->work_ready) {
    c->err = "bind_workspace must come before the first call that uses work vectors";
    return PFF_E_STATE;
  }
  const int m = std::max(1, c->prm.gmres_restart);
  if (bytes < c->layout_work(false, m)) {
    c->err = "workspace smaller than pff_workspace_bytes";
    return PFF_E_ARG;
  }
  GUARD_BEGIN
  c->ws = static_cast<char*>(ptr);
  c->ws_size = bytes;
  c->ws_restart = m;
  c->layout_work(true, m);
  c->ensure_work();
  return PFF_OK;
  GUARD_END(c)
}

int pff_sizes(const pff_ctx* c, int64_t* n_nodes, int32_t* n_levels, int64_t* level_nodes) {
  if (!c) return PFF_E_ARG;
  if (n_nodes) *n_nodes = c->n;
  if (n_levels) *n_levels = int32_t(c->nlev());
  if (level_nodes)
    for (int l = 0; l < c->nlev(); ++l) level_nodes[l] = c->lev(l).n;
  return PFF_OK;
}

int pff_lattice(const pff_ctx* c, int64_t* M) {
  if (!c || !M) return PFF_E_ARG;
  *M = c->mesh.M;
  return PFF_OK;
}

int pff_node_coords(const pff_ctx* c, int32_t level, int32_t* xy) {
  if (!c || !xy || level < -1 || level >= int32_t(c->nlev())) return PFF_E_ARG;
  const std::vector<int32_t>* Xp = level < 0 ? &c->mesh.NX : &c->mesh.levels[size_t(level)].NX;
  const std::vector<int32_t>* Yp = level < 0 ? &c->mesh.NY : &c->mesh.levels[size_t(level)].NY;
  if (level >= 0 && c->H == c->H_gc && c->has_gc) {
    const GcLevel& G = c->mesh.gc[size_t(level)];
    if (level == c->nlev() - 1) { Xp = &c->mesh.NX; Yp = &c->mesh.NY; }
    else if (G.own) { Xp = &G.NX; Yp = &G.NY; }
  }
  const std::vector<int32_t>& X = *Xp;
  const std::vector<int32_t>& Y = *Yp;
  std::memcpy(xy, X.data(), X.size() * sizeof(int32_t));
  std::memcpy(xy + X.size(), Y.data(), Y.size() * sizeof(int32_t));
  return PFF_OK;
}

int pff_node_flags(const pff_ctx* c, int32_t level, uint8_t* out) {
  if (!c || !out || level < -1 || level >= int32_t(c->nlev())) return PFF_E_ARG;
  const int64_t nn = level < 0 ? c->n : c->lev(level).n;
  const uint8_t* src = level < 0 ? c->flags : c->lev(level).flags;
  if (hipMemcpy(out, src, size_t(nn), hipMemcpyDeviceToHost) != hipSuccess) return PFF_E_HIP;
  return PFF_OK;
}

int pff_tile_stats(const pff_ctx* c, int32_t level, int64_t* n_tiles, int64_t* n_records, int64_t* max_cells) {
  if (!c || level < -1 || level >= int32_t(c->nlev())) return PFF_E_ARG;
  const DevTiles& t = level < 0 ? c->tiles : c->lev(level).tiles;
  if (n_tiles) *n_tiles = t.n_tiles;
  if (n_records) *n_records = t.n_rec;
  if (max_cells) *max_cells = t.max_cells;
  return PFF_OK;
}

int pff_set_state(pff_ctx* c, const double* U, const double* phi_old, const double* phi_tilde,
                  const uint8_t* active, int32_t setup_mg, void* stream) {
  if (!c || !U || !phi_old || !phi_tilde) return PFF_E_ARG;
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  c->ensure_work();
  const int64_t n = c->n;
  HIPCHK(hipMemcpyAsync(c->U, U, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, c->s));
  HIPCHK(hipMemcpyAsync(c->phio, phi_old, sizeof(double) * n, hipMemcpyDeviceToDevice, c->s));
  // keep the previous phi~ to tell whether it changed (wv[9] is free here)
  const bool compare = c->has_state && c->ucache;
  if (compare) HIPCHK(hipMemcpyAsync(c->wv[9], c->phit, sizeof(double) * n, hipMemcpyDeviceToDevice, c->s));
  HIPCHK(hipMemcpyAsync(c->phit, phi_tilde, sizeof(double) * n, hipMemcpyDeviceToDevice, c->s));
  if (c->n_hang) {
    const int np1 = c->p + 1;
    hipLaunchKernelGGL((k_distribute<double>), dim3(grid_for(3 * c->n_hang)), dim3(256), 0, c->s, c->U, n, 3, c->hang,
                       c->n_hang, np1);
    hipLaunchKernelGGL((k_distribute<double>), dim3(grid_for(c->n_hang)), dim3(256), 0, c->s, c->phit, n, 1, c->hang,
                       c->n_hang, np1);
    hipLaunchKernelGGL((k_distribute<double>), dim3(grid_for(c->n_hang)), dim3(256), 0, c->s, c->phio, n, 1, c->hang,
                       c->n_hang, np1);
  }
  if (compare) {
    hipLaunchKernelGGL(k_neq_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, c->s, c->wv[9], c->phit, n,
                       c->red_part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, c->s, c->red_part, RED_BLOCKS, 1,
                       c->red_out + 210);
    HIPCHK(hipMemcpyAsync(c->host_red + 210, c->red_out + 210, sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    if (c->host_red[210] != 0.0) c->ucache = false;
  } else {
    c->ucache = false;
  }
  if (active) {
    hipLaunchKernelGGL(k_set_active, dim3(grid_for(n)), dim3(256), 0, c->s, c->flags, active, n);
  } else {
    double* R = c->wv[2];
    c->residual(R, c->U);
    double* tau = c->red_out + 200;
    hipLaunchKernelGGL(k_lambda_max_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, c->s, R, c->mass + 2 * n,
                       c->flags, n, c->red_part);
    hipLaunchKernelGGL(k_reduce_max_final, dim3(1), dim3(RED_THREADS), 0, c->s, c->red_part, RED_BLOCKS, 1e-12, tau);
    hipLaunchKernelGGL(k_active_rule, dim3(grid_for(n)), dim3(256), 0, c->s, c->flags, R, c->mass + 2 * n,
                       c->U + 2 * n, c->phio, n, tau, c->prm.pdas_c);
  }
  HIPCHK(hipGetLastError());
  c->has_state = true;
  c->mg_ready = false;
  c->fp32_ready = false;
  if (setup_mg) {
    c->setup_mg();
    HIPCHK(hipStreamSynchronize(c->s));
  }
  return PFF_OK;
  GUARD_END(c)
}

int pff_get_active(pff_ctx* c, uint8_t* active, void* stream) {
  if (!c || !active) return PFF_E_ARG;
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_get_active, dim3(grid_for(c->n)), dim3(256), 0, c->s, active, c->flags, c->n);
  HIPCHK(hipGetLastError());
  return PFF_OK;
  GUARD_END(c)
}

int pff_extrapolate_phi(pff_ctx* c, const double* phi_prev, const double* phi_prev2, double theta, double* out,
                        void* stream) {
  if (!c || !phi_prev || !phi_prev2 || !out || !std::isfinite(theta) || theta < 0.0) return PFF_E_ARG;
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_extrapolate_phi, dim3(grid_for(c->n)), dim3(256), 0, c->s, out, phi_prev, phi_prev2, theta,
                     c->n);
  HIPCHK(hipGetLastError());
  return PFF_OK;
  GUARD_END(c)
}

int pff_vmult(pff_ctx* c, double* dst, const double* src, void* stream) {
  if (!c || !dst || !src || dst == src) return PFF_E_ARG;
  if (!c->has_state) { c->err = "vmult needs a state"; return PFF_E_STATE; }
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  c->apply_A(dst, src, false);
  return PFF_OK;
  GUARD_END(c)
}

int pff_vmult_noalloc(pff_ctx* c, double* dst, const double* src, void* stream) {
  if (!c || !dst || !src || dst == src) return PFF_E_ARG;
  const size_t need = size_t(3 * std::max<int64_t>(c->tiles.n_slots, 1)) * sizeof(double);
  if (need > size_t(PFF_NOALLOC_SCRATCH_BYTES)) {
    c->err = "vmult_noalloc: the mesh needs " + std::to_string(need) + " bytes of partial sums, above the " +
             std::to_string(size_t(PFF_NOALLOC_SCRATCH_BYTES)) + "-byte static scratch; use pff_vmult";
    return PFF_E_ARG;
  }
  if (!c->has_state) { c->err = "vmult_noalloc needs a state"; return PFF_E_STATE; }
  if (!c->scratch_dev) { c->err = "vmult_noalloc: scratch address not resolved"; return PFF_E_STATE; }
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  const double* st[4];
  c->leaf_state4(st);
  TileArgs<double> a{};
  a.src = src;
  a.dst = dst;
  for (int i = 0; i < 4; ++i) a.st[i] = st[i];
  c->launch_tile<double, MODE_J, EPI_PLAIN>(c->tiles, c->flags, c->n, a, c->scratch_dev,
                                            size_t(PFF_NOALLOC_SCRATCH_BYTES));
  return PFF_OK;
  GUARD_END(c)
}

int pff_vmult_T(pff_ctx* c, double* dst, const double* src, int32_t batch, void* stream) {
  if (!c || !dst || !src || dst == src || batch < 1) return PFF_E_ARG;
  if (!c->has_state) { c->err = "vmult_T needs a state"; return PFF_E_STATE; }
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  c->ensure_work();
  if (batch == 1) {
    c->apply_A(dst, src, true);
    return PFF_OK;
  }
  // chunks of at most JT_BATCH_MAX right-hand sides, the state read once per
  // tile and chunk
  for (int b = 0; b < batch; b += JT_BATCH_MAX) {
    const int nb = std::min(JT_BATCH_MAX, batch - b);
    c->leaf_jt_batch(dst + int64_t(b) * 3 * c->n, src + int64_t(b) * 3 * c->n, nb);
  }
  return PFF_OK;
  GUARD_END(c)
}

int pff_inverse_diagonal(pff_ctx* c, int32_t level, void* dst, int32_t fp32, void* stream) {
  if (!c || !dst || level < -1 || level >= int32_t(c->nlev())) return PFF_E_ARG;
  if (!c->has_state) { c->err = "inverse_diagonal needs a state"; return PFF_E_STATE; }
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  if (level < 0) {
    const double* st[4];
    c->leaf_state4(st);
    TileArgs<double> a{};
    a.dst = static_cast<double*>(dst);
    for (int i = 0; i < 4; ++i) a.st[i] = st[i];
    c->launch_tile<double, MODE_DIAG_LEAF, EPI_PLAIN>(c->tiles, c->flags, c->n, a);
    return PFF_OK;
  }
  if (!c->mg_ready) { c->err = "level diagonals need set_state with setup_mg"; return PFF_E_STATE; }
  DevLevel& D = c->lev(level);
  if (fp32) {
    if (!c->fp32_ready) c->setup_fp32();
    HIPCHK(hipMemcpyAsync(dst, D.w32.dinv, sizeof(float) * 3 * D.n, hipMemcpyDeviceToDevice, c->s));
  } else {
    HIPCHK(hipMemcpyAsync(dst, D.w64.dinv, sizeof(double) * 3 * D.n, hipMemcpyDeviceToDevice, c->s));
  }
  return PFF_OK;
  GUARD_END(c)
}

int pff_vcycle(pff_ctx* c, double* dst, const double* src, int32_t fp32, void* stream) {
  if (!c || !dst || !src || dst == src) return PFF_E_ARG;
  if (!c->has_state || !c->mg_ready) { c->err = "vcycle needs set_state with setup_mg"; return PFF_E_STATE; }
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  c->apply_Minv(dst, src, fp32 != 0);
  return PFF_OK;
  GUARD_END(c)
}

int pff_get_eigen(const pff_ctx* c, double* lam_max, double* lam_min0) {
  if (!c) return PFF_E_ARG;
  for (int l = 0; l < c->nlev(); ++l)
    for (int b = 0; b < 2; ++b)
      if (lam_max) lam_max[2 * l + b] = c->lev(l).lam_max[b];
  if (lam_min0)
    for (int b = 0; b < 2; ++b) lam_min0[b] = c->lev(0).lam_min[b];
  return PFF_OK;
}

int pff_set_eigen(pff_ctx* c, const double* lam_max, const double* lam_min0) {
  if (!c) return PFF_E_ARG;
  c->ucache = false;
  if (!lam_max) { c->eig_fixed = false; return PFF_OK; }
  for (int l = 0; l < c->nlev(); ++l)
    for (int b = 0; b < 2; ++b) c->lev(l).lam_max[b] = lam_max[2 * l + b];
  if (lam_min0)
    for (int b = 0; b < 2; ++b) c->lev(0).lam_min[b] = lam_min0[b];
  c->eig_fixed = true;
  return PFF_OK;
}

int pff_gmres_solve(pff_ctx* c, double* x, const double* b, int32_t transpose, double tol_override,
                    pff_gmres_info* info, void* stream) {
  if (!c || !x || !b || x == b) return PFF_E_ARG;
  if (!c->has_state || !c->mg_ready) { c->err = "gmres needs set_state with setup_mg"; return PFF_E_STATE; }
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  double tol = tol_override;
  if (!(tol > 0.0)) tol = std::max(c->prm.gmres_atol, c->prm.gmres_rtol * c->norm(b, 3 * c->n));
  return c->gmres(x, b, transpose != 0, tol, info, c->prm.vcycle_fp32 != 0);
  GUARD_END(c)
}

int pff_residual(pff_ctx* c, double* R, const double* U, int32_t masked, void* stream) {
  if (!c || !R || !U || R == U) return PFF_E_ARG;
  if (!c->has_state) { c->err = "residual needs a state"; return PFF_E_STATE; }
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  c->residual(R, U);
  if (masked) hipLaunchKernelGGL(k_mask_leaf, dim3(grid_for(3 * c->n)), dim3(256), 0, c->s, R, c->flags, c->n);
  HIPCHK(hipGetLastError());
  return PFF_OK;
  GUARD_END(c)
}

int pff_newton_step(pff_ctx* c, double* U, const double* phi_old, const double* phi_tilde, uint8_t* active_inout,
                    pff_newton_info* info, void* stream) {
  if (!c || !U || !phi_old || !phi_tilde) return PFF_E_ARG;
  GUARD_BEGIN
  using clk = std::chrono::steady_clock;
  auto t0 = clk::now();
  c->s = static_cast<hipStream_t>(stream);
  c->ensure_work();
  const int64_t n = c->n, N = 3 * n;
  pff_newton_info inf{};
  // state at U (hanging entries distributed), residual, active set
  int rc = pff_set_state(c, U, phi_old, phi_tilde, nullptr, 0, stream);
  if (rc) return rc;
  double* R = c->wv[2];
  double* Uc = c->wv[3];
  double* dU = c->wv[4];
  double* trial = c->wv[5];
  double* Rt = c->wv[6];
  c->residual(R, c->U);
  // counts of active entries and changes
  hipLaunchKernelGGL(k_count_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, c->s, c->flags, active_inout, n,
                     c->red_part);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, c->s, c->red_part, RED_BLOCKS, 2, c->red_out);
  HIPCHK(hipMemcpyAsync(c->host_red, c->red_out, 2 * sizeof(double), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  inf.n_active = int64_t(c->host_red[0]);
  inf.active_changed = int64_t(c->host_red[1]);
  // baseline |R~(U)|
  hipLaunchKernelGGL(k_mask_leaf, dim3(grid_for(N)), dim3(256), 0, c->s, R, c->flags, n);
  const double base = c->norm(R, N);
  inf.residual_before = base;
  if (!std::isfinite(base)) throw nonfinite_error("newton_step: |R~(U)| is not finite");
  // U_c and the right-hand side R~(U_c)
  HIPCHK(hipMemcpyAsync(Uc, c->U, sizeof(double) * N, hipMemcpyDeviceToDevice, c->s));
  hipLaunchKernelGGL(k_apply_active, dim3(grid_for(n)), dim3(256), 0, c->s, Uc, c->phio, c->flags, n);
  c->residual(Rt, Uc);
  hipLaunchKernelGGL(k_mask_leaf, dim3(grid_for(N)), dim3(256), 0, c->s, Rt, c->flags, n);
  inf.rhs_norm = c->norm(Rt, N);
  // multigrid setup at U
  c->setup_mg();
  HIPCHK(hipStreamSynchronize(c->s));
  auto t1 = clk::now();
  // GMRES
  const double tol = std::max(c->prm.gmres_atol, c->prm.gmres_rtol * inf.rhs_norm);
  pff_gmres_info gi{};
  int grc = c->gmres(dU, Rt, false, tol, &gi, c->prm.vcycle_fp32 != 0);
  inf.gmres_iterations = gi.iterations;
  inf.gmres_converged = gi.converged;
  auto t2 = clk::now();
  // dU = (U_c - U) + dU_f, hanging entries from masters
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(N)), dim3(256), 0, c->s, dU, Uc, 1.0, N);
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(N)), dim3(256), 0, c->s, dU, c->U, -1.0, N);
  if (c->n_hang)
    hipLaunchKernelGGL((k_distribute<double>), dim3(grid_for(3 * c->n_hang)), dim3(256), 0, c->s, dU, n, 3, c->hang,
                       c->n_hang, c->p + 1);
  // line search: trial = U + omega^(l-1) dU
  int ls = 0;
  double rn = base;
  bool decreased = false;
  for (int l = 1; l <= c->prm.ls_max; ++l) {
    const double om = std::pow(c->prm.ls_omega, double(l - 1));
    hipLaunchKernelGGL(k_waxpy, dim3(grid_for(N)), dim3(256), 0, c->s, trial, c->U, dU, om, N);
    c->residual(Rt, trial);
    hipLaunchKernelGGL(k_mask_leaf, dim3(grid_for(N)), dim3(256), 0, c->s, Rt, c->flags, n);
    rn = c->norm(Rt, N);
    ls = l;
    if (rn < base) { decreased = true; break; }
  }
  HIPCHK(hipMemcpyAsync(U, trial, sizeof(double) * N, hipMemcpyDeviceToDevice, c->s));
  if (active_inout)
    hipLaunchKernelGGL(k_get_active, dim3(grid_for(n)), dim3(256), 0, c->s, active_inout, c->flags, n);
  HIPCHK(hipStreamSynchronize(c->s));
  auto t3 = clk::now();
  inf.residual_after = rn;
  inf.ls_trials = ls;
  inf.setup_seconds = std::chrono::duration<double>(t1 - t0).count();
  inf.solve_seconds = std::chrono::duration<double>(t2 - t1).count();
  inf.linesearch_seconds = std::chrono::duration<double>(t3 - t2).count();
  if (info) *info = inf;
  if (grc) return grc;
  return decreased ? PFF_OK : PFF_W_LINESEARCH;
  GUARD_END(c)
}

int pff_tcv(pff_ctx* c, const double* U, double* tcv, double* dTCVdU, void* stream) {
  if (!c || !U) return PFF_E_ARG;
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  c->ensure_work();
  double* g = dTCVdU ? dTCVdU : c->wv[7];
  c->leaf_op<MODE_TCVGRAD>(g, U, nullptr);
  // TCV is bilinear: int u . grad phi = (dTCV/dphi) . phi over master nodes
  if (tcv) *tcv = c->dot(g + 2 * c->n, U + 2 * c->n, c->n);
  HIPCHK(hipStreamSynchronize(c->s));
  return PFF_OK;
  GUARD_END(c)
}

int pff_param_grad(pff_ctx* c, const double* z, double* out, void* stream) {
  if (!c || !z || !out) return PFF_E_ARG;
  if (!c->has_state) { c->err = "param_grad needs a state"; return PFF_E_STATE; }
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  const int64_t N = 3 * c->n;
  double* v = c->wv[7];
  double* zm = c->wv[6];
  HIPCHK(hipMemcpyAsync(zm, z, sizeof(double) * N, hipMemcpyDeviceToDevice, c->s));
  hipLaunchKernelGGL(k_mask_leaf, dim3(grid_for(N)), dim3(256), 0, c->s, zm, c->flags, c->n);
  const double* st[4] = {c->phit, nullptr, nullptr, nullptr};
  c->leaf_op<MODE_DGC>(v, c->U, st);
  out[0] = c->dot(zm, v, N);
  c->leaf_op<MODE_DE>(v, c->U, st);
  out[1] = c->dot(zm, v, N);
  c->leaf_op<MODE_DP>(v, c->U, st);
  out[2] = c->dot(zm, v, N);
  return PFF_OK;
  GUARD_END(c)
}

int pff_cod(pff_ctx* c, const double* U, const double* x, int32_t nx, double* cod, void* stream) {
  if (!c || !U || nx < 0 || (nx > 0 && (!x || !cod))) return PFF_E_ARG;
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  c->ensure_work();
  const DevTiles& t = c->tiles;
  TileArgs<double> a{};
  c->tile_args(t, c->flags, c->n, a, c->part);
  // lines per launch: at most COD_MAX_LINES and what the partial-sum buffer
  // holds for one partial per tile and line
  const int64_t cap = int64_t(c->part_bytes / sizeof(double)) / std::max(1, t.n_tiles);
  const int chunk = int(std::min<int64_t>(COD_MAX_LINES, cap));
  if (chunk < 1) throw std::runtime_error("cod: partial-sum buffer too small");
  for (int j0 = 0; j0 < nx; j0 += chunk) {
    CodLines L{};
    L.n = std::min(chunk, nx - j0);
    for (int j = 0; j < L.n; ++j) {
      const double xv = x[j0 + j];
      if (!std::isfinite(xv)) {
        c->err = "cod: a line position is not finite";
        return PFF_E_ARG;
      }
      L.X[j] = (xv + 10.0) * double(c->mesh.M) / 20.0;   // physical -> lattice
    }
    double* part = static_cast<double*>(c->part);
    auto launch = [&](auto kfn) {
      if (t.n_tiles > 0) hipLaunchKernelGGL(kfn, dim3(t.n_tiles), dim3(RED_THREADS), 0, c->s, a, c->nodeX, U, L, part);
    };
    const bool q1 = c->p == 1;
    if (L.n <= 8) launch(q1 ? k_cod_partial<1, 8> : k_cod_partial<2, 8>);
    else if (L.n <= 16) launch(q1 ? k_cod_partial<1, 16> : k_cod_partial<2, 16>);
    else if (L.n <= 32) launch(q1 ? k_cod_partial<1, 32> : k_cod_partial<2, 32>);
    else launch(q1 ? k_cod_partial<1, 64> : k_cod_partial<2, 64>);
    HIPCHK(hipGetLastError());
    if (t.n_tiles == 0) {
      for (int j = 0; j < L.n; ++j) cod[j0 + j] = 0.0;
      continue;
    }
    // per-line sums of the per-tile partials, in tile order
    hipLaunchKernelGGL(k_reduce_final, dim3(L.n), dim3(RED_THREADS), 0, c->s, (const double*)part, t.n_tiles, L.n,
                       c->red_out);
    HIPCHK(hipMemcpyAsync(c->host_red, c->red_out, sizeof(double) * L.n, hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    for (int j = 0; j < L.n; ++j) cod[j0 + j] = c->host_red[j];
  }
  return PFF_OK;
  GUARD_END(c)
}

int pff_adjoint_tcv(pff_ctx* c, const double* U, double* tcv, double* grad, double* z, double tol_override,
                    pff_gmres_info* info, void* stream) {
  if (!c || !U || !grad) return PFF_E_ARG;
  if (!c->has_state || !c->mg_ready) { c->err = "adjoint_tcv needs set_state with setup_mg"; return PFF_E_STATE; }
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  const int64_t N = 3 * c->n;
  double* g = c->wv[2];
  double* zz = z ? z : c->wv[3];
  // dTCV/dU (condensed) with constrained rows zeroed: the right-hand side
  // of the transposed system J~^T z = dTCV/dU
  c->leaf_op<MODE_TCVGRAD>(g, U, nullptr);
  const double t = c->dot(g + 2 * c->n, U + 2 * c->n, c->n);
  hipLaunchKernelGGL(k_mask_leaf, dim3(grid_for(N)), dim3(256), 0, c->s, g, c->flags, c->n);
  const double gn = c->norm(g, N);
  if (!std::isfinite(gn) || !std::isfinite(t)) throw nonfinite_error("adjoint_tcv: TCV or its gradient is not finite");
  const double tol = tol_override > 0.0 ? tol_override : std::max(c->prm.gmres_atol, c->prm.gmres_rtol * gn);
  pff_gmres_info gi{};
  const int grc = c->gmres(zz, g, true, tol, &gi, c->prm.vcycle_fp32 != 0);
  // dTCV/dtheta = -z^T dF~/dtheta (the state depends on theta through F~(U, theta) = 0)
  double dF[3];
  const int rc = pff_param_grad(c, zz, dF, stream);
  if (rc) return rc;
  for (int k = 0; k < 3; ++k) grad[k] = -dF[k];
  if (tcv) *tcv = t;
  if (info) *info = gi;
  return grc;
  GUARD_END(c)
}

int pff_extrapolate_phi_load(pff_ctx* c, const double* phi_prev, const double* phi_prev2, double t_prev2,
                             double t_prev, double t_next, double* out, void* stream) {
  if (!c) return PFF_E_ARG;
  const double den = t_prev - t_prev2;
  const double theta = (t_next - t_prev) / den;
  if (!std::isfinite(theta) || den == 0.0 || theta < 0.0) {
    c->err = "extrapolate_phi_load: the load parameters must increase (t_prev2 < t_prev <= t_next)";
    return PFF_E_ARG;
  }
  return pff_extrapolate_phi(c, phi_prev, phi_prev2, theta, out, stream);
}

int pff_distribute(pff_ctx* c, double* v, int32_t ncomp, void* stream) {
  if (!c || !v || ncomp < 1 || ncomp > 3) return PFF_E_ARG;
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  if (c->n_hang)
    hipLaunchKernelGGL((k_distribute<double>), dim3(grid_for(int64_t(ncomp) * c->n_hang)), dim3(256), 0, c->s, v, c->n,
                       ncomp, c->hang, c->n_hang, c->p + 1);
  HIPCHK(hipGetLastError());
  return PFF_OK;
  GUARD_END(c)
}

int pff_mask_constrained(pff_ctx* c, double* v, void* stream) {
  if (!c || !v) return PFF_E_ARG;
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_mask_leaf, dim3(grid_for(3 * c->n)), dim3(256), 0, c->s, v, c->flags, c->n);
  HIPCHK(hipGetLastError());
  return PFF_OK;
  GUARD_END(c)
}

int pff_dot(pff_ctx* c, const double* a, const double* b, int64_t len, double* out, void* stream) {
  if (!c || !a || !b || !out || len < 0) return PFF_E_ARG;
  GUARD_BEGIN
  c->s = static_cast<hipStream_t>(stream);
  *out = c->dot(a, b, len);
  return PFF_OK;
  GUARD_END(c)
}

const char* pff_last_error(const pff_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

}  // extern "C"
