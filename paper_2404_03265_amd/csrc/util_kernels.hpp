// Elementwise, transfer and reduction kernels of the solver. Grid-stride
// loops over nodes; reductions are two-stage with a fixed summation order so
// that results repeat bit for bit for a given size.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "mesh.hpp"

namespace pff {

constexpr int RED_BLOCKS = 2048;
constexpr int RED_THREADS = 256;

__device__ __forceinline__ bool leaf_constrained(uint8_t f, int c) {
  return c < 2 ? (f & (NODE_DIRICHLET | NODE_HANGING)) != 0 : (f & (NODE_ACTIVE | NODE_HANGING)) != 0;
}
__device__ __forceinline__ bool level_fixed(uint8_t f, int c) {
  return c < 2 ? (f & (NODE_DIRICHLET | NODE_EDGE)) != 0 : (f & (NODE_ACTIVE | NODE_EDGE)) != 0;
}

#define GRID_LOOP(i, N) for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < (N); i += int64_t(gridDim.x) * blockDim.x)

// hanging entries from their masters (Sec. 3.2: hanging-node constraints)
template <typename T>
__global__ void k_distribute(T* v, int64_t n, int ncomp, const Hanging* h, int nh, int np1) {
  GRID_LOOP(i, int64_t(nh) * ncomp) {
    const int c = int(i / nh);
    const Hanging& hg = h[i % nh];
    T s = T(0);
    for (int k = 0; k < np1; ++k) s += T(hg.weight[k]) * v[c * n + hg.master[k]];
    v[c * n + hg.node] = s;
  }
}

// identity on hanging rows: out = in
__global__ void k_copy_hanging(double* out, const double* in, int64_t n, const Hanging* h, int nh) {
  GRID_LOOP(i, int64_t(nh) * 3) {
    const int c = int(i / nh);
    const int64_t g = h[i % nh].node;
    out[c * n + g] = in[c * n + g];
  }
}

// active flags from a caller's byte array (hanging unknowns never active)
__global__ void k_set_active(uint8_t* flags, const uint8_t* active, int64_t n) {
  GRID_LOOP(i, n) {
    uint8_t f = flags[i] & uint8_t(~NODE_ACTIVE);
    if (active[i] && !(f & NODE_HANGING)) f |= NODE_ACTIVE;
    flags[i] = f;
  }
}

// Active-set rule of Sec. 2 / Alg. 2, lambda = R_phi / B: active <=>
// lambda + c (phi - phi_old) exceeds tau, tau = 1e-12 max |lambda| (*tau_ptr):
// exact ties that quadrature turns into rounding noise count as zero, i.e.
// inactive. c_fixed = 0 selects the per-unknown constant
// c_i = 2 |lambda_i / (phi_i - phi_old_i)| (c_i * 0 := 0); c_fixed > 0 is
// used for every unknown.
__global__ void k_active_rule(uint8_t* flags, const double* R, const double* mass, const double* phi,
                              const double* phio, int64_t n, const double* tau_ptr, double c_fixed) {
  const double tau = *tau_ptr;
  GRID_LOOP(i, n) {
    uint8_t f = flags[i] & uint8_t(~NODE_ACTIVE);
    if (!(f & NODE_HANGING)) {
      const double lam = R[2 * n + i] / mass[i];
      const double diff = phi[i] - phio[i];
      const double c = c_fixed > 0.0 ? c_fixed : (diff != 0.0 ? 2.0 * fabs(lam / diff) : 0.0);
      const double val = lam + c * diff;
      if (val > tau) f |= NODE_ACTIVE;
    }
    flags[i] = f;
  }
}

// Linearisation phase field extrapolated from two earlier load steps (Sec. 2):
// out = phi_prev + theta (phi_prev - phi_prev2), clipped to [0, 1]. Products
// and sums are rounded separately (no fused multiply-add), so the result is
// the correctly rounded value of each step.
__global__ void k_extrapolate_phi(double* out, const double* a, const double* b, double theta, int64_t n) {
#pragma clang fp contract(off)
  GRID_LOOP(i, n) {
    const double ai = a[i];
    const double step = theta * (ai - b[i]);
    out[i] = fmin(1.0, fmax(0.0, ai + step));
  }
}

// per-block maxima of |R_phi / B| over non-hanging nodes
__global__ void __launch_bounds__(RED_THREADS) k_lambda_max_partial(const double* R, const double* mass,
                                                                      const uint8_t* flags, int64_t n,
                                                                      double* part) {
  __shared__ double sh[RED_THREADS];
  double m = 0.0;
  GRID_LOOP(i, n) {
    if (!(flags[i] & NODE_HANGING)) m = fmax(m, fabs(R[2 * n + i] / mass[i]));
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out[0] = scale * max of part[0..nb)
__global__ void __launch_bounds__(RED_THREADS) k_reduce_max_final(const double* part, int nb, double scale,
                                                                    double* out) {
  __shared__ double sh[RED_THREADS];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, part[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = scale * sh[0];
}

__global__ void k_get_active(uint8_t* out, const uint8_t* flags, int64_t n) {
  GRID_LOOP(i, n) out[i] = (flags[i] & NODE_ACTIVE) ? 1 : 0;
}

// per-block partial counts of active entries and of entries that differ
// from `prev` (part[2 * blk], part[2 * blk + 1]); reduced by k_reduce_final
__global__ void __launch_bounds__(RED_THREADS) k_count_partial(const uint8_t* flags, const uint8_t* prev,
                                                                 int64_t n, double* part) {
  __shared__ double sa[RED_THREADS], sc[RED_THREADS];
  double a = 0.0, c = 0.0;
  GRID_LOOP(i, n) {
    const bool act = (flags[i] & NODE_ACTIVE) != 0;
    a += act ? 1.0 : 0.0;
    if (prev) c += (act != (prev[i] != 0)) ? 1.0 : 0.0;
  }
  sa[threadIdx.x] = a;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sc[threadIdx.x] += sc[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sa[0];
    part[2 * blockIdx.x + 1] = sc[0];
  }
}

// U_c: phase field set to phi_old on the active set
__global__ void k_apply_active(double* U, const double* phio, const uint8_t* flags, int64_t n) {
  GRID_LOOP(i, n) if (flags[i] & NODE_ACTIVE) U[2 * n + i] = phio[i];
}

// zero constrained rows of a leaf vector
__global__ void k_mask_leaf(double* v, const uint8_t* flags, int64_t n) {
  GRID_LOOP(k, n) {
    const uint8_t f = flags[k];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (leaf_constrained(f, c)) v[c * n + k] = 0.0;
  }
}

// level state injection: (u_x, u_y, phit) at the coinciding leaf position
template <typename T>
__global__ void k_inject(T* st, int64_t nl, const int32_t* leaf_index, const double* U, const double* phit,
                         int64_t n) {
  GRID_LOOP(i, nl) {
    const int64_t g = leaf_index[i];
    st[i] = T(U[g]);
    st[nl + i] = T(U[n + g]);
    st[2 * nl + i] = T(phit[g]);
  }
}

// Level active set (Sec. 3.2: inactive only if every fine unknown it
// interacts with is inactive): active if the leaf unknown at the same
// position is active or any finer unknown in the prolongation stencil is.
// home_rule (local smoothing): on the home level of a leaf unknown
// (NODE_COPY) only its own flag counts, so that no free leaf unknown is
// frozen on every level that holds it; global coarsening smooths every free
// leaf unknown on its finest level and passes home_rule = 0.
__global__ void k_level_active(uint8_t* fl, int64_t nl, const int32_t* leaf_index, const uint8_t* leaf_flags,
                               const int64_t* PT_ptr, const int32_t* PT_col, const uint8_t* fine_flags,
                               int home_rule) {
  GRID_LOOP(i, nl) {
    uint8_t f = fl[i] & uint8_t(~NODE_ACTIVE);
    const bool own = (leaf_flags[leaf_index[i]] & NODE_ACTIVE) != 0;
    bool act = own;
    if (!(home_rule && (f & NODE_COPY)) && PT_ptr && !act)
      for (int64_t e = PT_ptr[i]; e < PT_ptr[i + 1]; ++e)
        if (fine_flags[PT_col[e]] & NODE_ACTIVE) { act = true; break; }
    if (act && !(f & NODE_HANGING)) f |= NODE_ACTIVE;   // hanging unknowns are never active
    fl[i] = f;
  }
}

// The leaf <-> level copies of every level in one launch: the threads walk
// the concatenated level node ranges, start[l] .. start[l + 1] being level l.
// Every free non-hanging leaf unknown belongs to the one level whose leaf
// cells own it (the level nodes flagged NODE_COPY).
constexpr int COPY_MAX_LEVELS = 16;

template <typename T>
struct LevelCopyArgs {
  int nlev;
  int64_t start[COPY_MAX_LEVELS + 1];
  // first 256-thread block of each level: a block holds nodes of one level,
  // so the level and its pointers are uniform (scalar) in the kernels
  int bstart[COPY_MAX_LEVELS + 1];
  T* vec[COPY_MAX_LEVELS];                  // level vector (3 x n_l) written or read
  const uint8_t* fl[COPY_MAX_LEVELS];       // level node flags
  const int32_t* leaf_index[COPY_MAX_LEVELS];
};

// the block's level and its node k (launched with 256-thread blocks, one
// grid of bstart[nlev] blocks); false past the level's last node
template <typename T>
__device__ __forceinline__ bool copy_node_of(const LevelCopyArgs<T>& a, int& l, int64_t& k, int64_t& nl) {
  const int bid = int(blockIdx.x);
  l = 0;
#pragma unroll
  for (int j = 1; j < COPY_MAX_LEVELS; ++j)
    if (j < a.nlev && bid >= a.bstart[j]) l = j;
  nl = a.start[l + 1] - a.start[l];
  k = int64_t(bid - a.bstart[l]) * 256 + threadIdx.x;
  return k < nl;
}

// level vectors = the leaf values of their copy targets (zero elsewhere and on
// constrained leaf rows). The node's flag and leaf index go out together, then
// the leaf flag and values (branch-free: other nodes read leaf node 0).
template <typename T>
__global__ void __launch_bounds__(256) k_copy_to_levels(const LevelCopyArgs<T> a, const double* b,
                                                        const uint8_t* leaf_flags, int64_t n) {
  int l;
  int64_t k, nl;
  if (!copy_node_of(a, l, k, nl)) return;
  const uint8_t* flp = a.fl[l];
  const int32_t* lip = a.leaf_index[l];
  T* vp = a.vec[l];
  // the level's three pointers in one scalar round trip
  asm volatile("" ::"s"(flp), "s"(lip), "s"(vp));
  const uint8_t fl = flp[k];
  const int32_t gi = lip[k];
  const bool copy = fl & NODE_COPY;
  const int64_t g = copy ? int64_t(gi) : 0;
  const uint8_t lf = leaf_flags[g];
  double bv[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) bv[c] = b[c * n + g];
  // the four loads together (the compiler would otherwise branch on the
  // flag first and load the values behind it)
  asm volatile("" ::"v"(int(lf)), "v"(bv[0]), "v"(bv[1]), "v"(bv[2]));
#pragma unroll
  for (int c = 0; c < 3; ++c) vp[c * nl + k] = (copy && !leaf_constrained(lf, c)) ? T(bv[c]) : T(0);
}

// leaf rows = the value of their copy level (the input on constrained rows);
// every leaf node is the copy target of one level at most
template <typename T>
__global__ void __launch_bounds__(256) k_copy_from_levels(double* out, const LevelCopyArgs<T> a, const double* b,
                                                          const uint8_t* leaf_flags, int64_t n) {
  int l;
  int64_t k, nl;
  if (!copy_node_of(a, l, k, nl)) return;
  const uint8_t* flp = a.fl[l];
  const int32_t* lip = a.leaf_index[l];
  const T* vp = a.vec[l];
  // the level's three pointers in one scalar round trip
  asm volatile("" ::"s"(flp), "s"(lip), "s"(vp));
  const uint8_t fl = flp[k];
  const int32_t gi = lip[k];
  T xv[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) xv[c] = vp[c * nl + k];
  // the flag, leaf index and level values together (the compiler would
  // otherwise branch on the flag first and load the rest behind it)
  asm volatile("" ::"v"(int(fl)), "v"(gi), "v"(xv[0]), "v"(xv[1]), "v"(xv[2]));
  const bool copy = fl & NODE_COPY;
  const int64_t g = copy ? int64_t(gi) : 0;
  const uint8_t lf = leaf_flags[g];
  double bv[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) bv[c] = b[c * n + g];
  asm volatile("" ::"v"(int(lf)), "v"(bv[0]), "v"(bv[1]), "v"(bv[2]));
  if (copy) {
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * n + g] = leaf_constrained(lf, c) ? bv[c] : double(xv[c]);
  }
}

// Global coarsening: the finest level is the leaf mesh itself. Its right-hand
// side is the leaf vector with constrained rows set to zero; the output takes
// the level solution on free rows and the input on constrained ones.
template <typename T>
__global__ void k_leaf_to_level(T* d, const double* b, const uint8_t* leaf_flags, int64_t n) {
  GRID_LOOP(k, n) {
    const uint8_t f = leaf_flags[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c * n + k] = leaf_constrained(f, c) ? T(0) : T(b[c * n + k]);
  }
}
template <typename T>
__global__ void k_level_to_leaf(double* out, const T* x, const double* b, const uint8_t* leaf_flags, int64_t n) {
  GRID_LOOP(k, n) {
    const uint8_t f = leaf_flags[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * n + k] = leaf_constrained(f, c) ? b[c * n + k] : double(x[c * n + k]);
  }
}

// Grid transfers in a column-major ELL layout: entry e of row r at
// E[e * rows + r], so the entries of one step are read with unit stride
// across the lanes. An entry packs the column (low TRANSFER_COL_BITS bits) and
// the index of its weight in the level's table of distinct weights (high
// bits); the weights are exact dyadic values, the table holds them as float
// for both precisions, and index 0 is the weight 0 of padding entries.
constexpr int TRANSFER_COL_BITS = 27;   // levels up to 134 M nodes, 32 distinct weights
constexpr int TRANSFER_WEIGHTS = 1 << (32 - TRANSFER_COL_BITS);
constexpr uint32_t TRANSFER_COL_MASK = (1u << TRANSFER_COL_BITS) - 1u;

__device__ __forceinline__ void load_weight_table(float* W, const float* wtab) {
  for (int i = threadIdx.x; i < TRANSFER_WEIGHTS; i += blockDim.x) W[i] = wtab[i];
  __syncthreads();
}

// s_c += sum over the entries e of ELL row r (column-major, runtime width)
// of weight_e * x[c * nx + col_e] (c = 0, 1, 2)
template <typename T>
__device__ __forceinline__ void ell_row3(const uint32_t* E, int64_t stride, int64_t r, int width, const float* W,
                                         const T* x, int64_t nx, T& s0, T& s1, T& s2) {
  for (int e = 0; e < width; ++e) {
    const uint32_t t = E[int64_t(e) * stride + r];
    const int64_t col = t & TRANSFER_COL_MASK;
    const T w = T(W[t >> TRANSFER_COL_BITS]);
    s0 += w * x[col];
    s1 += w * x[nx + col];
    s2 += w * x[2 * nx + col];
  }
}

// the weights and gathers of WIDTH entries t of one ELL row held in registers
template <typename T, int WIDTH>
__device__ __forceinline__ void ell_gather3(const uint32_t (&t)[WIDTH], const float* W, const T* x, int64_t nx,
                                            T& s0, T& s1, T& s2) {
#pragma unroll
  for (int e = 0; e < WIDTH; ++e) {
    const int64_t col = t[e] & TRANSFER_COL_MASK;
    const T w = T(W[t[e] >> TRANSFER_COL_BITS]);
    s0 += w * x[col];
    s1 += w * x[nx + col];
    s2 += w * x[2 * nx + col];
  }
}

// With a compile-time row width each thread requests its (first) row's
// entries before the block loads the weight table and passes its barrier,
// so the two latencies overlap, and the next row's entries (when the grid
// does not cover the rows) before the current row's gathers are summed.
// Launched with 256-thread blocks. (The grouped form of the restriction
// below was slower here: one lane per fine row already gathers neighbouring
// coarse nodes, two fine rows sharing each.)

// x_f += P x_c on unknowns the fine level does not hold at zero
// (Dirichlet for u, active for phi)
template <typename T, int WIDTH>
__global__ void __launch_bounds__(256) k_prolong_add(T* xf, const T* xc, int64_t nf, int64_t nc, int width,
                                                     const uint32_t* E, const float* wtab, const uint8_t* ff) {
  __shared__ float W[TRANSFER_WEIGHTS];
  if constexpr (WIDTH > 0) {
    const int64_t st = int64_t(gridDim.x) * 256;
    int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    // a row's entries, flag and the values it adds to, requested together
    uint32_t t[WIDTH];
    uint8_t f = 0;
    T x0 = T(0), x1 = T(0), x2 = T(0);
    auto fetch = [&](int64_t row) {
#pragma unroll
      for (int e = 0; e < WIDTH; ++e) t[e] = E[int64_t(e) * nf + row];
      f = ff[row];
      x0 = xf[row];
      x1 = xf[nf + row];
      x2 = xf[2 * nf + row];
    };
    if (i < nf) fetch(i);
    load_weight_table(W, wtab);
    for (; i < nf; i += st) {
      T s0 = T(0), s1 = T(0), s2 = T(0);
      ell_gather3<T, WIDTH>(t, W, xc, nc, s0, s1, s2);
      const uint8_t fi = f;
      const T y0 = x0 + s0, y1 = x1 + s1, y2 = x2 + s2;
      if (i + st < nf) fetch(i + st);
      if (!(fi & NODE_DIRICHLET)) {
        xf[i] = y0;
        xf[nf + i] = y1;
      }
      if (!(fi & NODE_ACTIVE)) xf[2 * nf + i] = y2;
    }
  } else {
    load_weight_table(W, wtab);
    GRID_LOOP(i, nf) {
      T s0 = T(0), s1 = T(0), s2 = T(0);
      ell_row3<T>(E, nf, i, width, W, xc, nc, s0, s1, s2);
      const uint8_t f = ff[i];
      if (!(f & NODE_DIRICHLET)) {
        xf[i] += s0;
        xf[nf + i] += s1;
      }
      if (!(f & NODE_ACTIVE)) xf[2 * nf + i] += s2;
    }
  }
}

// Grouped restriction, for P^T of width G^2 (9 for Q1, 25 for Q2) whose rows
// are on average at least half full (local smoothing; not the identity rows
// of global coarsening away from the refined cells):
// the entries of one row are spread over G lanes, lane g of the row's group
// taking the entries j G + g (j < G), stored at E[(j * rows + row) * G + g].
// The row's entries are sorted by fine node and a coarse node's support
// holds G neighbouring fine nodes per grid line, so one load instruction
// gathers, for 64 / G consecutive rows, runs of neighbouring fine nodes
// instead of one fine node per row and lane spread over many cache lines.
// The group's first lane adds the G partial sums in lane order and updates
// the row. Each lane requests its first row's entries (with the row's
// receiving node) before the block loads the weight table and passes its
// barrier, and the next row's before the current row's sums (when the grid
// does not cover the rows).
// Launched with 256-thread blocks, 64 / G rows per wave; the lanes past the
// last group, and those past the last row, read row 0 and store nothing.

// sum over the lanes of a group (lane order), valid in the group's first lane
template <typename T, int G>
__device__ __forceinline__ T group_sum(T s, int lane) {
  T a = s;
#pragma unroll
  for (int k = 1; k < G; ++k) a += __shfl(s, lane + k < 64 ? lane + k : lane, 64);
  return a;
}

// d_c += P^T t_f over the coarse rows that receive fine contributions, one
// lane per row (WIDTH > 0: compile-time row width, as the prolongation)
template <typename T, int WIDTH>
__global__ void __launch_bounds__(256) k_restrict_add(T* dc, const T* tf, int64_t nc, int64_t nf, int64_t nrows,
                                                      const int32_t* rows, int width, const uint32_t* E,
                                                      const float* wtab) {
  __shared__ float W[TRANSFER_WEIGHTS];
  if constexpr (WIDTH > 0) {
    const int64_t st = int64_t(gridDim.x) * 256;
    int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
    // a row's entries and its receiving node, requested together
    uint32_t t[WIDTH];
    int64_t i = 0;
    auto fetch = [&](int64_t row) {
#pragma unroll
      for (int e = 0; e < WIDTH; ++e) t[e] = E[int64_t(e) * nrows + row];
      i = rows[row];
    };
    if (r < nrows) fetch(r);
    load_weight_table(W, wtab);
    for (; r < nrows; r += st) {
      // the values added to go out with the gathers
      const int64_t ir = i;
      const T d0 = dc[ir], d1 = dc[nc + ir], d2 = dc[2 * nc + ir];
      T s0 = T(0), s1 = T(0), s2 = T(0);
      ell_gather3<T, WIDTH>(t, W, tf, nf, s0, s1, s2);
      if (r + st < nrows) fetch(r + st);
      dc[ir] = d0 + s0;
      dc[nc + ir] = d1 + s1;
      dc[2 * nc + ir] = d2 + s2;
    }
  } else {
    load_weight_table(W, wtab);
    GRID_LOOP(r, nrows) {
      T s0 = T(0), s1 = T(0), s2 = T(0);
      ell_row3<T>(E, nrows, r, width, W, tf, nf, s0, s1, s2);
      const int64_t i = rows[r];
      dc[i] += s0;
      dc[nc + i] += s1;
      dc[2 * nc + i] += s2;
    }
  }
}

// d_c += P^T t_f over the coarse rows that receive fine contributions
template <typename T, int G>
__global__ void __launch_bounds__(256) k_restrict_add_grouped(T* dc, const T* tf, int64_t nc, int64_t nf,
                                                              int64_t nrows, const int32_t* rows, const uint32_t* E,
                                                              const float* wtab) {
  constexpr int RPW = 64 / G;   // rows per wave
  __shared__ float W[TRANSFER_WEIGHTS];
  const int lane = int(threadIdx.x) & 63, g = lane % G, rl = lane / G;
  const int64_t wst = int64_t(gridDim.x) * 4;
  int64_t w = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  uint32_t t[G];
  int64_t i = 0;
  // a row's entries of this lane and its receiving node, requested together
  auto fetch = [&](int64_t wv) {
    const int64_t r = wv * RPW + rl;
    const int64_t row = (rl < RPW && r < nrows) ? r : int64_t(0);
#pragma unroll
    for (int j = 0; j < G; ++j) t[j] = E[(int64_t(j) * nrows + row) * G + g];
    i = rows[row];
  };
  if (w * RPW < nrows) fetch(w);
  load_weight_table(W, wtab);
  for (; w * RPW < nrows; w += wst) {   // uniform per wave
    const int64_t r = w * RPW + rl;
    const bool store = rl < RPW && r < nrows && g == 0;
    const int64_t ir = i;
    const T d0 = dc[ir], d1 = dc[nc + ir], d2 = dc[2 * nc + ir];
    T s0 = T(0), s1 = T(0), s2 = T(0);
    ell_gather3<T, G>(t, W, tf, nf, s0, s1, s2);
    if ((w + wst) * RPW < nrows) fetch(w + wst);
    const T a0 = group_sum<T, G>(s0, lane), a1 = group_sum<T, G>(s1, lane), a2 = group_sum<T, G>(s2, lane);
    if (store) {
      dc[ir] = d0 + a0;
      dc[nc + ir] = d1 + a1;
      dc[2 * nc + ir] = d2 + a2;
    }
  }
}

// first Chebyshev update from x0 = 0: d = dinv b / theta, x = d
template <typename T>
__global__ void k_cheb_first(T* x, T* d, const T* b, const T* dinv, int64_t nl, T c2u, T c2p) {
  GRID_LOOP(i, 3 * nl) {
    const T c2 = (i < 2 * nl) ? c2u : c2p;
    const T v = c2 * dinv[i] * b[i];
    d[i] = v;
    x[i] = v;
  }
}

template <typename T>
__global__ void k_fill(T* v, T val, int64_t len) {
  GRID_LOOP(i, len) v[i] = val;
}

template <typename TO, typename TI>
__global__ void k_cast(TO* o, const TI* in, int64_t len) {
  GRID_LOOP(i, len) o[i] = TO(in[i]);
}

// Block-triangular preconditioner: out = the rows of one block of in (u
// rows for phi_block = 0, phi rows for 1), zero elsewhere; and t = b - t on
// the rows of one block, zero elsewhere
__global__ void k_block_select(double* out, const double* in, int64_t n, int phi_block) {
  GRID_LOOP(i, 3 * n) out[i] = ((i >= 2 * n) == (phi_block != 0)) ? in[i] : 0.0;
}
__global__ void k_block_rhs(double* t, const double* b, int64_t n, int phi_block) {
  GRID_LOOP(i, 3 * n) t[i] = ((i >= 2 * n) == (phi_block != 0)) ? b[i] - t[i] : 0.0;
}

// partials of the number of entries where a and b differ (bit for bit)
__global__ void __launch_bounds__(RED_THREADS) k_neq_partial(const double* a, const double* b, int64_t len,
                                                              double* part) {
  __shared__ double sh[RED_THREADS];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < len; i += int64_t(gridDim.x) * blockDim.x)
    s += (__double_as_longlong(a[i]) != __double_as_longlong(b[i])) ? 1.0 : 0.0;
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// y = a x + y
__global__ void k_axpy(double* y, const double* x, double a, int64_t len) {
  GRID_LOOP(i, len) y[i] += a * x[i];
}
// y = x + a z
__global__ void k_waxpy(double* y, const double* x, const double* z, double a, int64_t len) {
  GRID_LOOP(i, len) y[i] = x[i] + a * z[i];
}
__global__ void k_scale(double* y, const double* x, double a, int64_t len) {
  GRID_LOOP(i, len) y[i] = a * x[i];
}
__global__ void k_sub(double* y, const double* a, const double* b, int64_t len) {
  GRID_LOOP(i, len) y[i] = a[i] - b[i];
}
// w -= sum_j h_j V_j (V: k vectors of length len, contiguous)
__global__ void k_mcombine(double* w, const double* V, const double* h, int k, int64_t len, double sign) {
  GRID_LOOP(i, len) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += h[j] * V[int64_t(j) * len + i];
    w[i] += sign * s;
  }
}

// CG helpers for the eigenvalue estimate: r = 1 on free unknowns
// (inverse diagonal nonzero exactly there); z = a * b; r -= alpha q on free
// unknowns and z = dinv r
__global__ void k_free_ones(double* r, const double* dinv, int64_t len) {
  GRID_LOOP(i, len) r[i] = dinv[i] != 0.0 ? 1.0 : 0.0;
}
__global__ void k_mul(double* z, const double* a, const double* b, int64_t len) {
  GRID_LOOP(i, len) z[i] = a[i] * b[i];
}
__global__ void k_cg_update(double* r, double* z, const double* q, const double* dinv, double alpha, int64_t len) {
  GRID_LOOP(i, len) {
    if (dinv[i] != 0.0) r[i] -= alpha * q[i];
    z[i] = dinv[i] * r[i];
  }
}

// ---- eigenvalue-estimate CG with its scalars on the device ----------------
// Both blocks of a level (u rows, phi rows) run their CG at once; sc holds
// EIG_SC doubles per block: rz, pq, rz2, alpha, beta, rz0, active, steps,
// max_steps. The step kernels reproduce the host recurrence: alpha = rz / pq
// (stop if pq <= 0), beta = rz2 / rz, stop once rz2 <= 1e-24 rz0 or after
// max_steps; al / be collect the coefficients of the Lanczos tridiagonal.
constexpr int EIG_SC = 9;
constexpr int EIG_MAX_ITS = 200;   // largest accepted eig_cg_its / coarse_eig_its
enum { EIG_RZ = 0, EIG_PQ, EIG_RZ2, EIG_ALPHA, EIG_BETA, EIG_RZ0, EIG_ACTIVE, EIG_STEPS, EIG_MAX };

// start of the estimate from the two dots of the start vector (r.r = the
// number of free unknowns in the EIG_PQ slot, r.z in EIG_RZ): at most its_u
// (displacement block) or its_phi (phase-field block) steps and never more
// than the free unknowns; a block without free unknowns
// or with r.z = 0 takes no step
// skip_u: the displacement block takes no step (its estimate is kept)
__global__ void k_eig_init(double* sc, int its_u, int its_phi, int skip_u) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int b = 0; b < 2; ++b) {
    double* c = sc + EIG_SC * b;
    if (b == 0 && skip_u) {
      c[EIG_ACTIVE] = 0.0;
      c[EIG_STEPS] = 0.0;
      continue;
    }
    const double n_free = c[EIG_PQ];
    c[EIG_RZ0] = c[EIG_RZ];
    c[EIG_MAX] = fmin(double(b == 0 ? its_u : its_phi), n_free);
    c[EIG_ACTIVE] = (c[EIG_MAX] >= 1.0 && c[EIG_RZ] > 0.0) ? 1.0 : 0.0;
    c[EIG_STEPS] = 0.0;
  }
}

// stage 1 of a dot product: one partial per block, fixed order
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_dot_partial(const T* a, const T* b, int64_t len, double* part) {
  __shared__ double sh[RED_THREADS];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < len; i += int64_t(gridDim.x) * blockDim.x)
    s += double(a[i]) * double(b[i]);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Orthogonalisation kernels for GMRES (classical Gram-Schmidt, twice).
// V holds k vectors of length len back to back, k <= K (a compile-time
// bound, so the k running sums stay in registers). Each kernel streams w and
// the V[j] once and leaves one partial sum per block and product in
// part[block * k + j], reduced in fixed order by k_reduce_final.
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int K>
__device__ __forceinline__ void block_partials(const double (&s)[K], int k, double* part) {
  __shared__ double sh[RED_THREADS / 64][K];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (j < k) {
      const double t = wave_sum(s[j]);
      if (lane == 0) sh[wave][j] = t;
    }
  __syncthreads();
  if (threadIdx.x < k) {
    double t = 0.0;
    for (int q = 0; q < RED_THREADS / 64; ++q) t += sh[q][threadIdx.x];
    part[int64_t(blockIdx.x) * k + threadIdx.x] = t;
  }
}

// partials of V[j] . w
template <int K>
__global__ void __launch_bounds__(RED_THREADS) k_mdot_partial(const double* V, const double* w, int k,
                                                                int64_t len, double* part) {
  double s[K];
#pragma unroll
  for (int j = 0; j < K; ++j) s[j] = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < len; i += int64_t(gridDim.x) * blockDim.x) {
    const double wi = w[i];
    // all k values of element i requested before the first product
    double v[K];
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = j < k ? V[int64_t(j) * len + i] : 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) s[j] += v[j] * wi;
  }
  block_partials<K>(s, k, part);
}

// w -= sum_j h[j] V[j], then the partial of w . w
__global__ void __launch_bounds__(RED_THREADS) k_mcombine_sq_partial(const double* V, double* w, const double* h,
                                                                       int k, int64_t len, double* part) {
  double s[1] = {0.0};
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < len; i += int64_t(gridDim.x) * blockDim.x) {
    double wi = w[i];
    for (int j = 0; j < k; ++j) wi -= h[j] * V[int64_t(j) * len + i];
    w[i] = wi;
    s[0] += wi * wi;
  }
  block_partials<1>(s, 1, part);
}

// Second sweep of the delayed classical Gram-Schmidt step of GMRES: column j
// of V holds q_j (one projection done, second one pending with coefficients
// c), w = M^-1 A q_j. Per element:
//   v_j     = (q_j - sum_l c_l v_l) / rho_j            (written over q_j)
//   q_(j+1) = w / rho_j - sum_l d_l v_l - gamma v_j    (written to column j + 1)
// (l < j) and the partials of v_l . q_(j+1) (l <= j) and |q_(j+1)|^2, j + 2
// sums in all.
constexpr int DCGS_MAX = 64;
struct DcgsCoef {
  double c[DCGS_MAX];
  double d[DCGS_MAX];
  double inv_rho, gamma;
  int j;
};

template <int K>
__global__ void __launch_bounds__(RED_THREADS) k_dcgs2_partial(double* V, const double* w, const DcgsCoef cf,
                                                                 int64_t len, double* part) {
  const int j = cf.j;
  double s[K];
#pragma unroll
  for (int l = 0; l < K; ++l) s[l] = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < len; i += int64_t(gridDim.x) * blockDim.x) {
    const double q = V[int64_t(j) * len + i];
    const double wi = w[i];
    double vj, qn;
    if constexpr (K <= 32) {
      // the basis values of element i stay in registers for the products
      double v[K];
      double sc = 0.0, sd = 0.0;
#pragma unroll
      for (int l = 0; l < K; ++l) {
        v[l] = l < j ? V[int64_t(l) * len + i] : 0.0;
        sc += cf.c[l < j ? l : 0] * v[l];
        sd += cf.d[l < j ? l : 0] * v[l];
      }
      vj = (q - sc) * cf.inv_rho;
      qn = wi * cf.inv_rho - sd - cf.gamma * vj;
#pragma unroll
      for (int l = 0; l < K; ++l) s[l] += v[l] * qn;
    } else {
      double sc = 0.0, sd = 0.0;
      for (int l = 0; l < j; ++l) {
        const double vl = V[int64_t(l) * len + i];
        sc += cf.c[l] * vl;
        sd += cf.d[l] * vl;
      }
      vj = (q - sc) * cf.inv_rho;
      qn = wi * cf.inv_rho - sd - cf.gamma * vj;
#pragma unroll
      for (int l = 0; l < K; ++l)
        if (l < j) s[l] += V[int64_t(l) * len + i] * qn;
    }
    V[int64_t(j) * len + i] = vj;
    V[int64_t(j + 1) * len + i] = qn;
    // slots j and j + 1 (the padded register slots l >= j summed zero products)
#pragma unroll
    for (int l = 0; l < K; ++l) {
      if (l == j) s[l] += vj * qn;
      if (l == j + 1) s[l] += qn * qn;
    }
  }
  block_partials<K>(s, j + 2, part);
}

// stage 2: out[j] = sum over nb blocks of part[blk * k + j]
// (one block per column when launched with k blocks)
__global__ void __launch_bounds__(RED_THREADS) k_reduce_final(const double* part, int nb, int k, double* out) {
  __shared__ double sh[RED_THREADS / 64];
  for (int j = blockIdx.x; j < k; j += gridDim.x) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[int64_t(i) * k + j];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int q = 0; q < RED_THREADS / 64; ++q) t += sh[q];
      out[j] = t;
    }
    __syncthreads();
  }
}

// ---- eigenvalue-estimate CG, both blocks of a level per launch ------------
// Block 0 is rows [0, 2 nl) (u), block 1 rows [2 nl, 3 nl) (phi); sc holds the
// per-block scalars (EIG_*). Partial sums per workgroup and block go to
// part[2 * workgroup + block] and are reduced in fixed order.
__device__ __forceinline__ void eig_block_partials(double s0, double s1, double* part) {
  __shared__ double sh[2][RED_THREADS / 64];
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    sh[0][wave] = s0;
    sh[1][wave] = s1;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int w = 0; w < RED_THREADS / 64; ++w) t += sh[threadIdx.x][w];
    part[2 * blockIdx.x + threadIdx.x] = t;
  }
}
// sums of the two columns of part over nb workgroups (one thread each, fixed order)
__device__ __forceinline__ void eig_reduce2(const double* part, int nb, double* out2) {
  __shared__ double sh[2][RED_THREADS / 64];
  double s0 = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    s0 += part[2 * i];
    s1 += part[2 * i + 1];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    sh[0][wave] = s0;
    sh[1][wave] = s1;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int w = 0; w < RED_THREADS / 64; ++w) t += sh[threadIdx.x][w];
    out2[threadIdx.x] = t;
  }
  __syncthreads();
}

// partials of p.q per block
// Each block's rows run in a loop of their own with the thread index counted
// from the block's first row (begin = 2 nl: the displacement block is
// skipped), so the phase-field partial sums are the same with and without
// the other block.
template <class F>
__device__ __forceinline__ void eig_block_loops(int64_t nl, int64_t begin, F&& body) {
  // (launched with RED_THREADS-thread blocks: a compile-time block size
  // spares each workgroup a load of the dispatch packet)
  const int64_t st = int64_t(gridDim.x) * RED_THREADS;
  const int64_t t0 = int64_t(blockIdx.x) * RED_THREADS + threadIdx.x;
  if (begin == 0)
    for (int64_t i = t0; i < 2 * nl; i += st) body(0, i);
  for (int64_t i = 2 * nl + t0; i < 3 * nl; i += st) body(1, i);
}
__global__ void __launch_bounds__(RED_THREADS) k_eig_pq_partial(const double* p, const double* q, int64_t nl,
                                                                  int64_t begin, double* part) {
  double s[2] = {0.0, 0.0};
  eig_block_loops(nl, begin, [&](int b, int64_t i) { s[b] += p[i] * q[i]; });
  eig_block_partials(s[0], s[1], part);
}
// p.q per block, then alpha = r.z / p.q (a block with p.q <= 0 stops)
__global__ void __launch_bounds__(RED_THREADS) k_eig_alpha_reduce(const double* part, int nb, double* sc, double* al,
                                                                    int stride, int it) {
  __shared__ double pq[2];
  eig_reduce2(part, nb, pq);
  const int b = threadIdx.x;
  if (b >= 2) return;
  double* c = sc + EIG_SC * b;
  if (c[EIG_ACTIVE] == 0.0) return;
  if (!(pq[b] > 0.0)) {
    c[EIG_ACTIVE] = 0.0;
    return;
  }
  const double alpha = c[EIG_RZ] / pq[b];
  c[EIG_ALPHA] = alpha;
  al[b * stride + it] = alpha;
}
// r -= alpha q on free rows, z = D^-1 r (active blocks), partials of r.z
__global__ void __launch_bounds__(RED_THREADS) k_eig_update_partial(double* r, double* z, const double* q,
                                                                      const double* dinv, const double* sc,
                                                                      int64_t nl, int64_t begin, double* part) {
  const bool act[2] = {sc[EIG_ACTIVE] != 0.0, sc[EIG_SC + EIG_ACTIVE] != 0.0};
  const double alpha[2] = {sc[EIG_ALPHA], sc[EIG_SC + EIG_ALPHA]};
  double s[2] = {0.0, 0.0};
  eig_block_loops(nl, begin, [&](int b, int64_t i) {
    // all four loads at once (under the branches they waited in turn)
    double ri = r[i], zi = z[i];
    const double di = dinv[i], qi = q[i];
    if (act[b]) {
      ri = di != 0.0 ? ri - alpha[b] * qi : ri;
      zi = di * ri;
      r[i] = ri;
      z[i] = zi;
    }
    s[b] += ri * zi;
  });
  eig_block_partials(s[0], s[1], part);
}
// r.z per block, beta = r.z_new / r.z; stop once r.z <= 1e-24 r.z_0 or after
// the block's step count
__global__ void __launch_bounds__(RED_THREADS) k_eig_beta_reduce(const double* part, int nb, double* sc, double* be,
                                                                   int stride, int it) {
  __shared__ double rz2[2];
  eig_reduce2(part, nb, rz2);
  const int b = threadIdx.x;
  if (b >= 2) return;
  double* c = sc + EIG_SC * b;
  if (c[EIG_ACTIVE] == 0.0) return;
  const double beta = rz2[b] / c[EIG_RZ];
  c[EIG_BETA] = beta;
  be[b * stride + it] = beta;
  c[EIG_RZ] = rz2[b];
  c[EIG_STEPS] = double(it + 1);
  if (rz2[b] <= 1e-24 * c[EIG_RZ0] || double(it + 1) >= c[EIG_MAX]) c[EIG_ACTIVE] = 0.0;
}
// p = z + beta p on active blocks
// (launched with 256-thread blocks)
__global__ void __launch_bounds__(256) k_eig_waxpy(double* p, const double* z, const double* sc, int64_t nl,
                                                   int64_t begin) {
  const bool act[2] = {sc[EIG_ACTIVE] != 0.0, sc[EIG_SC + EIG_ACTIVE] != 0.0};
  const double beta[2] = {sc[EIG_BETA], sc[EIG_SC + EIG_BETA]};
  for (int64_t i = begin + int64_t(blockIdx.x) * 256 + threadIdx.x; i < 3 * nl; i += int64_t(gridDim.x) * 256) {
    const int b = i < 2 * nl ? 0 : 1;
    if (act[b]) p[i] = z[i] + beta[b] * p[i];
  }
}

// ---- coarse-level CG (one workgroup; the coarse level is small) ----------
// Jacobi-preconditioned CG from x = 0 on both blocks at once: block 0 is the
// displacement rows [0, 2n), block 1 the phase-field rows [2n, 3n); each has
// its own scalars. Free unknowns are those with dinv != 0. s[0..1] holds
// r.z per block between the kernels. An exactly zero r.z stops a block (its
// further steps change nothing).
constexpr int CCG_THREADS = 256;

__device__ __forceinline__ void ccg_reduce2(double& a0, double& a1, double* sh) {
  sh[threadIdx.x] = a0;
  sh[CCG_THREADS + threadIdx.x] = a1;
  __syncthreads();
  for (int w = CCG_THREADS / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      sh[threadIdx.x] += sh[threadIdx.x + w];
      sh[CCG_THREADS + threadIdx.x] += sh[CCG_THREADS + threadIdx.x + w];
    }
    __syncthreads();
  }
  a0 = sh[0];
  a1 = sh[CCG_THREADS];
  __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(CCG_THREADS) k_ccg_init(T* x, T* r, T* p, const T* b, const T* dinv, int64_t n,
                                                           double* s) {
  __shared__ double sh[2 * CCG_THREADS];
  double rz0 = 0.0, rz1 = 0.0;
  for (int64_t i = threadIdx.x; i < 3 * n; i += blockDim.x) {
    const T di = dinv[i];
    const T ri = di != T(0) ? b[i] : T(0);
    x[i] = T(0);
    r[i] = ri;
    p[i] = di * ri;
    const double c = double(ri) * double(di * ri);
    if (i < 2 * n) rz0 += c; else rz1 += c;
  }
  ccg_reduce2(rz0, rz1, sh);
  if (threadIdx.x == 0) { s[0] = rz0; s[1] = rz1; }
}

// one CG step after q = A p: mask q, alpha = r.z / p.q, x += alpha p,
// r -= alpha q, z = dinv r, beta = r.z_new / r.z, p = z + beta p
template <typename T>
__global__ void __launch_bounds__(CCG_THREADS) k_ccg_step(T* x, T* r, T* p, const T* q, const T* dinv, int64_t n,
                                                           double* s) {
  __shared__ double sh[2 * CCG_THREADS];
  const double rz[2] = {s[0], s[1]};
  double pq0 = 0.0, pq1 = 0.0;
  for (int64_t i = threadIdx.x; i < 3 * n; i += blockDim.x) {
    const double c = dinv[i] != T(0) ? double(p[i]) * double(q[i]) : 0.0;
    if (i < 2 * n) pq0 += c; else pq1 += c;
  }
  ccg_reduce2(pq0, pq1, sh);
  const double alpha[2] = {rz[0] == 0.0 ? 0.0 : rz[0] / pq0, rz[1] == 0.0 ? 0.0 : rz[1] / pq1};
  double rn0 = 0.0, rn1 = 0.0;
  for (int64_t i = threadIdx.x; i < 3 * n; i += blockDim.x) {
    const int blk = i < 2 * n ? 0 : 1;
    const T di = dinv[i];
    const T qi = di != T(0) ? q[i] : T(0);
    const T al = T(alpha[blk]);
    x[i] += al * p[i];
    const T ri = r[i] - al * qi;
    r[i] = ri;
    const double c = double(ri) * double(di * ri);
    if (blk == 0) rn0 += c; else rn1 += c;
  }
  ccg_reduce2(rn0, rn1, sh);
  const double beta[2] = {rz[0] == 0.0 ? 0.0 : rn0 / rz[0], rz[1] == 0.0 ? 0.0 : rn1 / rz[1]};
  for (int64_t i = threadIdx.x; i < 3 * n; i += blockDim.x) {
    const int blk = i < 2 * n ? 0 : 1;
    p[i] = dinv[i] * r[i] + T(beta[blk]) * p[i];
  }
  if (threadIdx.x == 0) { s[0] = rn0; s[1] = rn1; }
}

}  // namespace pff
