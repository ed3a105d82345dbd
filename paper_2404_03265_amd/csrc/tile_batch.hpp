// Transposed Jacobian J~^T for a batch of right-hand sides with the state read
// once per tile (the adjoint of the crack-volume functional, Sec. 4, needs
// J~^T; differentiating through several quantities applies it to several
// vectors at one state).
//
// One workgroup per tile as in tile_kernel: the state fields (u_x, u_y, phi,
// phit), the node flags and the state's hanging values are staged once; then,
// per right-hand side, the operand is staged (constrained columns masked,
// identity rows of constrained private nodes written at once), its hanging
// values interpolated, every cell evaluated with jacobian_t_cell, accumulated
// in colour phases, distributed from hanging nodes, and written: private rows
// directly, shared rows as partial sums into the right-hand side's own slot
// range. shared_fixup_jt_batch adds the slots of every shared node in
// ascending tile order for each right-hand side, in the order of the
// one-vector kernel.
#pragma once

#include "tile_kernel.hpp"

namespace pff {

constexpr int JT_BATCH_MAX = 8;   // right-hand sides per launch

// two waves per SIMD: left to itself the register allocator takes two
// accumulation registers beyond 256 for Q2 and halves the occupancy
template <int P>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
tile_kernel_jt_batch(const TileArgs<double> a, int nrhs) {
  using T = double;
  constexpr int N1 = P + 1, NL = N1 * N1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ML = a.max_local;
  T* opd = reinterpret_cast<T*>(smem_raw);   // [3][ML] operand, then the accumulators
  T* stl = opd + 3 * ML;                     // [4][ML] state
  uint8_t* lflag = reinterpret_cast<uint8_t*>(stl + 4 * ML);

  // XCD-aware tile order (as in tile_kernel)
  const int nb = int(gridDim.x), bid = int(blockIdx.x);
  const int xq = nb >> 3, xr = nb & 7, xcd = bid & 7;
  const int order_idx = xcd * xq + (xcd < xr ? xcd : xr) + (bid >> 3);
  const int tile = a.tile_base + order_idx;
  int ti[TILE_STRIDE];
  {
    const int32_t* tp = a.tile_info + TILE_STRIDE * tile;
#pragma unroll
    for (int k = 0; k < TILE_STRIDE; ++k) ti[k] = tp[k];
  }
  const int o0 = ti[TILE_OWNED0], no = ti[TILE_NOWNED];
  const int s0 = ti[TILE_SHARED0], ns = ti[TILE_NSHARED];
  const int c0 = ti[TILE_CELL0], nc = ti[TILE_NCELL];
  const int ncol = ti[TILE_NCOLOR];
  const int slot0 = ti[TILE_SLOT0];
  const int nrun = ti[TILE_NRUN];
  const int hr0 = ti[TILE_HANG0], nhang = ti[TILE_NHANG], nhcol = ti[TILE_NHCOLOR];
  const int nloc = no + ns;
  const int64_t n = a.n;
  const int bs = int(blockDim.x), tid = int(threadIdx.x);
  // nodes per thread and staging round, sized for the default tiles (Q1:
  // 16 x 16 cells on four waves, Q2: 8 x 8 cells on one wave)
  constexpr int KB = P == 1 ? 2 : 5;
  // global id of local node l: private range, then the shared list (from the
  // header's runs of consecutive ids, else the list)
  auto node_id = [&](int l) -> uint32_t {
    if (l < no) return uint32_t(o0 + l);
    const int r = l - no;
    if (nrun > 0) {
      int id = ti[TILE_RUN_START] + r;
#pragma unroll
      for (int k = 1; k < TILE_MAX_RUNS; ++k)
        if (k < nrun && r >= ti[TILE_RUN_OFF + k]) id = ti[TILE_RUN_START + k] + (r - ti[TILE_RUN_OFF + k]);
      return uint32_t(id);
    }
    return uint32_t(a.shared[s0 + r]);
  };
  // values at hanging nodes from their masters, fields [f0, f0 + nf) of base
  auto interp_hanging = [&](T* base, int nf) {
    for (int r = tid; r < nhang; r += bs) {
      const uint16_t* hr = a.hang_rec + 4 * int64_t(hr0 + r);
      const double* hw = a.hang_w + 3 * int64_t(hr0 + r);
      const int h = hr[0], m0 = hr[1], m1 = hr[2], m2 = hr[3];
      for (int f = 0; f < nf; ++f)
        base[f * ML + h] = hw[0] * base[f * ML + m0] + hw[1] * base[f * ML + m1] + hw[2] * base[f * ML + m2];
    }
  };

  // 1. state and flags, once (every load of a round before its stores)
  for (int l0 = 0; l0 < nloc; l0 += KB * bs) {
    uint32_t g[KB];
    uint8_t fl[KB];
    T v[KB][4];
#pragma unroll
    for (int k = 0; k < KB; ++k) g[k] = node_id(min(l0 + k * bs + tid, nloc - 1));
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      fl[k] = at32(a.flags, g[k]);
#pragma unroll
      for (int f = 0; f < 4; ++f) v[k][f] = at32(a.st[f], g[k]);
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int l = l0 + k * bs + tid;
      if (l < nloc) {
        lflag[l] = fl[k];
#pragma unroll
        for (int f = 0; f < 4; ++f) stl[f * ML + l] = v[k][f];
      }
    }
  }
  const int cell = tid;
  const bool live = cell < nc;
  int loc[NL];
  __syncthreads();
  if (nhang > 0) {
    interp_hanging(stl, 4);
    __syncthreads();
  }
  const Material& m = a.mat;
  const T kap = T(m.kappa), pr = T(m.pressure), Gc = T(m.Gc), ell = T(m.ell);
  const T mu = T(m.mu), lam = T(m.lam);
  const bool one_phase = bs <= 64;

  for (int b = 0; b < nrhs; ++b) {
    const T* src = a.src + int64_t(b) * 3 * n;
    T* dst = a.dst + int64_t(b) * 3 * n;
    T* part = a.part + int64_t(b) * 3 * a.n_slots;
    // 2. operand: constrained columns masked; identity rows of constrained
    //    private nodes written now. Per round every load is issued before the
    //    first store (a store to dst between loads of src would order them).
    for (int l0 = 0; l0 < nloc; l0 += KB * bs) {
      uint32_t g[KB];
      T v[KB][3];
#pragma unroll
      for (int k = 0; k < KB; ++k) g[k] = node_id(min(l0 + k * bs + tid, nloc - 1));
#pragma unroll
      for (int k = 0; k < KB; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) v[k][c] = at32(src + c * n, g[k]);
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const int l = l0 + k * bs + tid;
        if (l < nloc) {
          const uint8_t f = lflag[l];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            if (l < no) {
              const bool cons =
                  (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
              if (cons) at32(dst + c * n, g[k]) = v[k][c];
            }
            const bool fixed = (c < 2) ? (f & NODE_DIRICHLET) : (f & NODE_ACTIVE);
            opd[c * ML + l] = fixed ? T(0) : v[k][c];
          }
        }
      }
    }
    __syncthreads();
    if (nhang > 0) {
      interp_hanging(opd, 3);
      __syncthreads();
    }
    // 3. cells. The cell record is read again in every pass (from the
    //    caches): held across the passes, the LDS addresses derived from it
    //    would stay live for all fields and halve the occupancy.
    unsigned info = 0;
    if (live) {
      const int64_t rec = int64_t(c0) + cell;
#pragma unroll
      for (int k = 0; k < NL; ++k) loc[k] = a.cell_loc[rec * NL + k];
      info = a.cell_info[rec];
    }
    const int color = live ? int((info >> CELL_COLOR_SHIFT) & 15u) : -1;
    const T H = live ? T(ldexp(double(a.H0), -int((info >> CELL_LEVEL_SHIFT) & 31u))) : T(1);
    T out[3][NL];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < NL; ++k) out[c][k] = T(0);
    if (live) {
      auto gather = [&](int field, T(&u)[NL]) {
        const T* base = field < 3 ? opd + field * ML : stl + (field - 3) * ML;
#pragma unroll
        for (int k = 0; k < NL; ++k) u[k] = base[loc[k]];
      };
      jacobian_t_cell<P, T>(H, mu, lam, kap, pr, Gc, ell, gather, out);
    }
    __syncthreads();   // every gather done: the operand arrays become the accumulators
    for (int l = tid; l < nloc; l += bs) {
      opd[l] = T(0);
      opd[ML + l] = T(0);
      opd[2 * ML + l] = T(0);
    }
    __syncthreads();
    const int nphase = one_phase ? 1 : ncol;
    for (int col = 0; col < nphase; ++col) {
      if (live && (one_phase || color == col)) {
#pragma unroll
        for (int k = 0; k < NL; ++k) {
          const int l = loc[k];
#pragma unroll
          for (int c = 0; c < 3; ++c)
            __hip_atomic_fetch_add(&opd[c * ML + l], out[c][k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
      __syncthreads();
    }
    // contributions at hanging nodes to their masters (records of one colour
    // share no master)
    for (int col = 0; col < nhcol; ++col) {
      for (int r = tid; r < nhang; r += bs) {
        if (a.hang_col[hr0 + r] != col) continue;
        const uint16_t* hr = a.hang_rec + 4 * int64_t(hr0 + r);
        const double* hw = a.hang_w + 3 * int64_t(hr0 + r);
        const int h = hr[0];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T v = opd[c * ML + h];
#pragma unroll
          for (int k = 0; k <= P; ++k)
            __hip_atomic_fetch_add(&opd[c * ML + hr[1 + k]], hw[k] * v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
      __syncthreads();
    }
    // 4. private rows (free ones; constrained ones were written while
    //    staging), shared rows into this right-hand side's slots
    for (int l = tid; l < no; l += bs) {
      const uint8_t f = lflag[l];
      const uint32_t g = uint32_t(o0 + l);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const bool cons = (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
        if (!cons) at32(dst + c * n, g) = opd[c * ML + l];
      }
    }
    for (int r = tid; r < ns; r += bs) {
#pragma unroll
      for (int c = 0; c < 3; ++c) at32(part + c * a.n_slots, uint32_t(slot0 + r)) = opd[c * ML + no + r];
    }
    __syncthreads();   // the next operand overwrites the accumulators
  }
}

// Shared nodes of every right-hand side: the partial sums in ascending tile
// order, then the transposed operator's rows (identity on constrained rows).
__global__ void __launch_bounds__(256) shared_fixup_jt_batch(const TileArgs<double> a, int nrhs) {
  const int64_t total = a.n_shared * int64_t(nrhs);
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t b = t / a.n_shared, s = t - b * a.n_shared;
    const double* part = a.part + b * 3 * a.n_slots;
    const double* src = a.src + b * 3 * a.n;
    double* dst = a.dst + b * 3 * a.n;
    const int64_t g = a.n_private + s;
    const uint8_t f = a.flags[g];
    double v[3] = {0.0, 0.0, 0.0};
    if (a.sh_w == SHARED_SLOTS) {
      const int4 sl = reinterpret_cast<const int4*>(a.sh_tab)[s];
      const int slot[SHARED_SLOTS] = {sl.x, sl.y, sl.z, sl.w};
#pragma unroll
      for (int j = 0; j < SHARED_SLOTS; ++j)
        if (slot[j] >= 0) {
#pragma unroll
          for (int c = 0; c < 3; ++c) v[c] += part[c * a.n_slots + slot[j]];
        }
    } else {
      for (int j = 0; j < a.sh_w; ++j) {
        const int slot = a.sh_tab[s * a.sh_w + j];
        if (slot < 0) break;
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] += part[c * a.n_slots + slot];
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = c * a.n + g;
      const bool cons = (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
      dst[i] = cons ? src[i] : v[c];
    }
  }
}

}  // namespace pff
