// Persistent, double-buffered form of the tile kernel for one-wave tiles of
// the leaf Jacobian and its transpose (Q2, at most 64 cells per tile).
//
// The partition of cells into tiles, the per-tile arithmetic, the summation
// order and the partial sums of shared nodes are those of tile_kernel, so the
// results are bitwise the same. What changes is how a wave meets memory
// latency: each workgroup (one wave) walks a contiguous chunk of the tile
// list, and while it computes tile t its next tile's nodal fields are already
// on their way into the other of two LDS buffers through gfx950's direct
// global-to-LDS loads (global_load_lds_dwordx4 for the private node range of
// each field, global_load_lds_dword for the shared nodes). These loads hold no
// registers, so the staging of tile t + 1 overlaps the compute of tile t
// without the register cost that a prefetch into VGPRs would have. The two
// buffers are distinct __shared__ arrays and the loop is unrolled by two, so
// the compiler's wait counts separate the buffer being read from the one
// being filled.
//
// LDS layout of a buffer: NF field regions of PIPE_FIELD doubles. Private
// node l of field f sits at index s_f + l and shared entry r at
// PIPE_SHOFF + s_f + r, where s_f in {0, 1} is the parity of the field's
// global element address of the tile's first private node (the 16-byte
// loads start at the even element at or below it).
#pragma once

#include "tile_kernel.hpp"

namespace pff {

constexpr int PIPE_PRIV = 256;                       // private nodes per tile
constexpr int PIPE_SH = 64;                          // shared nodes per tile
constexpr int PIPE_SHOFF = PIPE_PRIV;                // first shared slot
constexpr int PIPE_FIELD = PIPE_PRIV + 2 + PIPE_SH;  // 322: private, shift slack, shared
constexpr int PIPE_CELLS = 64;                       // cells per tile (one per lane)
constexpr int PIPE_NF = 7;                           // staged fields: src (3) + leaf state (4)

// What the prefetch of a tile leaves in registers for its processing.
struct PipeStaged {
  int o0, no, ns, c0, nc, slot0, hr0, nhang, nhcol;
  bool skip;               // shared list not in runs: tile_kernel processes the tile
  unsigned sbits;          // bit f: the shift s_f of field f
  uint8_t fp[4], fsh;      // node flags: private l = 64 k + lane, shared r = lane
  int loc[9];              // the lane's cell: local ids
  unsigned info;           // the lane's cell: info word
  int hn, hm0, hm1, hm2;   // the lane's hanging record (lane < nhang): local ids
  double hw0, hw1, hw2;
  int hcol;
};

template <int MODE>
__device__ __forceinline__ const double* pipe_field_ptr(const TileArgs<double>& a, int f) {
  // fields 0..2: the operand's components, 3..6: u_x, u_y, phi, phi~
  return f < 3 ? a.src + f * a.n : a.st[f - 3];
}

// The read-only tables and the two outputs as separate restrict-qualified
// kernel arguments: with them the compiler knows that the loop's stores do
// not clobber the tables, and reads the tile headers with scalar loads
// (tracked by lgkmcnt) instead of vector loads, whose waits would also wait
// for the other buffer's direct-to-LDS loads.
struct PipePtrs {
  const int32_t* __restrict__ tile_info;
  const int32_t* __restrict__ shared;
  const uint16_t* __restrict__ cell_loc;
  const uint16_t* __restrict__ cell_info;
  const uint8_t* __restrict__ flags;
  const uint16_t* __restrict__ hang_rec;
  const double* __restrict__ hang_w;
  const uint8_t* __restrict__ hang_col;
  double* __restrict__ dst;
  double* __restrict__ part;
};

__device__ __forceinline__ int pipe_lidx(int l, int no) { return l < no ? l : PIPE_SHOFF + (l - no); }

// Phase boundary of a one-wave workgroup. The LDS executes one wave's
// operations in the order they are issued, so lanes see each other's
// earlier LDS writes without a wait; what is needed is that the compiler
// keeps the phases in program order (a compiler barrier on memory). A fence
// is not used: even restricted to LDS it waits for every LDS write in
// flight, the direct-to-LDS loads of the other buffer included.
__device__ __forceinline__ void pipe_sync() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

template <int MODE>
__device__ __forceinline__ PipeStaged pipe_prefetch(const TileArgs<double>& a, const PipePtrs& pp, int tile, double* buf,
                                                    int n_hang_rec) {
  using LdsPtr = __attribute__((address_space(3))) void*;
  PipeStaged s;
  const int lane = int(threadIdx.x);
  int ti[TILE_STRIDE];
  {
    const int32_t* tp = pp.tile_info + TILE_STRIDE * tile;
#pragma unroll
    for (int k = 0; k < TILE_STRIDE; ++k) ti[k] = tp[k];
  }
  const int o0 = ti[TILE_OWNED0], no = ti[TILE_NOWNED];
  const int s0 = ti[TILE_SHARED0], ns = ti[TILE_NSHARED];
  const int nrun = ti[TILE_NRUN];
  s.o0 = o0;
  s.no = no;
  s.ns = ns;
  s.c0 = ti[TILE_CELL0];
  s.nc = ti[TILE_NCELL];
  s.slot0 = ti[TILE_SLOT0];
  s.hr0 = ti[TILE_HANG0];
  s.nhang = ti[TILE_NHANG];
  s.nhcol = ti[TILE_NHCOLOR];
  // global id of shared entry r (clamped into the list; ns >= 1 on the
  // pipelined path) from the runs of consecutive ids in the header, ALU
  // only. A tile whose shared list has more runs than the header holds is
  // skipped here (it stages an in-range dummy and writes nothing) and
  // processed by tile_kernel over the list of such tiles: a load of the
  // list before the direct-to-LDS loads would make their issue wait for
  // every load in flight, the other buffer's included.
  s.skip = nrun == 0;
  (void)s0;
  auto shared_id = [&](int r) -> int64_t {
    r = min(r, ns - 1);
    int id = nrun > 0 ? ti[TILE_RUN_START] + r : o0;
#pragma unroll
    for (int k = 1; k < TILE_MAX_RUNS; ++k)
      if (k < nrun && r >= ti[TILE_RUN_OFF + k]) id = ti[TILE_RUN_START + k] + (r - ti[TILE_RUN_OFF + k]);
    return id;
  };
  const int64_t sid0 = shared_id(lane >> 1), sid1 = shared_id(32 + (lane >> 1));
  const int half = lane & 1;
  unsigned sbits = 0;
#pragma unroll
  for (int f = 0; f < PIPE_NF; ++f) {
    const double* ep = pipe_field_ptr<MODE>(a, f);
    const int sf = int((reinterpret_cast<uintptr_t>(ep + o0) >> 3) & 1u);
    sbits |= unsigned(sf) << f;
    // private range: 16-byte chunks from the even element at or below o0;
    // lanes past the last chunk re-read it and fill unused slots
    const double* g0 = ep + (o0 - sf);
    const int jl = (sf + no - 1) >> 1;
    double* fb = buf + f * PIPE_FIELD;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int j = min(64 * i + lane, jl);
      __builtin_amdgcn_global_load_lds((const void*)(g0 + 2 * j), (LdsPtr)(fb + 128 * i), 16, 0, 0);
    }
    // shared entries, one dword per lane: entry r = d / 2, half d % 2
    const char* gs0 = reinterpret_cast<const char*>(ep + sid0) + 4 * half;
    const char* gs1 = reinterpret_cast<const char*>(ep + sid1) + 4 * half;
    char* sb = reinterpret_cast<char*>(fb + PIPE_SHOFF + sf);
    __builtin_amdgcn_global_load_lds((const void*)gs0, (LdsPtr)sb, 4, 0, 0);
    __builtin_amdgcn_global_load_lds((const void*)gs1, (LdsPtr)(sb + 256), 4, 0, 0);
  }
  s.sbits = sbits;
  // node flags, the lane's cell record and hanging record into registers
  const int64_t n = a.n;
#pragma unroll
  for (int k = 0; k < 4; ++k) s.fp[k] = pp.flags[min(int64_t(o0) + min(64 * k + lane, no - 1), n - 1)];
  s.fsh = pp.flags[shared_id(lane)];
  {
    const int64_t rec = int64_t(s.c0) + min(lane, s.nc - 1);
#pragma unroll
    for (int k = 0; k < 9; ++k) s.loc[k] = pp.cell_loc[rec * 9 + k];
    s.info = pp.cell_info[rec];
  }
  {
    const int r = max(0, min(s.hr0 + min(lane, s.nhang - 1), n_hang_rec - 1));
    const uint16_t* hr = pp.hang_rec + 4 * int64_t(r);
    const double* hw = pp.hang_w + 3 * int64_t(r);
    s.hn = hr[0];
    s.hm0 = hr[1];
    s.hm1 = hr[2];
    s.hm2 = hr[3];
    s.hw0 = hw[0];
    s.hw1 = hw[1];
    s.hw2 = hw[2];
    s.hcol = pp.hang_col[r];
  }
  return s;
}

template <int MODE>
__device__ __forceinline__ void pipe_process(const TileArgs<double>& a, const PipePtrs& pp, const PipeStaged& s,
                                             double* buf, uint8_t* lflag) {
  constexpr int P = 2, NL = 9;
  using T = double;
  const int lane = int(threadIdx.x);
  const int no = s.no, ns = s.ns;
  const int64_t n = a.n;
  auto sh = [&](int f) { return int((s.sbits >> f) & 1u); };
  // node flags into LDS (index = local slot without shift)
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (64 * k + lane < no) lflag[64 * k + lane] = s.fp[k];
  if (lane < ns) lflag[PIPE_SHOFF + lane] = s.fsh;
  // the raw operand of the lane's private rows (identity rows of
  // constrained unknowns), before masking and hanging interpolation
  T raw[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) raw[k][c] = buf[c * PIPE_FIELD + sh(c) + min(64 * k + lane, PIPE_PRIV - 1)];
  pipe_sync();
  // constrained columns of the operand: Dirichlet u, active phi
  for (int l = lane; l < no + ns; l += 64) {
    const int li = pipe_lidx(l, no);
    const uint8_t f = lflag[li];
    if (f & NODE_DIRICHLET) {
      buf[0 * PIPE_FIELD + sh(0) + li] = T(0);
      buf[1 * PIPE_FIELD + sh(1) + li] = T(0);
    }
    if (f & NODE_ACTIVE) buf[2 * PIPE_FIELD + sh(2) + li] = T(0);
  }
  pipe_sync();
  // hanging nodes from their masters (masters are never hanging)
  if (s.nhang > 0) {
    if (lane < s.nhang) {
      const int h = pipe_lidx(s.hn, no), m0 = pipe_lidx(s.hm0, no), m1 = pipe_lidx(s.hm1, no),
                m2 = pipe_lidx(s.hm2, no);
#pragma unroll
      for (int f = 0; f < PIPE_NF; ++f) {
        double* fb = buf + f * PIPE_FIELD + sh(f);
        fb[h] = s.hw0 * fb[m0] + s.hw1 * fb[m1] + s.hw2 * fb[m2];
      }
    }
    pipe_sync();
  }
  // one cell per lane
  const bool live = lane < s.nc;
  int li[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) li[k] = pipe_lidx(s.loc[k], no);
  T out[3][NL];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < NL; ++k) out[c][k] = T(0);
  if (live) {
    const int lev = int((s.info >> CELL_LEVEL_SHIFT) & 31u);
    const T H = T(ldexp(double(a.H0), -lev));
    auto gather = [&](int field, T(&u)[NL]) {
      const double* fb = buf + field * PIPE_FIELD + sh(field);
#pragma unroll
      for (int k = 0; k < NL; ++k) u[k] = fb[li[k]];
    };
    compute_cell<P, T, MODE>(a, H, false, s.info, gather, out);
  }
  // every gather is done: the accumulators take over the operand's regions
  pipe_sync();
  double* acc = buf;
  for (int l = lane; l < 3 * PIPE_FIELD; l += 64) acc[l] = T(0);
  pipe_sync();
  // one phase: two distinct cells never have the same node at the same
  // local position, and a wave's adds execute in program order
  if (live) {
#pragma unroll
    for (int k = 0; k < NL; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        __hip_atomic_fetch_add(&acc[c * PIPE_FIELD + li[k]], out[c][k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  pipe_sync();
  // contributions at hanging nodes go to their masters, records of one
  // colour sharing no master
  for (int col = 0; col < s.nhcol; ++col) {
    if (lane < s.nhang && s.hcol == col) {
      const int h = pipe_lidx(s.hn, no);
      const int m[3] = {pipe_lidx(s.hm0, no), pipe_lidx(s.hm1, no), pipe_lidx(s.hm2, no)};
      const T w[3] = {s.hw0, s.hw1, s.hw2};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T v = acc[c * PIPE_FIELD + h];
#pragma unroll
        for (int k = 0; k <= P; ++k)
          __hip_atomic_fetch_add(&acc[c * PIPE_FIELD + m[k]], w[k] * v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
    pipe_sync();
  }
  // private rows: identity on constrained unknowns, else the sum
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int l = 64 * k + lane;
    if (l < no && !s.skip) {
      const uint8_t f = lflag[l];
      const int64_t g = int64_t(s.o0) + l;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const bool cons = (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
        pp.dst[c * n + g] = cons ? raw[k][c] : acc[c * PIPE_FIELD + l];
      }
    }
  }
  // shared nodes: this tile's partial sums
  if (lane < ns && !s.skip) {
#pragma unroll
    for (int c = 0; c < 3; ++c) pp.part[c * a.n_slots + s.slot0 + lane] = acc[c * PIPE_FIELD + PIPE_SHOFF + lane];
  }
  // the buffer is refilled by the next prefetch: every read of it is done
  pipe_sync();
}

// One wave per workgroup; workgroup w (in XCD-major order) walks the tiles
// [begin_w, end_w) of an even split of the tile list.
template <int MODE>
__global__ void __launch_bounds__(64)
    tile_pipe_kernel(const TileArgs<double> a, const int32_t* __restrict__ tile_info,
                     const int32_t* __restrict__ shared, const uint16_t* __restrict__ cell_loc,
                     const uint16_t* __restrict__ cell_info, const uint8_t* __restrict__ flags,
                     const uint16_t* __restrict__ hang_rec, const double* __restrict__ hang_w,
                     const uint8_t* __restrict__ hang_col, double* __restrict__ dst, double* __restrict__ part,
                     int n_tiles, int n_hang_rec) {
  const PipePtrs pp{tile_info, shared, cell_loc, cell_info, flags, hang_rec, hang_w, hang_col, dst, part};
  __shared__ __align__(16) double bufA[PIPE_NF * PIPE_FIELD];
  __shared__ __align__(16) double bufB[PIPE_NF * PIPE_FIELD];
  __shared__ uint8_t lflag[PIPE_FIELD];
  const int nb = int(gridDim.x), bid = int(blockIdx.x);
  const int xq = nb >> 3, xr = nb & 7, xcd = bid & 7;
  const int w = xcd * xq + (xcd < xr ? xcd : xr) + (bid >> 3);
  const int q = n_tiles / nb, r = n_tiles % nb;
  const int t0 = w * q + (w < r ? w : r);
  const int t1 = t0 + q + (w < r ? 1 : 0);
  if (t0 >= t1) return;
  // every prefetch is unconditional (past the end of the chunk it repeats the
  // last tile, whose result is not used), so that the number of memory
  // operations between a buffer's loads and its first read is the same on
  // every path and the wait for one buffer never includes the other's loads
  // Each half of the loop body: wait until the buffer about to be processed
  // has landed (its loads were issued one tile earlier, so with a tile's
  // compute longer than the memory latency this wait is free), then start
  // the other buffer's loads, then compute. The explicit vmcnt(0) comes
  // before the other buffer's loads are issued, so it never waits for them.
  constexpr unsigned kWaitVm0 = 0x0F70u;   // vmcnt(0), expcnt and lgkmcnt unconstrained
  PipeStaged sA = pipe_prefetch<MODE>(a, pp, t0, bufA, n_hang_rec);
  for (int t = t0; t < t1; t += 2) {
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    const PipeStaged sB = pipe_prefetch<MODE>(a, pp, min(t + 1, t1 - 1), bufB, n_hang_rec);
    pipe_process<MODE>(a, pp, sA, bufA, lflag);
    if (t + 1 >= t1) break;
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    sA = pipe_prefetch<MODE>(a, pp, min(t + 2, t1 - 1), bufA, n_hang_rec);
    pipe_process<MODE>(a, pp, sB, bufB, lflag);
  }
  // the last prefetch is still in flight: the workgroup's LDS must not be
  // released before its direct-to-LDS loads have landed
  __builtin_amdgcn_s_waitcnt(0);
}

}  // namespace pff
