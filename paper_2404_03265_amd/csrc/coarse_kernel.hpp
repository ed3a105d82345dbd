// Coarse-level solve in one kernel (Sec. 3.2: the level-0 solve of the
// V-cycle). The block operator is block diagonal, so its two blocks are
// solved by two workgroups at once (blockIdx.x 0: the displacement rows,
// 1: the phase-field rows). Each holds the level's operand, accumulator, state
// and iteration vectors in LDS and runs every step of the fixed-length solve
// of its block: Chebyshev from x = 0 over [lambda_min, upper_factor *
// lambda_max], or Jacobi-preconditioned CG from x = 0 with the block's
// scalars. Each thread evaluates its block's rows of one level-0 cell with
// the cell routines of the tile kernels (the state coefficients once, kept in
// registers for every step) and adds them into the accumulator in colour
// phases (cells of one colour share no node), so the summation order is
// fixed; unknown i belongs to thread i mod COARSE_THREADS in both blocks.
// Replaces 2-3 launches per step (tile kernel, shared-node fix-up, CG
// scalars) by one launch.
#pragma once

#include "tile_kernel.hpp"
#include "util_kernels.hpp"

namespace pff {

constexpr int COARSE_THREADS = 256;    // one cell per thread: level 0 has at most 256 cells
constexpr int COARSE_MAX_STEPS = 64;
constexpr int COARSE_MAX_COLORS = 8;
constexpr int COARSE_PER_THREAD = 16;  // unknowns per thread: 3 n0 <= COARSE_THREADS * COARSE_PER_THREAD

template <typename T>
struct CoarseArgs {
  int n0;                                // level-0 nodes
  int ncell;                             // level-0 cells, sorted by colour
  int ncolor;
  int cstart[COARSE_MAX_COLORS + 1];     // colour c: cells [cstart[c], cstart[c + 1])
  int steps;                             // Chebyshev updates / CG steps
  int cg;                                // 0: Chebyshev, 1: CG
  const int32_t* cell_nodes;             // [ncell][(p+1)^2] level-0 node ids
  const uint8_t* flags;                  // [n0]
  const T* state;                        // [3][n0] level state (u_x, u_y, phit)
  const T* b;                            // [3][n0] right-hand side
  const T* dinv;                         // [3][n0] inverse diagonal (0 on held rows)
  T* x;                                  // [3][n0] result
  T H;                                   // cell edge on level 0
  Material mat;
  T c1[COARSE_MAX_STEPS][2], c2[COARSE_MAX_STEPS][2];   // Chebyshev coefficients per step and block
};

// deterministic sums over the workgroup of two per-thread values
__device__ __forceinline__ void coarse_sum2(double& a0, double& a1, double* red) {
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    red[2 * wave] = a0;
    red[2 * wave + 1] = a1;
  }
  __syncthreads();
  a0 = 0.0;
  a1 = 0.0;
  for (int w = 0; w < COARSE_THREADS / 64; ++w) {
    a0 += red[2 * w];
    a1 += red[2 * w + 1];
  }
}

// LDS: five vectors of 3 n0 doubles (operand, accumulator, state, two
// iteration vectors) and the flags.
template <int P, typename T>
__global__ void __launch_bounds__(COARSE_THREADS) coarse_kernel(const CoarseArgs<T> a) {
  constexpr int NL = (P + 1) * (P + 1);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[2 * (COARSE_THREADS / 64)];
  const int n0 = a.n0, N = 3 * n0, tid = int(threadIdx.x);
  const int blk = int(blockIdx.x);                    // 0: u_x, u_y rows; 1: phi rows
  const int r0 = blk == 0 ? 0 : 2 * n0, r1 = blk == 0 ? 2 * n0 : N;
  const int c0 = blk == 0 ? 0 : 2, c1e = blk == 0 ? 2 : 3;   // components [c0, c1e)
  double* xo = reinterpret_cast<double*>(smem_raw);   // operand of A: x (Chebyshev) or p (CG)
  double* acc = xo + N;                               // A * operand
  double* st = acc + N;                               // state
  double* v1 = st + N;                                // Chebyshev: d; CG: r
  double* v2 = v1 + N;                                // CG: x
  uint8_t* fl = reinterpret_cast<uint8_t*>(v2 + N);
  for (int i = tid; i < N; i += COARSE_THREADS) st[i] = double(a.state[i]);
  for (int i = tid; i < n0; i += COARSE_THREADS) fl[i] = a.flags[i];

  const bool live = tid < a.ncell;
  int nodes[NL];
  int color = -1;
  if (live) {
#pragma unroll
    for (int k = 0; k < NL; ++k) nodes[k] = a.cell_nodes[int64_t(tid) * NL + k];
    for (int c = 0; c < a.ncolor; ++c)
      if (tid >= a.cstart[c] && tid < a.cstart[c + 1]) color = c;
  }
  const Material& m = a.mat;
  const T kap = T(m.kappa), pr = T(m.pressure), Gc = T(m.Gc), ell = T(m.ell);
  const T mu = T(m.mu), lam = T(m.lam);
  auto gather = [&](int f, T(&u)[NL]) {
#pragma unroll
    for (int k = 0; k < NL; ++k) u[k] = T(xo[f * n0 + nodes[k]]);
  };
  __syncthreads();
  // the state enters every step only through the block's coefficients (g
  // for the displacement rows, H^2 c1 for the phase-field rows)
  T cf[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) cf[k] = T(0);
  if (live) {
    auto gather_state = [&](int f, T(&u)[NL]) {
#pragma unroll
      for (int k = 0; k < NL; ++k) u[k] = T(st[f * n0 + nodes[k]]);
    };
    T cg[NL], cc1[NL];
    level_coefs<P, T>(a.H, mu, lam, kap, pr, Gc, ell, gather_state, cg, cc1);
#pragma unroll
    for (int k = 0; k < NL; ++k) cf[k] = blk == 0 ? cg[k] : cc1[k];
  }
  // acc = A xo on the block's rows (held columns of xo are zero)
  auto apply = [&]() {
    for (int i = r0 + tid; i < r1; i += COARSE_THREADS) acc[i] = 0.0;
    __syncthreads();
    T out[2][NL];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int k = 0; k < NL; ++k) out[c][k] = T(0);
    if (live) {
      if (blk == 0) level_cell_u<P, T>(mu, lam, cf, gather, out[0], out[1]);
      else level_cell_phi<P, T>(Gc * ell, cf, [&](int, T(&u)[NL]) { gather(2, u); }, out[0]);
    }
    for (int col = 0; col < a.ncolor; ++col) {
      if (color == col) {
#pragma unroll
        for (int k = 0; k < NL; ++k)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            if (c0 + c < c1e)
              __hip_atomic_fetch_add(&acc[(c0 + c) * n0 + nodes[k]], double(out[c][k]), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      __syncthreads();
    }
  };

  if (!a.cg) {
    // Chebyshev: d = c2 D^-1 b, x = d; then r = b - A x,
    // d = c1 d + c2 D^-1 r and x += d on free rows (d = 0 on held rows).
    // b, D^-1 and the held flag of the thread's unknowns stay in registers.
    T bi[COARSE_PER_THREAD], di[COARSE_PER_THREAD];
    bool held[COARSE_PER_THREAD];
#pragma unroll
    for (int k = 0; k < COARSE_PER_THREAD; ++k) {
      const int i = tid + k * COARSE_THREADS;
      bi[k] = T(0);
      di[k] = T(0);
      held[k] = true;
      if (i >= r0 && i < r1) {
        const int c = i / n0;
        const uint8_t f = a.flags[i - c * n0];
        bi[k] = a.b[i];
        di[k] = a.dinv[i];
        held[k] = (c < 2) ? (f & (NODE_DIRICHLET | NODE_EDGE)) : (f & (NODE_ACTIVE | NODE_EDGE));
        const T v = a.c2[0][blk] * di[k] * bi[k];
        v1[i] = double(v);
        xo[i] = double(v);
      }
    }
    __syncthreads();
    for (int j = 1; j < a.steps; ++j) {
      apply();
#pragma unroll
      for (int k = 0; k < COARSE_PER_THREAD; ++k) {
        const int i = tid + k * COARSE_THREADS;
        if (i >= r0 && i < r1) {
          if (held[k]) {
            v1[i] = 0.0;
          } else {
            const T r = bi[k] - T(acc[i]);
            const T dn = a.c1[j][blk] * T(v1[i]) + a.c2[j][blk] * di[k] * r;
            v1[i] = double(dn);
            xo[i] = double(T(xo[i]) + dn);
          }
        }
      }
      __syncthreads();
    }
    for (int i = r0 + tid; i < r1; i += COARSE_THREADS) a.x[i] = T(xo[i]);
    return;
  }

  // CG: r = b on free rows, x = 0, p = D^-1 r; per step alpha = r.z / p.q,
  // x += alpha p, r -= alpha q, beta = r.z_new / r.z, p = D^-1 r + beta p;
  // a block whose r.z is exactly zero stays where it is. D^-1 of the thread's
  // unknowns stays in registers.
  T di[COARSE_PER_THREAD];
  double rz0 = 0.0, rz1 = 0.0;
#pragma unroll
  for (int k = 0; k < COARSE_PER_THREAD; ++k) {
    const int i = tid + k * COARSE_THREADS;
    di[k] = T(0);
    if (i >= r0 && i < r1) {
      di[k] = a.dinv[i];
      const T ri = di[k] != T(0) ? a.b[i] : T(0);
      v2[i] = 0.0;
      v1[i] = double(ri);
      xo[i] = double(di[k] * ri);
      const double c = double(ri) * double(di[k] * ri);
      if (i < 2 * n0) rz0 += c; else rz1 += c;
    }
  }
  coarse_sum2(rz0, rz1, red);
  double rz[2] = {rz0, rz1};
  for (int it = 0; it < a.steps; ++it) {
    apply();
    double pq0 = 0.0, pq1 = 0.0;
#pragma unroll
    for (int k = 0; k < COARSE_PER_THREAD; ++k) {
      const int i = tid + k * COARSE_THREADS;
      if (i >= r0 && i < r1) {
        const double c = di[k] != T(0) ? double(T(xo[i])) * double(T(acc[i])) : 0.0;
        if (i < 2 * n0) pq0 += c; else pq1 += c;
      }
    }
    coarse_sum2(pq0, pq1, red);
    const double alpha[2] = {rz[0] == 0.0 ? 0.0 : rz[0] / pq0, rz[1] == 0.0 ? 0.0 : rz[1] / pq1};
    double rn0 = 0.0, rn1 = 0.0;
#pragma unroll
    for (int k = 0; k < COARSE_PER_THREAD; ++k) {
      const int i = tid + k * COARSE_THREADS;
      if (i >= r0 && i < r1) {
        const T qi = di[k] != T(0) ? T(acc[i]) : T(0);
        const T al = T(alpha[blk]);
        v2[i] = double(T(v2[i]) + al * T(xo[i]));
        const T ri = T(v1[i]) - al * qi;
        v1[i] = double(ri);
        const double c = double(ri) * double(di[k] * ri);
        if (blk == 0) rn0 += c; else rn1 += c;
      }
    }
    coarse_sum2(rn0, rn1, red);
    const double beta[2] = {rz[0] == 0.0 ? 0.0 : rn0 / rz[0], rz[1] == 0.0 ? 0.0 : rn1 / rz[1]};
#pragma unroll
    for (int k = 0; k < COARSE_PER_THREAD; ++k) {
      const int i = tid + k * COARSE_THREADS;
      if (i >= r0 && i < r1) {
        xo[i] = double(di[k] * T(v1[i]) + T(beta[blk]) * T(xo[i]));
      }
    }
    rz[0] = rn0;
    rz[1] = rn1;
    __syncthreads();
  }
  for (int i = r0 + tid; i < r1; i += COARSE_THREADS) a.x[i] = T(v2[i]);
}

}  // namespace pff
