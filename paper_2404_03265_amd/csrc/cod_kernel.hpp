// Crack opening displacement (Sec. 4): COD(x) = the integral over y of
// u . grad phi along the vertical line at x, for up to COD_MAX_LINES lines per
// launch.
//
// One workgroup per leaf tile, one cell per thread (the tile's cell records
// give the cell's nodes; values are read directly from the global vectors in
// the per-cell constraint form: hanging faces from the coarse face's nodes).
// A cell contributes to line j if x_j lies in its x-range [X_c, X_c + S) on
// the node lattice (a line on a cell edge belongs to the cell on its right).
// In reference coordinates x = x_c + s H, y = y_c + t H the contribution is
//   int_0^1 [u_x d_s phi + u_y d_t phi](s, t) dt
// (dy = H dt cancels the 1 / H of the gradient), with p + 1 Gauss points in t.
// Per-thread sums per line, then per-workgroup partials reduced in a fixed
// order by k_reduce_final.
#pragma once

#include "tile_kernel.hpp"
#include "util_kernels.hpp"

namespace pff {

constexpr int COD_MAX_LINES = 64;

struct CodLines {
  double X[COD_MAX_LINES];   // line positions in lattice units
  int n;
};

// Lagrange basis of degree P on the equispaced nodes of [0, 1] and its
// derivative at s
template <int P>
__device__ __forceinline__ void lagrange_at(double s, double (&v)[P + 1], double (&d)[P + 1]) {
  if constexpr (P == 1) {
    v[0] = 1.0 - s;
    v[1] = s;
    d[0] = -1.0;
    d[1] = 1.0;
  } else {
    v[0] = 2.0 * (s - 0.5) * (s - 1.0);
    v[1] = -4.0 * s * (s - 1.0);
    v[2] = 2.0 * s * (s - 0.5);
    d[0] = 4.0 * s - 3.0;
    d[1] = 4.0 - 8.0 * s;
    d[2] = 4.0 * s - 1.0;
  }
}

template <int P, int K>
__global__ void __launch_bounds__(RED_THREADS) k_cod_partial(const TileArgs<double> a, const int32_t* nodeX,
                                                               const double* U, const CodLines lines,
                                                               double* part) {
  constexpr int N1 = P + 1, NL = N1 * N1;
  const int tile = int(blockIdx.x);
  const int32_t* ti = a.tile_info + TILE_STRIDE * tile;
  const int o0 = ti[TILE_OWNED0], no = ti[TILE_NOWNED];
  const int s0 = ti[TILE_SHARED0];
  const int c0 = ti[TILE_CELL0], nc = ti[TILE_NCELL];
  const int64_t n = a.n;
  double acc[K];
#pragma unroll
  for (int j = 0; j < K; ++j) acc[j] = 0.0;
  const int cell = int(threadIdx.x);
  constexpr Basis<double> BC = basis_table<P, double>();
  if (cell < nc) {
    const int64_t rec = int64_t(c0) + cell;
    const unsigned info = a.cell_info[rec];
    auto gid = [&](int l) -> int64_t { return l < no ? int64_t(o0) + l : int64_t(a.shared[s0 + (l - no)]); };
    // x-range on the lattice from the cell's own lower corners
    const int64_t X0 = nodeX[gid(a.cell_loc[rec * NL + 0])];
    const int64_t X1 = nodeX[gid(a.cell_loc[rec * NL + P])];
    const double S = double(X1 - X0);
    // nodal values in the per-cell constraint form
    double ux[NL], uy[NL], ph[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int64_t g = gid(a.cell_loc_sub[rec * NL + k]);
      ux[k] = U[g];
      uy[k] = U[n + g];
      ph[k] = U[2 * n + g];
    }
    if (info & 15u) {
      hang_apply<P, double>(ux, info);
      hang_apply<P, double>(uy, info);
      hang_apply<P, double>(ph, info);
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (j >= lines.n) break;
      const double Xl = lines.X[j];
      if (!(Xl >= double(X0) && Xl < double(X1))) continue;
      const double s = (Xl - double(X0)) / S;
      double vs[N1], ds[N1];
      lagrange_at<P>(s, vs, ds);
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < N1; ++q) {
        // values along the line at t_q: f = sum_ab f_ab l_a(s) l_b(t_q)
        double fx = 0.0, fy = 0.0, fs = 0.0, ft = 0.0;
#pragma unroll
        for (int b = 0; b < N1; ++b) {
          double rx = 0.0, ry = 0.0, rs = 0.0, rv = 0.0;
#pragma unroll
          for (int a2 = 0; a2 < N1; ++a2) {
            const int k = a2 + N1 * b;
            rx += ux[k] * vs[a2];
            ry += uy[k] * vs[a2];
            rs += ph[k] * ds[a2];
            rv += ph[k] * vs[a2];
          }
          fx += BC.v[q][b] * rx;
          fy += BC.v[q][b] * ry;
          fs += BC.v[q][b] * rs;
          ft += BC.d[q][b] * rv;
        }
        sum += BC.w[q] * (fx * fs + fy * ft);
      }
      acc[j] += sum;
    }
  }
  block_partials<K>(acc, lines.n, part);
}

}  // namespace pff
