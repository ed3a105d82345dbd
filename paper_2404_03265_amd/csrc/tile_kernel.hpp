// Cell-partition tile kernel for every cell-based operator of the solver.
//
// The tiles partition the cells (one block of cells of one refinement level
// per tile). One workgroup per tile, one thread per cell:
//   1. stage the tile's local nodes (private range, then shared list) into
//      LDS, masking constrained columns;
//   2. each thread gathers its cell's nodal values from LDS, applies the
//      hanging-node interpolation, runs the sum-factorised pointwise law,
//      integrates and applies the transposed hanging-node map;
//   3. accumulation into LDS accumulators over all local nodes with
//      no-return LDS atomic adds, in colour phases (cells of one colour share
//      no node) when the tile spans several waves or uses substituted
//      footprints, in one phase for one-wave tiles (one lane's k-th node is
//      never another lane's k-th node, and a wave's LDS operations execute in
//      program order): the summation order is fixed either way;
//   4. private nodes are complete and go through the mode's epilogue in one
//      coalesced write; shared nodes leave a partial sum in the tile's slots,
//      which shared_fixup adds in ascending tile order before the epilogue.
// Every cell is evaluated exactly once and every output written once.
#pragma once

#include "cell.hpp"
#include "mesh.hpp"

namespace pff {

enum Mode : int {
  MODE_J = 0,      // leaf Jacobian (Sec. 3.1), identity on constrained rows
  MODE_JT,         // its transpose
  MODE_LEVEL,      // level block operator diag(G_uu, G_phiphi) (Sec. 3.2)
  MODE_RESID,      // leaf residual R = -F(U) condensed (Problem 2)
  MODE_DIAG_LEAF,  // inverse diagonal of the leaf operator
  MODE_DIAG_LEVEL, // inverse diagonal of a level operator
  MODE_TCVGRAD,    // d TCV / dU (Sec. 4)
  MODE_DGC,        // dF/dGc
  MODE_DE,         // dF/dE
  MODE_DP,         // dF/dp
  MODE_MASS,       // lumped phase-field mass (row sums)
  MODE_LEVEL_COEF, // state coefficients of a level operator at its Gauss points
};

// EPI_CHEB_FIRST: the first two Chebyshev updates from x = 0 in one pass: the
// operand x = d_0 = c0 D^-1 b is formed while staging (never stored), then the
// EPI_CHEB update with d_old = d_0.
// EPI_PHI (level operator): the phase-field rows alone, from the phase-field
// operand alone (the block operator has no coupling); the displacement rows
// of dst are not written.
enum Epi : int { EPI_PLAIN = 0, EPI_RESID = 1, EPI_CHEB = 2, EPI_CHEB_FIRST = 3, EPI_PHI = 4 };

template <typename T>
struct TileArgs {
  int tile_base;               // this launch handles tiles tile_base + [0, n_grid)
  int n_grid;                  // = gridDim.x, beside tile_base and tile_info so that one scalar
                               // load brings all three
  const int32_t* tile_info;
  const int32_t* shared;       // global ids of the tiles' shared local nodes
  const uint16_t* cell_loc;       // own nodes per cell (hanging nodes included)
  const uint16_t* cell_loc_sub;   // hanging faces replaced by the coarse face's nodes
  const uint16_t* cell_info;
  // hanging nodes per tile: (node, masters) local ids, weights, colour
  const uint16_t* hang_rec;
  const double* hang_w;
  const uint8_t* hang_col;
  const uint8_t* flags;
  int64_t n;
  int max_local;
  // shared nodes: partial sums, [3][n_slots], tile-major; the slots of
  // shared node s are sh_tab[s * sh_w ..], ascending tile order, padded
  // with -1 (sh_w = SHARED_SLOTS unless a node touches more tiles)
  T* part;
  int64_t n_slots;
  int64_t n_private;
  int64_t n_shared;
  const int32_t* sh_tab;
  int sh_w;
  T H0;             // cell edge on level 0; level l has H0 / 2^l
  Material mat;
  const T* src;      // 3n input (operand / state U)
  const T* st[4];    // state fields: leaf (ux, uy, phi, phit); level (ux, uy, phit: inverse diagonal, coefficients)
  T* dst;            // 3n output
  // level epilogues
  const T* b;        // right-hand side (EPI_RESID, EPI_CHEB)
  const T* dold;     // previous Chebyshev direction (nullable)
  const T* dinv;     // inverse diagonal
  T* xnew;
  T c1[2], c2[2];    // Chebyshev coefficients per block (u, phi)
  T c0[2];           // EPI_CHEB_FIRST: coefficient of the first update d_0 = c0 D^-1 b
  // level operator state coefficients per cell record (MODE_LEVEL reads,
  // MODE_LEVEL_COEF writes): [2 (p+1)^2][n_coef], g at the Gauss points,
  // then H^2 c1 (see level_coefs)
  T* coef;
  int64_t n_coef;
};

// Element i of a device array addressed as a uniform base plus a 32-bit
// byte offset (the scalar-base form of the global loads and stores): one
// 32-bit register per node serves every field of the node, where a 64-bit
// address per load would hold two. Arrays of at most 2^29 elements of 8
// bytes (the host checks the node count).
template <typename T>
__device__ __forceinline__ const T& at32(const T* base, uint32_t i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + uint64_t(i * uint32_t(sizeof(T))));
}
template <typename T>
__device__ __forceinline__ T& at32(T* base, uint32_t i) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + uint64_t(i * uint32_t(sizeof(T))));
}

template <int MODE>
struct ModeTraits {
  static constexpr bool leaf = !(MODE == MODE_LEVEL || MODE == MODE_DIAG_LEVEL || MODE == MODE_LEVEL_COEF);
  static constexpr int n_src = (MODE == MODE_J || MODE == MODE_JT || MODE == MODE_LEVEL) ? 3
                               : (MODE == MODE_RESID || MODE == MODE_TCVGRAD || MODE == MODE_DGC ||
                                  MODE == MODE_DE || MODE == MODE_DP) ? 3 : 0;
  // state fields staged besides src (the level operator reads its state
  // through the per-cell coefficients of MODE_LEVEL_COEF instead)
  static constexpr int n_state = (MODE == MODE_J || MODE == MODE_JT || MODE == MODE_DIAG_LEAF) ? 4
                                 : (MODE == MODE_DIAG_LEVEL || MODE == MODE_LEVEL_COEF) ? 3
                                 : (MODE == MODE_RESID || MODE == MODE_DGC || MODE == MODE_DE || MODE == MODE_DP) ? 1
                                 : 0;
  // src columns are masked (constrained columns of the operator)
  static constexpr bool mask_src = (MODE == MODE_J || MODE == MODE_JT || MODE == MODE_LEVEL);
};

// Output of one node component: private nodes in the tile kernel, shared
// nodes in shared_fixup. v is the accumulated cell sum of row i = c n + g.
// With EARLY (private nodes of the tile kernel), the identity rows of the
// Jacobian modes were already written while staging and are skipped here.
template <int MODE, int EPI, bool EARLY, typename T>
__device__ __forceinline__ void node_epilogue(const TileArgs<T>& a, int c, int64_t g, uint8_t f, T v) {
  const int64_t i = c * a.n + g;
  if constexpr (MODE == MODE_J || MODE == MODE_JT) {
    const bool cons = (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
    if (EARLY) {
      if (!cons) a.dst[i] = v;
    } else {
      a.dst[i] = cons ? a.src[i] : v;
    }
  } else if constexpr (MODE == MODE_LEVEL) {
    if constexpr (EPI == EPI_PLAIN || EPI == EPI_PHI) {
      a.dst[i] = v;
    } else if constexpr (EPI == EPI_RESID) {
      // residual to restrict: zero on rows held at zero on this level
      const bool held = (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
      a.dst[i] = held ? T(0) : a.b[i] - v;
    } else {
      const bool fixed = (c < 2) ? (f & (NODE_DIRICHLET | NODE_EDGE | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_EDGE | NODE_HANGING));
      const int blk = c < 2 ? 0 : 1;
      T x, dp;
      if constexpr (EPI == EPI_CHEB_FIRST) {
        x = a.c0[blk] * a.dinv[i] * a.b[i];
        dp = x;
      } else {
        x = a.src[i];
        dp = a.dold ? a.dold[i] : T(0);
      }
      if (fixed) {
        a.dst[i] = T(0);
        a.xnew[i] = x;
      } else {
        const T r = a.b[i] - v;
        const T dn = a.c1[blk] * dp + a.c2[blk] * a.dinv[i] * r;
        a.dst[i] = dn;
        a.xnew[i] = x + dn;
      }
    }
  } else if constexpr (MODE == MODE_RESID) {
    a.dst[i] = (f & NODE_HANGING) ? T(0) : -v;
  } else if constexpr (MODE == MODE_DIAG_LEAF) {
    const bool cons = (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
    a.dst[i] = cons ? T(1) : T(1) / v;
  } else if constexpr (MODE == MODE_DIAG_LEVEL) {
    const bool fixed = (c < 2) ? (f & (NODE_DIRICHLET | NODE_EDGE | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_EDGE | NODE_HANGING));
    a.dst[i] = fixed ? T(0) : T(1) / v;
  } else {
    a.dst[i] = (f & NODE_HANGING) ? T(0) : v;
  }
}

// One cell of the Jacobian: gather(f, u) fetches the cell's nodal values of
// field f (0..2 the operand, then the state fields: u_x, u_y, phi, phit), out
// receives the cell's contributions to its nodes.
template <int P, typename T, class Gather>
__device__ __forceinline__ void jacobian_cell(T H, T mu, T lam, T kap, T pr, T Gc, T ell,
                                              Gather&& gather, T (&out)[3][(P + 1) * (P + 1)]) {
  constexpr int N1 = P + 1, NL = N1 * N1, NQ = NL;
  // Jacobian (Sec. 3.1) in reference units (gradients of the unit square,
  // Gauss weights in the integration tables); with e^, sigma^ the
  // reference strain and stress (e = e^ / H):
  //   u rows:   g(phit) sigma^(du) : grad^ psi
  //   phi rows: [H^2 c1 dphi + H B : e(du)] psi + Gc l grad^ dphi . grad^ psi
  //   H^2 c1 = (1-k) S^ + 2 p H tr e^ + H^2 Gc/l,
  //   H B    = 2 (1-k) phi sigma^(u) + 2 p H phi I   (the coupling G_phi,u)
  // The level block operator diag(G_uu, G_phiphi) (Sec. 3.2) is the same
  // without the coupling term (level_coefs, level_cell).
  constexpr int FUX = 3, FUY = 4, FPHI = 5, FPT = 6;
  const T twopH = T(2) * pr * H, gcl2 = H * H * Gc / ell, gcell = Gc * ell;
  T c1[NQ], bxx[NQ], byy[NQ], bxy[NQ];
  {
    T u[NL], sx1[NQ], sy1[NQ], sx2[NQ], sy2[NQ];
    gather(FUX, u);
    interp_g<P, T>(u, sx1, sy1);
    gather(FUY, u);
    interp_g<P, T>(u, sx2, sy2);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const T exx = sx1[q], eyy = sy2[q], exy = T(0.5) * (sy1[q] + sx2[q]);
      const T tr = exx + eyy;
      const T sxx = T(2) * mu * exx + lam * tr, syy = T(2) * mu * eyy + lam * tr, sxy = T(2) * mu * exy;
      const T S = sxx * exx + syy * eyy + T(2) * sxy * exy;
      c1[q] = (T(1) - kap) * S + twopH * tr + gcl2;
      bxx[q] = sxx;
      byy[q] = syy;
      bxy[q] = sxy;
    }
  }
  {
    T u[NL], pq[NQ];
    gather(FPHI, u);
    interp_v<P, T>(u, pq);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const T f = T(2) * (T(1) - kap) * pq[q], t = twopH * pq[q];
      bxx[q] = f * bxx[q] + t;
      byy[q] = f * byy[q] + t;
      bxy[q] = f * bxy[q];
    }
  }
  T dxx[NQ], dxy[NQ], dyx[NQ], dyy[NQ], be[NQ];
  {
    T u[NL];
    gather(0, u);
    interp_g<P, T>(u, dxx, dxy);
    gather(1, u);
    interp_g<P, T>(u, dyx, dyy);
#pragma unroll
    for (int q = 0; q < NQ; ++q) be[q] = bxx[q] * dxx[q] + byy[q] * dyy[q] + bxy[q] * (dxy[q] + dyx[q]);
  }
  {
    T u[NL], tq[NQ];
    gather(FPT, u);
    interp_v<P, T>(u, tq);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const T gq = (T(1) - kap) * tq[q] * tq[q] + kap;
      const T exx = dxx[q], eyy = dyy[q], exy2 = dxy[q] + dyx[q];
      const T tr = exx + eyy;
      const T sxx = T(2) * mu * exx + lam * tr, syy = T(2) * mu * eyy + lam * tr, sxy = mu * exy2;
      dxx[q] = gq * sxx;
      dxy[q] = gq * sxy;
      dyx[q] = gq * sxy;
      dyy[q] = gq * syy;
    }
  }
  integrate_gw<P, T>(dxx, dxy, out[0]);
  integrate_gw<P, T>(dyx, dyy, out[1]);
  {
    T u[NL], pv[NQ], px[NQ], py[NQ];
    gather(2, u);
    interp_vg<P, T>(u, pv, px, py);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      pv[q] = c1[q] * pv[q] + be[q];
      px[q] = gcell * px[q];
      py[q] = gcell * py[q];
    }
    integrate_w<P, T>(pv, px, py, out[2]);
  }
}

// State coefficients of the level block operator at the Gauss points of one
// cell, in the reference units of jacobian_cell (fields: 0, 1 the state
// u_x, u_y; 2 phit):
//   g = (1-k) phit^2 + k,   H^2 c1 = (1-k) S^ + 2 p H tr e^ + H^2 Gc/l.
// The level state is fixed for a multigrid set-up, so they are evaluated
// once per set-up (MODE_LEVEL_COEF) rather than in every application.
template <int P, typename T, class Gather>
__device__ __forceinline__ void level_coefs(T H, T mu, T lam, T kap, T pr, T Gc, T ell,
                                            Gather&& gather, T (&g)[(P + 1) * (P + 1)],
                                            T (&c1)[(P + 1) * (P + 1)]) {
  constexpr int NL = (P + 1) * (P + 1), NQ = NL;
  const T twopH = T(2) * pr * H, gcl2 = H * H * Gc / ell;
  {
    T u[NL], sx1[NQ], sy1[NQ], sx2[NQ], sy2[NQ];
    gather(0, u);
    interp_g<P, T>(u, sx1, sy1);
    gather(1, u);
    interp_g<P, T>(u, sx2, sy2);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const T exx = sx1[q], eyy = sy2[q], exy = T(0.5) * (sy1[q] + sx2[q]);
      const T tr = exx + eyy;
      const T sxx = T(2) * mu * exx + lam * tr, syy = T(2) * mu * eyy + lam * tr, sxy = T(2) * mu * exy;
      const T S = sxx * exx + syy * eyy + T(2) * sxy * exy;
      c1[q] = (T(1) - kap) * S + twopH * tr + gcl2;
    }
  }
  T u[NL], tq[NQ];
  gather(2, u);
  interp_v<P, T>(u, tq);
#pragma unroll
  for (int q = 0; q < NQ; ++q) g[q] = (T(1) - kap) * tq[q] * tq[q] + kap;
}

// The phase-field rows of the level block operator (level_cell): gather(0, u)
// fetches the phase-field operand, c1 holds H^2 c1 at the Gauss points.
template <int P, typename T, class Gather>
__device__ __forceinline__ void level_cell_phi(T gcell, const T (&c1)[(P + 1) * (P + 1)],
                                               Gather&& gather, T (&out)[(P + 1) * (P + 1)]) {
  constexpr int NL = (P + 1) * (P + 1), NQ = NL;
  T u[NL], pv[NQ], px[NQ], py[NQ];
  gather(0, u);
  interp_vg<P, T>(u, pv, px, py);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    pv[q] = c1[q] * pv[q];
    px[q] = gcell * px[q];
    py[q] = gcell * py[q];
  }
  integrate_w<P, T>(pv, px, py, out);
}

// One cell of the level block operator diag(G_uu, G_phiphi) (Sec. 3.2) from
// its state coefficients (level_coefs); gather(f, u), f = 0..2, fetches the
// operand. The same arithmetic as jacobian_cell without the coupling.
// level_cell_u: the displacement rows (ox, oy) from g.
template <int P, typename T, class Gather>
__device__ __forceinline__ void level_cell_u(T mu, T lam, const T (&g)[(P + 1) * (P + 1)],
                                             Gather&& gather, T (&ox)[(P + 1) * (P + 1)],
                                             T (&oy)[(P + 1) * (P + 1)]) {
  constexpr int NL = (P + 1) * (P + 1), NQ = NL;
  T u[NL], dxx[NQ], dxy[NQ], dyx[NQ], dyy[NQ];
  gather(0, u);
  interp_g<P, T>(u, dxx, dxy);
  gather(1, u);
  interp_g<P, T>(u, dyx, dyy);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const T gq = g[q];
    const T exx = dxx[q], eyy = dyy[q], exy2 = dxy[q] + dyx[q];
    const T tr = exx + eyy;
    const T sxx = T(2) * mu * exx + lam * tr, syy = T(2) * mu * eyy + lam * tr, sxy = mu * exy2;
    dxx[q] = gq * sxx;
    dxy[q] = gq * sxy;
    dyx[q] = gq * sxy;
    dyy[q] = gq * syy;
  }
  integrate_gw<P, T>(dxx, dxy, ox);
  integrate_gw<P, T>(dyx, dyy, oy);
}

template <int P, typename T, class Gather>
__device__ __forceinline__ void level_cell(T mu, T lam, T gcell, const T (&g)[(P + 1) * (P + 1)],
                                           const T (&c1)[(P + 1) * (P + 1)], Gather&& gather,
                                           T (&out)[3][(P + 1) * (P + 1)]) {
  constexpr int NL = (P + 1) * (P + 1);
  level_cell_u<P, T>(mu, lam, g, gather, out[0], out[1]);
  level_cell_phi<P, T>(gcell, c1, [&](int, T(&u)[NL]) { gather(2, u); }, out[2]);
}

// One cell of the transposed Jacobian, in the reference units of
// jacobian_cell: the coupling block G_phi,u moves from the phi rows to the u
// rows, weighted by the phase-field operand,
//   u rows:   [g(phit) sigma^(du) + dphi H B] : grad^ psi
//   phi rows: H^2 c1 dphi psi + Gc l grad^ dphi . grad^ psi
// (same fields and the same H B, c1 as the forward routine). The order keeps
// few values live: state coefficients, then the phase-field rows (whose
// operand scales H B in place), then the displacement rows.
template <int P, typename T, class Gather>
__device__ __forceinline__ void jacobian_t_cell(T H, T mu, T lam, T kap, T pr, T Gc, T ell,
                                                Gather&& gather, T (&out)[3][(P + 1) * (P + 1)]) {
  constexpr int N1 = P + 1, NL = N1 * N1, NQ = NL;
  constexpr int FUX = 3, FUY = 4, FPHI = 5, FPT = 6;
  const T twopH = T(2) * pr * H, gcl2 = H * H * Gc / ell, gcell = Gc * ell;
  T bxx[NQ], byy[NQ], bxy[NQ];
  {
    T c1[NQ];
    {
      T u[NL], sx1[NQ], sy1[NQ], sx2[NQ], sy2[NQ];
      gather(FUX, u);
      interp_g<P, T>(u, sx1, sy1);
      gather(FUY, u);
      interp_g<P, T>(u, sx2, sy2);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const T exx = sx1[q], eyy = sy2[q], exy = T(0.5) * (sy1[q] + sx2[q]);
        const T tr = exx + eyy;
        const T sxx = T(2) * mu * exx + lam * tr, syy = T(2) * mu * eyy + lam * tr, sxy = T(2) * mu * exy;
        const T S = sxx * exx + syy * eyy + T(2) * sxy * exy;
        c1[q] = (T(1) - kap) * S + twopH * tr + gcl2;
        bxx[q] = sxx;
        byy[q] = syy;
        bxy[q] = sxy;
      }
    }
    {
      T u[NL], pq[NQ];
      gather(FPHI, u);
      interp_v<P, T>(u, pq);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const T f = T(2) * (T(1) - kap) * pq[q], t = twopH * pq[q];
        bxx[q] = f * bxx[q] + t;
        byy[q] = f * byy[q] + t;
        bxy[q] = f * bxy[q];
      }
    }
    // phi rows; the operand dphi then scales H B for the u rows
    T u[NL], pv[NQ], px[NQ], py[NQ];
    gather(2, u);
    interp_vg<P, T>(u, pv, px, py);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      bxx[q] *= pv[q];
      byy[q] *= pv[q];
      bxy[q] *= pv[q];
      pv[q] = c1[q] * pv[q];
      px[q] = gcell * px[q];
      py[q] = gcell * py[q];
    }
    integrate_w<P, T>(pv, px, py, out[2]);
  }
  T dxx[NQ], dxy[NQ], dyx[NQ], dyy[NQ];
  {
    T u[NL];
    gather(0, u);
    interp_g<P, T>(u, dxx, dxy);
    gather(1, u);
    interp_g<P, T>(u, dyx, dyy);
  }
  {
    T u[NL], tq[NQ];
    gather(FPT, u);
    interp_v<P, T>(u, tq);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const T gq = (T(1) - kap) * tq[q] * tq[q] + kap;
      const T exx = dxx[q], eyy = dyy[q], exy2 = dxy[q] + dyx[q];
      const T tr = exx + eyy;
      const T sxx = T(2) * mu * exx + lam * tr, syy = T(2) * mu * eyy + lam * tr, sxy = mu * exy2;
      dxx[q] = gq * sxx + bxx[q];
      dxy[q] = gq * sxy + bxy[q];
      dyx[q] = gq * sxy + bxy[q];
      dyy[q] = gq * syy + byy[q];
    }
  }
  integrate_gw<P, T>(dxx, dxy, out[0]);
  integrate_gw<P, T>(dyx, dyy, out[1]);
}

// One cell of an operator mode: gather(f, u) fetches the cell's nodal values
// of staged field f, out receives the cell's contributions to its (p+1)^2
// nodes (per component). H: the cell edge; hang: the per-cell constraint form
// of the inverse diagonal.
template <int P, typename T, int MODE, class Gather>
__device__ __forceinline__ void compute_cell(const TileArgs<T>& a, T H, bool hang, unsigned info, Gather&& gather,
                                             T (&out)[3][(P + 1) * (P + 1)]) {
  constexpr int N1 = P + 1, NL = N1 * N1, NQ = NL;
  using TR = ModeTraits<MODE>;
  const Material& m = a.mat;
  const T kap = T(m.kappa), pr = T(m.pressure), Gc = T(m.Gc), ell = T(m.ell);
  const T mu = T(m.mu), lam = T(m.lam);
  (void)info;
  (void)hang;
  constexpr Basis<T> BW = basis_table<P, T>();
  T wq[NQ];
#pragma unroll
  for (int qy = 0; qy < N1; ++qy)
#pragma unroll
    for (int qx = 0; qx < N1; ++qx) wq[qy * N1 + qx] = BW.w[qx] * BW.w[qy];
  const T invH = T(1) / H;

  if constexpr (MODE == MODE_J) {
    jacobian_cell<P, T>(H, mu, lam, kap, pr, Gc, ell, gather, out);
  } else if constexpr (MODE == MODE_JT) {
    jacobian_t_cell<P, T>(H, mu, lam, kap, pr, Gc, ell, gather, out);
  } else if constexpr (MODE == MODE_DIAG_LEAF || MODE == MODE_DIAG_LEVEL) {
    // state-derived coefficients at the Gauss points:
    //   g = (1-k) phit^2 + k, c1 = (1-k) S + 2 p tr e(u) + Gc/l
    // (the leaf stages u_x, u_y, phi, phit; a level u_x, u_y, phit)
    constexpr int SU = TR::n_src;
    constexpr int FPT = SU + (TR::leaf ? 3 : 2);
    T cg[NQ], cc1[NQ];
    {
      T u[NL], gx1[NQ], gy1[NQ], gx2[NQ], gy2[NQ], tq[NQ];
      gather(SU + 0, u);
      interp_g<P, T>(u, gx1, gy1);
      gather(SU + 1, u);
      interp_g<P, T>(u, gx2, gy2);
      gather(FPT, u);
      interp_v<P, T>(u, tq);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const T exx = gx1[q] * invH, eyy = gy2[q] * invH, exy = T(0.5) * (gy1[q] + gx2[q]) * invH;
        const T tr = exx + eyy;
        const T sxx = T(2) * mu * exx + lam * tr, syy = T(2) * mu * eyy + lam * tr, sxy = T(2) * mu * exy;
        const T S = sxx * exx + syy * eyy + T(2) * sxy * exy;
        cg[q] = (T(1) - kap) * tq[q] * tq[q] + kap;
        cc1[q] = (T(1) - kap) * S + T(2) * pr * tr + Gc / ell;
      }
    }
    // diagonal of the block-diagonal part for each local master dof:
    // interpolate the (hanging-mapped) unit vector and evaluate the forms
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      T u[NL], vq[NQ], gxq[NQ], gyq[NQ];
#pragma unroll
      for (int j = 0; j < NL; ++j) u[j] = (j == k) ? T(1) : T(0);
      if (hang) hang_apply<P, T>(u, info);
      interp_vg<P, T>(u, vq, gxq, gyq);
      T dux = T(0), duy = T(0), dph = T(0);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const T gx = gxq[q] * invH, gy = gyq[q] * invH, JxW = H * H * wq[q];
        dux += JxW * cg[q] * ((T(2) * mu + lam) * gx * gx + mu * gy * gy);
        duy += JxW * cg[q] * (mu * gx * gx + (T(2) * mu + lam) * gy * gy);
        dph += JxW * (cc1[q] * vq[q] * vq[q] + Gc * ell * (gx * gx + gy * gy));
      }
      out[0][k] = dux;
      out[1][k] = duy;
      out[2][k] = dph;
    }
  } else if constexpr (MODE == MODE_RESID || MODE == MODE_DGC || MODE == MODE_DE || MODE == MODE_DP) {
    // residual F(U) of Problem 2 (phi~ in degradation and u-pressure):
    //   u rows:   g(phit) sigma(u) : e(psi) + p phit^2 div psi
    //   phi rows: (1-k) phi S + 2 p phi tr e(u) - (Gc/l)(1 - phi), Gc l grad phi
    // the parameter derivatives keep the terms linear in Gc, E or p.
    T gx1[NQ], gy1[NQ], gx2[NQ], gy2[NQ], pv[NQ], px[NQ], py[NQ], tq[NQ];
    {
      T u[NL];
      gather(0, u);
      interp_g<P, T>(u, gx1, gy1);
      gather(1, u);
      interp_g<P, T>(u, gx2, gy2);
      gather(2, u);
      interp_vg<P, T>(u, pv, px, py);
      gather(3, u);
      interp_v<P, T>(u, tq);
    }
    constexpr T sig = (MODE == MODE_RESID || MODE == MODE_DE) ? T(1) : T(0);
    const T spr = (MODE == MODE_RESID) ? pr : (MODE == MODE_DP ? T(1) : T(0));
    const T sgc = (MODE == MODE_RESID) ? Gc : (MODE == MODE_DGC ? T(1) : T(0));
    const T invE = (MODE == MODE_DE) ? T(1.0 / m.E) : T(1);   // sigma is linear in E at fixed nu
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const T exx = gx1[q] * invH, eyy = gy2[q] * invH, exy = T(0.5) * (gy1[q] + gx2[q]) * invH;
      const T tr = exx + eyy;
      const T sxx = T(2) * mu * exx + lam * tr, syy = T(2) * mu * eyy + lam * tr, sxy = T(2) * mu * exy;
      const T S = sxx * exx + syy * eyy + T(2) * sxy * exy;
      const T g = (T(1) - kap) * tq[q] * tq[q] + kap;
      const T ph = pv[q];
      const T wg = H * wq[q], wv = H * H * wq[q];
      const T pt2 = spr * tq[q] * tq[q];
      gx1[q] = wg * (sig * invE * g * sxx + pt2);
      gy1[q] = wg * (sig * invE * g * sxy);
      gx2[q] = wg * (sig * invE * g * sxy);
      gy2[q] = wg * (sig * invE * g * syy + pt2);
      pv[q] = wv * (sig * invE * (T(1) - kap) * ph * S + spr * T(2) * ph * tr - sgc / ell * (T(1) - ph));
      px[q] = wq[q] * sgc * ell * px[q];
      py[q] = wq[q] * sgc * ell * py[q];
    }
    integrate_g<P, T>(gx1, gy1, out[0]);
    integrate_g<P, T>(gx2, gy2, out[1]);
    integrate<P, T>(pv, px, py, out[2]);
  } else if constexpr (MODE == MODE_TCVGRAD) {
    // TCV = int u . grad phi; derivative: (v . grad phi) for u, (u . grad psi) for phi
    T vx[NQ], vy[NQ], px[NQ], py[NQ], zero[NQ];
    {
      T u[NL], d1[NQ], d2[NQ];
      gather(0, u);
      interp_v<P, T>(u, vx);
      gather(1, u);
      interp_v<P, T>(u, vy);
      gather(2, u);
      interp_g<P, T>(u, px, py);
      (void)d1;
      (void)d2;
    }
    T f0[NQ], f1[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      zero[q] = T(0);
      const T wv = H * H * wq[q], wg = H * wq[q];
      f0[q] = wv * px[q] * invH;
      f1[q] = wv * py[q] * invH;
      px[q] = wg * vx[q];
      py[q] = wg * vy[q];
    }
    integrate<P, T>(f0, zero, zero, out[0]);
    integrate<P, T>(f1, zero, zero, out[1]);
    integrate<P, T>(zero, px, py, out[2]);
  } else if constexpr (MODE == MODE_MASS) {
    T f[NQ], zero[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      f[q] = H * H * wq[q];
      zero[q] = T(0);
    }
    integrate<P, T>(f, zero, zero, out[2]);
  }
}

// FIXED: the launch uses the default tile's block (64 threads for Q2, 256
// for Q1), known at compile time: reading blockDim.x would cost every
// workgroup a vector load of the dispatch packet ahead of its node loads.
template <int P, typename T, int MODE, int EPI, bool HANG, bool FIXED>
__global__ void __launch_bounds__(256) tile_kernel(const TileArgs<T> a) {
  constexpr int N1 = P + 1, NL = N1 * N1, NQ = NL;
  using TR = ModeTraits<MODE>;
  // EPI_PHI stages the phase-field operand alone (field 0 is component 2)
  constexpr bool PHI = MODE == MODE_LEVEL && EPI == EPI_PHI;
  constexpr int NF = PHI ? 1 : TR::n_src + TR::n_state;
  constexpr int C0 = PHI ? 2 : 0;   // first output component
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ML = a.max_local;
  using LT = double;   // LDS values (FP64 for both precisions)
  LT* lds = reinterpret_cast<LT*>(smem_raw);   // staged fields [NF][max_local]
  // the accumulators [3][max_local] reuse the first three field arrays once
  // every cell has gathered its values (one LDS region of max(NF, 3) arrays
  // keeps the footprint per tile, and so the tiles per CU, at its minimum)
  LT* acc = lds;
  uint8_t* lflag = reinterpret_cast<uint8_t*>(lds + (NF > 3 ? NF : 3) * ML);     // [max_local]

  // XCD-aware order: workgroups go to the 8 XCDs round-robin, so XCD x
  // receives a contiguous chunk of the tile list and neighbouring tiles (which
  // share nodes) run on the same XCD and hit the same L2.
  const int nb = a.n_grid, bid = int(blockIdx.x);
  const int xq = nb >> 3, xr = nb & 7, xcd = bid & 7;
  const int order_idx = xcd * xq + (xcd < xr ? xcd : xr) + (bid >> 3);
  const int tile = a.tile_base + order_idx;
  // the whole tile header goes into scalar registers in one batch of loads;
  // reading it field by field under the branches below would serialise a
  // scalar-load round trip per run. The empty asm statements take every
  // word, so that the compiler cannot sink a word's load into the branch
  // that first uses it.
  int ti[TILE_STRIDE];
  {
    const int32_t* tp = a.tile_info + TILE_STRIDE * tile;
#pragma unroll
    for (int k = 0; k < TILE_STRIDE; ++k) ti[k] = tp[k];
#pragma unroll
    for (int k = 0; k < TILE_STRIDE; ++k) asm volatile("" ::"s"(ti[k]));
  }
  const int o0 = ti[TILE_OWNED0], no = ti[TILE_NOWNED];
  const int s0 = ti[TILE_SHARED0], ns = ti[TILE_NSHARED];
  const int c0 = ti[TILE_CELL0], nc = ti[TILE_NCELL];
  const int ncol = ti[TILE_NCOLOR];
  const int slot0 = ti[TILE_SLOT0];
  const int nrun = ti[TILE_NRUN];
  // global id of shared entry r from the runs of consecutive ids in the tile
  // header (no dependent lookup); tiles with more runs use the shared list
  auto run_id = [&](int r) -> int64_t {
    int id = ti[TILE_RUN_START] + r;
#pragma unroll
    for (int k = 1; k < TILE_MAX_RUNS; ++k)
      if (k < nrun && r >= ti[TILE_RUN_OFF + k]) id = ti[TILE_RUN_START + k] + (r - ti[TILE_RUN_OFF + k]);
    return id;
  };
  // Hanging nodes: every mode but the inverse diagonal applies the
  // constraints on the tile's nodes (interpolate after staging, distribute
  // after accumulation); the inverse diagonal needs the per-cell form.
  // (the level operator too: the levels of global-coarsening multigrid have
  // hanging nodes; local-smoothing levels have no records, nhang = 0)
  constexpr bool NODE_HANG = (TR::leaf && MODE != MODE_DIAG_LEAF) || MODE == MODE_LEVEL || MODE == MODE_LEVEL_COEF;
  const int hr0 = NODE_HANG ? ti[TILE_HANG0] : 0, nhang = NODE_HANG ? ti[TILE_NHANG] : 0;
  const int nhcol = NODE_HANG ? ti[TILE_NHCOLOR] : 0;
  const int nloc = no + ns;
  const int64_t n = a.n;
  const Material& m = a.mat;
  const T kap = T(m.kappa), pr = T(m.pressure), Gc = T(m.Gc), ell = T(m.ell);
  const T mu = T(m.mu), lam = T(m.lam);

  const int cell = int(threadIdx.x);
  const bool live = cell < nc;
  int loc[NL];
  unsigned info = 0;
  // level operator: the cell's state coefficients (g, then H^2 c1)
  constexpr int NCF = MODE == MODE_LEVEL ? (PHI ? NQ : 2 * NQ) : 1;
  T cf[NCF];
  // the cell record is requested after the first round's node loads (see
  // below): its latency overlaps theirs instead of preceding them
  auto load_cell_record = [&]() {
    if (live) {
      const int64_t rec = int64_t(c0) + cell;
      const uint16_t* cl = (MODE == MODE_DIAG_LEAF || MODE == MODE_DIAG_LEVEL) ? a.cell_loc_sub : a.cell_loc;
#pragma unroll
      for (int k = 0; k < NL; ++k) loc[k] = cl[rec * NL + k];
      info = a.cell_info[rec];
      if constexpr (MODE == MODE_LEVEL) {
        // EPI_PHI: H^2 c1 alone
#pragma unroll
        for (int k = 0; k < NCF; ++k) cf[k] = a.coef[((PHI ? NQ : 0) + k) * a.n_coef + rec];
      }
    }
  };

  // 1. stage local nodes. Per round: the shared ids (from the header runs,
  //    else the list), then every node load of the round as one batch, the
  //    cell record in the first round, and one LDS store pass at the end, so
  //    that a tile waits for memory about once. The Jacobian modes write
  //    their identity rows (constrained private nodes) here, from the raw
  //    values.
  constexpr bool JMODE = (MODE == MODE_J || MODE == MODE_JT);
  // private / shared nodes per thread and round, sized for the default tiles
  // (Q1: 16 x 16 cells on four waves, Q2: 8 x 8 cells on one wave) so that
  // one round covers a tile without many idle lanes
  constexpr int SP = P == 1 ? 1 : 4, SS = P == 1 ? 1 : 2;
  const int bs = FIXED ? (P == 1 ? 256 : 64) : int(blockDim.x), tid = int(threadIdx.x);
  // When one round covers the private range, each thread keeps what the
  // epilogue of its private rows needs in registers: the raw source values
  // (Jacobian identity rows, smoother iterate) and, for the level smoother
  // and residual, b, D^-1 and the previous update, requested here with the
  // node loads so that the epilogue issues no dependent load. The Jacobian
  // modes otherwise write their identity rows while staging.
  constexpr bool FIRST = MODE == MODE_LEVEL && EPI == EPI_CHEB_FIRST;
  constexpr bool CHEB = MODE == MODE_LEVEL && (EPI == EPI_CHEB || FIRST);
  constexpr bool LPRE = CHEB || (MODE == MODE_LEVEL && EPI == EPI_RESID);
  constexpr int NPRE = (JMODE || LPRE) ? SP : 1;
  const bool keep_raw = (JMODE || LPRE) && no <= SP * bs;
  T raw[NPRE][3], pb[LPRE ? SP : 1][3], pdi[CHEB ? SP : 1][3], pdo[CHEB ? SP : 1][3];
  // Requested after the first round's node loads and cell records: issued
  // before them, they would be waited for first (the shared ids of a tile
  // without runs come from a load whose register the other path writes,
  // and the compiler waits for every load in flight there).
  auto load_epilogue_inputs = [&]() {
    if constexpr (LPRE) {
#pragma unroll
      for (int k = 0; k < SP; ++k) {
        const uint32_t g = uint32_t(min(o0 + min(k * bs + tid, max(no - 1, 0)), int(n - 1)));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          pb[k][c] = at32(a.b + c * n, g);
          if constexpr (CHEB) {
            pdi[k][c] = at32(a.dinv + c * n, g);
            if constexpr (!FIRST) pdo[k][c] = a.dold ? at32(a.dold + c * n, g) : T(0);
          }
        }
      }
    }
  };
  bool first = true;
  for (int rp = 0, rs = 0; rp < no || rs < ns; rp += SP * bs, rs += SS * bs) {
    // shared ids before any load is in flight: with the list, the wait for
    // the ids then holds nothing else up
    // (out-of-range entries read node 0 and are discarded)
    uint32_t gsh[SS];
    if (nrun > 0) {
#pragma unroll
      for (int k = 0; k < SS; ++k) {
        const int r = rs + k * bs + tid;
        gsh[k] = r < ns ? uint32_t(run_id(r)) : 0u;
      }
    } else {
#pragma unroll
      for (int k = 0; k < SS; ++k) {
        const int r = rs + k * bs + tid;
        gsh[k] = r < ns ? uint32_t(a.shared[s0 + r]) : 0u;
      }
    }
    // loads without branches (out-of-range lanes read an in-range node and
    // discard it), so that they issue as one batch
    uint8_t fp_[SP], fsh[SS];
    T vp[SP][NF > 0 ? NF : 1], vsh[SS][NF > 0 ? NF : 1];
#pragma unroll
    for (int k = 0; k < SP; ++k) {
      const int l = rp + k * bs + tid;
      const uint32_t g = uint32_t(min(o0 + min(l, max(no - 1, 0)), int(n - 1)));
      fp_[k] = at32(a.flags, g);
      if constexpr (NF > 0) {
        if constexpr (FIRST) {
#pragma unroll
          for (int c = 0; c < 3; ++c) vp[k][c] = a.c0[c < 2 ? 0 : 1] * at32(a.dinv + c * n, g) * at32(a.b + c * n, g);
        } else if constexpr (PHI) {
          vp[k][0] = at32(a.src + 2 * n, g);
        } else if constexpr (TR::n_src > 0) {
#pragma unroll
          for (int c = 0; c < 3; ++c) vp[k][c] = at32(a.src + c * n, g);
        }
#pragma unroll
        for (int st = 0; st < TR::n_state; ++st) vp[k][TR::n_src + st] = at32(a.st[st], g);
      }
    }
#pragma unroll
    for (int k = 0; k < SS; ++k) {
      const uint32_t g = gsh[k];
      fsh[k] = at32(a.flags, g);
      if constexpr (NF > 0) {
        if constexpr (FIRST) {
#pragma unroll
          for (int c = 0; c < 3; ++c) vsh[k][c] = a.c0[c < 2 ? 0 : 1] * at32(a.dinv + c * n, g) * at32(a.b + c * n, g);
        } else if constexpr (PHI) {
          vsh[k][0] = at32(a.src + 2 * n, g);
        } else if constexpr (TR::n_src > 0) {
#pragma unroll
          for (int c = 0; c < 3; ++c) vsh[k][c] = at32(a.src + c * n, g);
        }
#pragma unroll
        for (int st = 0; st < TR::n_state; ++st) vsh[k][TR::n_src + st] = at32(a.st[st], g);
      }
    }
    if (first) {
      load_cell_record();
      load_epilogue_inputs();
    }
    first = false;
    auto put = [&](int l, uint8_t f, const T* v) {
      lflag[l] = f;
      if constexpr (NF > 0) {
#pragma unroll
        for (int c = 0; c < NF; ++c) {
          T x = v[c];
          if constexpr (TR::mask_src) {
            if (c < 3) {
              const bool fixed = (C0 + c < 2) ? (f & NODE_DIRICHLET) : (f & NODE_ACTIVE);
              if (fixed) x = T(0);
            }
          }
          lds[c * ML + l] = LT(x);
        }
      }
    };
#pragma unroll
    for (int k = 0; k < SP; ++k) {
      const int l = rp + k * bs + tid;
      if (l < no) {
        put(l, fp_[k], vp[k]);
        if constexpr (LPRE) {
#pragma unroll
          for (int c = 0; c < 3; ++c) raw[k][c] = vp[k][c];
        }
        if constexpr (JMODE) {
          const uint8_t f = fp_[k];
          const uint32_t g = uint32_t(o0 + l);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            raw[k][c] = vp[k][c];
            const bool cons = (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
            if (cons && !keep_raw) at32(a.dst + c * n, g) = vp[k][c];
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < SS; ++k) {
      const int r = rs + k * bs + tid;
      if (r < ns) put(no + r, fsh[k], vsh[k]);
    }
  }
  if (first) {
    load_cell_record();
    load_epilogue_inputs();
  }
  __syncthreads();
  if constexpr (NODE_HANG && NF > 0) {
    if (nhang > 0) {
      // values at hanging nodes from their masters (masters are never hanging)
      for (int r = threadIdx.x; r < nhang; r += bs) {
        const uint16_t* hr = a.hang_rec + 4 * int64_t(hr0 + r);
        const double* hw = a.hang_w + 3 * int64_t(hr0 + r);
        const int h = hr[0], m0 = hr[1], m1 = hr[2], m2 = hr[3];
        const T w0 = T(hw[0]), w1 = T(hw[1]), w2 = T(hw[2]);
#pragma unroll
        for (int f = 0; f < NF; ++f)
          lds[f * ML + h] = LT(w0 * T(lds[f * ML + m0]) + w1 * T(lds[f * ML + m1]) + w2 * T(lds[f * ML + m2]));
      }
      __syncthreads();
    }
  }

  if constexpr (MODE == MODE_LEVEL_COEF) {
    // the level state's coefficients of every cell; no accumulation
    if (live) {
      const int lev = int((info >> CELL_LEVEL_SHIFT) & 31u);
      const T H = T(ldexp(double(a.H0), -lev));
      auto gather = [&](int field, T(&u)[NL]) {
#pragma unroll
        for (int k = 0; k < NL; ++k) u[k] = T(lds[field * ML + loc[k]]);
      };
      T g[NQ], c1[NQ];
      level_coefs<P, T>(H, mu, lam, kap, pr, Gc, ell, gather, g, c1);
      const int64_t rec = int64_t(c0) + cell;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        a.coef[q * a.n_coef + rec] = g[q];
        a.coef[(NQ + q) * a.n_coef + rec] = c1[q];
      }
    }
    return;
  }

  // 2./3. one cell per thread, colour-phased accumulation
  {
    T out[3][NL];
    int color = -1;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < NL; ++k) out[c][k] = T(0);
    if (live) {
      color = int((info >> CELL_COLOR_SHIFT) & 15u);
      const int lev = int((info >> CELL_LEVEL_SHIFT) & 31u);
      const T H = T(ldexp(double(a.H0), -lev));
      // per-cell constraint form (inverse diagonal only)
      const bool hang = HANG && (MODE == MODE_DIAG_LEAF || MODE == MODE_DIAG_LEVEL) && (info & 15u);
      auto gather = [&](int field, T(&u)[NL]) {
#pragma unroll
        for (int k = 0; k < NL; ++k) u[k] = T(lds[field * ML + loc[k]]);
        if (hang) hang_apply<P, T>(u, info);
      };
      if constexpr (PHI) {
        T c1[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) c1[q] = cf[q];
        level_cell_phi<P, T>(Gc * ell, c1, gather, out[2]);
      } else if constexpr (MODE == MODE_LEVEL) {
        T g[NQ], c1[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          g[q] = cf[q];
          c1[q] = cf[NQ + q];
        }
        level_cell<P, T>(mu, lam, Gc * ell, g, c1, gather, out);
      } else {
        compute_cell<P, T, MODE>(a, H, hang, info, gather, out);
      }
    }
    // every gather is done: the accumulators take over the field arrays
    __syncthreads();
    for (int l = threadIdx.x; l < nloc; l += bs) {
#pragma unroll
      for (int c = C0; c < 3; ++c) acc[c * ML + l] = LT(0);
    }
    __syncthreads();
    // LDS atomic adds without return: no read-modify-write round trip per
    // entry. Within a phase no two lanes address the same node in one
    // instruction, and a wave's adds execute in program order, so the
    // summation order is fixed. A one-wave tile over the cells' own nodes
    // needs no colour phases: two distinct cells never have the same node at
    // the same local position.
    const bool one_phase = !HANG && bs <= 64;
    const int nphase = one_phase ? 1 : ncol;
    for (int col = 0; col < nphase; ++col) {
      if (live && (one_phase || color == col)) {
#pragma unroll
        for (int k = 0; k < NL; ++k) {
          const int l = loc[k];
#pragma unroll
          for (int c = C0; c < 3; ++c)
            __hip_atomic_fetch_add(&acc[c * ML + l], LT(out[c][k]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
      __syncthreads();
    }
  }
  if constexpr (NODE_HANG) {
    // contributions at hanging nodes go to their masters; records of one
    // colour share no master
    for (int col = 0; col < nhcol; ++col) {
      for (int r = threadIdx.x; r < nhang; r += bs) {
        if (a.hang_col[hr0 + r] != col) continue;
        const uint16_t* hr = a.hang_rec + 4 * int64_t(hr0 + r);
        const double* hw = a.hang_w + 3 * int64_t(hr0 + r);
        const int h = hr[0];
#pragma unroll
        for (int c = C0; c < 3; ++c) {
          const LT v = acc[c * ML + h];
#pragma unroll
          for (int k = 0; k <= P; ++k)
            __hip_atomic_fetch_add(&acc[c * ML + hr[1 + k]], LT(T(hw[k])) * v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
      __syncthreads();
    }
  }

  // 4. private nodes through the epilogue, shared nodes into the tile's slots
  if (keep_raw) {
#pragma unroll
    for (int k = 0; k < NPRE; ++k) {
      const int l = k * bs + int(threadIdx.x);
      if (l < no) {
        const uint8_t f = lflag[l];
        const uint32_t g = uint32_t(o0 + l);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T& di = at32(a.dst + c * n, g);
          const T v = T(acc[c * ML + l]);
          if constexpr (JMODE) {
            const bool cons = (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
            di = cons ? raw[k][c] : v;
          } else if constexpr (CHEB) {
            // the level smoother step, as in node_epilogue
            const bool fixed = (c < 2) ? (f & (NODE_DIRICHLET | NODE_EDGE | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_EDGE | NODE_HANGING));
            const int blk = c < 2 ? 0 : 1;
            const T x = raw[k][c];
            // (EPI_CHEB_FIRST: the previous update is d_0 = c0 D^-1 b)
            const T dold = FIRST ? a.c0[blk] * pdi[k][c] * pb[k][c] : pdo[k][c];
            const T dn = a.c1[blk] * dold + a.c2[blk] * pdi[k][c] * (pb[k][c] - v);
            di = fixed ? T(0) : dn;
            at32(a.xnew + c * n, g) = fixed ? x : x + dn;
          } else if constexpr (LPRE) {
            const bool held =
                (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
            di = held ? T(0) : pb[k][c] - v;
          }
        }
      }
    }
  } else {
    for (int l = threadIdx.x; l < no; l += bs) {
      const uint8_t f = lflag[l];
#pragma unroll
      for (int c = C0; c < 3; ++c) node_epilogue<MODE, EPI, true, T>(a, c, int64_t(o0) + l, f, T(acc[c * ML + l]));
    }
  }
  for (int r = threadIdx.x; r < ns; r += bs) {
#pragma unroll
    for (int c = C0; c < 3; ++c) at32(a.part + c * a.n_slots, uint32_t(slot0 + r)) = T(acc[c * ML + no + r]);
  }
}

// Shared nodes: add the partial sums of every tile touching the node in
// ascending tile order, then apply the mode's epilogue.
template <typename T, int MODE, int EPI>
__global__ void __launch_bounds__(256) shared_fixup(const TileArgs<T> a) {
  constexpr int C0 = (MODE == MODE_LEVEL && EPI == EPI_PHI) ? 2 : 0;
  constexpr bool JM = MODE == MODE_J || MODE == MODE_JT;
  constexpr bool LRES = MODE == MODE_LEVEL && EPI == EPI_RESID;
  constexpr bool LCHEB = MODE == MODE_LEVEL && (EPI == EPI_CHEB || EPI == EPI_CHEB_FIRST);
  const int64_t n = a.n;
  // launched with 256-thread blocks (a compile-time block size spares each
  // workgroup a load of the dispatch packet)
  for (int64_t s = int64_t(blockIdx.x) * 256 + threadIdx.x; s < a.n_shared; s += int64_t(gridDim.x) * 256) {
    const uint32_t g = uint32_t(a.n_private + s);
    // Every load that does not depend on another goes out first: the node
    // flag, the slot list and what the epilogue reads besides the sum; then
    // the partial sums of all slots (an unused slot reads slot 0 and is
    // dropped) and, on constrained rows of the Jacobian modes, the operand.
    // Two memory round trips per node, where a branch per slot and loads
    // inside the epilogue had made nine.
    // (the slot table has SHARED_SLOTS or more entries per node, so this
    // 16-byte read stays inside it whatever its width)
    const int4 sl = reinterpret_cast<const int4*>(a.sh_tab)[s];
    const uint8_t f = at32(a.flags, g);
    T eb[3], ed[3], ex[3], ep[3], es[3];
#pragma unroll
    for (int c = C0; c < 3; ++c) {
      if constexpr (LRES || LCHEB) eb[c] = at32(a.b + c * n, g);
      if constexpr (LCHEB) ed[c] = at32(a.dinv + c * n, g);
      if constexpr (MODE == MODE_LEVEL && EPI == EPI_CHEB) {
        ex[c] = at32(a.src + c * n, g);
        ep[c] = a.dold ? at32(a.dold + c * n, g) : T(0);
      }
    }
    if constexpr (JM) {
      // the operand on constrained rows (identity rows). Branch-free: the
      // other lanes read element 0 (one cached line), since a load under a
      // branch would make the compiler wait for every load before it
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const bool cons = (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
        es[c] = at32(a.src + c * n, cons ? g : 0u);
      }
    }
    // partial sums of the four slots, loaded without a branch (a load under
    // a branch is sunk there and waited for apart); with a wider slot table
    // (sh_w > SHARED_SLOTS, rare) they read in-range slots of other nodes and
    // the loop below sums the node's own
    const bool four = a.sh_w == SHARED_SLOTS;
    const int slot[SHARED_SLOTS] = {sl.x, sl.y, sl.z, sl.w};
    T pv[SHARED_SLOTS][3];
#pragma unroll
    for (int j = 0; j < SHARED_SLOTS; ++j)
#pragma unroll
      for (int c = C0; c < 3; ++c) pv[j][c] = at32(a.part + c * a.n_slots, uint32_t(max(slot[j], 0)));
    // ascending tile order, the used slots only (computed on every path, so
    // that the loads above stay ahead of the branch)
    T v[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < SHARED_SLOTS; ++j)
#pragma unroll
      for (int c = C0; c < 3; ++c) v[c] = slot[j] >= 0 ? v[c] + pv[j][c] : v[c];
    if (!four) {
#pragma unroll
      for (int c = C0; c < 3; ++c) v[c] = T(0);
      for (int j = 0; j < a.sh_w; ++j) {
        const int sj = a.sh_tab[s * a.sh_w + j];
        if (sj < 0) break;
#pragma unroll
        for (int c = C0; c < 3; ++c) v[c] += at32(a.part + c * a.n_slots, uint32_t(sj));
      }
    }
#pragma unroll
    for (int c = C0; c < 3; ++c) {
      T& d = at32(a.dst + c * n, g);
      if constexpr (JM) {
        const bool cons = (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
        d = cons ? es[c] : v[c];
      } else if constexpr (LCHEB) {
        // the level smoother step (as node_epilogue)
        const bool fixed =
            (c < 2) ? (f & (NODE_DIRICHLET | NODE_EDGE | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_EDGE | NODE_HANGING));
        const int blk = c < 2 ? 0 : 1;
        T x, dp;
        if constexpr (EPI == EPI_CHEB_FIRST) {
          x = a.c0[blk] * ed[c] * eb[c];
          dp = x;
        } else {
          x = ex[c];
          dp = ep[c];
        }
        T& xn = at32(a.xnew + c * n, g);
        if (fixed) {
          d = T(0);
          xn = x;
        } else {
          const T r = eb[c] - v[c];
          const T dn = a.c1[blk] * dp + a.c2[blk] * ed[c] * r;
          d = dn;
          xn = x + dn;
        }
      } else if constexpr (LRES) {
        const bool held = (c < 2) ? (f & (NODE_DIRICHLET | NODE_HANGING)) : (f & (NODE_ACTIVE | NODE_HANGING));
        d = held ? T(0) : eb[c] - v[c];
      } else {
        node_epilogue<MODE, EPI, false, T>(a, c, int64_t(g), f, v[c]);
      }
    }
  }
}

}  // namespace pff
