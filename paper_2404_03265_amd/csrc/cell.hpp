// Device-side cell arithmetic for the matrix-free phase-field operators:
// tensor-product (sum-factorised) interpolation to Gauss points, the
// pointwise laws of the residual and the Jacobian (Kolditz & Wick, Sec. 2,
// Problem 2, and Sec. 3.1), and the transposed integration against test
// functions. One thread handles one cell; everything is unrolled for the
// degree P at compile time.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace pff {

// 1-D Lagrange basis (equispaced nodes) at the P+1 Gauss points of [0, 1],
// the Gauss weights, and the 1-D face-interpolation matrices of the two
// halves of a coarse face (hanging nodes); built at compile time by
// basis_table.
template <typename T>
struct Basis {
  T v[3][3];      // v[q][a] = l_a(g_q)
  T d[3][3];      // d[q][a] = l_a'(g_q)
  T w[3];         // Gauss weights on [0, 1]
  T vw[3][3];     // vw[q][a] = w_q l_a(g_q): weighted tables for integration
  T dw[3][3];     // dw[q][a] = w_q l_a'(g_q)
  T hang[2][3][3];  // hang[sub][t][k] = l_k((sub + t/P) / 2)
};

// The tables as compile-time constants (nodes a / P, Gauss points
// 1/2 -+ sqrt(3)/6 for P = 1 and 1/2 -+ sqrt(15)/10, 1/2 for P = 2, the
// offsets written as correctly rounded binary64 literals). The cell routines
// read them as constants, so the compiler drops the exact zeros and unit
// factors of the tables (for P = 2 the middle Gauss point is a node: its
// values are (0, 1, 0), its derivatives (-1, 0, 1)): about a quarter of the
// FP64 instructions of the Jacobian cell routine.
namespace basis_detail {
constexpr double gauss_point(int p, int q) {
  return p == 1 ? (q == 0 ? 0.5 - 0x1.279a74590331dp-2 : 0.5 + 0x1.279a74590331dp-2)
                : (q == 0 ? 0.5 - 0x1.8c97ef43f7248p-2 : q == 1 ? 0.5 : 0.5 + 0x1.8c97ef43f7248p-2);
}
constexpr double gauss_weight(int p, int q) { return p == 1 ? 0.5 : (q == 1 ? 8.0 / 18.0 : 5.0 / 18.0); }
// Lagrange polynomial k of the nodes m / p, and its derivative, at t
constexpr double lagrange(int p, int k, double t) {
  double v = 1.0;
  for (int m = 0; m <= p; ++m)
    if (m != k) v *= (t - double(m) / p) / (double(k - m) / p);
  return v;
}
constexpr double lagrange_d(int p, int k, double t) {
  double s = 0.0;
  for (int r = 0; r <= p; ++r) {
    if (r == k) continue;
    double v = 1.0 / (double(k - r) / p);
    for (int m = 0; m <= p; ++m)
      if (m != k && m != r) v *= (t - double(m) / p) / (double(k - m) / p);
    s += v;
  }
  return s;
}
}  // namespace basis_detail

template <int P, typename T>
constexpr Basis<T> basis_table() {
  using namespace basis_detail;
  Basis<T> B{};
  for (int q = 0; q <= P; ++q) {
    const double g = gauss_point(P, q), w = gauss_weight(P, q);
    B.w[q] = T(w);
    for (int a = 0; a <= P; ++a) {
      B.v[q][a] = T(lagrange(P, a, g));
      B.d[q][a] = T(lagrange_d(P, a, g));
      B.vw[q][a] = T(w * lagrange(P, a, g));
      B.dw[q][a] = T(w * lagrange_d(P, a, g));
    }
  }
  for (int sub = 0; sub < 2; ++sub)
    for (int t = 0; t <= P; ++t)
      for (int k = 0; k <= P; ++k) B.hang[sub][t][k] = T(lagrange(P, k, (sub + double(t) / P) / 2.0));
  return B;
}

// s = sum_a c[a] x[a] for compile-time coefficients (unrolled loops over
// constant tables): exact zeros are skipped and the sum starts from the
// first non-zero term, so a node-valued Gauss point costs no arithmetic.
template <typename T>
struct CSum {
  T s = T(0);
  bool started = false;
  __device__ __forceinline__ void add(T c, T x) {
    if (c == T(0)) return;
    s = started ? s + c * x : c * x;
    started = true;
  }
};

struct Material {
  double E, mu, lam, kappa, pressure, Gc, ell;
};

// ---------------------------------------------------------------------------
// sum factorisation (B: a table of basis_table, so that the coefficients are
// compile-time constants after unrolling; CSum drops their exact zeros)
template <int P, typename T>
__device__ __forceinline__ void interp_vg(const T (&u)[(P + 1) * (P + 1)],
                                          T (&val)[(P + 1) * (P + 1)], T (&gx)[(P + 1) * (P + 1)],
                                          T (&gy)[(P + 1) * (P + 1)]) {
  constexpr int N = P + 1;
  constexpr Basis<T> B = basis_table<P, T>();
  T V[N][N], D[N][N];  // [node row b][qx]
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      CSum<T> sv, sd;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        sv.add(B.v[q][a], u[b * N + a]);
        sd.add(B.d[q][a], u[b * N + a]);
      }
      V[b][q] = sv.s;
      D[b][q] = sd.s;
    }
#pragma unroll
  for (int qy = 0; qy < N; ++qy)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) {
      CSum<T> s0, s1, s2;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        s0.add(B.v[qy][b], V[b][qx]);
        s1.add(B.v[qy][b], D[b][qx]);
        s2.add(B.d[qy][b], V[b][qx]);
      }
      val[qy * N + qx] = s0.s;
      gx[qy * N + qx] = s1.s;
      gy[qy * N + qx] = s2.s;
    }
}

template <int P, typename T>
__device__ __forceinline__ void interp_g(const T (&u)[(P + 1) * (P + 1)],
                                         T (&gx)[(P + 1) * (P + 1)], T (&gy)[(P + 1) * (P + 1)]) {
  constexpr int N = P + 1;
  constexpr Basis<T> B = basis_table<P, T>();
  T V[N][N], D[N][N];
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      CSum<T> sv, sd;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        sv.add(B.v[q][a], u[b * N + a]);
        sd.add(B.d[q][a], u[b * N + a]);
      }
      V[b][q] = sv.s;
      D[b][q] = sd.s;
    }
#pragma unroll
  for (int qy = 0; qy < N; ++qy)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) {
      CSum<T> s1, s2;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        s1.add(B.v[qy][b], D[b][qx]);
        s2.add(B.d[qy][b], V[b][qx]);
      }
      gx[qy * N + qx] = s1.s;
      gy[qy * N + qx] = s2.s;
    }
}

template <int P, typename T>
__device__ __forceinline__ void interp_v(const T (&u)[(P + 1) * (P + 1)],
                                         T (&val)[(P + 1) * (P + 1)]) {
  constexpr int N = P + 1;
  constexpr Basis<T> B = basis_table<P, T>();
  T V[N][N];
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      CSum<T> sv;
#pragma unroll
      for (int a = 0; a < N; ++a) sv.add(B.v[q][a], u[b * N + a]);
      V[b][q] = sv.s;
    }
#pragma unroll
  for (int qy = 0; qy < N; ++qy)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) {
      CSum<T> s0;
#pragma unroll
      for (int b = 0; b < N; ++b) s0.add(B.v[qy][b], V[b][qx]);
      val[qy * N + qx] = s0.s;
    }
}

// out_k = sum_q (fv_q N_k + fx_q dN_k/dx^ + fy_q dN_k/dy^) (reference derivatives);
// TV, TD: the value and derivative tables (plain, or with the Gauss weights
// folded in), HAS_V / HAS_X / HAS_Y: which point values take part
template <int P, typename T, bool WEIGHTED, bool HAS_V, bool HAS_X, bool HAS_Y>
__device__ __forceinline__ void integrate_tab(const T (&fv)[(P + 1) * (P + 1)], const T (&fx)[(P + 1) * (P + 1)],
                                              const T (&fy)[(P + 1) * (P + 1)], T (&out)[(P + 1) * (P + 1)]) {
  constexpr int N = P + 1;
  constexpr Basis<T> B = basis_table<P, T>();
  auto TV = [&](int q, int a) -> T { return WEIGHTED ? B.vw[q][a] : B.v[q][a]; };
  auto TD = [&](int q, int a) -> T { return WEIGHTED ? B.dw[q][a] : B.d[q][a]; };
  T A[N][N], C[N][N];  // [node row b][qx]
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) {
      CSum<T> sa, sc;
#pragma unroll
      for (int qy = 0; qy < N; ++qy) {
        if (HAS_V) sa.add(TV(qy, b), fv[qy * N + qx]);
        if (HAS_Y) sa.add(TD(qy, b), fy[qy * N + qx]);
        if (HAS_X) sc.add(TV(qy, b), fx[qy * N + qx]);
      }
      A[b][qx] = sa.s;
      C[b][qx] = sc.s;
    }
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int a = 0; a < N; ++a) {
      CSum<T> s;
#pragma unroll
      for (int qx = 0; qx < N; ++qx) {
        if (HAS_V || HAS_Y) s.add(TV(qx, a), A[b][qx]);
        if (HAS_X) s.add(TD(qx, a), C[b][qx]);
      }
      out[b * N + a] = s.s;
    }
}

template <int P, typename T>
__device__ __forceinline__ void integrate(const T (&fv)[(P + 1) * (P + 1)],
                                          const T (&fx)[(P + 1) * (P + 1)],
                                          const T (&fy)[(P + 1) * (P + 1)], T (&out)[(P + 1) * (P + 1)]) {
  integrate_tab<P, T, false, true, true, true>(fv, fx, fy, out);
}

// out_k = sum_q (fx_q dN_k/dx^ + fy_q dN_k/dy^)
template <int P, typename T>
__device__ __forceinline__ void integrate_g(const T (&fx)[(P + 1) * (P + 1)],
                                            const T (&fy)[(P + 1) * (P + 1)], T (&out)[(P + 1) * (P + 1)]) {
  integrate_tab<P, T, false, false, true, true>(fx, fx, fy, out);
}

// Weighted variants: the Gauss weights sit in the tables (vw, dw), so the
// point values passed in carry no weight factor.
template <int P, typename T>
__device__ __forceinline__ void integrate_w(const T (&fv)[(P + 1) * (P + 1)],
                                            const T (&fx)[(P + 1) * (P + 1)],
                                            const T (&fy)[(P + 1) * (P + 1)], T (&out)[(P + 1) * (P + 1)]) {
  integrate_tab<P, T, true, true, true, true>(fv, fx, fy, out);
}

template <int P, typename T>
__device__ __forceinline__ void integrate_gw(const T (&fx)[(P + 1) * (P + 1)],
                                             const T (&fy)[(P + 1) * (P + 1)], T (&out)[(P + 1) * (P + 1)]) {
  integrate_tab<P, T, true, false, true, true>(fx, fx, fy, out);
}

// ---------------------------------------------------------------------------
// hanging-node constraints inside a cell: slots of a hanging face hold the
// coarse face's nodes; interpolate them to the fine face positions (forward)
// or distribute fine-face contributions back to the coarse nodes (transpose).
// Corner slots are fixed points of both faces' maps, so faces commute.
// FACE: 0 left (a = 0), 1 right (a = P), 2 bottom (b = 0), 3 top (b = P);
// all slot indices are compile-time so the local arrays stay in registers.
template <int P, int FACE>
struct FaceSlots {
  static constexpr int N = P + 1;
  static constexpr int start = FACE == 0 ? 0 : FACE == 1 ? P : FACE == 2 ? 0 : P * N;
  static constexpr int stride = FACE < 2 ? N : 1;
};

template <int P, int FACE, typename T>
__device__ __forceinline__ void hang_face(T (&u)[(P + 1) * (P + 1)], int sub) {
  constexpr int N = P + 1, S0 = FaceSlots<P, FACE>::start, ST = FaceSlots<P, FACE>::stride;
  constexpr Basis<T> B = basis_table<P, T>();
  T c[N];
#pragma unroll
  for (int k = 0; k < N; ++k) c[k] = u[S0 + k * ST];
#pragma unroll
  for (int t = 0; t < N; ++t) {
    T s = T(0);
#pragma unroll
    for (int k = 0; k < N; ++k) s += (sub ? B.hang[1][t][k] : B.hang[0][t][k]) * c[k];
    u[S0 + t * ST] = s;
  }
}

template <int P, int FACE, typename T>
__device__ __forceinline__ void hang_face_T(T (&u)[(P + 1) * (P + 1)], int sub) {
  constexpr int N = P + 1, S0 = FaceSlots<P, FACE>::start, ST = FaceSlots<P, FACE>::stride;
  constexpr Basis<T> B = basis_table<P, T>();
  T f[N];
#pragma unroll
  for (int t = 0; t < N; ++t) f[t] = u[S0 + t * ST];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    T s = T(0);
#pragma unroll
    for (int t = 0; t < N; ++t) s += (sub ? B.hang[1][t][k] : B.hang[0][t][k]) * f[t];
    u[S0 + k * ST] = s;
  }
}

// info bits: 0..3 hanging faces (L, R, B, T), 4 cx, 5 cy. Vertical faces
// are halves of the coarse face selected by cy, horizontal ones by cx.
template <int P, typename T>
__device__ __forceinline__ void hang_apply(T (&u)[(P + 1) * (P + 1)], unsigned info) {
  const int cx = (info >> 4) & 1, cy = (info >> 5) & 1;
  if (info & 1u) hang_face<P, 0, T>(u, cy);
  if (info & 2u) hang_face<P, 1, T>(u, cy);
  if (info & 4u) hang_face<P, 2, T>(u, cx);
  if (info & 8u) hang_face<P, 3, T>(u, cx);
}

template <int P, typename T>
__device__ __forceinline__ void hang_apply_T(T (&u)[(P + 1) * (P + 1)], unsigned info) {
  const int cx = (info >> 4) & 1, cy = (info >> 5) & 1;
  if (info & 1u) hang_face_T<P, 0, T>(u, cy);
  if (info & 2u) hang_face_T<P, 1, T>(u, cy);
  if (info & 4u) hang_face_T<P, 2, T>(u, cx);
  if (info & 8u) hang_face_T<P, 3, T>(u, cx);
}

}  // namespace pff
