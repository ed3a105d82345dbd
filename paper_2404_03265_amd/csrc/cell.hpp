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
// halves of a coarse face (hanging nodes). Filled on the host.
template <typename T>
struct Basis {
  T v[3][3];      // v[q][a] = l_a(g_q)
  T d[3][3];      // d[q][a] = l_a'(g_q)
  T w[3];         // Gauss weights on [0, 1]
  T vw[3][3];     // vw[q][a] = w_q l_a(g_q): weighted tables for integration
  T dw[3][3];     // dw[q][a] = w_q l_a'(g_q)
  T hang[2][3][3];  // hang[sub][t][k] = l_k((sub + t/P) / 2)
};

struct Material {
  double E, mu, lam, kappa, pressure, Gc, ell;
};

// ---------------------------------------------------------------------------
// sum factorisation
template <int P, typename T>
__device__ __forceinline__ void interp_vg(const Basis<T>& B, const T (&u)[(P + 1) * (P + 1)],
                                          T (&val)[(P + 1) * (P + 1)], T (&gx)[(P + 1) * (P + 1)],
                                          T (&gy)[(P + 1) * (P + 1)]) {
  constexpr int N = P + 1;
  T V[N][N], D[N][N];  // [node row b][qx]
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      T sv = T(0), sd = T(0);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        sv += B.v[q][a] * u[b * N + a];
        sd += B.d[q][a] * u[b * N + a];
      }
      V[b][q] = sv;
      D[b][q] = sd;
    }
#pragma unroll
  for (int qy = 0; qy < N; ++qy)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) {
      T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
      for (int b = 0; b < N; ++b) {
        s0 += B.v[qy][b] * V[b][qx];
        s1 += B.v[qy][b] * D[b][qx];
        s2 += B.d[qy][b] * V[b][qx];
      }
      val[qy * N + qx] = s0;
      gx[qy * N + qx] = s1;
      gy[qy * N + qx] = s2;
    }
}

template <int P, typename T>
__device__ __forceinline__ void interp_g(const Basis<T>& B, const T (&u)[(P + 1) * (P + 1)],
                                         T (&gx)[(P + 1) * (P + 1)], T (&gy)[(P + 1) * (P + 1)]) {
  constexpr int N = P + 1;
  T V[N][N], D[N][N];
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      T sv = T(0), sd = T(0);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        sv += B.v[q][a] * u[b * N + a];
        sd += B.d[q][a] * u[b * N + a];
      }
      V[b][q] = sv;
      D[b][q] = sd;
    }
#pragma unroll
  for (int qy = 0; qy < N; ++qy)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) {
      T s1 = T(0), s2 = T(0);
#pragma unroll
      for (int b = 0; b < N; ++b) {
        s1 += B.v[qy][b] * D[b][qx];
        s2 += B.d[qy][b] * V[b][qx];
      }
      gx[qy * N + qx] = s1;
      gy[qy * N + qx] = s2;
    }
}

template <int P, typename T>
__device__ __forceinline__ void interp_v(const Basis<T>& B, const T (&u)[(P + 1) * (P + 1)],
                                         T (&val)[(P + 1) * (P + 1)]) {
  constexpr int N = P + 1;
  T V[N][N];
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      T sv = T(0);
#pragma unroll
      for (int a = 0; a < N; ++a) sv += B.v[q][a] * u[b * N + a];
      V[b][q] = sv;
    }
#pragma unroll
  for (int qy = 0; qy < N; ++qy)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) {
      T s0 = T(0);
#pragma unroll
      for (int b = 0; b < N; ++b) s0 += B.v[qy][b] * V[b][qx];
      val[qy * N + qx] = s0;
    }
}

// out_k = sum_q (fv_q N_k + fx_q dN_k/dx^ + fy_q dN_k/dy^) (reference derivatives)
template <int P, typename T>
__device__ __forceinline__ void integrate(const Basis<T>& B, const T (&fv)[(P + 1) * (P + 1)],
                                          const T (&fx)[(P + 1) * (P + 1)],
                                          const T (&fy)[(P + 1) * (P + 1)], T (&out)[(P + 1) * (P + 1)]) {
  constexpr int N = P + 1;
  T A[N][N], C[N][N];  // [node row b][qx]
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) {
      T sa = T(0), sc = T(0);
#pragma unroll
      for (int qy = 0; qy < N; ++qy) {
        sa += B.v[qy][b] * fv[qy * N + qx] + B.d[qy][b] * fy[qy * N + qx];
        sc += B.v[qy][b] * fx[qy * N + qx];
      }
      A[b][qx] = sa;
      C[b][qx] = sc;
    }
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int a = 0; a < N; ++a) {
      T s = T(0);
#pragma unroll
      for (int qx = 0; qx < N; ++qx) s += B.v[qx][a] * A[b][qx] + B.d[qx][a] * C[b][qx];
      out[b * N + a] = s;
    }
}

// out_k = sum_q (fx_q dN_k/dx^ + fy_q dN_k/dy^)
template <int P, typename T>
__device__ __forceinline__ void integrate_g(const Basis<T>& B, const T (&fx)[(P + 1) * (P + 1)],
                                            const T (&fy)[(P + 1) * (P + 1)], T (&out)[(P + 1) * (P + 1)]) {
  constexpr int N = P + 1;
  T A[N][N], C[N][N];
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) {
      T sa = T(0), sc = T(0);
#pragma unroll
      for (int qy = 0; qy < N; ++qy) {
        sa += B.d[qy][b] * fy[qy * N + qx];
        sc += B.v[qy][b] * fx[qy * N + qx];
      }
      A[b][qx] = sa;
      C[b][qx] = sc;
    }
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int a = 0; a < N; ++a) {
      T s = T(0);
#pragma unroll
      for (int qx = 0; qx < N; ++qx) s += B.v[qx][a] * A[b][qx] + B.d[qx][a] * C[b][qx];
      out[b * N + a] = s;
    }
}

// Weighted variants: the Gauss weights sit in the tables (vw, dw), so the
// point values passed in carry no weight factor.
template <int P, typename T>
__device__ __forceinline__ void integrate_w(const Basis<T>& B, const T (&fv)[(P + 1) * (P + 1)],
                                            const T (&fx)[(P + 1) * (P + 1)],
                                            const T (&fy)[(P + 1) * (P + 1)], T (&out)[(P + 1) * (P + 1)]) {
  constexpr int N = P + 1;
  T A[N][N], C[N][N];
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) {
      T sa = T(0), sc = T(0);
#pragma unroll
      for (int qy = 0; qy < N; ++qy) {
        sa += B.vw[qy][b] * fv[qy * N + qx] + B.dw[qy][b] * fy[qy * N + qx];
        sc += B.vw[qy][b] * fx[qy * N + qx];
      }
      A[b][qx] = sa;
      C[b][qx] = sc;
    }
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int a = 0; a < N; ++a) {
      T s = T(0);
#pragma unroll
      for (int qx = 0; qx < N; ++qx) s += B.vw[qx][a] * A[b][qx] + B.dw[qx][a] * C[b][qx];
      out[b * N + a] = s;
    }
}

template <int P, typename T>
__device__ __forceinline__ void integrate_gw(const Basis<T>& B, const T (&fx)[(P + 1) * (P + 1)],
                                             const T (&fy)[(P + 1) * (P + 1)], T (&out)[(P + 1) * (P + 1)]) {
  constexpr int N = P + 1;
  T A[N][N], C[N][N];
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) {
      T sa = T(0), sc = T(0);
#pragma unroll
      for (int qy = 0; qy < N; ++qy) {
        sa += B.dw[qy][b] * fy[qy * N + qx];
        sc += B.vw[qy][b] * fx[qy * N + qx];
      }
      A[b][qx] = sa;
      C[b][qx] = sc;
    }
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int a = 0; a < N; ++a) {
      T s = T(0);
#pragma unroll
      for (int qx = 0; qx < N; ++qx) s += B.vw[qx][a] * A[b][qx] + B.dw[qx][a] * C[b][qx];
      out[b * N + a] = s;
    }
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
__device__ __forceinline__ void hang_face(const Basis<T>& B, T (&u)[(P + 1) * (P + 1)], int sub) {
  constexpr int N = P + 1, S0 = FaceSlots<P, FACE>::start, ST = FaceSlots<P, FACE>::stride;
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
__device__ __forceinline__ void hang_face_T(const Basis<T>& B, T (&u)[(P + 1) * (P + 1)], int sub) {
  constexpr int N = P + 1, S0 = FaceSlots<P, FACE>::start, ST = FaceSlots<P, FACE>::stride;
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
__device__ __forceinline__ void hang_apply(const Basis<T>& B, T (&u)[(P + 1) * (P + 1)], unsigned info) {
  const int cx = (info >> 4) & 1, cy = (info >> 5) & 1;
  if (info & 1u) hang_face<P, 0, T>(B, u, cy);
  if (info & 2u) hang_face<P, 1, T>(B, u, cy);
  if (info & 4u) hang_face<P, 2, T>(B, u, cx);
  if (info & 8u) hang_face<P, 3, T>(B, u, cx);
}

template <int P, typename T>
__device__ __forceinline__ void hang_apply_T(const Basis<T>& B, T (&u)[(P + 1) * (P + 1)], unsigned info) {
  const int cx = (info >> 4) & 1, cy = (info >> 5) & 1;
  if (info & 1u) hang_face_T<P, 0, T>(B, u, cy);
  if (info & 2u) hang_face_T<P, 1, T>(B, u, cy);
  if (info & 4u) hang_face_T<P, 2, T>(B, u, cx);
  if (info & 8u) hang_face_T<P, 3, T>(B, u, cx);
}

}  // namespace pff
