// Even/odd folded 1D tables and the small-matvec helpers shared by the
// plane-ownership operator kernels (box and trilinear cells).  The GLL nodes
// and Gauss points are symmetric about 0, so B[n-1-a][n-1-i] = B[a][i] and D,
// Dg are antisymmetric: a 1D contraction splits into an even and an odd half
// of size n/2 each.
#pragma once
#include "tdfe_internal.h"
#include "tdfe_rule1d.h"

namespace {

constexpr int EO_MAX_H = 5;  // (9 + 1) / 2

// folded form of one N x N matrix with reflection symmetry S (+1 or -1), in the
// kernel's working precision (no conversions at the point of use)
template <typename T>
struct Folded {
  T E[EO_MAX_H * EO_MAX_H];  // (A[a][i] + A[a][N-1-i]) / 2, a, i < H
  T O[EO_MAX_H * EO_MAX_H];  // (A[a][i] - A[a][N-1-i]) / 2
  T mc[EO_MAX_H];            // A[a][H] (odd N)
  T mr[EO_MAX_H + 1];        // A[H][i], i <= H (odd N)
};

// the six folded tables of order N (B, B^T, D, D^T, Dg, Dg^T) and the Gauss
// weights, evaluated at compile time: a kernel declares
//   constexpr FoldSet<N> FS = make_foldset<N>();
// and every coefficient becomes a constant of the instruction stream
template <int N>
struct FoldSet {
  Folded<double> B, Bt, D, Dt, G, Gt;
  double wq[TDFE_MAXN];
};

constexpr void fold_c(const double* A, int N, int S, bool transpose, Folded<double>& F) {
  const int H = N / 2;
  for (int a = 0; a < H; ++a)
    for (int i = 0; i < H; ++i) {
      const double ai = transpose ? A[i * TDFE_MAXN + a] : A[a * TDFE_MAXN + i];
      const double aj = transpose ? A[(N - 1 - i) * TDFE_MAXN + a] : A[a * TDFE_MAXN + N - 1 - i];
      F.E[a * EO_MAX_H + i] = 0.5 * (ai + aj);
      F.O[a * EO_MAX_H + i] = 0.5 * (ai - aj);
    }
  if (N & 1) {
    for (int a = 0; a < H; ++a) F.mc[a] = transpose ? A[H * TDFE_MAXN + a] : A[a * TDFE_MAXN + H];
    for (int i = 0; i <= H; ++i) F.mr[i] = transpose ? A[i * TDFE_MAXN + H] : A[H * TDFE_MAXN + i];
    if (S < 0) F.mr[H] = 0.0;
  }
}

template <int N>
constexpr FoldSet<N> make_foldset() {
  const tdfe1d::Rule R = tdfe1d::make_rule(N - 1);
  FoldSet<N> F{};
  fold_c(R.B, N, 1, false, F.B);
  fold_c(R.B, N, 1, true, F.Bt);
  fold_c(R.D, N, -1, false, F.D);
  fold_c(R.D, N, -1, true, F.Dt);
  fold_c(R.Dg, N, -1, false, F.G);
  fold_c(R.Dg, N, -1, true, F.Gt);
  for (int i = 0; i < TDFE_MAXN; ++i) F.wq[i] = R.wq[i];
  return F;
}

// quadratic form: FP32 kernels sum each line in FP32 and promote the line
// sums; FP64 kernels accumulate directly
template <typename T>
__device__ __forceinline__ void acc_energy(double& e, T& line, T v) {
  if constexpr (sizeof(T) == 4)
    line += v;
  else
    e += v;
}
template <typename T>
__device__ __forceinline__ void flush_energy(double& e, T line) {
  if constexpr (sizeof(T) == 4) e += (double)line;
}

// logical block of physical block p in a grid of G: the dispatcher hands
// blocks to the 8 XCDs round robin (block p to XCD p mod 8), and XCD x takes
// the contiguous logical range starting at x q + min(x, r) (q = G / 8,
// r = G mod 8; q + 1 blocks for x < r), so that neighbouring cells, which
// share nodes, run under one L2
__device__ __forceinline__ int remap_block(int p, int G) {
  const int q = G >> 3, r = G & 7, x = p & 7;
  return x * q + min(x, r) + (p >> 3);
}

// out[a] = sum_i A[a][i] in[i] by even/odd folding; A given folded (in any
// precision, converted to T), symmetry S
template <typename T, int N, int S, typename FT>
__device__ __forceinline__ void eo(const Folded<FT>& F, const T* in, T* out) {
  constexpr int H = N / 2;
  T e[H > 0 ? H : 1], o[H > 0 ? H : 1];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    e[i] = in[i] + in[N - 1 - i];
    o[i] = in[i] - in[N - 1 - i];
  }
  // coefficients that are exactly zero (for odd N the middle row of B, whose
  // middle Gauss point is a GLL node, and the middle column of B^T) are
  // skipped: the tables are compile-time constants, so the tests fold away
#pragma unroll
  for (int a = 0; a < H; ++a) {
    T Pv = 0, Qv = 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      if (F.E[a * EO_MAX_H + i] != 0) Pv += (T)F.E[a * EO_MAX_H + i] * e[i];
      if (F.O[a * EO_MAX_H + i] != 0) Qv += (T)F.O[a * EO_MAX_H + i] * o[i];
    }
    if constexpr (N & 1)
      if (F.mc[a] != 0) Pv += (T)F.mc[a] * in[H];
    out[a] = Pv + Qv;
    out[N - 1 - a] = S > 0 ? Pv - Qv : Qv - Pv;
  }
  if constexpr (N & 1) {
    T m = 0;
    if constexpr (S > 0) {
#pragma unroll
      for (int i = 0; i < H; ++i)
        if (F.mr[i] != 0) m += (T)F.mr[i] * e[i];
      if (F.mr[H] != 0) m += (T)F.mr[H] * in[H];
    } else {
#pragma unroll
      for (int i = 0; i < H; ++i)
        if (F.mr[i] != 0) m += (T)F.mr[i] * o[i];
    }
    out[H] = m;
  }
}

// two matrices on the same input line share the fold
template <typename T, int N, int S1, int S2, typename FT>
__device__ __forceinline__ void eo2(const Folded<FT>& F1, const Folded<FT>& F2, const T* in, T* out1, T* out2) {
  eo<T, N, S1>(F1, in, out1);
  eo<T, N, S2>(F2, in, out2);
}

// host: fold an N x N table (row-major, stride TDFE_MAXN) with symmetry S
template <typename T>
void fold(const double* A, int N, int S, bool transpose, Folded<T>& F) {
  auto at = [&](int a, int i) { return transpose ? A[i * TDFE_MAXN + a] : A[a * TDFE_MAXN + i]; };
  const int H = N / 2;
  for (int a = 0; a < H; ++a)
    for (int i = 0; i < H; ++i) {
      F.E[a * EO_MAX_H + i] = (T)(0.5 * (at(a, i) + at(a, N - 1 - i)));
      F.O[a * EO_MAX_H + i] = (T)(0.5 * (at(a, i) - at(a, N - 1 - i)));
    }
  if (N & 1) {
    for (int a = 0; a < H; ++a) F.mc[a] = (T)at(a, H);
    for (int i = 0; i <= H; ++i) F.mr[i] = (T)at(H, i);
    if (S < 0) F.mr[H] = (T)0;
  }
}

}  // namespace
