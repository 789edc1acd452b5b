// Operator kernel for rectilinear (box) cells, even n: two lanes per plane.
//
// The same operator and phase order as the plane kernel (Eq. DiscreteHamiltonian
// in the Loewdin form, Eq. TDKSMatVecStandard), but the n x n plane of one
// column is shared by an adjacent lane pair: each lane holds the half of the z
// index range that is its own, lane 0 the indices 0..n/2-1 and lane 1 their
// mirror images n-1..n/2, both in local order.  Contractions along x and y stay
// inside a lane (even/odd folded, as in the plane kernel); a contraction along
// z forms, in each lane, the partial sums over its own inputs for its own
// outputs and for the partner's, and swaps the latter with the partner by a DPP
// quad permutation.  The mirror symmetry of the 1D tables
// (A[n-1-c][n-1-k] = S A[c][k], S = +1 for B, -1 for D and Dg) makes the two
// lanes run identical code with identical coefficients: lane 1 only multiplies
// its inputs by S.  All tables are compile-time constants (make_pairset).  A
// lane then keeps half the registers of a plane-owning thread, which lets FP64
// run two waves per SIMD.
#include "tdfe_fold.h"

namespace {

constexpr int PH = 4;  // largest half order (n = 8)

// folded table of an even-order matrix (no middle row or column)
template <typename T>
struct FoldE {
  T E[PH * PH];  // (A[a][i] + A[a][n-1-i]) / 2, a, i < n/2
  T O[PH * PH];  // (A[a][i] - A[a][n-1-i]) / 2
};

// split table of a matrix for a contraction along the paired direction:
// own[cc][kk] = A[cc][kk], oth[cc][kk] = A[n-1-cc][kk]
template <typename T>
struct SplitT {
  T own[PH * PH];
  T oth[PH * PH];
};

template <typename T>
struct PairParams {
  const void* x;
  void* y;
  int ld, cols, nchunks;
  const double* colscale;
  double kin;
  const void* vw;
  const double* m1x;  // separable M^-1/2 factors: minv(I,J,K) = m1x[I] m1y[J] m1z[K]
  const double* m1y;
  const double* m1z;
  const double* cellgeo;
  double* energy;
  const int* done;
  int ncx, ncy, ncz, p, Nx, Ny, Nz;
  int64_t n_cell;
  int lowdin, fullgrid;
  double wq[TDFE_MAXN];
};

// the kernel's tables for order N, evaluated at compile time
struct PairSet {
  FoldE<double> fB, fBt, fD, fDt, fG, fGt;  // B, B^T, D, D^T, Dg, Dg^T (x and y directions)
  SplitT<double> zB, zBt, zG, zGt;          // B, B^T, Dg, Dg^T along z
  double wq[TDFE_MAXN];
};

constexpr void fold_even(const double* A, int N, bool transpose, FoldE<double>& F) {
  const int H = N / 2;
  for (int a = 0; a < H; ++a)
    for (int i = 0; i < H; ++i) {
      const double ai = transpose ? A[i * TDFE_MAXN + a] : A[a * TDFE_MAXN + i];
      const double aj = transpose ? A[(N - 1 - i) * TDFE_MAXN + a] : A[a * TDFE_MAXN + N - 1 - i];
      F.E[a * PH + i] = 0.5 * (ai + aj);
      F.O[a * PH + i] = 0.5 * (ai - aj);
    }
}

constexpr void split_tab(const double* A, int N, bool transpose, SplitT<double>& F) {
  const int H = N / 2;
  for (int c = 0; c < H; ++c)
    for (int k = 0; k < H; ++k) {
      F.own[c * PH + k] = transpose ? A[k * TDFE_MAXN + c] : A[c * TDFE_MAXN + k];
      F.oth[c * PH + k] = transpose ? A[k * TDFE_MAXN + N - 1 - c] : A[(N - 1 - c) * TDFE_MAXN + k];
    }
}

template <int N>
constexpr PairSet make_pairset() {
  const tdfe1d::Rule R = tdfe1d::make_rule(N - 1);
  PairSet F{};
  fold_even(R.B, N, false, F.fB);
  fold_even(R.B, N, true, F.fBt);
  fold_even(R.D, N, false, F.fD);
  fold_even(R.D, N, true, F.fDt);
  fold_even(R.Dg, N, false, F.fG);
  fold_even(R.Dg, N, true, F.fGt);
  split_tab(R.B, N, false, F.zB);
  split_tab(R.B, N, true, F.zBt);
  split_tab(R.Dg, N, false, F.zG);
  split_tab(R.Dg, N, true, F.zGt);
  for (int i = 0; i < TDFE_MAXN; ++i) F.wq[i] = R.wq[i];
  return F;
}

// out[a] = sum_i A[a][i] in[i], A folded with symmetry S (even N)
template <typename T, int N, int S>
__device__ __forceinline__ void eoe(const FoldE<double>& F, const T* in, T* out) {
  constexpr int H = N / 2;
  T e[H], o[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    e[i] = in[i] + in[N - 1 - i];
    o[i] = in[i] - in[N - 1 - i];
  }
#pragma unroll
  for (int a = 0; a < H; ++a) {
    T Pv = 0, Qv = 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      Pv += (T)F.E[a * PH + i] * e[i];
      Qv += (T)F.O[a * PH + i] * o[i];
    }
    out[a] = Pv + Qv;
    out[N - 1 - a] = S > 0 ? Pv - Qv : Qv - Pv;
  }
}

// value of the partner lane (lane ^ 1)
template <typename T>
__device__ __forceinline__ T pair_swap(T v) {
  if constexpr (sizeof(T) == 8) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0xB1, 0xf, 0xf, false);  // quad_perm 1,0,3,2
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0xB1, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
  } else {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, false));
  }
}

// contraction along the paired direction: in/out hold this lane's H local
// entries; sg = S on lane 1, 1 on lane 0
template <typename T, int N>
__device__ __forceinline__ void zsplit(const SplitT<double>& F, const T* in, T* out, T sg) {
  constexpr int H = N / 2;
  T x[H], own[H], oth[H];
#pragma unroll
  for (int k = 0; k < H; ++k) x[k] = sg * in[k];
#pragma unroll
  for (int c = 0; c < H; ++c) {
    T a = 0, b = 0;
#pragma unroll
    for (int k = 0; k < H; ++k) {
      a += (T)F.own[c * PH + k] * x[k];
      b += (T)F.oth[c * PH + k] * x[k];
    }
    own[c] = a;
    oth[c] = b;
  }
#pragma unroll
  for (int c = 0; c < H; ++c) out[c] = own[c] + pair_swap(oth[c]);
}

template <typename T, int N>
constexpr int pair_wpe() {
  return sizeof(T) == 8 ? 2 : 3;
}

template <typename T, int N, int CB, int CPB>
__global__ void __launch_bounds__(2 * CPB * N * CB) __attribute__((amdgpu_waves_per_eu(pair_wpe<T, N>())))
    pair_kernel(PairParams<T> P) {
  static_assert(N % 2 == 0 && N / 2 <= PH, "even n <= 8");
  constexpr int H = N / 2;
  constexpr int VOL = N * N * N;
  constexpr int THREADS = 2 * CPB * N * CB;
  constexpr PairSet FS = make_pairset<N>();
  __shared__ T sX[CPB * VOL * CB];
  __shared__ T sV[CPB * VOL];
  __shared__ double sRed[THREADS];
  if (P.done && *P.done) return;

  const int t = threadIdx.x;
  const int h = t & 1;  // half of the z range
  const int r = t >> 1;
  const int L = remap_block(blockIdx.x, gridDim.x);
  const int chunk = L % P.nchunks;
  const int group = L / P.nchunks;
  const int col = r % CB;
  const int pl = (r / CB) % N;
  const int slot = r / (CB * N);
  const int64_t cell = (int64_t)group * CPB + slot;
  const bool cell_ok = cell < P.n_cell;
  const int colg = chunk * CB + col;
  const bool act = cell_ok && colg < P.cols;
  const T sgn = h ? (T)-1 : (T)1;  // S = -1 tables on lane 1
  // global z index of local entry q
  auto zg = [&](int q) { return h ? N - 1 - q : q; };

  int cx = 0, cy = 0, cz = 0;
  if (cell_ok) {
    cx = (int)(cell % P.ncx);
    cy = (int)((cell / P.ncx) % P.ncy);
    cz = (int)(cell / ((int64_t)P.ncx * P.ncy));
  }
  const T* __restrict__ X = (const T*)P.x;
  T* __restrict__ Y = (T*)P.y;
  T cs = (T)1;
  if (P.colscale && act) cs = (T)P.colscale[colg >> 1];

  // block staging (as in the plane kernel): potential, M^-1/2 factors along
  // x, y, z and the metric of the block's cells; loads issued before the
  // phase A gather, LDS stores after it, one wait for memory per wave
  constexpr int NFC = 3 * N + 3;
  constexpr int NV = (CPB * VOL + THREADS - 1) / THREADS;
  constexpr int NF = (CPB * NFC + THREADS - 1) / THREADS;
  __shared__ double sF[CPB * NFC];
  const int64_t c0 = (int64_t)group * CPB;
  T vr[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int q = t + k * THREADS;
    const int64_t ce = c0 + q / VOL;
    const bool ok = P.vw && q < CPB * VOL && ce < P.n_cell;
    vr[k] = ok ? ((const T*)P.vw)[ce * VOL + q % VOL] : (T)0;
  }
  double fr[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const int f = t + k * THREADS;
    const int r = f % NFC;
    const int64_t ce = c0 + f / NFC;
    const bool ok = f < CPB * NFC && ce < P.n_cell;
    const int64_t cv = ok ? ce : 0;
    const int ex = (int)(cv % P.ncx), ey = (int)((cv / P.ncx) % P.ncy);
    const int ez = (int)(cv / ((int64_t)P.ncx * P.ncy));
    const double* src = r < N ? P.m1x + (ex * P.p + r)
                        : r < 2 * N ? P.m1y + (ey * P.p + r - N)
                        : r < 3 * N ? P.m1z + (ez * P.p + r - 2 * N)
                                    : P.cellgeo + (cv * 4 + r - 3 * N);
    const double val = *src;
    fr[k] = ok ? val : 0.0;
  }
  const double* sFc = sF + slot * NFC;
  auto sidx = [&](int y, int x, int z) { return (((slot * N + y) * N + x) * N + z) * CB + col; };
  const int NxI = P.Nx - 2, NyI = P.Ny - 2;

  // node masks, element offsets and Loewdin factors of node plane j = pl
  // (phases A and C; recomputed in C rather than held through B): fx, fz
  // and my are the x, z and y factors of M^-1/2
  struct PlaneNodes {
    unsigned imask, kmask;  // kmask over local z entries
    int64_t e0, kstride;
    T fx[N], fz[H], my;
  };
  auto plane_nodes = [&](PlaneNodes& Q, bool factors) {
    const int J = cy * P.p + pl;
    const bool jok = P.fullgrid ? true : (J > 0 && J < P.Ny - 1);
    Q.imask = 0;
    Q.kmask = 0;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const int I = cx * P.p + q;
      if (P.fullgrid || (I > 0 && I < P.Nx - 1)) Q.imask |= 1u << q;
    }
#pragma unroll
    for (int q = 0; q < H; ++q) {
      const int K = cz * P.p + zg(q);
      if (P.fullgrid || (K > 0 && K < P.Nz - 1)) Q.kmask |= 1u << q;
    }
    if (!act || !jok) Q.imask = 0;
    if (P.fullgrid) {
      Q.e0 = ((int64_t)cx * P.p + (int64_t)P.Nx * ((int64_t)J + (int64_t)P.Ny * cz * P.p)) * P.ld + colg;
      Q.kstride = (int64_t)P.Nx * P.Ny * P.ld;
    } else {
      Q.e0 = ((int64_t)(cx * P.p - 1) + (int64_t)NxI * ((int64_t)(J - 1) + (int64_t)NyI * (cz * P.p - 1))) * P.ld +
             colg;
      Q.kstride = (int64_t)NxI * NyI * P.ld;
    }
    Q.my = (T)1;
#pragma unroll
    for (int q = 0; q < N; ++q) Q.fx[q] = (T)1;
#pragma unroll
    for (int q = 0; q < H; ++q) Q.fz[q] = (T)1;
    if (factors && P.lowdin && Q.imask) {
      Q.my = (T)sFc[N + pl];
#pragma unroll
      for (int q = 0; q < N; ++q)
        if ((Q.imask >> q) & 1u) Q.fx[q] = (T)sFc[q];
#pragma unroll
      for (int q = 0; q < H; ++q)
        if ((Q.kmask >> q) & 1u) Q.fz[q] = (T)sFc[2 * N + zg(q)];
    }
  };

  // ---------------- A: plane j = pl, values (i, local k) ---------------------------------
  T tu[N][H], tx[N][H];  // [x point][local z]
  {
    PlaneNodes Q;
    plane_nodes(Q, false);
    T u[N][H];
#pragma unroll
    for (int k = 0; k < H; ++k)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const bool ok = ((Q.imask >> i) & (Q.kmask >> k) & 1u) != 0;
        const int64_t e = ok ? Q.e0 + (int64_t)i * P.ld + (int64_t)zg(k) * Q.kstride : 0;
        const T val = X[e];
        u[i][k] = ok ? val : (T)0;
      }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int q = t + k * THREADS;
      if (q < CPB * VOL) sV[q] = vr[k];
    }
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int f = t + k * THREADS;
      if (f < CPB * NFC) sF[f] = fr[k];
    }
    __syncthreads();
    plane_nodes(Q, true);
#pragma unroll
    for (int k = 0; k < H; ++k)
#pragma unroll
      for (int i = 0; i < N; ++i) u[i][k] *= Q.fx[i] * Q.fz[k] * (Q.my * cs);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      T line[N], o1[N], o2[N];
#pragma unroll
      for (int i = 0; i < N; ++i) line[i] = u[i][k];
      eoe<T, N, 1>(FS.fB, line, o1);
      eoe<T, N, -1>(FS.fD, line, o2);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        tu[a][k] = o1[a];
        tx[a][k] = o2[a];
      }
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
      T o1[H], o2[H];
      zsplit<T, N>(FS.zB, tu[a], o1, (T)1);
      zsplit<T, N>(FS.zB, tx[a], o2, (T)1);
#pragma unroll
      for (int c = 0; c < H; ++c) {
        tu[a][c] = o1[c];
        tx[a][c] = o2[c];
      }
    }
  }
  // ---------------- transpose: (j; a, c) -> (a; j, c) ---------------------------------------
  T v[N][H], w[N][H];  // [y node][local z] at x point a = pl
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int c = 0; c < H; ++c) sX[sidx(pl, a, zg(c))] = tu[a][c];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int c = 0; c < H; ++c) v[j][c] = sX[sidx(j, pl, zg(c))];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int c = 0; c < H; ++c) sX[sidx(pl, a, zg(c))] = tx[a][c];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int c = 0; c < H; ++c) w[j][c] = sX[sidx(j, pl, zg(c))];
  __syncthreads();

  // ---------------- B: plane a = pl, Gauss points (b, local c) ---------------------------------
  double energy = 0.0;
  T gx = 0, gy = 0, gz = 0;
  if (cell_ok) {
    T wa = (T)FS.wq[0];  // selected from the constants: no per-lane memory load
#pragma unroll
    for (int q = 1; q < N; ++q) wa = pl == q ? (T)FS.wq[q] : wa;
    gx = (T)(P.kin * sFc[3 * N + 0]) * wa;
    gy = (T)(P.kin * sFc[3 * N + 1]) * wa;
    gz = (T)(P.kin * sFc[3 * N + 2]) * wa;
  }
  // z Gauss weights of this lane's points: the rule's weights are symmetric
  // (bitwise, for every order), so the mirror point's weight is wq[c] itself
  T wc[H];
#pragma unroll
  for (int c = 0; c < H; ++c) wc[c] = (T)FS.wq[c];
  // B1: x flux from w, transposed y interpolation, into the transpose buffer
#pragma unroll
  for (int c = 0; c < H; ++c) {
    T l[N], o[N];
#pragma unroll
    for (int j = 0; j < N; ++j) l[j] = w[j][c];
    eoe<T, N, 1>(FS.fB, l, o);
    T le = 0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const T f = gx * ((T)FS.wq[b] * wc[c]) * o[b];
      acc_energy<T>(energy, le, f * o[b]);
      o[b] = f;
    }
    flush_energy<T>(energy, le);
    eoe<T, N, 1>(FS.fBt, o, l);
#pragma unroll
    for (int j = 0; j < N; ++j) sX[sidx(j, pl, zg(c))] = l[j];
    __builtin_amdgcn_sched_barrier(0);
  }
  // B2: u_q, potential, z and y fluxes, transposed y interpolation
  T s[N][H];  // [y node][local z]
  {
    T uq[N][H], acc[N][H];
#pragma unroll
    for (int c = 0; c < H; ++c) {
      T l[N], o[N];
#pragma unroll
      for (int j = 0; j < N; ++j) l[j] = v[j][c];
      eoe<T, N, 1>(FS.fB, l, o);
      T le = 0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        uq[b][c] = o[b];
        const T pot = P.vw ? sV[slot * VOL + pl + N * (b + N * zg(c))] * o[b] : (T)0;
        acc_energy<T>(energy, le, pot * o[b]);
        acc[b][c] = pot;
      }
      flush_energy<T>(energy, le);
      __builtin_amdgcn_sched_barrier(0);
    }
    // z flux, per y point (paired contractions)
#pragma unroll
    for (int b = 0; b < N; ++b) {
      T d[H], rr[H];
      zsplit<T, N>(FS.zG, uq[b], d, sgn);
      T le = 0;
#pragma unroll
      for (int c = 0; c < H; ++c) {
        const T f = gz * ((T)FS.wq[b] * wc[c]) * d[c];
        acc_energy<T>(energy, le, f * d[c]);
        d[c] = f;
      }
      flush_energy<T>(energy, le);
      zsplit<T, N>(FS.zGt, d, rr, sgn);
#pragma unroll
      for (int c = 0; c < H; ++c) acc[b][c] += rr[c];
    }
    // y flux and transposed y interpolation, per local z point
#pragma unroll
    for (int c = 0; c < H; ++c) {
      T l[N], d[N], rr[N];
#pragma unroll
      for (int b = 0; b < N; ++b) l[b] = uq[b][c];
      eoe<T, N, -1>(FS.fG, l, d);
      T le = 0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const T f = gy * ((T)FS.wq[b] * wc[c]) * d[b];
        acc_energy<T>(energy, le, f * d[b]);
        d[b] = f;
      }
      flush_energy<T>(energy, le);
      eoe<T, N, -1>(FS.fGt, d, rr);
#pragma unroll
      for (int b = 0; b < N; ++b) rr[b] += acc[b][c];
      eoe<T, N, 1>(FS.fBt, rr, l);
#pragma unroll
      for (int j = 0; j < N; ++j) s[j][c] = l[j];
    }
  }
  // ---------------- transposes: (a; j, c) -> (j; a, c) ---------------------------------------
  sRed[t] = act ? energy : 0.0;
  T s2[N][H], sx2[N][H];  // [x point][local z] at node plane j = pl
  __syncthreads();
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int c = 0; c < H; ++c) sx2[a][c] = sX[sidx(pl, a, zg(c))];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int c = 0; c < H; ++c) sX[sidx(j, pl, zg(c))] = s[j][c];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int c = 0; c < H; ++c) s2[a][c] = sX[sidx(pl, a, zg(c))];

  // ---------------- C: plane j = pl: x transposed, z transposed (paired), scatter -------------------
  {
    T hh[N][H];  // [x node][local z point]
#pragma unroll
    for (int c = 0; c < H; ++c) {
      T l1[N], l2[N], o1[N], o2[N];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        l1[a] = s2[a][c];
        l2[a] = sx2[a][c];
      }
      eoe<T, N, 1>(FS.fBt, l1, o1);
      eoe<T, N, -1>(FS.fDt, l2, o2);
#pragma unroll
      for (int i = 0; i < N; ++i) hh[i][c] = o1[i] + o2[i];
    }
    PlaneNodes Q;
    plane_nodes(Q, true);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T o[H];
      zsplit<T, N>(FS.zBt, hh[i], o, (T)1);
#pragma unroll
      for (int k = 0; k < H; ++k) {
        if (((Q.imask >> i) & (Q.kmask >> k) & 1u) != 0)
          unsafeAtomicAdd(Y + (Q.e0 + (int64_t)i * P.ld + (int64_t)zg(k) * Q.kstride), o[k] * (Q.fx[i] * Q.fz[k] * Q.my));
      }
    }
  }
  // ---------------- per-column quadratic form ----------------------------------------------------
  if (P.energy) {
    __syncthreads();
    if (t < CB) {
      double acc = 0.0;
      for (int u = 2 * t; u < THREADS; u += 2 * CB) acc += sRed[u] + sRed[u + 1];
      if (chunk * CB + t < P.cols) P.energy[(int64_t)group * P.cols + chunk * CB + t] = acc;
    }
  }
}

// ----------------------------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------------------------

template <typename T, int N, int CB>
constexpr int pair_lds(int cpb) {
  constexpr int VOL = N * N * N;
  return cpb * VOL * CB * (int)sizeof(T) + cpb * VOL * (int)sizeof(T) + 2 * cpb * N * CB * 8 + cpb * (3 * N + 3) * 8;
}

// cells per block: at most 256 threads (blocks of a few waves pack the CUs
// at two or more waves per SIMD) and LDS for the occupancy pair_wpe asks for
template <typename T, int N, int CB>
constexpr int pair_cpb() {
  constexpr int budget = sizeof(T) == 8 ? 64 * 1024 : 40 * 1024;
  int cpb = 1;
  while (2 * cpb * 2 * N * CB <= 256 && pair_lds<T, N, CB>(cpb * 2) <= budget) cpb *= 2;
  return cpb;
}

template <typename T, int N, int CB>
tdfe_status launch_pair(tdfe_ctx* c, PairParams<T>& P, int64_t* groups_out) {
  constexpr int CPB = pair_cpb<T, N, CB>();
  static_assert(pair_lds<T, N, CB>(CPB) <= 160 * 1024, "LDS");
  const int64_t groups = (c->n_cell + CPB - 1) / CPB;
  P.nchunks = (P.cols + CB - 1) / CB;
  if (groups_out) *groups_out = groups;
  hipLaunchKernelGGL((pair_kernel<T, N, CB, CPB>), dim3((unsigned)(groups * P.nchunks)), dim3(2 * CPB * N * CB), 0,
                     c->stream, P);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

template <typename T, int N>
tdfe_status launch_pair_n(tdfe_ctx* c, PairParams<T>& P, int64_t* g) {
  if (P.cols <= 1) return launch_pair<T, N, 1>(c, P, g);
  if (P.cols <= 2) return launch_pair<T, N, 2>(c, P, g);
  if (P.cols <= 4) return launch_pair<T, N, 4>(c, P, g);
  if (P.cols <= 8) return launch_pair<T, N, 8>(c, P, g);
  return launch_pair<T, N, 16>(c, P, g);
}

template <typename T>
tdfe_status launch_pair_box(tdfe_ctx* c, const ApplyArgs& a) {
  static_assert(sizeof(PairParams<T>) <= 4096, "kernel arguments exceed 4 KB");
  PairParams<T> P{};
  P.x = a.x;
  P.y = a.y;
  P.ld = a.ld;
  P.cols = a.cols;
  P.colscale = a.colscale;
  P.kin = a.kin;
  P.vw = a.fp32 ? (const void*)a.vw32 : (const void*)a.vw;
  P.m1x = c->m1x;
  P.m1y = c->m1y;
  P.m1z = c->m1z;
  P.cellgeo = c->cellgeo;
  P.energy = a.energy;
  P.done = a.done_flag;
  P.ncx = c->ncx;
  P.ncy = c->ncy;
  P.ncz = c->ncz;
  P.p = c->p;
  P.Nx = c->Nx;
  P.Ny = c->Ny;
  P.Nz = c->Nz;
  P.n_cell = c->n_cell;
  P.lowdin = a.lowdin;
  P.fullgrid = a.fullgrid;
  const int N = c->n;
  for (int i = 0; i < N; ++i) P.wq[i] = c->wq[i];
  switch (N) {
    case 2: return launch_pair_n<T, 2>(c, P, a.n_blocks_out);
    case 4: return launch_pair_n<T, 4>(c, P, a.n_blocks_out);
    case 6: return launch_pair_n<T, 6>(c, P, a.n_blocks_out);
    case 8: return launch_pair_n<T, 8>(c, P, a.n_blocks_out);
  }
  return tdfe_fail(c, TDFE_EINVAL, "paired box operator: order p=%d is not odd", c->p);
}

}  // namespace

// true if the lane-pair box kernel can handle this context (rectilinear mesh, odd p <= 7)
bool tdfe_pair_kernel_ok(const tdfe_ctx* c) { return c->box && c->n % 2 == 0 && c->n <= 8; }

tdfe_status tdfe_launch_apply_pair(tdfe_ctx* c, const ApplyArgs& a) {
  if (a.cols < 1) return tdfe_fail(c, TDFE_EINVAL, "apply: cols < 1");
  if (!tdfe_pair_kernel_ok(c)) return tdfe_fail(c, TDFE_EINVAL, "paired box operator: unsupported mesh or order");
  return a.fp32 ? launch_pair_box<float>(c, a) : launch_pair_box<double>(c, a);
}
