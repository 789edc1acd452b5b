// Box-cell operator with its 1D contractions on the matrix cores.
//
// The same operator as the VALU box kernels (Eq. DiscreteHamiltonian in the
// Loewdin form, Eq. TDKSMatVecStandard; Gauss quadrature with n = p + 1
// points, the x derivative through D on the nodes, the y and z derivatives
// by collocation at the Gauss points), with every 1D contraction of a cell
// issued as 16 x 16 matrix-core products:
//
//   C[m][col] (+)= sum_k A[m][k] X[k][col]
//
// A is a 1D table (its rows are the outputs along the contracted axis, up to
// two tables stacked, zero padded to 16 x 16), X holds one line of the cell
// (the inputs along that axis, up to two arrays stacked along k) for the
// block's 16 real columns, and C lands in the layout the next LDS store needs.
// A block is one cell and 16 columns (four waves); the cell lives in LDS in
// three arrays [node or point][16 columns] and is swept axis by axis:
//
//   x: A0 <- B u,  A1 <- D u                        (u gathered, x M^-1/2)
//   y: A0 <- B A0, A1 <- B A1
//   z: A0 <- B A0 (= u_q),  A1 <- fx(B A1)           (x flux)
//   y: A2 <- fy(Dg A0);  A2 <- Dg^T A2 + V u_q
//   z: A0 <- fz(Dg A0);  A2 <- Dg^T A0 + A2;  A2 <- B^T A2;  A1 <- B^T A1
//   y: A2 <- B^T A2, A1 <- B^T A1
//   x: A2 <- B^T A2 + D^T A1                          (scatter-add x M^-1/2)
//
// with f_d = kin g_d w_a w_b w_c d (g_d the cell's metric factor) and the
// quadratic form sum f_d d + V u_q^2 per column (alpha of the Lanczos step).
// A wave owns whole lines within a sweep; where a line's next contraction
// reads what the previous one stored, a wavefront fence orders the LDS
// accesses (no workgroup barrier).
//
// Engines: FP64 (v_mfma_f64_16x16x4, k in steps of 4), FP32
// (v_mfma_f32_16x16x4), and split BF16 (v_mfma_f32_16x16x16_bf16: table and
// data each split into a BF16 head and a BF16 remainder, three products
// head*head + head*rem + rem*head accumulated in FP32, about 2^-16 relative).
#include "tdfe_fold.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

constexpr int ENG_F64 = 0, ENG_F32 = 1, ENG_BF16X3 = 2;
constexpr int MTHREADS = 256;  // four waves
constexpr int MCOLS = 16;      // real columns per block (the products' N)
constexpr int NTAB = 6;        // x forward [B;D], B, Dg, Dg^T, B^T, x backward [B^T | D^T]

template <int E>
struct Eng;
template <>
struct Eng<ENG_F64> {
  using T = double;
  using V = v4d;
};
template <>
struct Eng<ENG_F32> {
  using T = float;
  using V = v4f;
};
template <>
struct Eng<ENG_BF16X3> {
  using T = float;
  using V = v4f;
};

// BF16 bits of x, rounded to nearest even (x finite)
__device__ __forceinline__ short bf16_rn(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(short h) { return __uint_as_float(((unsigned)(unsigned short)h) << 16); }

// the lane's operand of a table: FP64 / FP32 hold A[m][4 s + g] for the k
// steps s; BF16 holds A[m][4 g + q], q = 0..3, as head and remainder
template <int E>
struct TabOp {
  typename Eng<E>::T a[4];
};
template <>
struct TabOp<ENG_BF16X3> {
  v4s hi, lo;
};

template <int E>
__device__ __forceinline__ TabOp<E> load_tab(const double* __restrict__ tab, int t, int m, int g) {
  TabOp<E> A;
  const double* row = tab + t * 256 + m * 16;
  if constexpr (E == ENG_BF16X3) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float x = (float)row[4 * g + q];
      const short h = bf16_rn(x);
      A.hi[q] = h;
      A.lo[q] = bf16_rn(x - bf16_val(h));
    }
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) A.a[s] = (typename Eng<E>::T)row[4 * s + g];
  }
  return A;
}

template <int E>
__device__ __forceinline__ typename Eng<E>::V zero_acc() {
  typename Eng<E>::V v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = 0;
  return v;
}

// acc += A X for one line: X's k-th input is in0[(base + k stride) RS + c]
// for k < N and in1[(base + (k - N) stride) RS + c] for N <= k < K
template <int E, int N, int K, int RS>
__device__ __forceinline__ void contract(const TabOp<E>& A, const typename Eng<E>::T* in0,
                                         const typename Eng<E>::T* in1, int base, int stride, int g, int c,
                                         typename Eng<E>::V& acc) {
  using T = typename Eng<E>::T;
  static_assert(K <= 16, "k <= 16");
  auto ld = [&](int k) -> T {
    if (k >= K) return (T)0;
    const T* src = k < N ? in0 : in1;
    const int kk = k < N ? k : k - N;
    return src[(base + kk * stride) * RS + c];
  };
  if constexpr (E == ENG_BF16X3) {
    v4s bh, bl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float x = ld(4 * g + q);
      const short h = bf16_rn(x);
      bh[q] = h;
      bl[q] = bf16_rn(x - bf16_val(h));
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.lo, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.hi, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.hi, bh, acc, 0, 0, 0);
  } else {
    constexpr int KS = (K + 3) / 4;
    T b[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) b[s] = ld(4 * s + g);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      if constexpr (E == ENG_F64)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A.a[s], b[s], acc, 0, 0, 0);
      else
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a[s], b[s], acc, 0, 0, 0);
    }
  }
}

// output row of register r in lane group g: the FP32 and BF16 products hold
// rows 4 g .. 4 g + 3, the FP64 product rows g, g + 4, g + 8, g + 12
template <int E>
__device__ __forceinline__ int out_row(int g, int r) {
  return E == ENG_F64 ? g + 4 * r : 4 * g + r;
}

// rows m = out_row(g, r) of acc: m < N to out0, N <= m < M to out1
template <int E, int N, int M, int RS>
__device__ __forceinline__ void store_rows(const typename Eng<E>::V& acc, typename Eng<E>::T* out0,
                                           typename Eng<E>::T* out1, int base, int stride, int g, int c) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = out_row<E>(g, r);
    if (m < M) {
      auto* dst = m < N ? out0 : out1;
      dst[(base + (m < N ? m : m - N) * stride) * RS + c] = acc[r];
    }
  }
}

template <int E, int N, int RS>
__device__ __forceinline__ typename Eng<E>::V load_rows(const typename Eng<E>::T* src, int base, int stride, int g,
                                                        int c) {
  auto v = zero_acc<E>();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = out_row<E>(g, r);
    if (m < N) v[r] = src[(base + m * stride) * RS + c];
  }
  return v;
}

// orders this wave's LDS stores before its following LDS loads (other lanes read them)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct MParams {
  const void* x;
  void* y;
  int ld, cols, nchunks;
  const double* colscale;
  double kin;
  const void* vw;
  const double* m1x;  // separable M^-1/2 factors along x, y, z
  const double* m1y;
  const double* m1z;
  const double* cellgeo;  // [n_cell][4]: metric factors g_x, g_y, g_z, det J
  const double* tab;      // [NTAB][16][16]
  double* energy;
  const int* done;
  int ncx, ncy, ncz, p, Nx, Ny, Nz;
  int64_t n_cell;
  double wq[TDFE_MAXN];
};

template <int E, int N>
constexpr int mfma_lds() {
  return 3 * N * N * N * MCOLS * (int)sizeof(typename Eng<E>::T) + N * N * N * (int)sizeof(typename Eng<E>::T) +
         TDFE_MAXN * 8 + MTHREADS * 8;
}

template <int E, int N, int LB>
__global__ void __launch_bounds__(MTHREADS) mfma_box_kernel(MParams P) {
  using T = typename Eng<E>::T;
  using V = typename Eng<E>::V;
  constexpr int VOL = N * N * N;
  constexpr int NL = N * N;  // lines per sweep
  constexpr int RS = MCOLS;  // row stride of the LDS arrays
  __shared__ T sA[3 * VOL * RS];
  __shared__ T sV[VOL];
  __shared__ double sW[TDFE_MAXN];
  __shared__ double sRed[MTHREADS];
  if (P.done && *P.done) return;

  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int L = remap_block(blockIdx.x, gridDim.x);
  const int chunk = L % P.nchunks;
  const int64_t cell = L / P.nchunks;
  const int cx = (int)(cell % P.ncx), cy = (int)((cell / P.ncx) % P.ncy);
  const int cz = (int)(cell / ((int64_t)P.ncx * P.ncy));
  const T* __restrict__ X = (const T*)P.x;
  T* __restrict__ Y = (T*)P.y;
  T* A0 = sA;
  T* A1 = sA + VOL * RS;
  T* A2 = sA + 2 * VOL * RS;
  const int NxI = P.Nx - 2, NyI = P.Ny - 2;

  // gather (x M^-1/2 x column scale); Dirichlet nodes and absent columns are 0
  for (int q = t; q < VOL * MCOLS; q += MTHREADS) {
    const int r = q >> 4, cc = q & 15;
    const int i = r % N, j = (r / N) % N, k = r / (N * N);
    const int I = cx * P.p + i, J = cy * P.p + j, K = cz * P.p + k;
    const int colg = chunk * MCOLS + cc;
    const bool ok = colg < P.cols && I > 0 && I < P.Nx - 1 && J > 0 && J < P.Ny - 1 && K > 0 && K < P.Nz - 1;
    T v = (T)0;
    if (ok) {
      const int64_t e = ((int64_t)(I - 1) + (int64_t)NxI * ((int64_t)(J - 1) + (int64_t)NyI * (K - 1))) * P.ld + colg;
      const double s = P.m1x[I] * P.m1y[J] * P.m1z[K] * (P.colscale ? P.colscale[colg >> 1] : 1.0);
      v = X[e] * (T)s;
    }
    A0[r * RS + cc] = v;
  }
  for (int q = t; q < VOL; q += MTHREADS) sV[q] = P.vw ? ((const T*)P.vw)[cell * VOL + q] : (T)0;
  if (t < TDFE_MAXN) sW[t] = P.wq[t];
  const double gx = P.kin * P.cellgeo[cell * 4 + 0];
  const double gy = P.kin * P.cellgeo[cell * 4 + 1];
  const double gz = P.kin * P.cellgeo[cell * 4 + 2];
  const TabOp<E> Tx = load_tab<E>(P.tab, 0, c, g);   // [B; D]
  const TabOp<E> Tb = load_tab<E>(P.tab, 1, c, g);   // B
  const TabOp<E> Tg = load_tab<E>(P.tab, 2, c, g);   // Dg
  const TabOp<E> Tgt = load_tab<E>(P.tab, 3, c, g);  // Dg^T
  const TabOp<E> Tbt = load_tab<E>(P.tab, 4, c, g);  // B^T
  const TabOp<E> Txt = load_tab<E>(P.tab, 5, c, g);  // [B^T | D^T]
  double en = 0.0;
  __syncthreads();

  // line L of a sweep: x lines (j, k), y lines (i, k), z lines (i, j)
  auto xbase = [](int l) { return N * (l % N) + N * N * (l / N); };
  auto ybase = [](int l) { return (l % N) + N * N * (l / N); };
  auto zbase = [](int l) { return (l % N) + N * (l / N); };

  // ---- x: A0 <- B u, A1 <- D u ----
  for (int l0 = wv * LB; l0 < NL; l0 += 4 * LB) {
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      const int l = l0 + b;
      if (l < NL) {
        V acc = zero_acc<E>();
        contract<E, N, N, RS>(Tx, A0, A0, xbase(l), 1, g, c, acc);
        store_rows<E, N, 2 * N, RS>(acc, A0, A1, xbase(l), 1, g, c);
      }
    }
  }
  __syncthreads();
  // ---- y: A0 <- B A0, A1 <- B A1 ----
  for (int l0 = wv * LB; l0 < NL; l0 += 4 * LB) {
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      const int l = l0 + b;
      if (l < NL) {
        V a0 = zero_acc<E>(), a1 = zero_acc<E>();
        contract<E, N, N, RS>(Tb, A0, A0, ybase(l), N, g, c, a0);
        contract<E, N, N, RS>(Tb, A1, A1, ybase(l), N, g, c, a1);
        store_rows<E, N, N, RS>(a0, A0, A0, ybase(l), N, g, c);
        store_rows<E, N, N, RS>(a1, A1, A1, ybase(l), N, g, c);
      }
    }
  }
  __syncthreads();
  // ---- z: A0 <- B A0 (u_q), A1 <- fx(B A1) ----
  for (int l0 = wv * LB; l0 < NL; l0 += 4 * LB) {
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      const int l = l0 + b;
      if (l < NL) {
        V a0 = zero_acc<E>(), a1 = zero_acc<E>();
        contract<E, N, N, RS>(Tb, A0, A0, zbase(l), N * N, g, c, a0);
        contract<E, N, N, RS>(Tb, A1, A1, zbase(l), N * N, g, c, a1);
        const double wl = sW[l % N] * sW[l / N];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = out_row<E>(g, r);
          if (m < N) {
            const T d = a1[r];
            const T f = (T)(gx * wl * sW[m]) * d;
            en += (double)f * (double)d;
            a1[r] = f;
          }
        }
        store_rows<E, N, N, RS>(a0, A0, A0, zbase(l), N * N, g, c);
        store_rows<E, N, N, RS>(a1, A1, A1, zbase(l), N * N, g, c);
      }
    }
  }
  __syncthreads();
  // ---- y: A2 <- fy(Dg A0); A2 <- Dg^T A2 + V u_q ----
  for (int l0 = wv * LB; l0 < NL; l0 += 4 * LB) {
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      const int l = l0 + b;
      if (l < NL) {
        const int base = ybase(l);
        V d = zero_acc<E>();
        contract<E, N, N, RS>(Tg, A0, A0, base, N, g, c, d);
        const double wl = sW[l % N] * sW[l / N];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = out_row<E>(g, r);
          if (m < N) {
            const T f = (T)(gy * wl * sW[m]) * d[r];
            en += (double)f * (double)d[r];
            d[r] = f;
          }
        }
        store_rows<E, N, N, RS>(d, A2, A2, base, N, g, c);
        // seed: V u_q at the line's points
        V s = load_rows<E, N, RS>(A0, base, N, g, c);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = out_row<E>(g, r);
          if (m < N) {
            const T u = s[r];
            const T pv = sV[base + m * N] * u;
            en += (double)pv * (double)u;
            s[r] = pv;
          }
        }
        wave_sync();
        contract<E, N, N, RS>(Tgt, A2, A2, base, N, g, c, s);
        wave_sync();
        store_rows<E, N, N, RS>(s, A2, A2, base, N, g, c);
      }
    }
  }
  __syncthreads();
  // ---- z: A0 <- fz(Dg A0); A2 <- Dg^T A0 + A2; A2 <- B^T A2; A1 <- B^T A1 ----
  for (int l0 = wv * LB; l0 < NL; l0 += 4 * LB) {
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      const int l = l0 + b;
      if (l < NL) {
        const int base = zbase(l);
        constexpr int S = N * N;
        V d = zero_acc<E>();
        contract<E, N, N, RS>(Tg, A0, A0, base, S, g, c, d);
        const double wl = sW[l % N] * sW[l / N];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = out_row<E>(g, r);
          if (m < N) {
            const T f = (T)(gz * wl * sW[m]) * d[r];
            en += (double)f * (double)d[r];
            d[r] = f;
          }
        }
        V a1 = zero_acc<E>();
        contract<E, N, N, RS>(Tbt, A1, A1, base, S, g, c, a1);
        store_rows<E, N, N, RS>(d, A0, A0, base, S, g, c);
        store_rows<E, N, N, RS>(a1, A1, A1, base, S, g, c);
        V s = load_rows<E, N, RS>(A2, base, S, g, c);
        wave_sync();
        contract<E, N, N, RS>(Tgt, A0, A0, base, S, g, c, s);
        wave_sync();
        store_rows<E, N, N, RS>(s, A2, A2, base, S, g, c);
        wave_sync();
        V o = zero_acc<E>();
        contract<E, N, N, RS>(Tbt, A2, A2, base, S, g, c, o);
        wave_sync();
        store_rows<E, N, N, RS>(o, A2, A2, base, S, g, c);
      }
    }
  }
  __syncthreads();
  // ---- y: A2 <- B^T A2, A1 <- B^T A1 ----
  for (int l0 = wv * LB; l0 < NL; l0 += 4 * LB) {
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      const int l = l0 + b;
      if (l < NL) {
        V a2 = zero_acc<E>(), a1 = zero_acc<E>();
        contract<E, N, N, RS>(Tbt, A2, A2, ybase(l), N, g, c, a2);
        contract<E, N, N, RS>(Tbt, A1, A1, ybase(l), N, g, c, a1);
        store_rows<E, N, N, RS>(a2, A2, A2, ybase(l), N, g, c);
        store_rows<E, N, N, RS>(a1, A1, A1, ybase(l), N, g, c);
      }
    }
  }
  __syncthreads();
  // ---- x: A2 <- B^T A2 + D^T A1 ----
  for (int l0 = wv * LB; l0 < NL; l0 += 4 * LB) {
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      const int l = l0 + b;
      if (l < NL) {
        V acc = zero_acc<E>();
        contract<E, N, 2 * N, RS>(Txt, A2, A1, xbase(l), 1, g, c, acc);
        store_rows<E, N, N, RS>(acc, A2, A2, xbase(l), 1, g, c);
      }
    }
  }
  sRed[t] = en;
  __syncthreads();
  // scatter-add (x M^-1/2)
  for (int q = t; q < VOL * MCOLS; q += MTHREADS) {
    const int r = q >> 4, cc = q & 15;
    const int i = r % N, j = (r / N) % N, k = r / (N * N);
    const int I = cx * P.p + i, J = cy * P.p + j, K = cz * P.p + k;
    const int colg = chunk * MCOLS + cc;
    if (colg < P.cols && I > 0 && I < P.Nx - 1 && J > 0 && J < P.Ny - 1 && K > 0 && K < P.Nz - 1) {
      const int64_t e = ((int64_t)(I - 1) + (int64_t)NxI * ((int64_t)(J - 1) + (int64_t)NyI * (K - 1))) * P.ld + colg;
      unsafeAtomicAdd(Y + e, A2[r * RS + cc] * (T)(P.m1x[I] * P.m1y[J] * P.m1z[K]));
    }
  }
  // per-column quadratic form: lanes of column c in the four waves and four lane groups
  if (P.energy && t < MCOLS) {
    double acc = 0.0;
    for (int u = 0; u < 16; ++u) acc += sRed[(u >> 2) * 64 + (u & 3) * 16 + t];
    const int colg = chunk * MCOLS + t;
    if (colg < P.cols) P.energy[cell * P.cols + colg] = acc;
  }
}

template <int E, int N>
tdfe_status launch_mfma_n(tdfe_ctx* c, MParams& P, int64_t* groups_out) {
  static_assert(mfma_lds<E, N>() <= 160 * 1024, "LDS");
  P.nchunks = (P.cols + MCOLS - 1) / MCOLS;
  if (groups_out) *groups_out = c->n_cell;
  hipLaunchKernelGGL((mfma_box_kernel<E, N, 2>), dim3((unsigned)(c->n_cell * P.nchunks)), dim3(MTHREADS), 0,
                     c->stream, P);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

template <int E>
tdfe_status launch_mfma_e(tdfe_ctx* c, MParams& P, int64_t* g) {
  switch (c->n) {
    case 2: return launch_mfma_n<E, 2>(c, P, g);
    case 3: return launch_mfma_n<E, 3>(c, P, g);
    case 4: return launch_mfma_n<E, 4>(c, P, g);
    case 5: return launch_mfma_n<E, 5>(c, P, g);
    case 6: return launch_mfma_n<E, 6>(c, P, g);
    case 7: return launch_mfma_n<E, 7>(c, P, g);
  }
  if constexpr (E != ENG_F64) {
    if (c->n == 8) return launch_mfma_n<E, 8>(c, P, g);
  }
  return tdfe_fail(c, TDFE_EINVAL, "matrix-core operator: order p=%d not supported", c->p);
}

}  // namespace

bool tdfe_mfma_kernel_ok(const tdfe_ctx* c, const ApplyArgs& a) {
  // launches in the context's own storage precision (an FP64 launch in an
  // FP32 matrix-core context takes the VALU kernels)
  return c->box && c->mfma_tab && a.lowdin && !a.fullgrid && a.fp32 == tdfe_fp32(c) &&
         (c->n <= 7 || (a.fp32 && c->n <= 8));
}

// the stacked, zero-padded 16 x 16 tables of the matrix-core operator,
// [NTAB][16][16] (host side; uploaded at bind)
void tdfe_mfma_tables(int p, double* out) {
  const tdfe1d::Rule R = tdfe1d::make_rule(p);
  const int N = p + 1;
  for (int i = 0; i < NTAB * 256; ++i) out[i] = 0.0;
  auto at = [&](int t, int m, int k) -> double& { return out[t * 256 + m * 16 + k]; };
  for (int a = 0; a < N; ++a)
    for (int i = 0; i < N; ++i) {
      const double B = R.B[a * TDFE_MAXN + i], D = R.D[a * TDFE_MAXN + i], G = R.Dg[a * TDFE_MAXN + i];
      at(0, a, i) = B;
      at(0, N + a, i) = D;
      at(1, a, i) = B;
      at(2, a, i) = G;
      at(3, i, a) = G;
      at(4, i, a) = B;
      at(5, i, a) = B;
      at(5, i, N + a) = D;
    }
}

tdfe_status tdfe_launch_apply_mfma(tdfe_ctx* c, const ApplyArgs& a) {
  if (a.cols < 1) return tdfe_fail(c, TDFE_EINVAL, "apply: cols < 1");
  if (!tdfe_mfma_kernel_ok(c, a)) return tdfe_fail(c, TDFE_EINVAL, "matrix-core operator: unsupported mesh or launch");
  static_assert(sizeof(MParams) <= 4096, "kernel arguments exceed 4 KB");
  MParams P{};
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
  P.tab = c->mfma_tab;
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
  for (int i = 0; i < c->n; ++i) P.wq[i] = c->wq[i];
  if (!a.fp32) return launch_mfma_e<ENG_F64>(c, P, a.n_blocks_out);
  if (c->precision == TDFE_BF16_MFMA) return launch_mfma_e<ENG_BF16X3>(c, P, a.n_blocks_out);
  return launch_mfma_e<ENG_F32>(c, P, a.n_blocks_out);
}
