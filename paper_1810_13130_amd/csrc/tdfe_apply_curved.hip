// Operator kernel for trilinear (curved) cells in the plane layout of the box
// kernel (Eq. DiscreteHamiltonian in the Loewdin form, Eq. TDKSMatVecStandard).
//
// A thread owns an n x n plane of one column of one cell:
//   A  (plane at node y = j): gather u(i,k) (x M^-1/2); x: B u, D u; z: B on both
//   -- LDS transpose of the two arrays -->
//   B  (plane at Gauss x = a): y: B on both -> u_q, d_x u_q; d_y u_q and d_z u_q
//      by the Gauss collocation derivative; the full metric
//      G = w detJ J^-1 J^-T (6 values per Gauss point, from the 8 cell corners,
//      staged in LDS per block) gives the three fluxes; V u_q; the y and z
//      transposed derivatives; transposed y interpolation of (V u_q + ...) and of
//      the x flux
//   -- LDS transpose of the two arrays -->
//   C  (plane at node y = j): x: B^T s + D^T s_x; z: B^T; scatter-add (x M^-1/2).
// The x derivative is taken on the nodes (D = Dg B along x) so that x never
// crosses threads; only y does.  Contractions use the even/odd folded tables.
#include "tdfe_fold.h"

namespace {

template <typename T>
struct CurvedParams {
  const void* x;
  void* y;
  int ld, cols, nchunks;
  const double* colscale;
  double kin;
  const void* vw;
  const double* minv;
  const float* minv32;  // FP32 copy (FP32 kernels)
  const double* corners;  // [n_cell][2][2][2][3]
  double* energy;
  const int* done;
  int ncx, ncy, ncz, p, Nx, Ny, Nz;
  int64_t n_cell;
  int lowdin, fullgrid;
  double eta[TDFE_MAXN];  // Gauss points on [-1, 1]
  double wq[TDFE_MAXN];   // Gauss weights
};

template <typename T, int N>
constexpr int cplane_wpe() {
  return sizeof(T) == 4 ? 2 : 1;
}

template <typename T, int N, int CB, int CPB>
__global__ void __launch_bounds__(CPB * N * CB) __attribute__((amdgpu_waves_per_eu(cplane_wpe<T, N>())))
    cplane_kernel(CurvedParams<T> P) {
  constexpr int VOL = N * N * N;
  constexpr int THREADS = CPB * N * CB;
  // 1D tables of order N, folded, as compile-time constants
  constexpr FoldSet<N> FS = make_foldset<N>();
  __shared__ T sX[CPB * VOL * CB];
  __shared__ T sV[CPB * VOL];
  __shared__ T sG[CPB * VOL * 6];
  __shared__ T sM[CPB * VOL];
  __shared__ double sRed[THREADS];
  if (P.done && *P.done) return;

  const int t = threadIdx.x;
  const int L = remap_block(blockIdx.x, gridDim.x);
  const int chunk = L % P.nchunks;
  const int group = L / P.nchunks;
  const int col = t % CB;
  const int pl = (t / CB) % N;
  const int slot = t / (CB * N);
  const int64_t cell = (int64_t)group * CPB + slot;
  const bool cell_ok = cell < P.n_cell;
  const int colg = chunk * CB + col;
  const bool act = cell_ok && colg < P.cols;

  int cx = 0, cy = 0, cz = 0;
  if (cell_ok) {
    cx = (int)(cell % P.ncx);
    cy = (int)((cell / P.ncx) % P.ncy);
    cz = (int)(cell / ((int64_t)P.ncx * P.ncy));
  }
  const T* __restrict__ X = (const T*)P.x;
  T* __restrict__ Y = (T*)P.y;
  // M^-1/2 in the kernel's precision (a conversion right after each load
  // would make the gather wait for every value)
  using MT = T;
  const MT* __restrict__ MV;
  if constexpr (sizeof(T) == 8)
    MV = (const MT*)P.minv;
  else
    MV = (const MT*)P.minv32;
  T cs = act ? (T)1 : (T)0;
  if (P.colscale && act) cs = (T)P.colscale[colg >> 1];

  // block staging in three steps, so that a wave waits for memory once and
  // computes while its gather is in flight: (1) the block's potential and cell
  // corners are loaded into registers and the phase A gather (values and
  // M^-1/2 per node) is issued; (2) potential and corners go to LDS; (3) the
  // metric of every Gauss point of the block is computed from the LDS corners;
  // only then are the gathered values used.
  constexpr int NV = (CPB * VOL + THREADS - 1) / THREADS;
  constexpr int NCR = (CPB * 24 + THREADS - 1) / THREADS;
  __shared__ double sC[CPB * 24];
  __shared__ double sEW[2 * N];  // Gauss points, then weights
  {
    constexpr tdfe1d::Rule R = tdfe1d::make_rule(N - 1);
    if (t < 2 * N) {
      double v = R.eta[0];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        v = t == q ? R.eta[q] : v;
        v = t == N + q ? R.wq[q] : v;
      }
      sEW[t] = v;
    }
  }
  const int64_t c0 = (int64_t)group * CPB;
  // per-node scale of the block's cells, staged once per block (the column
  // lanes of a plane share it): M^-1/2 on DoFs (1 without the Loewdin
  // scaling) and 0 on Dirichlet nodes and past the last cell, which zeroes
  // their gathered values and their scattered contributions
  constexpr int NM = NV;
  T mr[NM];
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    const int q = t + k * THREADS;
    const int64_t ce = c0 + q / VOL;
    const int r = q % VOL;
    bool in = q < CPB * VOL && ce < P.n_cell;
    int64_t idx = 0;
    if (in) {
      const int ex = (int)(ce % P.ncx), ey = (int)((ce / P.ncx) % P.ncy), ez = (int)(ce / ((int64_t)P.ncx * P.ncy));
      const int I = ex * P.p + r % N, Jn = ey * P.p + (r / N) % N, K = ez * P.p + r / (N * N);
      if (!P.fullgrid) {
        in = I > 0 && I < P.Nx - 1 && Jn > 0 && Jn < P.Ny - 1 && K > 0 && K < P.Nz - 1;
        idx = (int64_t)(I - 1) + (int64_t)(P.Nx - 2) * ((int64_t)(Jn - 1) + (int64_t)(P.Ny - 2) * (K - 1));
      }
    }
    const T mval = MV[(in && P.lowdin) ? idx : 0];
    mr[k] = in ? (P.lowdin ? mval : (T)1) : (T)0;
  }
  T vr[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int q = t + k * THREADS;
    const int64_t ce = c0 + q / VOL;
    // zeros without a potential, so that phase B needs no branch on it
    const bool ok = P.vw && q < CPB * VOL && ce < P.n_cell;
    vr[k] = ok ? ((const T*)P.vw)[ce * VOL + q % VOL] : (T)0;
  }
  double cr[NCR];
#pragma unroll
  for (int k = 0; k < NCR; ++k) {
    const int f = t + k * THREADS;
    const bool ok = f < CPB * 24 && c0 + f / 24 < P.n_cell;
    const double val = P.corners[ok ? c0 * 24 + f : 0];
    cr[k] = ok ? val : 0.0;
  }
  auto sidx = [&](int y, int x, int z) { return (((slot * N + y) * N + x) * N + z) * CB + col; };
  const int NxI = P.Nx - 2, NyI = P.Ny - 2;

  // node (i, j, k) of this cell -> element offset and inside flag
  const int J = cy * P.p + pl;
  const bool jok = P.fullgrid ? true : (J > 0 && J < P.Ny - 1);
  unsigned imask = 0, kmask = 0;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const int I = cx * P.p + q, K = cz * P.p + q;
    if (P.fullgrid || (I > 0 && I < P.Nx - 1)) imask |= 1u << q;
    if (P.fullgrid || (K > 0 && K < P.Nz - 1)) kmask |= 1u << q;
  }
  if (!act || !jok) imask = 0;
  int64_t n0, nk;  // node index of (0, j, 0) and the node stride along z
  if (P.fullgrid) {
    n0 = (int64_t)cx * P.p + (int64_t)P.Nx * ((int64_t)J + (int64_t)P.Ny * cz * P.p);
    nk = (int64_t)P.Nx * P.Ny;
  } else {
    n0 = (int64_t)(cx * P.p - 1) + (int64_t)NxI * ((int64_t)(J - 1) + (int64_t)NyI * (cz * P.p - 1));
    nk = (int64_t)NxI * NyI;
  }

  // metric of the block's Gauss points from the LDS corners (read in phase B,
  // after the transposes' barriers); Gauss points and weights from LDS
  auto compute_metric = [&]() {
      for (int it = t; it < CPB * VOL; it += THREADS) {
        const int sl = it / VOL, q = it % VOL;
        const int64_t ce = c0 + sl;
        T* g = sG + it * 6;
        if (ce >= P.n_cell) {
          for (int w6 = 0; w6 < 6; ++w6) g[w6] = (T)0;
          continue;
        }
        const int a = q % N, b = (q / N) % N, c = q / (N * N);
        const double xa = sEW[a], xb = sEW[b], xc = sEW[c];
        const double f[2][3] = {{0.5 * (1 - xa), 0.5 * (1 - xb), 0.5 * (1 - xc)},
                                {0.5 * (1 + xa), 0.5 * (1 + xb), 0.5 * (1 + xc)}};
        const double* C = sC + sl * 24;
        double Jm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int vz = 0; vz < 2; ++vz)
          for (int vy = 0; vy < 2; ++vy)
            for (int vx = 0; vx < 2; ++vx) {
              const double* X3 = C + ((vz * 2 + vy) * 2 + vx) * 3;
              const double d0 = (vx ? 0.5 : -0.5) * f[vy][1] * f[vz][2];
              const double d1 = f[vx][0] * (vy ? 0.5 : -0.5) * f[vz][2];
              const double d2 = f[vx][0] * f[vy][1] * (vz ? 0.5 : -0.5);
              for (int d = 0; d < 3; ++d) {
                Jm[d][0] += X3[d] * d0;
                Jm[d][1] += X3[d] * d1;
                Jm[d][2] += X3[d] * d2;
              }
            }
        double A[3][3];  // adjugate rows: J^-1 = A / det
        A[0][0] = Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1];
        A[0][1] = Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2];
        A[0][2] = Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1];
        A[1][0] = Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2];
        A[1][1] = Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0];
        A[1][2] = Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2];
        A[2][0] = Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0];
        A[2][1] = Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1];
        A[2][2] = Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0];
        const double det = Jm[0][0] * A[0][0] + Jm[0][1] * A[1][0] + Jm[0][2] * A[2][0];
        const double s = P.kin * sEW[N + a] * sEW[N + b] * sEW[N + c] / det;
        g[0] = (T)(s * (A[0][0] * A[0][0] + A[0][1] * A[0][1] + A[0][2] * A[0][2]));
        g[1] = (T)(s * (A[0][0] * A[1][0] + A[0][1] * A[1][1] + A[0][2] * A[1][2]));
        g[2] = (T)(s * (A[0][0] * A[2][0] + A[0][1] * A[2][1] + A[0][2] * A[2][2]));
        g[3] = (T)(s * (A[1][0] * A[1][0] + A[1][1] * A[1][1] + A[1][2] * A[1][2]));
        g[4] = (T)(s * (A[1][0] * A[2][0] + A[1][1] * A[2][1] + A[1][2] * A[2][2]));
        g[5] = (T)(s * (A[2][0] * A[2][0] + A[2][1] * A[2][1] + A[2][2] * A[2][2]));
      }
  };

  // ---------------- A: plane j = pl -------------------------------------------------------------
  T tu[N][N], tx[N][N];  // [x][z]
  {
    // FP64 (one wave per SIMD): the gather is issued first and the metric is
    // computed while it is in flight.  FP32 (fewer registers to spare): metric
    // first, then the gather.
    if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const int q = t + k * THREADS;
        if (q < CPB * VOL) {
          sV[q] = vr[k];
          sM[q] = mr[k];
        }
      }
#pragma unroll
      for (int k = 0; k < NCR; ++k) {
        const int f = t + k * THREADS;
        if (f < CPB * 24) sC[f] = cr[k];
      }
      __syncthreads();
      compute_metric();
    }
    // The gather reads through a buffer resource that starts at the block's
    // first node row: nodes outside the array (the Dirichlet planes at the
    // domain faces) have negative offsets or offsets past the end and read
    // 0; Dirichlet nodes inside its range (I = 0 or Nx-1, which alias a
    // neighbouring row's DoF) read a value that the zero in sM cancels.  No
    // address is selected and no value is masked.  The range is kept below
    // 2^31 bytes, so every negative 32-bit offset is out of range; a block
    // spans at most (n-1)(1 + row + plane) rows, far below that.
    T u[N][N];  // [i][k]: gathered values, all loads in flight together
    {
      // the resource is built from the block's first cell (the lowest rows
      // any of its cells touches) and made explicitly wave-uniform
      const int64_t rows = P.fullgrid ? (int64_t)P.Nx * P.Ny * P.Nz : (int64_t)NxI * NyI * (P.Nz - 2);
      const int bx = (int)(c0 % P.ncx), by = (int)((c0 / P.ncx) % P.ncy), bz = (int)(c0 / ((int64_t)P.ncx * P.ncy));
      const int64_t first = P.fullgrid ? (int64_t)bx * P.p + (int64_t)P.Nx * ((int64_t)by * P.p +
                                                                              (int64_t)P.Ny * bz * P.p)
                                       : (int64_t)(bx * P.p - 1) + (int64_t)NxI * ((int64_t)(by * P.p - 1) +
                                                                                 (int64_t)NyI * (bz * P.p - 1));
      const int64_t base = first > 0 ? first : 0;
      const int64_t bytes = (rows - base) * P.ld * (int64_t)sizeof(T);
      const uint64_t addr = (uint64_t)(uintptr_t)(X + base * P.ld);
      const uint32_t alo = __builtin_amdgcn_readfirstlane((uint32_t)addr);
      const uint32_t ahi = __builtin_amdgcn_readfirstlane((uint32_t)(addr >> 32));
      const int nrec = __builtin_amdgcn_readfirstlane((int)(bytes < 0x7fffffff ? bytes : 0x7fffffff));
      const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(uintptr_t)(((uint64_t)ahi << 32) | alo), 0, nrec, 0x00020000);
      const int ldb = P.ld * (int)sizeof(T);
      const int64_t kst = nk * ldb;
      const int64_t off0 = ((n0 - base) * P.ld + colg) * (int64_t)sizeof(T);
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const int ok = (int)(off0 + k * kst);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          if constexpr (sizeof(T) == 8)
            u[i][k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rx, ok + i * ldb, 0, 0));
          else
            u[i][k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, ok + i * ldb, 0, 0));
        }
      }
    }
    // keep the scaling below from being interleaved with the loads (which
    // would make each load wait for its own value)
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (sizeof(T) == 8) {
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const int q = t + k * THREADS;
        if (q < CPB * VOL) {
          sV[q] = vr[k];
          sM[q] = mr[k];
        }
      }
#pragma unroll
      for (int k = 0; k < NCR; ++k) {
        const int f = t + k * THREADS;
        if (f < CPB * 24) sC[f] = cr[k];
      }
      __syncthreads();
      compute_metric();
    }
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
      for (int i = 0; i < N; ++i) u[i][k] *= sM[slot * VOL + i + N * (pl + N * k)] * cs;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      T line[N], o1[N], o2[N];
#pragma unroll
      for (int i = 0; i < N; ++i) line[i] = u[i][k];
      eo2<T, N, 1, -1>(FS.B, FS.D, line, o1, o2);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        tu[a][k] = o1[a];
        tx[a][k] = o2[a];
      }
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
      T o1[N], o2[N];
      eo<T, N, 1>(FS.B, tu[a], o1);
      eo<T, N, 1>(FS.B, tx[a], o2);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        tu[a][c] = o1[c];
        tx[a][c] = o2[c];
      }
    }
  }
  // ---------------- transpose: (j; a, c) -> (a; j, c) --------------------------------------------
  T v[N][N], w[N][N];  // [y node][z point] at x point a = pl
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int c = 0; c < N; ++c) sX[sidx(pl, a, c)] = tu[a][c];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int c = 0; c < N; ++c) v[j][c] = sX[sidx(j, pl, c)];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int c = 0; c < N; ++c) sX[sidx(pl, a, c)] = tx[a][c];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int c = 0; c < N; ++c) w[j][c] = sX[sidx(j, pl, c)];
  __syncthreads();

  // ---------------- B: plane a = pl, Gauss points (b, c) ------------------------------------------
  double energy = 0.0;
  T dx[N][N], uq[N][N], dy[N][N];  // [b][c]; reused in place for the fluxes
#pragma unroll
  for (int c = 0; c < N; ++c) {
    T l1[N], l2[N], o1[N], o2[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      l1[j] = v[j][c];
      l2[j] = w[j][c];
    }
    eo<T, N, 1>(FS.B, l1, o1);
    eo<T, N, 1>(FS.B, l2, o2);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      uq[b][c] = o1[b];
      dx[b][c] = o2[b];
    }
  }
#pragma unroll
  for (int c = 0; c < N; ++c) {
    T l[N], d[N];
#pragma unroll
    for (int b = 0; b < N; ++b) l[b] = uq[b][c];
    eo<T, N, -1>(FS.G, l, d);
#pragma unroll
    for (int b = 0; b < N; ++b) dy[b][c] = d[b];
  }
  // per y line: z derivative, the three fluxes, the potential term and the
  // transposed z derivative; dx <- f_x, dy <- f_y, uq <- V u + Dg_z^T f_z
#pragma unroll
  for (int b = 0; b < N; ++b) {
    T dz[N], fz[N], r[N];
    eo<T, N, -1>(FS.G, uq[b], dz);
    T le = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const int q = pl + N * (b + N * c);
      const T* g = sG + (slot * VOL + q) * 6;
      const T ux = dx[b][c], uy = dy[b][c], uz = dz[c];
      const T fx = g[0] * ux + g[1] * uy + g[2] * uz;
      const T fy = g[1] * ux + g[3] * uy + g[4] * uz;
      const T f3 = g[2] * ux + g[4] * uy + g[5] * uz;
      const T pot = sV[slot * VOL + q] * uq[b][c];
      acc_energy<T>(energy, le, fx * ux + fy * uy + f3 * uz + pot * uq[b][c]);
      dx[b][c] = fx;
      dy[b][c] = fy;
      fz[c] = f3;
      uq[b][c] = pot;
    }
    flush_energy<T>(energy, le);
    eo<T, N, -1>(FS.Gt, fz, r);
#pragma unroll
    for (int c = 0; c < N; ++c) uq[b][c] += r[c];
    __builtin_amdgcn_sched_barrier(0);
  }
  // per z line: transposed y derivative of f_y, then transposed y interpolation
  // of both arrays: s_x = B_y^T f_x goes straight into the transpose buffer
  // (every thread has finished reading w), s = B_y^T (uq + Dg_y^T f_y) stays
  T s[N][N];  // [j][c]
#pragma unroll
  for (int c = 0; c < N; ++c) {
    T l[N], r[N], o[N];
#pragma unroll
    for (int b = 0; b < N; ++b) l[b] = dx[b][c];
    eo<T, N, 1>(FS.Bt, l, o);
#pragma unroll
    for (int j = 0; j < N; ++j) sX[sidx(j, pl, c)] = o[j];
#pragma unroll
    for (int b = 0; b < N; ++b) l[b] = dy[b][c];
    eo<T, N, -1>(FS.Gt, l, r);
#pragma unroll
    for (int b = 0; b < N; ++b) l[b] = uq[b][c] + r[b];
    eo<T, N, 1>(FS.Bt, l, o);
#pragma unroll
    for (int j = 0; j < N; ++j) s[j][c] = o[j];
  }
  // ---------------- transposes: (a; j, c) -> (j; a, c) -------------------------------------------
  // the quadratic form is parked in LDS first (keeps its accumulation chain
  // from being sunk into the final reduction)
  sRed[t] = act ? energy : 0.0;
  T s2[N][N], sx2[N][N];  // [x point a][z point c] at node plane j = pl
  __syncthreads();
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int c = 0; c < N; ++c) sx2[a][c] = sX[sidx(pl, a, c)];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int c = 0; c < N; ++c) sX[sidx(j, pl, c)] = s[j][c];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int c = 0; c < N; ++c) s2[a][c] = sX[sidx(pl, a, c)];

  // ---------------- C: plane j = pl: x then z transposed, scatter ---------------------------------
  {
    T h[N][N];  // [i][c]
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T l1[N], l2[N], o1[N], o2[N];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        l1[a] = s2[a][c];
        l2[a] = sx2[a][c];
      }
      eo<T, N, 1>(FS.Bt, l1, o1);
      eo<T, N, -1>(FS.Dt, l2, o2);
#pragma unroll
      for (int i = 0; i < N; ++i) h[i][c] = o1[i] + o2[i];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      // the line's M^-1/2 values are loaded before its contraction, so that
      // one wait per line covers them
      T ml[N];
#pragma unroll
      for (int k = 0; k < N; ++k) ml[k] = sM[slot * VOL + i + N * (pl + N * k)];
      T o[N];
      eo<T, N, 1>(FS.Bt, h[i], o);
      // imask / kmask depend on the cell only, so these branches are uniform
      // whenever a wave holds one cell; act and the plane's own row test are
      // folded into imask
      if ((imask >> i) & 1u) {
        T* yrow = Y + ((n0 + i) * P.ld + colg);
#pragma unroll
        for (int k = 0; k < N; ++k)
          if ((kmask >> k) & 1u) unsafeAtomicAdd(yrow + (int64_t)k * nk * P.ld, o[k] * ml[k]);
      }
    }
  }
  // ---------------- per-column quadratic form ------------------------------------------------------
  if (P.energy) {
    __syncthreads();
    if (t < CB) {
      double acc = 0.0;
      for (int u = t; u < THREADS; u += CB) acc += sRed[u];
      if (chunk * CB + t < P.cols) P.energy[(int64_t)group * P.cols + chunk * CB + t] = acc;
    }
  }
}

// LDS bytes of one block of cpb cells (transpose buffer, potential, 6 metric
// entries per Gauss point, quadratic-form partials)
template <typename T, int N, int CB>
constexpr int cplane_lds(int cpb) {
  constexpr int VOL = N * N * N;
  return cpb * VOL * CB * (int)sizeof(T) + cpb * VOL * (int)sizeof(T) * 8 + cpb * N * CB * 8 + cpb * 24 * 8;
}

// cells per block: at most 512 threads; the metric makes a cell's LDS about
// 1.4x that of a box cell, so the budgets are larger than the box kernel's
// (an FP64 block still runs alone on its CU at one wave per SIMD)
template <typename T, int N, int CB>
constexpr int cplane_cpb() {
  constexpr int budget = sizeof(T) == 8 ? 96 * 1024 : 48 * 1024;
  int cpb = 1;
  while (cpb * 2 * N * CB <= 512 && cplane_lds<T, N, CB>(cpb * 2) <= budget) cpb *= 2;
  return cpb;
}

template <typename T, int N, int CB>
tdfe_status launch_cplane(tdfe_ctx* c, CurvedParams<T>& P, int64_t* groups_out) {
  constexpr int CPB = cplane_cpb<T, N, CB>();
  static_assert(cplane_lds<T, N, CB>(CPB) <= 160 * 1024, "LDS");
  const int64_t groups = (c->n_cell + CPB - 1) / CPB;
  P.nchunks = (P.cols + CB - 1) / CB;
  if (groups_out) *groups_out = groups;
  hipLaunchKernelGGL((cplane_kernel<T, N, CB, CPB>), dim3((unsigned)(groups * P.nchunks)), dim3(CPB * N * CB), 0,
                     c->stream, P);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

// columns per block: the next power of two up to 16; FP32 launches of more
// than 16 columns take 32 per block, so that a node's row of columns (128 B)
// is read by one block and the block's metric serves all of them (two blocks
// of 16 each fetched half of every row and computed the metric twice:
// 2.3x the algorithmic HBM traffic on the graded workload)
template <typename T, int N>
tdfe_status launch_cplane_n(tdfe_ctx* c, CurvedParams<T>& P, int64_t* g) {
  if (P.cols <= 1) return launch_cplane<T, N, 1>(c, P, g);
  if (P.cols <= 2) return launch_cplane<T, N, 2>(c, P, g);
  if (P.cols <= 4) return launch_cplane<T, N, 4>(c, P, g);
  if (P.cols <= 8) return launch_cplane<T, N, 8>(c, P, g);
  if constexpr (sizeof(T) == 4)
    if (P.cols > 16) return launch_cplane<T, N, 32>(c, P, g);
  return launch_cplane<T, N, 16>(c, P, g);
}

// ------------------------------------------------------------------------------------------------
// Lane-pair variant: the n x n plane of one column is shared by an adjacent
// lane pair, each lane holding its half of the z index range (lane 0 the
// indices 0..H-1, lane 1 their mirror images n-1..n-H, H = n/2) plus, for odd
// n, a copy of the middle index H.  x and y contractions stay in the lane;
// a z contraction forms in each lane the partial sums over its own entries
// for its own outputs and for the partner's and swaps the latter by a DPP quad
// permutation.  The tables' mirror symmetry A[n-1-c][n-1-k] = S A[c][k] lets
// both lanes run the same code (lane 1 multiplies its inputs by S); the shared
// middle entry enters each lane's partial sums with half its weight, so both
// lanes end with the same middle outputs; only lane 0 scatters them, and each
// lane counts them in the quadratic form with half weight.  A lane keeps
// about 4/7 of a plane-owning thread's registers, which lets FP64 run two
// waves per SIMD.
// ------------------------------------------------------------------------------------------------
constexpr int CP_HZ = 4;  // largest local z count: (n + 1) / 2 for n <= 8

// split table of one matrix for the paired direction: own[c][k] for the
// lane's local outputs c < HZ, oth[c][k] for the partner's (c < H), local
// inputs k < HZ; the middle input (k = H, odd n) at half weight
struct ZSplit {
  double own[CP_HZ * CP_HZ];
  double oth[CP_HZ * CP_HZ];
};

struct CPairSet {
  ZSplit B, Bt, G, Gt;  // B, B^T, Dg, Dg^T along z
};

constexpr void zsplit_table(const double* A, int N, bool transpose, ZSplit& F) {
  const int H = N / 2, HZ = (N + 1) / 2;
  for (int c = 0; c < HZ; ++c)
    for (int k = 0; k < HZ; ++k) {
      const double half = k == H ? 0.5 : 1.0;  // k == H only for odd n
      const double a_own = transpose ? A[k * TDFE_MAXN + c] : A[c * TDFE_MAXN + k];
      F.own[c * CP_HZ + k] = half * a_own;
      double a_oth = 0.0;
      if (c < H) a_oth = transpose ? A[k * TDFE_MAXN + N - 1 - c] : A[(N - 1 - c) * TDFE_MAXN + k];
      F.oth[c * CP_HZ + k] = half * a_oth;
    }
}

template <int N>
constexpr CPairSet make_cpairset() {
  const tdfe1d::Rule R = tdfe1d::make_rule(N - 1);
  CPairSet F{};
  zsplit_table(R.B, N, false, F.B);
  zsplit_table(R.B, N, true, F.Bt);
  zsplit_table(R.Dg, N, false, F.G);
  zsplit_table(R.Dg, N, true, F.Gt);
  return F;
}

// value held by the partner lane (lane ^ 1): a DPP quad permutation, every
// lane a valid source (the move needs no initialised destination)
template <typename T>
__device__ __forceinline__ T partner(T v) {
  if constexpr (sizeof(T) == 8) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xf, 0xf, true);  // quad_perm 1,0,3,2
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
  } else {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xf, 0xf, true));
  }
}

// contraction along z: in/out hold the lane's HZ local entries; sg = S on
// lane 1 and 1 on lane 0
template <typename T, int N>
__device__ __forceinline__ void zpair(const ZSplit& F, const T* in, T* out, T sg) {
  constexpr int H = N / 2, HZ = (N + 1) / 2;
  T x[HZ], own[HZ], oth[H];
#pragma unroll
  for (int k = 0; k < HZ; ++k) x[k] = sg * in[k];
  // (entries that are exactly zero -- the middle row of B for odd n, the
  // centre of Dg -- are skipped at compile time)
#pragma unroll
  for (int c = 0; c < HZ; ++c) {
    T a = 0;
#pragma unroll
    for (int k = 0; k < HZ; ++k)
      if (F.own[c * CP_HZ + k] != 0.0) a += (T)F.own[c * CP_HZ + k] * x[k];
    own[c] = a;
  }
#pragma unroll
  for (int c = 0; c < H; ++c) {
    T b = 0;
#pragma unroll
    for (int k = 0; k < HZ; ++k)
      if (F.oth[c * CP_HZ + k] != 0.0) b += (T)F.oth[c * CP_HZ + k] * x[k];
    oth[c] = b;
  }
#pragma unroll
  for (int c = 0; c < H; ++c) out[c] = own[c] + partner(oth[c]);
  // both lanes' middle outputs are the same sum, in either order
  if constexpr (N & 1) out[H] = own[H] + partner(own[H]);
}

// the 6 entries of kin w detJ J^-1 J^-T at every Gauss point of the block's
// cells, from the corners staged in LDS (the plane kernel's computation)
template <typename T, int N, int CPB, int THREADS>
__device__ __forceinline__ void block_metric(int t, T* sG, const double* sC, const double* sEW, int64_t c0,
                                             int64_t n_cell, double kin) {
  constexpr int VOL = N * N * N;
  for (int it = t; it < CPB * VOL; it += THREADS) {
    const int sl = it / VOL, q = it % VOL;
    T* g = sG + it * 6;
    if (c0 + sl >= n_cell) {
      for (int w6 = 0; w6 < 6; ++w6) g[w6] = (T)0;
      continue;
    }
    const int a = q % N, b = (q / N) % N, c = q / (N * N);
    const double xa = sEW[a], xb = sEW[b], xc = sEW[c];
    const double f[2][3] = {{0.5 * (1 - xa), 0.5 * (1 - xb), 0.5 * (1 - xc)},
                            {0.5 * (1 + xa), 0.5 * (1 + xb), 0.5 * (1 + xc)}};
    const double* C = sC + sl * 24;
    double Jm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int vz = 0; vz < 2; ++vz)
      for (int vy = 0; vy < 2; ++vy)
        for (int vx = 0; vx < 2; ++vx) {
          const double* X3 = C + ((vz * 2 + vy) * 2 + vx) * 3;
          const double d0 = (vx ? 0.5 : -0.5) * f[vy][1] * f[vz][2];
          const double d1 = f[vx][0] * (vy ? 0.5 : -0.5) * f[vz][2];
          const double d2 = f[vx][0] * f[vy][1] * (vz ? 0.5 : -0.5);
          for (int d = 0; d < 3; ++d) {
            Jm[d][0] += X3[d] * d0;
            Jm[d][1] += X3[d] * d1;
            Jm[d][2] += X3[d] * d2;
          }
        }
    double A[3][3];  // adjugate: J^-1 = A / det
    A[0][0] = Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1];
    A[0][1] = Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2];
    A[0][2] = Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1];
    A[1][0] = Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2];
    A[1][1] = Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0];
    A[1][2] = Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2];
    A[2][0] = Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0];
    A[2][1] = Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1];
    A[2][2] = Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0];
    const double det = Jm[0][0] * A[0][0] + Jm[0][1] * A[1][0] + Jm[0][2] * A[2][0];
    const double s = kin * sEW[N + a] * sEW[N + b] * sEW[N + c] / det;
    g[0] = (T)(s * (A[0][0] * A[0][0] + A[0][1] * A[0][1] + A[0][2] * A[0][2]));
    g[1] = (T)(s * (A[0][0] * A[1][0] + A[0][1] * A[1][1] + A[0][2] * A[1][2]));
    g[2] = (T)(s * (A[0][0] * A[2][0] + A[0][1] * A[2][1] + A[0][2] * A[2][2]));
    g[3] = (T)(s * (A[1][0] * A[1][0] + A[1][1] * A[1][1] + A[1][2] * A[1][2]));
    g[4] = (T)(s * (A[1][0] * A[2][0] + A[1][1] * A[2][1] + A[1][2] * A[2][2]));
    g[5] = (T)(s * (A[2][0] * A[2][0] + A[2][1] * A[2][1] + A[2][2] * A[2][2]));
  }
}

template <typename T, int N>
constexpr int cpair_wpe() {
  return 2;
}

template <typename T, int N, int CB, int CPB>
__global__ void __launch_bounds__(2 * CPB * N * CB) __attribute__((amdgpu_waves_per_eu(cpair_wpe<T, N>())))
    cpair_kernel(CurvedParams<T> P) {
  constexpr int H = N / 2;
  constexpr int HZ = (N + 1) / 2;  // local z entries per lane (the middle one shared for odd n)
  constexpr bool ODD = (N & 1) != 0;
  constexpr int VOL = N * N * N;
  constexpr int THREADS = 2 * CPB * N * CB;
  constexpr FoldSet<N> FS = make_foldset<N>();
  constexpr CPairSet ZS = make_cpairset<N>();
  __shared__ T sX[CPB * VOL * CB];
  __shared__ T sV[CPB * VOL];
  __shared__ T sG[CPB * VOL * 6];
  __shared__ T sM[CPB * VOL];
  __shared__ double sRed[THREADS];
  __shared__ double sC[CPB * 24];
  __shared__ double sEW[2 * N];  // Gauss points, then weights
  if (P.done && *P.done) return;

  const int t = threadIdx.x;
  const int h = t & 1;  // which half of the z range
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
  auto zg = [&](int q) { return q == H ? H : (h ? N - 1 - q : q); };

  int cx = 0, cy = 0, cz = 0;
  if (cell_ok) {
    cx = (int)(cell % P.ncx);
    cy = (int)((cell / P.ncx) % P.ncy);
    cz = (int)(cell / ((int64_t)P.ncx * P.ncy));
  }
  T* __restrict__ Y = (T*)P.y;
  const T* __restrict__ MV;
  if constexpr (sizeof(T) == 8)
    MV = (const T*)P.minv;
  else
    MV = (const T*)P.minv32;
  T cs = act ? (T)1 : (T)0;
  if (P.colscale && act) cs = (T)P.colscale[colg >> 1];

  // block staging as in the plane kernel: potential, per-node M^-1/2 (0 on
  // Dirichlet nodes and past the last cell) and corners into registers, the
  // gather issued, then LDS and the metric while the gather is in flight
  constexpr int NV = (CPB * VOL + THREADS - 1) / THREADS;
  constexpr int NCR = (CPB * 24 + THREADS - 1) / THREADS;
  {
    constexpr tdfe1d::Rule R = tdfe1d::make_rule(N - 1);
    if (t < 2 * N) {
      double v = R.eta[0];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        v = t == q ? R.eta[q] : v;
        v = t == N + q ? R.wq[q] : v;
      }
      sEW[t] = v;
    }
  }
  const int64_t c0 = (int64_t)group * CPB;
  T mr[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int q = t + k * THREADS;
    const int64_t ce = c0 + q / VOL;
    const int rr = q % VOL;
    bool in = q < CPB * VOL && ce < P.n_cell;
    int64_t idx = 0;
    if (in) {
      const int ex = (int)(ce % P.ncx), ey = (int)((ce / P.ncx) % P.ncy), ez = (int)(ce / ((int64_t)P.ncx * P.ncy));
      const int I = ex * P.p + rr % N, Jn = ey * P.p + (rr / N) % N, K = ez * P.p + rr / (N * N);
      if (!P.fullgrid) {
        in = I > 0 && I < P.Nx - 1 && Jn > 0 && Jn < P.Ny - 1 && K > 0 && K < P.Nz - 1;
        idx = (int64_t)(I - 1) + (int64_t)(P.Nx - 2) * ((int64_t)(Jn - 1) + (int64_t)(P.Ny - 2) * (K - 1));
      }
    }
    const T mval = MV[(in && P.lowdin) ? idx : 0];
    mr[k] = in ? (P.lowdin ? mval : (T)1) : (T)0;
  }
  T vr[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int q = t + k * THREADS;
    const int64_t ce = c0 + q / VOL;
    const bool ok = P.vw && q < CPB * VOL && ce < P.n_cell;
    vr[k] = ok ? ((const T*)P.vw)[ce * VOL + q % VOL] : (T)0;
  }
  double cr[NCR];
#pragma unroll
  for (int k = 0; k < NCR; ++k) {
    const int f = t + k * THREADS;
    const bool ok = f < CPB * 24 && c0 + f / 24 < P.n_cell;
    const double val = P.corners[ok ? c0 * 24 + f : 0];
    cr[k] = ok ? val : 0.0;
  }
  auto sidx = [&](int y, int x, int z) { return (((slot * N + y) * N + x) * N + z) * CB + col; };
  const int NxI = P.Nx - 2, NyI = P.Ny - 2;

  // scatter masks: node rows i of the plane and this lane's local z entries
  // that are DoFs; the shared middle entry is scattered by lane 0 only
  const int J = cy * P.p + pl;
  const bool jok = P.fullgrid ? true : (J > 0 && J < P.Ny - 1);
  unsigned imask = 0, kmask = 0;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const int I = cx * P.p + q;
    if (P.fullgrid || (I > 0 && I < P.Nx - 1)) imask |= 1u << q;
  }
#pragma unroll
  for (int q = 0; q < HZ; ++q) {
    const int K = cz * P.p + zg(q);
    if (P.fullgrid || (K > 0 && K < P.Nz - 1)) kmask |= 1u << q;
  }
  if (ODD && h) kmask &= ~(1u << H);
  if (!act || !jok) imask = 0;
  int64_t n0, nk;  // node index of (0, j, 0) and the node stride along z
  if (P.fullgrid) {
    n0 = (int64_t)cx * P.p + (int64_t)P.Nx * ((int64_t)J + (int64_t)P.Ny * cz * P.p);
    nk = (int64_t)P.Nx * P.Ny;
  } else {
    n0 = (int64_t)(cx * P.p - 1) + (int64_t)NxI * ((int64_t)(J - 1) + (int64_t)NyI * (cz * P.p - 1));
    nk = (int64_t)NxI * NyI;
  }

  // ---------------- A: plane j = pl, values (i, local k) -----------------------------------------
  T tu[N][HZ], tx[N][HZ];  // [x point][local z]
  {
    T u[N][HZ];
    {
      // buffer resource from the block's first cell, wave-uniform (see the
      // plane kernel): out-of-range nodes read 0, Dirichlet nodes inside the
      // range read a value that the zero in sM cancels
      const int64_t rows = P.fullgrid ? (int64_t)P.Nx * P.Ny * P.Nz : (int64_t)NxI * NyI * (P.Nz - 2);
      const int bx = (int)(c0 % P.ncx), by = (int)((c0 / P.ncx) % P.ncy), bz = (int)(c0 / ((int64_t)P.ncx * P.ncy));
      const int64_t first = P.fullgrid ? (int64_t)bx * P.p + (int64_t)P.Nx * ((int64_t)by * P.p +
                                                                              (int64_t)P.Ny * bz * P.p)
                                       : (int64_t)(bx * P.p - 1) + (int64_t)NxI * ((int64_t)(by * P.p - 1) +
                                                                                 (int64_t)NyI * (bz * P.p - 1));
      const int64_t base = first > 0 ? first : 0;
      const int64_t bytes = (rows - base) * P.ld * (int64_t)sizeof(T);
      const uint64_t addr = (uint64_t)(uintptr_t)((const T*)P.x + base * P.ld);
      const uint32_t alo = __builtin_amdgcn_readfirstlane((uint32_t)addr);
      const uint32_t ahi = __builtin_amdgcn_readfirstlane((uint32_t)(addr >> 32));
      const int nrec = __builtin_amdgcn_readfirstlane((int)(bytes < 0x7fffffff ? bytes : 0x7fffffff));
      const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(uintptr_t)(((uint64_t)ahi << 32) | alo), 0, nrec, 0x00020000);
      const int ldb = P.ld * (int)sizeof(T);
      const int64_t kst = nk * ldb;
      const int64_t off0 = ((n0 - base) * P.ld + colg) * (int64_t)sizeof(T);
#pragma unroll
      for (int k = 0; k < HZ; ++k) {
        const int ok = (int)(off0 + zg(k) * kst);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          if constexpr (sizeof(T) == 8)
            u[i][k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rx, ok + i * ldb, 0, 0));
          else
            u[i][k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, ok + i * ldb, 0, 0));
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int q = t + k * THREADS;
      if (q < CPB * VOL) {
        sV[q] = vr[k];
        sM[q] = mr[k];
      }
    }
#pragma unroll
    for (int k = 0; k < NCR; ++k) {
      const int f = t + k * THREADS;
      if (f < CPB * 24) sC[f] = cr[k];
    }
    __syncthreads();
    block_metric<T, N, CPB, THREADS>(t, sG, sC, sEW, c0, P.n_cell, P.kin);
#pragma unroll
    for (int k = 0; k < HZ; ++k)
#pragma unroll
      for (int i = 0; i < N; ++i) u[i][k] *= sM[slot * VOL + i + N * (pl + N * zg(k))] * cs;
#pragma unroll
    for (int k = 0; k < HZ; ++k) {
      T line[N], o1[N], o2[N];
#pragma unroll
      for (int i = 0; i < N; ++i) line[i] = u[i][k];
      eo2<T, N, 1, -1>(FS.B, FS.D, line, o1, o2);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        tu[a][k] = o1[a];
        tx[a][k] = o2[a];
      }
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
      T o1[HZ], o2[HZ];
      zpair<T, N>(ZS.B, tu[a], o1, (T)1);
      zpair<T, N>(ZS.B, tx[a], o2, (T)1);
#pragma unroll
      for (int c = 0; c < HZ; ++c) {
        tu[a][c] = o1[c];
        tx[a][c] = o2[c];
      }
    }
  }
  // ---------------- transpose: (j; a, c) -> (a; j, c) --------------------------------------------
  // (both lanes of a pair write the same middle entries with the same value)
  T v[N][HZ], w[N][HZ];  // [y node][local z] at x point a = pl
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int c = 0; c < HZ; ++c) sX[sidx(pl, a, zg(c))] = tu[a][c];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int c = 0; c < HZ; ++c) v[j][c] = sX[sidx(j, pl, zg(c))];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int c = 0; c < HZ; ++c) sX[sidx(pl, a, zg(c))] = tx[a][c];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int c = 0; c < HZ; ++c) w[j][c] = sX[sidx(j, pl, zg(c))];
  __syncthreads();

  // ---------------- B: plane a = pl, Gauss points (b, local c) -----------------------------------
  double energy = 0.0;
  T dx[N][HZ], uq[N][HZ], dy[N][HZ];  // [b][local c]; reused in place for the fluxes
#pragma unroll
  for (int c = 0; c < HZ; ++c) {
    T l1[N], l2[N], o1[N], o2[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      l1[j] = v[j][c];
      l2[j] = w[j][c];
    }
    eo<T, N, 1>(FS.B, l1, o1);
    eo<T, N, 1>(FS.B, l2, o2);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      uq[b][c] = o1[b];
      dx[b][c] = o2[b];
    }
  }
#pragma unroll
  for (int c = 0; c < HZ; ++c) {
    T l[N], d[N];
#pragma unroll
    for (int b = 0; b < N; ++b) l[b] = uq[b][c];
    eo<T, N, -1>(FS.G, l, d);
#pragma unroll
    for (int b = 0; b < N; ++b) dy[b][c] = d[b];
  }
  // per y point: z derivative (paired), the three fluxes, the potential term
  // and the transposed z derivative; dx <- f_x, dy <- f_y, uq <- V u + Dg_z^T f_z
#pragma unroll
  for (int b = 0; b < N; ++b) {
    T dz[HZ], fz[HZ], rz[HZ];
    zpair<T, N>(ZS.G, uq[b], dz, sgn);
    T le = 0;
#pragma unroll
    for (int c = 0; c < HZ; ++c) {
      const int q = pl + N * (b + N * zg(c));
      const T* g = sG + (slot * VOL + q) * 6;
      const T ux = dx[b][c], uy = dy[b][c], uz = dz[c];
      const T fx = g[0] * ux + g[1] * uy + g[2] * uz;
      const T fy = g[1] * ux + g[3] * uy + g[4] * uz;
      const T f3 = g[2] * ux + g[4] * uy + g[5] * uz;
      const T pot = sV[slot * VOL + q] * uq[b][c];
      const T e = fx * ux + fy * uy + f3 * uz + pot * uq[b][c];
      acc_energy<T>(energy, le, (ODD && c == H) ? (T)0.5 * e : e);
      dx[b][c] = fx;
      dy[b][c] = fy;
      fz[c] = f3;
      uq[b][c] = pot;
    }
    flush_energy<T>(energy, le);
    zpair<T, N>(ZS.Gt, fz, rz, sgn);
#pragma unroll
    for (int c = 0; c < HZ; ++c) uq[b][c] += rz[c];
    __builtin_amdgcn_sched_barrier(0);
  }
  // per local z point: transposed y derivative of f_y, then transposed y
  // interpolation of both arrays: s_x = B_y^T f_x goes straight into the
  // transpose buffer, s = B_y^T (uq + Dg_y^T f_y) stays
  T s[N][HZ];  // [j][local c]
#pragma unroll
  for (int c = 0; c < HZ; ++c) {
    T l[N], rr[N], o[N];
#pragma unroll
    for (int b = 0; b < N; ++b) l[b] = dx[b][c];
    eo<T, N, 1>(FS.Bt, l, o);
#pragma unroll
    for (int j = 0; j < N; ++j) sX[sidx(j, pl, zg(c))] = o[j];
#pragma unroll
    for (int b = 0; b < N; ++b) l[b] = dy[b][c];
    eo<T, N, -1>(FS.Gt, l, rr);
#pragma unroll
    for (int b = 0; b < N; ++b) l[b] = uq[b][c] + rr[b];
    eo<T, N, 1>(FS.Bt, l, o);
#pragma unroll
    for (int j = 0; j < N; ++j) s[j][c] = o[j];
  }
  // ---------------- transposes: (a; j, c) -> (j; a, c) -------------------------------------------
  sRed[t] = act ? energy : 0.0;
  T s2[N][HZ], sx2[N][HZ];  // [x point][local z] at node plane j = pl
  __syncthreads();
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int c = 0; c < HZ; ++c) sx2[a][c] = sX[sidx(pl, a, zg(c))];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int c = 0; c < HZ; ++c) sX[sidx(j, pl, zg(c))] = s[j][c];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int c = 0; c < HZ; ++c) s2[a][c] = sX[sidx(pl, a, zg(c))];

  // ---------------- C: plane j = pl: x transposed, z transposed (paired), scatter ------------------
  {
    T hh[N][HZ];  // [x node][local z point]
#pragma unroll
    for (int c = 0; c < HZ; ++c) {
      T l1[N], l2[N], o1[N], o2[N];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        l1[a] = s2[a][c];
        l2[a] = sx2[a][c];
      }
      eo<T, N, 1>(FS.Bt, l1, o1);
      eo<T, N, -1>(FS.Dt, l2, o2);
#pragma unroll
      for (int i = 0; i < N; ++i) hh[i][c] = o1[i] + o2[i];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T ml[HZ];
#pragma unroll
      for (int k = 0; k < HZ; ++k) ml[k] = sM[slot * VOL + i + N * (pl + N * zg(k))];
      T o[HZ];
      zpair<T, N>(ZS.Bt, hh[i], o, (T)1);
      if ((imask >> i) & 1u) {
        T* yrow = Y + ((n0 + i) * P.ld + colg);
#pragma unroll
        for (int k = 0; k < HZ; ++k)
          if ((kmask >> k) & 1u) unsafeAtomicAdd(yrow + (int64_t)zg(k) * nk * P.ld, o[k] * ml[k]);
      }
    }
  }
  // ---------------- per-column quadratic form ------------------------------------------------------
  if (P.energy) {
    __syncthreads();
    if (t < CB) {
      double acc = 0.0;
      for (int u = 2 * t; u < THREADS; u += 2 * CB) acc += sRed[u] + sRed[u + 1];
      if (chunk * CB + t < P.cols) P.energy[(int64_t)group * P.cols + chunk * CB + t] = acc;
    }
  }
}

// LDS bytes of one block of cpb cells (transpose buffer, potential, metric,
// M^-1/2, quadratic-form partials of both lanes, corners)
template <typename T, int N, int CB>
constexpr int cpair_lds(int cpb) {
  constexpr int VOL = N * N * N;
  return cpb * VOL * CB * (int)sizeof(T) + cpb * VOL * (int)sizeof(T) * 8 + 2 * cpb * N * CB * 8 + cpb * 24 * 8 +
         2 * N * 8;
}

// cells per block: at most 512 threads, LDS for two blocks per CU
template <typename T, int N, int CB>
constexpr int cpair_cpb() {
  int cpb = 1;
  while (2 * cpb * 2 * N * CB <= 512 && cpair_lds<T, N, CB>(cpb * 2) <= 80 * 1024) cpb *= 2;
  return cpb;
}

template <typename T, int N, int CB>
tdfe_status launch_cpair(tdfe_ctx* c, CurvedParams<T>& P, int64_t* groups_out) {
  constexpr int CPB = cpair_cpb<T, N, CB>();
  static_assert(cpair_lds<T, N, CB>(CPB) <= 160 * 1024, "LDS");
  const int64_t groups = (c->n_cell + CPB - 1) / CPB;
  P.nchunks = (P.cols + CB - 1) / CB;
  if (groups_out) *groups_out = groups;
  hipLaunchKernelGGL((cpair_kernel<T, N, CB, CPB>), dim3((unsigned)(groups * P.nchunks)), dim3(2 * CPB * N * CB), 0,
                     c->stream, P);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

// columns per block: the next power of two up to 16
template <typename T, int N>
tdfe_status launch_cpair_n(tdfe_ctx* c, CurvedParams<T>& P, int64_t* g) {
  if (P.cols <= 2) return launch_cpair<T, N, 2>(c, P, g);
  if (P.cols <= 4) return launch_cpair<T, N, 4>(c, P, g);
  if (P.cols <= 8) return launch_cpair<T, N, 8>(c, P, g);
  return launch_cpair<T, N, 16>(c, P, g);
}

template <typename T>
tdfe_status launch_curved(tdfe_ctx* c, const ApplyArgs& a) {
  static_assert(sizeof(CurvedParams<T>) <= 4096, "kernel arguments exceed 4 KB");
  CurvedParams<T> P{};
  P.x = a.x;
  P.y = a.y;
  P.ld = a.ld;
  P.cols = a.cols;
  P.colscale = a.colscale;
  P.kin = a.kin;
  P.vw = a.fp32 ? (const void*)a.vw32 : (const void*)a.vw;
  P.minv = c->minv;
  P.minv32 = c->minv32;
  P.corners = c->corners;
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
  for (int i = 0; i < N; ++i) {
    P.eta[i] = c->eta[i];
    P.wq[i] = c->wq[i];
  }
  // lane pairs for FP64 (two waves per SIMD instead of one) and for FP32 at
  // n = 8 (162 VGPRs against the plane kernel's 256: 1.75 against 1.98 ms per
  // 2-orbital launch of the all-electron workload); plane ownership for FP32
  // otherwise (at n = 7 both run two waves per SIMD and the pairs' duplicated
  // z work loses: 2.24 against 1.50 ms per 16-orbital graded launch)
  const bool pair = c->variant == TDFE_VARIANT_PAIR || (c->variant == 0 && (sizeof(T) == 8 || N == 8));
  if (pair) {
    switch (N) {
      case 2: return launch_cpair_n<T, 2>(c, P, a.n_blocks_out);
      case 3: return launch_cpair_n<T, 3>(c, P, a.n_blocks_out);
      case 4: return launch_cpair_n<T, 4>(c, P, a.n_blocks_out);
      case 5: return launch_cpair_n<T, 5>(c, P, a.n_blocks_out);
      case 6: return launch_cpair_n<T, 6>(c, P, a.n_blocks_out);
      case 7: return launch_cpair_n<T, 7>(c, P, a.n_blocks_out);
      case 8: return launch_cpair_n<T, 8>(c, P, a.n_blocks_out);
    }
    return tdfe_fail(c, TDFE_EINVAL, "curved operator: unsupported order p=%d", c->p);
  }
  switch (N) {
    case 2: return launch_cplane_n<T, 2>(c, P, a.n_blocks_out);
    case 3: return launch_cplane_n<T, 3>(c, P, a.n_blocks_out);
    case 4: return launch_cplane_n<T, 4>(c, P, a.n_blocks_out);
    case 5: return launch_cplane_n<T, 5>(c, P, a.n_blocks_out);
    case 6: return launch_cplane_n<T, 6>(c, P, a.n_blocks_out);
    case 7: return launch_cplane_n<T, 7>(c, P, a.n_blocks_out);
    case 8: return launch_cplane_n<T, 8>(c, P, a.n_blocks_out);
  }
  return tdfe_fail(c, TDFE_EINVAL, "curved operator: unsupported order p=%d", c->p);
}

}  // namespace

// true if the curved plane kernel handles this launch: trilinear cells, p <= 7,
// two or more real columns (one column leaves n threads per cell with the
// metric staged for the whole cell: the line kernel is faster there, 0.64 ms
// against 2.2 ms for the one-column stiffness products of the Hartree solve on
// the graded mesh)
bool tdfe_curved_kernel_ok(const tdfe_ctx* c, int cols, bool fp32) {
  (void)fp32;
  return !c->box && cols >= 2 && c->n <= 8;
}

tdfe_status tdfe_launch_apply_curved(tdfe_ctx* c, const ApplyArgs& a) {
  if (a.cols < 1) return tdfe_fail(c, TDFE_EINVAL, "apply: cols < 1");
  if (!tdfe_curved_kernel_ok(c, a.cols, a.fp32)) return tdfe_fail(c, TDFE_EINVAL, "curved operator: unsupported mesh or order");
  // M^-1/2 exists on the interior DoFs only
  if (a.lowdin && a.fullgrid) return tdfe_fail(c, TDFE_EINVAL, "apply: Loewdin scaling on the full node grid");
  return a.fp32 ? launch_curved<float>(c, a) : launch_curved<double>(c, a);
}
