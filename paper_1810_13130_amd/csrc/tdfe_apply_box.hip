// Operator kernel for rectilinear (box) cells: "plane" sum factorisation.
//
// Same operator as tdfe_apply.hip (Eq. DiscreteHamiltonian in the Loewdin
// form, Eq. TDKSMatVecStandard), organised for the register file of CDNA4:
// each thread owns one column and an n x n plane of a cell's values.
//
//   A  (plane at fixed y node j):  gather u(i,k); x: B u, D u; z: B on both
//   -- LDS transpose of the two arrays -->
//   B  (plane at fixed x point a): y: B on both -> u_q, d_x u_q; then in
//      registers d_y u_q, d_z u_q by the Gauss collocation derivative,
//      the box fluxes (diagonal metric), the potential term, the y and z
//      transposed derivatives and the transposed y interpolation of the two
//      results (s, s_x)
//   -- LDS transpose of the two arrays -->
//   C  (plane at fixed y node j):  x: B^T s + D^T s_x; z: B^T; scatter-add.
//
// Only the y direction crosses threads, so the cell data make four LDS
// round trips (two arrays each way) instead of fifteen.  Every 1D contraction
// uses the reflection symmetry of the GLL nodes and Gauss points
// (B[n-1-a][n-1-i] = B[a][i], D and Dg antisymmetric): even/odd folding halves
// the multiply-adds.  The folded tables are evaluated at compile time for the
// kernel's order (make_foldset), so each coefficient is an instruction
// constant: no table loads, and no scalar-memory waits that would also wait
// for the LDS transposes.
#include "tdfe_fold.h"

namespace {

template <typename T>
struct PlaneParams {
  const void* x;
  void* y;
  int ld, cols, nchunks;
  const double* colscale;
  double kin;
  const void* vw;
  const double* minv;
  const double* m1x;  // separable M^-1/2 factors of a box mesh: minv(I,J,K) = m1x[I] m1y[J] m1z[K]
  const double* m1y;
  const double* m1z;
  const double* cellgeo;
  double* energy;
  const int* done;
  int ncx, ncy, ncz, p, Nx, Ny, Nz;
  int64_t n_cell;
  int lowdin, fullgrid;
  double wq[TDFE_MAXN];  // Gauss weights (indexed by the thread's plane)
};

// occupancy target: FP64 planes of n >= 6 need more than 256 registers per
// lane, so they run one wave per SIMD and use the accumulation registers
template <typename T, int N>
constexpr int plane_wpe() {
  return sizeof(T) == 4 ? (N == 5 || N == 6 ? 3 : 2) : (N >= 6 ? 1 : 2);
}

// hold both transposed arrays in LDS at once (fewer barriers) instead of
// passing them through one buffer in turn; measured slower on both precisions
// at n = 6 (more live registers), kept selectable
template <typename T, int N>
constexpr bool plane_two_buffers() {
  return false;
}

template <typename T, int N, int CB, int CPB>
__global__ void __launch_bounds__(CPB * N * CB) __attribute__((amdgpu_waves_per_eu(plane_wpe<T, N>())))
    plane_kernel(PlaneParams<T> P) {
  constexpr int VOL = N * N * N;
  constexpr int THREADS = CPB * N * CB;
  constexpr bool TWO = plane_two_buffers<T, N>();
  // 1D tables of order N, folded, as compile-time constants
  constexpr FoldSet<N> FS = make_foldset<N>();
  auto wprod = [&](int b, int c) { return (T)(FS.wq[b] * FS.wq[c]); };
  __shared__ T sX[CPB * VOL * CB];
  __shared__ T sY[TWO ? CPB * VOL * CB : 1];
  __shared__ T sV[CPB * VOL];  // weighted potential of the block's cells
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
  T cs = (T)1;
  if (P.colscale && act) cs = (T)P.colscale[colg >> 1];

  // block staging: the weighted potential of the block's cells, their M^-1/2
  // factors along x, y and z and their metric go to LDS.  The loads are issued
  // here, the phase A gather right after them, and the LDS stores follow both,
  // so that a wave waits for memory once rather than once per array.
  constexpr int NFC = 3 * N + 3;  // per cell: m_x[N], m_y[N], m_z[N], metric[3]
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
    // one load from a selected (always valid) address: no branches
    const double* src = r < N ? P.m1x + (ex * P.p + r)
                        : r < 2 * N ? P.m1y + (ey * P.p + r - N)
                        : r < 3 * N ? P.m1z + (ez * P.p + r - 2 * N)
                                    : P.cellgeo + (cv * 4 + r - 3 * N);
    const double val = *src;
    fr[k] = ok ? val : 0.0;
  }
  const double* sFc = sF + slot * NFC;  // this thread's cell
  // LDS index: slot, y index, x index, z index, column
  auto sidx = [&](int y, int x, int z) { return (((slot * N + y) * N + x) * N + z) * CB + col; };
  const int NxI = P.Nx - 2, NyI = P.Ny - 2;

  // ---------------- A: plane j = pl, values (i, k) -------------------------------------
  T tu[N][N], tx[N][N];  // [x][z]
  {
    const int j = pl;
    const int J = cy * P.p + j;
    T u[N][N];  // [i][k]
    // node (I, J, K) -> element offset; all loads are issued unconditionally
    // from a valid address (masked entries read element 0 and are zeroed)
    const bool jok = P.fullgrid ? true : (J > 0 && J < P.Ny - 1);
    unsigned imask = 0, kmask = 0;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const int I = cx * P.p + q, K = cz * P.p + q;
      if (P.fullgrid || (I > 0 && I < P.Nx - 1)) imask |= 1u << q;
      if (P.fullgrid || (K > 0 && K < P.Nz - 1)) kmask |= 1u << q;
    }
    if (!act || !jok) imask = 0;
    // element index of (i, k): e0 + i * ld + k * kstride
    int64_t e0, kstride;
    if (P.fullgrid) {
      e0 = ((int64_t)cx * P.p + (int64_t)P.Nx * ((int64_t)J + (int64_t)P.Ny * cz * P.p)) * P.ld + colg;
      kstride = (int64_t)P.Nx * P.Ny * P.ld;
    } else {
      e0 = ((int64_t)(cx * P.p - 1) + (int64_t)NxI * ((int64_t)(J - 1) + (int64_t)NyI * (cz * P.p - 1))) * P.ld + colg;
      kstride = (int64_t)NxI * NyI * P.ld;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const bool ok = ((imask >> i) & (kmask >> k) & 1u) != 0;
        const int64_t e = ok ? e0 + (int64_t)i * P.ld + (int64_t)k * kstride : 0;
        const T val = X[e];
        u[i][k] = ok ? val : (T)0;
      }
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
    T my = (T)1;
    if (P.lowdin && imask) my = (T)sFc[N + j] * cs;
    else my = cs;
    if (P.lowdin) {
      T fx[N], fz[N];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        fx[q] = ((imask >> q) & 1u) ? (T)sFc[q] : (T)0;
        fz[q] = ((kmask >> q) & 1u) ? (T)sFc[2 * N + q] : (T)0;
      }
#pragma unroll
      for (int k = 0; k < N; ++k)
#pragma unroll
        for (int i = 0; i < N; ++i) u[i][k] *= fx[i] * fz[k] * my;
    } else {
#pragma unroll
      for (int k = 0; k < N; ++k)
#pragma unroll
        for (int i = 0; i < N; ++i) u[i][k] *= my;
    }
    // x: interpolation and nodal derivative at the Gauss points, per z line
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
    // z: interpolation of both, per x point
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
  // ---------------- transpose: (j; a, c) -> (a; j, c) ------------------------------------
  T v[N][N], w[N][N];  // [y][z] at x point a = pl
  if constexpr (TWO) {
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
      for (int c = 0; c < N; ++c) {
        sX[sidx(pl, a, c)] = tu[a][c];
        sY[sidx(pl, a, c)] = tx[a][c];
      }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int c = 0; c < N; ++c) {
        v[j][c] = sX[sidx(j, pl, c)];
        w[j][c] = sY[sidx(j, pl, c)];
      }
    __syncthreads();
  } else {
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
  }

  // ---------------- B: plane a = pl, quadrature values (b, c) --------------------------------
  double energy = 0.0;
  T gx = 0, gy = 0, gz = 0;
  const bool havev = P.vw != nullptr;
  if (cell_ok) {
    // Gauss weight of this thread's x point, selected from the constants (an
    // array indexed per lane would be a memory load and a wait)
    T wa = (T)FS.wq[0];
#pragma unroll
    for (int q = 1; q < N; ++q) wa = pl == q ? (T)FS.wq[q] : wa;
    gx = (T)(P.kin * sFc[3 * N + 0]) * wa;
    gy = (T)(P.kin * sFc[3 * N + 1]) * wa;
    gz = (T)(P.kin * sFc[3 * N + 2]) * wa;
  }
  // B1: x flux from w, transposed y interpolation, straight into the transpose
  // buffer (free: every thread has finished reading w)
#pragma unroll
  for (int c = 0; c < N; ++c) {
    T l[N], o[N];
#pragma unroll
    for (int j = 0; j < N; ++j) l[j] = w[j][c];
    eo<T, N, 1>(FS.B, l, o);  // u_x at (pl, b, c)
    T le = 0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const T f = gx * wprod(b, c) * o[b];
      acc_energy<T>(energy, le, f * o[b]);
      o[b] = f;
    }
    flush_energy<T>(energy, le);
    eo<T, N, 1>(FS.Bt, o, l);
#pragma unroll
    for (int j = 0; j < N; ++j) sX[sidx(j, pl, c)] = l[j];
    __builtin_amdgcn_sched_barrier(0);
  }
  // B2: u_q, potential, y and z fluxes, transposed y interpolation
  T s[N][N];  // [j][c]
  {
    T uq[N][N], acc[N][N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T l[N], o[N];
#pragma unroll
      for (int j = 0; j < N; ++j) l[j] = v[j][c];
      eo<T, N, 1>(FS.B, l, o);
      T le = 0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        uq[b][c] = o[b];
        const T pot = havev ? sV[slot * VOL + pl + N * (b + N * c)] * o[b] : (T)0;
        acc_energy<T>(energy, le, pot * o[b]);
        acc[b][c] = pot;
      }
      flush_energy<T>(energy, le);
      // keep the potential reads of later lines from being hoisted here
      __builtin_amdgcn_sched_barrier(0);
    }
    // z flux, per y line
#pragma unroll
    for (int b = 0; b < N; ++b) {
      T d[N], r[N];
      eo<T, N, -1>(FS.G, uq[b], d);
      T le = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const T f = gz * wprod(b, c) * d[c];
        acc_energy<T>(energy, le, f * d[c]);
        d[c] = f;
      }
      flush_energy<T>(energy, le);
      eo<T, N, -1>(FS.Gt, d, r);
#pragma unroll
      for (int c = 0; c < N; ++c) acc[b][c] += r[c];
    }
    // y flux and transposed y interpolation, per z line
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T l[N], d[N], r[N];
#pragma unroll
      for (int b = 0; b < N; ++b) l[b] = uq[b][c];
      eo<T, N, -1>(FS.G, l, d);
      T le = 0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const T f = gy * wprod(b, c) * d[b];
        acc_energy<T>(energy, le, f * d[b]);
        d[b] = f;
      }
      flush_energy<T>(energy, le);
      eo<T, N, -1>(FS.Gt, d, r);
#pragma unroll
      for (int b = 0; b < N; ++b) r[b] += acc[b][c];
      eo<T, N, 1>(FS.Bt, r, l);
      if constexpr (TWO) {
#pragma unroll
        for (int j = 0; j < N; ++j) sY[sidx(j, pl, c)] = l[j];
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) s[j][c] = l[j];
      }
    }
  }
  // ---------------- transposes: (a; j, c) -> (j; a, c) ----------------------------------------
  // the quadratic form is parked in LDS here, unconditionally: otherwise the
  // compiler sinks its whole accumulation chain into the final reduction and
  // keeps every partial product alive across phase C
  sRed[t] = act ? energy : 0.0;
  T s2[N][N], sx2[N][N];  // [x point a][z point c] at node plane j = pl (one-buffer blocks)
  __syncthreads();
  if constexpr (!TWO) {
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
  }

  // ---------------- C: plane j = pl: x then z transposed, scatter ------------------------------
  {
    const int j = pl;
    T h[N][N];  // [i][c]
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T l1[N], l2[N], o1[N], o2[N];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        if constexpr (TWO) {
          l1[a] = sY[sidx(pl, a, c)];
          l2[a] = sX[sidx(pl, a, c)];
        } else {
          l1[a] = s2[a][c];
          l2[a] = sx2[a][c];
        }
      }
      eo<T, N, 1>(FS.Bt, l1, o1);
      eo<T, N, -1>(FS.Dt, l2, o2);
#pragma unroll
      for (int i = 0; i < N; ++i) h[i][c] = o1[i] + o2[i];
    }
    const int J = cy * P.p + j;
    const bool jok = P.fullgrid ? true : (J > 0 && J < P.Ny - 1);
    unsigned imask = 0, kmask = 0;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const int I = cx * P.p + q, K = cz * P.p + q;
      if (P.fullgrid || (I > 0 && I < P.Nx - 1)) imask |= 1u << q;
      if (P.fullgrid || (K > 0 && K < P.Nz - 1)) kmask |= 1u << q;
    }
    if (!act || !jok) imask = 0;
    int64_t e0, kstride;
    if (P.fullgrid) {
      e0 = ((int64_t)cx * P.p + (int64_t)P.Nx * ((int64_t)J + (int64_t)P.Ny * cz * P.p)) * P.ld + colg;
      kstride = (int64_t)P.Nx * P.Ny * P.ld;
    } else {
      e0 = ((int64_t)(cx * P.p - 1) + (int64_t)NxI * ((int64_t)(J - 1) + (int64_t)NyI * (cz * P.p - 1))) * P.ld + colg;
      kstride = (int64_t)NxI * NyI * P.ld;
    }
    T fx[N], fz[N];
    T my = (T)1;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      fx[q] = (T)1;
      fz[q] = (T)1;
    }
    if (P.lowdin && imask) {
      my = (T)sFc[N + j];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        if ((imask >> q) & 1u) fx[q] = (T)sFc[q];
        if ((kmask >> q) & 1u) fz[q] = (T)sFc[2 * N + q];
      }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T o[N];
      eo<T, N, 1>(FS.Bt, h[i], o);
#pragma unroll
      for (int k = 0; k < N; ++k) {
        if (((imask >> i) & (kmask >> k) & 1u) != 0)
          unsafeAtomicAdd(Y + (e0 + (int64_t)i * P.ld + (int64_t)k * kstride), o[k] * fx[i] * fz[k] * my);
      }
    }
  }
  // ---------------- per-column quadratic form -------------------------------------------------
  if (P.energy) {
    __syncthreads();
    if (t < CB) {
      double acc = 0.0;
      for (int u = t; u < THREADS; u += CB) acc += sRed[u];
      if (chunk * CB + t < P.cols) P.energy[(int64_t)group * P.cols + chunk * CB + t] = acc;
    }
  }
}

// ----------------------------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------------------------

// LDS bytes of one block of cpb cells
template <typename T, int N, int CB>
constexpr int plane_lds(int cpb) {
  constexpr int VOL = N * N * N;
  return cpb * VOL * CB * (int)sizeof(T) * (plane_two_buffers<T, N>() ? 2 : 1) + cpb * VOL * (int)sizeof(T) +
         cpb * N * CB * 8 + cpb * (3 * N + 3) * 8;
}

// cells per block: at most 512 threads, and LDS small enough for the
// occupancy plane_wpe asks for (an FP64 block must also fit one CU at one wave
// per SIMD: at most four waves)
template <typename T, int N, int CB>
constexpr int plane_cpb() {
  constexpr int budget = sizeof(T) == 8 ? 64 * 1024 : 40 * 1024;
  int cpb = 1;
  while (cpb * 2 * N * CB <= 512 && plane_lds<T, N, CB>(cpb * 2) <= budget) cpb *= 2;
  return cpb;
}

template <typename T, int N, int CB>
tdfe_status launch_plane(tdfe_ctx* c, PlaneParams<T>& P, int64_t* groups_out) {
  constexpr int CPB = plane_cpb<T, N, CB>();
  const int64_t groups = (c->n_cell + CPB - 1) / CPB;
  P.nchunks = (P.cols + CB - 1) / CB;
  if (groups_out) *groups_out = groups;
  hipLaunchKernelGGL((plane_kernel<T, N, CB, CPB>), dim3((unsigned)(groups * P.nchunks)), dim3(CPB * N * CB), 0,
                     c->stream, P);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

template <typename T, int N>
tdfe_status launch_plane_n(tdfe_ctx* c, PlaneParams<T>& P, int64_t* g) {
  if (P.cols <= 1) return launch_plane<T, N, 1>(c, P, g);
  if (P.cols <= 2) return launch_plane<T, N, 2>(c, P, g);
  if (P.cols <= 4) return launch_plane<T, N, 4>(c, P, g);
  if (P.cols <= 8) return launch_plane<T, N, 8>(c, P, g);
  return launch_plane<T, N, 16>(c, P, g);
}

template <typename T>
tdfe_status launch_plane_p(tdfe_ctx* c, PlaneParams<T>& P, int64_t* g) {
  switch (c->n) {
    case 2: return launch_plane_n<T, 2>(c, P, g);
    case 3: return launch_plane_n<T, 3>(c, P, g);
    case 4: return launch_plane_n<T, 4>(c, P, g);
    case 5: return launch_plane_n<T, 5>(c, P, g);
    case 6: return launch_plane_n<T, 6>(c, P, g);
    case 7: return launch_plane_n<T, 7>(c, P, g);
    case 8: return launch_plane_n<T, 8>(c, P, g);
  }
  return tdfe_fail(c, TDFE_EINVAL, "box operator: unsupported order p=%d", c->p);
}


template <typename T>
tdfe_status launch_box(tdfe_ctx* c, const ApplyArgs& a) {
  static_assert(sizeof(PlaneParams<T>) <= 4096, "kernel arguments exceed 4 KB");
  PlaneParams<T> P{};
  P.x = a.x;
  P.y = a.y;
  P.ld = a.ld;
  P.cols = a.cols;
  P.colscale = a.colscale;
  P.kin = a.kin;
  P.vw = a.fp32 ? (const void*)a.vw32 : (const void*)a.vw;
  P.minv = c->minv;
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
  return launch_plane_p<T>(c, P, a.n_blocks_out);
}

}  // namespace

// true if the box kernel handles this context (rectilinear mesh, p <= 7)
bool tdfe_box_kernel_ok(const tdfe_ctx* c) { return c->box && c->n <= 8; }

tdfe_status tdfe_launch_apply_box(tdfe_ctx* c, const ApplyArgs& a) {
  if (a.cols < 1) return tdfe_fail(c, TDFE_EINVAL, "apply: cols < 1");
  return a.fp32 ? launch_box<float>(c, a) : launch_box<double>(c, a);
}
