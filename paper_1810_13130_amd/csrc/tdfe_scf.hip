// Density, dipole, Hartree/XC potential and the Magnus step (tdfe C ABI).
//
// * density: rho_q = sum_alpha f_alpha |psi_alpha(x_q)|^2 with
//   psi = M^-1/2 psibar interpolated to the Gauss points (Sec. TDKS
//   equations, Eq. TDKSMatVecStandard);
// * dipole mu = sum_q varpi_q detJ_q x_q rho_q, charge = sum_q varpi_q detJ_q rho_q;
// * Hartree: K phi = 4 pi c, c_j = int rho N_j, phi = f on the boundary with
//   f = sum_I Z_I / |x - R_I| at the boundary nodes (Eqs. Poisson,
//   VHDiscretePoisson; the appendix's boundary interpolant).  On a
//   rectilinear grid with Gauss quadrature the interior stiffness is exactly
//   the Kronecker sum Kx(x)My(x)Mz + Mx(x)Ky(x)Mz + Mx(x)My(x)Kz of 1D
//   matrices, so it is inverted exactly by the fast diagonalisation method
//   (1D generalised eigenvectors S with S^T M S = I, S^T K S = Lambda):
//   K^-1 = (S x S x S) diag(1/(lx+ly+lz)) (S x S x S)^T.  Curved meshes use
//   Jacobi-preconditioned conjugate gradients.
// * ALDA exchange (and Perdew-Zunger 81 correlation) at the Gauss points.
// * magnus_step: the predictor-corrector second-order Magnus step.
#include <algorithm>
#include <cmath>

// the solution-index queries of rocBLAS are in its beta interface
#define ROCBLAS_BETA_FEATURES_API
#include <rocblas/rocblas.h>

#include "tdfe_internal.h"
#include "tdfe_fold.h"

namespace {

constexpr int EW = 256;  // elementwise block size

inline unsigned nblk(int64_t n, int b = EW) { return (unsigned)((n + b - 1) / b); }

constexpr int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

__device__ __forceinline__ int64_t dof_of(int I, int J, int K, int Nx, int Ny) {
  return (int64_t)(I - 1) + (int64_t)(Nx - 2) * ((int64_t)(J - 1) + (int64_t)(Ny - 2) * (K - 1));
}

// ------------------------------------------------------------------------------------------------
// density: per cell, all orbitals; rho at the Gauss points and dipole partials
// ------------------------------------------------------------------------------------------------
struct DensParams {
  const double* psi;  // [n_dof][2 n_orb]
  int cols;           // 2 n_orb
  const double* occ;  // [n_orb]
  const double* minv;
  const double* tab;
  const double* wdet;
  const double* xq;
  double* rho;
  double* partial;  // [block][4]
  int ncx, ncy, ncz, p, Nx, Ny, Nz;
  int64_t n_cell;
};

template <int N, int CB>
__global__ void __launch_bounds__(N* N* CB) density_kernel(DensParams P) {
  constexpr int VOL = N * N * N;
  constexpr int T = N * N * CB;
  // folded interpolation table B as compile-time constants
  constexpr FoldSet<N> FS = make_foldset<N>();
  __shared__ double sU[VOL * CB];
  __shared__ double sred[T];
  const int t = threadIdx.x;
  const int col = t % CB, line = t / CB;
  const int64_t cell = blockIdx.x;
  const int cx = (int)(cell % P.ncx), cy = (int)((cell / P.ncx) % P.ncy), cz = (int)(cell / ((int64_t)P.ncx * P.ncy));
  double racc[N];
#pragma unroll
  for (int a = 0; a < N; ++a) racc[a] = 0.0;
  auto L = [&](int z, int y, int x) { return ((z * N + y) * N + x) * CB + col; };
  for (int c0 = 0; c0 < P.cols; c0 += CB) {
    const int cg = c0 + col;
    const bool ok = cg < P.cols;
    double r1[N];
    {
      const int i = line % N, j = line / N;
      const int I = cx * P.p + i, J = cy * P.p + j;
      // branch-free gather: all loads of the z-line (values and M^-1/2) are
      // issued from valid addresses before any is used
      double v[N], m[N];
      unsigned inm = 0;  // interior nodes of the line
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const int K = cz * P.p + k;
        const bool in = ok && I > 0 && I < P.Nx - 1 && J > 0 && J < P.Ny - 1 && K > 0 && K < P.Nz - 1;
        if (in) inm |= 1u << k;
        const int64_t d = in ? dof_of(I, J, K, P.Nx, P.Ny) : 0;
        v[k] = P.psi[d * P.cols + (in ? cg : 0)];
        m[k] = P.minv[d];
      }
#pragma unroll
      for (int k = 0; k < N; ++k) r1[k] = ((inm >> k) & 1u) ? v[k] * m[k] : 0.0;
      double o[N];
      eo<double, N, 1>(FS.B, r1, o);
#pragma unroll
      for (int c = 0; c < N; ++c) sU[L(c, j, i)] = o[c];
    }
    __syncthreads();
    {
      const int i = line % N, c = line / N;
#pragma unroll
      for (int j = 0; j < N; ++j) r1[j] = sU[L(c, j, i)];
      double o[N];
      eo<double, N, 1>(FS.B, r1, o);
#pragma unroll
      for (int b = 0; b < N; ++b) sU[L(c, b, i)] = o[b];
    }
    __syncthreads();
    {
      const int b = line % N, c = line / N;
#pragma unroll
      for (int i = 0; i < N; ++i) r1[i] = sU[L(c, b, i)];
      const double f = ok ? P.occ[cg >> 1] : 0.0;
      double o[N];
      eo<double, N, 1>(FS.B, r1, o);
#pragma unroll
      for (int a = 0; a < N; ++a) racc[a] += f * o[a] * o[a];
    }
    __syncthreads();
  }
  // sum over the column lanes of each x-line
  {
    const int b = line % N, c = line / N;
#pragma unroll
    for (int a = 0; a < N; ++a) sU[L(c, b, a)] = racc[a];
  }
  __syncthreads();
  double ch = 0, mx = 0, my = 0, mz = 0;
  for (int q = t; q < VOL; q += T) {
    double s = 0.0;
    for (int cc = 0; cc < CB; ++cc) s += sU[q * CB + cc];
    const int64_t g = cell * VOL + q;
    P.rho[g] = s;
    const double w = P.wdet[g] * s;
    ch += w;
    mx += w * P.xq[g * 3 + 0];
    my += w * P.xq[g * 3 + 1];
    mz += w * P.xq[g * 3 + 2];
  }
  double vals[4] = {ch, mx, my, mz};
  if constexpr (T % 64 == 0) {
    // whole wavefronts: lane shuffles, then one pass over the block's waves (fixed order)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      for (int off = 32; off > 0; off >>= 1) vals[v] += __shfl_xor(vals[v], off);
    constexpr int NW = T / 64;
    if ((t & 63) == 0)
#pragma unroll
      for (int v = 0; v < 4; ++v) sred[(t >> 6) * 4 + v] = vals[v];
    __syncthreads();
    if (t < 4) {
      double acc = 0.0;
      for (int w = 0; w < NW; ++w) acc += sred[w * 4 + t];
      P.partial[cell * 4 + t] = acc;
    }
  } else {
    constexpr int PW = pow2_floor(T);
    for (int v = 0; v < 4; ++v) {
      sred[t] = vals[v];
      __syncthreads();
      if (t < T - PW) sred[t] += sred[t + PW];  // fold the part beyond the largest power of two
      __syncthreads();
      for (int s = PW / 2; s > 0; s >>= 1) {
        if (t < s) sred[t] += sred[t + s];
        __syncthreads();
      }
      if (t == 0) P.partial[cell * 4 + v] = sred[0];
      __syncthreads();
    }
  }
}

// sum of [nblocks][4] partials in a fixed order
// (one block per value, launched with 4 blocks; the same order as a serial
// pass over the four values)
__global__ void finalize4_kernel(const double* partial, int64_t nblocks, double* out) {
  __shared__ double sred[256];
  const int v = blockIdx.x;
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += 256) acc += partial[b * 4 + v];
  sred[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sred[threadIdx.x] += sred[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = sred[0];
}

// ------------------------------------------------------------------------------------------------
// load vector c_j = sum_e sum_q varpi_q detJ_q rho_q N_j(x_q), all nodes (full grid).
// LOAD_CPB(N) cells per block, N^2 threads per cell (one 1D line of the cell
// per thread and pass), so that the block fills whole wavefronts.
// ------------------------------------------------------------------------------------------------
constexpr int load_cpb(int N) { return (N * N * N * 16 <= 4096) ? 16 : 8; }

template <int N>
__global__ void __launch_bounds__(load_cpb(N) * N * N)
    load_kernel(const double* rho, const double* wdet, const double* tab, double* cload, int64_t n_cell, int ncx,
                int ncy, int p, int Nx, int Ny, int weighted) {
  constexpr int VOL = N * N * N;
  constexpr int CPB = load_cpb(N);
  __shared__ double sU[CPB * VOL];
  __shared__ double sB[N * N];
  const int slot = threadIdx.x / (N * N);
  const int t = threadIdx.x % (N * N);
  const int64_t cell = (int64_t)blockIdx.x * CPB + slot;
  const bool ok = cell < n_cell;
  double* U = sU + slot * VOL;
  if (threadIdx.x < N * N) sB[threadIdx.x] = tab[TAB_B + (threadIdx.x / N) * TDFE_MAXN + (threadIdx.x % N)];
  __syncthreads();
  const int cx = (int)(cell % ncx), cy = (int)((cell / ncx) % ncy), cz = (int)(cell / ((int64_t)ncx * ncy));
  double r1[N];
  {
    const int a = t % N, b = t / N;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const int64_t g = (ok ? cell : 0) * VOL + a + N * (b + N * c);
      r1[c] = ok ? (weighted ? wdet[g] * rho[g] : rho[g]) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double s = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) s += sB[c * N + k] * r1[c];
      U[(k * N + b) * N + a] = s;
    }
  }
  __syncthreads();
  {
    const int a = t % N, k = t / N;
#pragma unroll
    for (int b = 0; b < N; ++b) r1[b] = U[(k * N + b) * N + a];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double s = 0;
#pragma unroll
      for (int b = 0; b < N; ++b) s += sB[b * N + j] * r1[b];
      U[(k * N + j) * N + a] = s;
    }
  }
  __syncthreads();
  if (!ok) return;
  {
    // last pass with x across lanes: each atomic instruction touches N
    // consecutive nodes per z line instead of one node per lane
    const int i = t % N, k = t / N;
#pragma unroll
    for (int a = 0; a < N; ++a) r1[a] = sB[a * N + i];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double s = 0;
#pragma unroll
      for (int a = 0; a < N; ++a) s += r1[a] * U[(k * N + j) * N + a];
      const int64_t node = (int64_t)(cx * p + i) + (int64_t)Nx * ((int64_t)(cy * p + j) + (int64_t)Ny * (cz * p + k));
      unsafeAtomicAdd(cload + node, s);
    }
  }
}

// ------------------------------------------------------------------------------------------------
// nodal field (full grid) -> Gauss points, fused with the XC potential:
//   W_q = phi(x_q) + V_xc(rho_q)
// ------------------------------------------------------------------------------------------------
__device__ double vxc(double rho, int mode) {
  if (mode == TDFE_XC_NONE || !(rho > 1e-300)) return 0.0;
  double v = -cbrt(3.0 * rho / M_PI);
  if (mode == TDFE_XC_XC) {
    const double rs = cbrt(3.0 / (4.0 * M_PI * rho));
    if (rs >= 1.0) {
      const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
      const double sq = sqrt(rs);
      const double den = 1.0 + b1 * sq + b2 * rs;
      v += g * (1.0 + 7.0 / 6.0 * b1 * sq + 4.0 / 3.0 * b2 * rs) / (den * den);
    } else {
      const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
      const double lr = log(rs);
      v += A * lr + (B - A / 3.0) + 2.0 / 3.0 * C * rs * lr + (2.0 * D - C) / 3.0 * rs;
    }
  }
  return v;
}

template <int N>
__global__ void __launch_bounds__(N* N) interp_xc_kernel(const double* phi, const double* rho, const double* tab,
                                                          double* W, int hartree, int xcmode, int ncx, int ncy, int p,
                                                          int Nx, int Ny) {
  constexpr int VOL = N * N * N;
  __shared__ double sU[VOL];
  __shared__ double sB[N * N];
  const int t = threadIdx.x;
  const int64_t cell = blockIdx.x;
  if (t < N * N) sB[t] = tab[TAB_B + (t / N) * TDFE_MAXN + (t % N)];
  __syncthreads();
  const int cx = (int)(cell % ncx), cy = (int)((cell / ncx) % ncy), cz = (int)(cell / ((int64_t)ncx * ncy));
  double r1[N];
  {
    const int i = t % N, j = t / N;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int64_t node = (int64_t)(cx * p + i) + (int64_t)Nx * ((int64_t)(cy * p + j) + (int64_t)Ny * (cz * p + k));
      r1[k] = hartree ? phi[node] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < N; ++c) {
      double s = 0;
#pragma unroll
      for (int k = 0; k < N; ++k) s += sB[c * N + k] * r1[k];
      sU[(c * N + j) * N + i] = s;
    }
  }
  __syncthreads();
  {
    const int i = t % N, c = t / N;
#pragma unroll
    for (int j = 0; j < N; ++j) r1[j] = sU[(c * N + j) * N + i];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      double s = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) s += sB[b * N + j] * r1[j];
      sU[(c * N + b) * N + i] = s;
    }
  }
  __syncthreads();
  {
    const int b = t % N, c = t / N;
#pragma unroll
    for (int i = 0; i < N; ++i) r1[i] = sU[(c * N + b) * N + i];
#pragma unroll
    for (int a = 0; a < N; ++a) {
      double s = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) s += sB[a * N + i] * r1[i];
      const int64_t g = cell * VOL + a + N * (b + N * c);
      W[g] = s + (rho != nullptr ? vxc(rho[g], xcmode) : 0.0);
    }
  }
}

// vw = wdet * (vext - E z + ca * A + cb * B)   (A, B may be null)
// (Ex, Ey, Ez) = E_n times the field direction: V_field = -E_n (d . r) (Eq. VField)
__global__ void assemble_vw_kernel(const double* vext, const double* xq, const double* wdet, const double* A, double ca,
                                   const double* Bv, double cb, const double* Cv, double cc, double Ex, double Ey,
                                   double Ez, double* vw, float* vw32, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = vext[i] - (Ex * xq[i * 3] + Ey * xq[i * 3 + 1] + Ez * xq[i * 3 + 2]);
  if (A) v += ca * A[i];
  if (Bv) v += cb * Bv[i];
  if (Cv) v += cc * Cv[i];
  const double x = wdet[i] * v;
  vw[i] = x;
  if (vw32) vw32[i] = (float)x;
}

__global__ void copy4_kernel(const double* src, double* dst) {
  if (threadIdx.x < 4) dst[threadIdx.x] = src[threadIdx.x];
}

// fold one Lanczos result slot (k, status, error per orbital; overflow flag)
// into acc = {max k, sum k, max error, not-converged flag, overflow flag}
__global__ void accum_results_kernel(const double* slot, int n_orb, int nm, double* acc) {
  if (threadIdx.x != 0) return;
  for (int o = 0; o < n_orb; ++o) {
    const double k = slot[o];
    acc[0] = fmax(acc[0], k);
    acc[1] += k;
    acc[2] = fmax(acc[2], slot[2 * nm + o]);
    if (slot[nm + o] == 2.0) acc[3] = 1.0;
    if (slot[nm + o] == 4.0) acc[5] = 1.0;
  }
  if (slot[3 * nm] != 0.0) acc[4] = 1.0;
}

// out = ca A + cb B (+ cc C)
__global__ void combine3_kernel(const double* A, double ca, const double* B, double cb, const double* C, double cc,
                                double* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = ca * A[i] + cb * B[i];
  if (C) v += cc * C[i];
  out[i] = v;
}

// self-consistent midpoint: wmid <- (w1 + wn)/2; part[block] = largest |change|
// (a NaN anywhere propagates to the result)
constexpr int SC_BLOCKS = 256;
__global__ void __launch_bounds__(EW) midpoint_update_kernel(const double* w1, const double* wn, double* wmid, int64_t n,
                                                            double* part) {
  __shared__ double s[EW];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x; i < n; i += (int64_t)gridDim.x * EW) {
    const double v = 0.5 * (w1[i] + wn[i]);
    const double d = fabs(v - wmid[i]);
    wmid[i] = v;
    if (!(d <= m)) m = d;
  }
  s[threadIdx.x] = m;
  __syncthreads();
  for (int w = EW / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w && !(s[threadIdx.x + w] <= s[threadIdx.x])) s[threadIdx.x] = s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void max_final_kernel(const double* part, int nb, double* out) {
  if (threadIdx.x != 0) return;
  double m = 0.0;
  for (int b = 0; b < nb; ++b)
    if (!(part[b] <= m)) m = part[b];
  *out = m;
}

// Lagrange weights of the instants t_{n-1}, t_{n-2}, t_{n-3} (abscissae 0, -1,
// -2 in steps) at abscissa s; order 1 uses the first two
void extrapolation_weights(double s, int order, double l[3]) {
  if (order <= 1) {
    l[0] = 1.0 + s;
    l[1] = -s;
    l[2] = 0.0;
    return;
  }
  l[0] = (s + 1.0) * (s + 2.0) / 2.0;
  l[1] = -s * (s + 2.0);
  l[2] = s * (s + 1.0) / 2.0;
}

// ------------------------------------------------------------------------------------------------
// Poisson: boundary data, right-hand side, fast diagonalisation
// ------------------------------------------------------------------------------------------------
__global__ void boundary_values_kernel(const double* nodexyz, const double* ZR, int nnuc, double* fb, double* phi,
                                       int Nx, int Ny, int Nz) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)Nx * Ny * Nz;
  if (idx >= nn) return;
  const int I = (int)(idx % Nx), J = (int)((idx / Nx) % Ny), K = (int)(idx / ((int64_t)Nx * Ny));
  const bool bnd = I == 0 || I == Nx - 1 || J == 0 || J == Ny - 1 || K == 0 || K == Nz - 1;
  double f = 0.0;
  if (bnd) {
    for (int a = 0; a < nnuc; ++a) {
      const double dx = nodexyz[idx * 3 + 0] - ZR[a * 4 + 1];
      const double dy = nodexyz[idx * 3 + 1] - ZR[a * 4 + 2];
      const double dz = nodexyz[idx * 3 + 2] - ZR[a * 4 + 3];
      f += ZR[a * 4 + 0] / sqrt(dx * dx + dy * dy + dz * dz);
    }
  }
  fb[idx] = f;
  phi[idx] = f;
}

// interior entries of a full-grid array -> DoF numbering, out = s * full[node] - sub[dof]
__global__ void gather_interior_kernel(const double* full, const double* sub, double s, double* out, int Nx, int Ny,
                                       int Nz) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nd = (int64_t)(Nx - 2) * (Ny - 2) * (Nz - 2);
  if (d >= nd) return;
  const int i = (int)(d % (Nx - 2)), j = (int)((d / (Nx - 2)) % (Ny - 2)), k = (int)(d / ((int64_t)(Nx - 2) * (Ny - 2)));
  const int64_t node = (int64_t)(i + 1) + (int64_t)Nx * ((int64_t)(j + 1) + (int64_t)Ny * (k + 1));
  out[d] = s * full[node] - (sub ? sub[d] : 0.0);
}

__global__ void scatter_interior_kernel(const double* in, double* full, int Nx, int Ny, int Nz) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nd = (int64_t)(Nx - 2) * (Ny - 2) * (Nz - 2);
  if (d >= nd) return;
  const int i = (int)(d % (Nx - 2)), j = (int)((d / (Nx - 2)) % (Ny - 2)), k = (int)(d / ((int64_t)(Nx - 2) * (Ny - 2)));
  const int64_t node = (int64_t)(i + 1) + (int64_t)Nx * ((int64_t)(j + 1) + (int64_t)Ny * (k + 1));
  full[node] = in[d];
}

// Register-tiled form of the same transform: a block stages FDM_TB lines and
// the whole 1D matrix R (R = S for the transposed product, S^T otherwise) in
// LDS; the FDM_G groups of FDM_TB lanes each own output modes
// [g MPT, g MPT + MPT) of every line and sweep the input modes once (a row
// of R is read at one address per group: LDS broadcasts in distinct banks).
// lam scaling is supported along z only.
constexpr int FDM_TB = 16, FDM_G = 16;
// rows of R are padded with zeros to FDM_G * MPT entries, so the inner loop needs no bounds test
inline size_t fdm_tile_lds(int nax, int mpt) {
  return ((size_t)nax * FDM_G * mpt + (size_t)nax * FDM_TB) * sizeof(double);
}
template <int MPT>
__global__ void __launch_bounds__(FDM_TB* FDM_G) fdm_tile_kernel(const double* __restrict__ in, double* __restrict__ out,
                                                                 const double* __restrict__ R, int n1x, int n1y,
                                                                 int n1z, int axis, const double* lx, const double* ly,
                                                                 const double* lz) {
  extern __shared__ double lds[];
  const int nax = axis == 0 ? n1x : (axis == 1 ? n1y : n1z);
  constexpr int RP = FDM_G * MPT;
  double* sR = lds;                        // [nax][RP], zero beyond column nax
  double* tile = lds + (size_t)nax * RP;   // [nax][FDM_TB]; reused as [FDM_TB][nax] for x-line output
  const int64_t nlines = (int64_t)n1x * n1y * n1z / nax;
  const int64_t l0 = (int64_t)blockIdx.x * FDM_TB;
  const int t = threadIdx.x;
  auto base_stride = [&](int64_t line, int64_t& base, int64_t& stride) {
    if (axis == 0) {
      base = line * n1x;
      stride = 1;
    } else if (axis == 1) {
      const int64_t i = line % n1x, k = line / n1x;
      base = i + k * (int64_t)n1x * n1y;
      stride = n1x;
    } else {
      base = line;
      stride = (int64_t)n1x * n1y;
    }
  };
  // staging: eight loads in flight per thread before their LDS stores
  constexpr int NT = FDM_TB * FDM_G, UNR = 8;
  for (int i0 = t; i0 < nax * RP; i0 += NT * UNR) {
    double v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = i0 + u * NT;
      const int m = idx / RP, mp = idx % RP;
      v[u] = (idx < nax * RP && mp < nax) ? R[m * nax + mp] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = i0 + u * NT;
      if (idx < nax * RP) sR[idx] = v[u];
    }
  }
  for (int i0 = t; i0 < nax * FDM_TB; i0 += NT * UNR) {
    double v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = i0 + u * NT;
      v[u] = 0.0;
      if (idx < nax * FDM_TB) {
        int m, l;
        if (axis == 0) {
          l = idx / nax;
          m = idx % nax;
        } else {
          m = idx / FDM_TB;
          l = idx % FDM_TB;
        }
        const int64_t line = l0 + l;
        if (line < nlines) {
          int64_t b, st;
          base_stride(line, b, st);
          v[u] = in[b + m * st];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = i0 + u * NT;
      if (idx < nax * FDM_TB) {
        const int m = axis == 0 ? idx % nax : idx / FDM_TB;
        const int l = axis == 0 ? idx / nax : idx % FDM_TB;
        tile[m * FDM_TB + l] = v[u];
      }
    }
  }
  __syncthreads();
  const int l = t % FDM_TB;
  const int g = t / FDM_TB;
  const int mp0 = g * MPT;
  double acc[MPT];
#pragma unroll
  for (int q = 0; q < MPT; ++q) acc[q] = 0.0;
  if (mp0 < nax) {
    for (int m = 0; m < nax; ++m) {
      const double v = tile[m * FDM_TB + l];
      const double* Rm = sR + m * RP + mp0;
#pragma unroll
      for (int q = 0; q < MPT; ++q) acc[q] += Rm[q] * v;
    }
  }
  const int64_t line = l0 + l;
  if (axis == 0) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MPT; ++q)
      if (mp0 + q < nax) tile[l * nax + mp0 + q] = acc[q];
    __syncthreads();
    for (int idx = t; idx < nax * FDM_TB; idx += FDM_TB * FDM_G) {
      const int ll = idx / nax, mp = idx % nax;
      if (l0 + ll < nlines) out[(l0 + ll) * n1x + mp] = tile[ll * nax + mp];
    }
    return;
  }
  if (line >= nlines) return;
  int64_t b, st;
  base_stride(line, b, st);
  double lxy = 0.0;
  if (lx) lxy = lx[line % n1x] + ly[line / n1x];  // axis 2: line = i + n1x j
#pragma unroll
  for (int q = 0; q < MPT; ++q) {
    const int mp = mp0 + q;
    if (mp < nax) out[b + (int64_t)mp * st] = lx ? acc[q] / (lxy + lz[mp]) : acc[q];
  }
}

// Axes of more than 128 interior nodes: the 1D transform is a plain dense
// product of the n1 x n1 table with every grid line along the axis, done by
// rocBLAS DGEMM (FP64 matrix cores) on the context's stream.  The interior
// grid, index i + n1x (j + n1y k), is read as column-major matrices:
//   x: (n1x) x (n1y n1z), ld n1x            out = Op x
//   y: n1z slabs of (n1x) x (n1y), ld n1x    out = slab Op^T   (strided batched)
//   z: (n1x n1y) x (n1z), ld n1x n1y        out = in Op^T
// with Op = S^T (trans = 1) or S (trans = 0); S is stored row-major, i.e. as
// the column-major S^T.  The scaling by 1 / (lx_i + ly_j + lz_k) follows as
// its own pass.
__global__ void fdm_scale_kernel(double* v, int n1x, int n1y, int n1z, const double* lx, const double* ly,
                                 const double* lz) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= (int64_t)n1x * n1y * n1z) return;
  const int i = (int)(d % n1x), j = (int)((d / n1x) % n1y), k = (int)(d / ((int64_t)n1x * n1y));
  v[d] /= lx[i] + ly[j] + lz[k];
}

tdfe_status blas_ready(tdfe_ctx* c) {
  if (c->blas) return TDFE_OK;
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success)
    return tdfe_fail(c, TDFE_EDEVICE, "rocblas_create_handle failed");
  if (rocblas_set_stream(h, c->stream) != rocblas_status_success) {
    rocblas_destroy_handle(h);
    return tdfe_fail(c, TDFE_EDEVICE, "rocblas_set_stream failed");
  }
  c->blas = (void*)h;
  return TDFE_OK;
}

// one fast-diagonalisation pass as a rocBLAS product: axis 0 and 2 one
// DGEMM over the whole array, axis 1 a strided batch over z slabs
struct FdmGemm {
  rocblas_operation ta, tb;
  int m, n, k;
  const double* A;
  int lda;
  rocblas_stride sa;
  const double* B;
  int ldb;
  rocblas_stride sb;
  int ldc;
  rocblas_stride sc;
  int batch;  // 0: a single product
};

rocblas_status fdm_gemm(rocblas_handle h, const FdmGemm& g, double* out, rocblas_gemm_algo algo, int32_t sol) {
  const double one = 1.0, zero = 0.0;
  const rocblas_datatype f64 = rocblas_datatype_f64_r;
  if (g.batch == 0)
    return rocblas_gemm_ex(h, g.ta, g.tb, g.m, g.n, g.k, &one, g.A, f64, g.lda, g.B, f64, g.ldb, &zero, out, f64,
                           g.ldc, out, f64, g.ldc, f64, algo, sol, 0);
  return rocblas_gemm_strided_batched_ex(h, g.ta, g.tb, g.m, g.n, g.k, &one, g.A, f64, g.lda, g.sa, g.B, f64, g.ldb,
                                         g.sb, &zero, out, f64, g.ldc, g.sc, out, f64, g.ldc, g.sc, g.batch, f64, algo,
                                         sol, 0);
}

// rocBLAS's default kernel for these shapes (K = one axis, some hundreds;
// the other dimension the rest of the grid) runs at about 10-30 TFLOP/s; at
// a pass's first use every solution rocBLAS lists for it is timed on the
// stream (the output is overwritten, the input is not touched) and the
// fastest kept: 272^3 passes 228-273 -> 175-186 us, 185^3 85 -> 47 us
void fdm_tune(tdfe_ctx* c, rocblas_handle h, const FdmGemm& g, double* out, int* algo_out, int* sol_out) {
  *algo_out = (int)rocblas_gemm_algo_standard;
  *sol_out = 0;
  const double one = 1.0, zero = 0.0;
  const rocblas_datatype f64 = rocblas_datatype_f64_r;
  const rocblas_gemm_algo idx = rocblas_gemm_algo_solution_index;
  rocblas_int cnt = 0;
  auto list = [&](rocblas_int* arr) {
    if (g.batch == 0)
      return rocblas_gemm_ex_get_solutions(h, g.ta, g.tb, g.m, g.n, g.k, &one, g.A, f64, g.lda, g.B, f64, g.ldb, &zero,
                                           out, f64, g.ldc, out, f64, g.ldc, f64, idx, 0, arr, &cnt);
    return rocblas_gemm_strided_batched_ex_get_solutions(h, g.ta, g.tb, g.m, g.n, g.k, &one, g.A, f64, g.lda, g.sa, g.B,
                                                         f64, g.ldb, g.sb, &zero, out, f64, g.ldc, g.sc, out, f64,
                                                         g.ldc, g.sc, g.batch, f64, idx, 0, arr, &cnt);
  };
  if (list(nullptr) != rocblas_status_success || cnt <= 0) return;
  std::vector<rocblas_int> sols((size_t)cnt);
  if (list(sols.data()) != rocblas_status_success) return;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    return;
  }
  auto time_one = [&](rocblas_gemm_algo a, int32_t s) -> float {
    if (fdm_gemm(h, g, out, a, s) != rocblas_status_success) return -1.f;  // warm-up
    if (hipEventRecord(e0, c->stream) != hipSuccess) return -1.f;
    for (int r = 0; r < 3; ++r)
      if (fdm_gemm(h, g, out, a, s) != rocblas_status_success) return -1.f;
    float ms = -1.f;
    if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return -1.f;
    return ms;
  };
  float best = time_one(rocblas_gemm_algo_standard, 0);
  for (const rocblas_int s : sols) {
    const float t = time_one(idx, s);
    if (t > 0.f && (best < 0.f || t < best)) {
      best = t;
      *algo_out = (int)idx;
      *sol_out = s;
    }
  }
  (void)hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

tdfe_status fdm_blas_pass(tdfe_ctx* c, const double* in, double* out, const double* S, int axis, int trans) {
  TDFE_TRY(blas_ready(c));
  rocblas_handle h = (rocblas_handle)c->blas;
  const int n1x = c->Nx - 2, n1y = c->Ny - 2, n1z = c->Nz - 2;
  const rocblas_operation nt = rocblas_operation_none, tr = rocblas_operation_transpose;
  FdmGemm g{};
  if (axis == 0) {
    g = FdmGemm{trans ? nt : tr, nt, n1x, n1y * n1z, n1x, S, n1x, 0, in, n1x, 0, n1x, 0, 0};
  } else if (axis == 1) {
    const rocblas_stride slab = (rocblas_stride)n1x * n1y;
    g = FdmGemm{nt, trans ? tr : nt, n1x, n1y, n1y, in, n1x, slab, S, n1y, 0, n1x, slab, n1z};
  } else {
    g = FdmGemm{nt, trans ? tr : nt, n1x * n1y, n1z, n1z, in, n1x * n1y, 0, S, n1z, 0, n1x * n1y, 0, 0};
  }
  const int tq = trans ? 1 : 0;
  if (!c->fdm_tuned[axis][tq]) {
    fdm_tune(c, h, g, out, &c->fdm_algo[axis][tq], &c->fdm_sol[axis][tq]);
    c->fdm_tuned[axis][tq] = 1;
  }
  const rocblas_status st = fdm_gemm(h, g, out, (rocblas_gemm_algo)c->fdm_algo[axis][tq], c->fdm_sol[axis][tq]);
  if (st != rocblas_status_success) return tdfe_fail(c, TDFE_EDEVICE, "rocBLAS DGEMM failed (status %d)", (int)st);
  return TDFE_OK;
}

// ---- host linear algebra for the 1D fast-diagonalisation tables ------------------------------
void cholesky(std::vector<double>& A, int n) {  // lower, in place
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
    A[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = t / A[j * n + j];
    }
    for (int k = j + 1; k < n; ++k) A[j * n + k] = 0.0;
  }
}

// cyclic Jacobi eigenvalue algorithm for a symmetric matrix: A = U diag(lam) U^T
void jacobi_eigen(std::vector<double> A, int n, std::vector<double>& lam, std::vector<double>& U) {
  U.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double v = A[(size_t)i * n + j] * A[(size_t)i * n + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(tt * tt + 1.0), sn = tt * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = cs * akp - sn * akq;
          A[(size_t)k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = cs * apk - sn * aqk;
          A[(size_t)q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double ukp = U[(size_t)k * n + p], ukq = U[(size_t)k * n + q];
          U[(size_t)k * n + p] = cs * ukp - sn * ukq;
          U[(size_t)k * n + q] = sn * ukp + cs * ukq;
        }
        // the rotation annihilates a_pq: store the zero rather than the
        // rounding residue, or the off-diagonal sum never meets the stop test
        A[(size_t)p * n + q] = A[(size_t)q * n + p] = 0.0;
      }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = A[(size_t)i * n + i];
}

// 1D interior stiffness and mass of one axis; returns S (row-major, S[m][mode]) and lambda
void fdm_axis(const tdfe_ctx* c, const std::vector<double>& ax, std::vector<double>& S, std::vector<double>& lam) {
  const int p = c->p, n = c->n, nq = c->nq;
  const int ncell = (int)ax.size() - 1;
  const int nn = ncell * p + 1;
  std::vector<double> K((size_t)nn * nn, 0.0), M((size_t)nn * nn, 0.0);
  for (int e = 0; e < ncell; ++e) {
    const double h = ax[e + 1] - ax[e];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double kk = 0.0, mm = 0.0;
        for (int a = 0; a < nq; ++a) {
          kk += c->wq[a] * c->D[a * TDFE_MAXN + i] * c->D[a * TDFE_MAXN + j];
          mm += c->wq[a] * c->B[a * TDFE_MAXN + i] * c->B[a * TDFE_MAXN + j];
        }
        const int I = e * p + i, J = e * p + j;
        K[(size_t)I * nn + J] += kk * 2.0 / h;
        M[(size_t)I * nn + J] += mm * h / 2.0;
      }
  }
  const int m = nn - 2;
  std::vector<double> Ki((size_t)m * m), Mi((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      Ki[(size_t)i * m + j] = K[(size_t)(i + 1) * nn + (j + 1)];
      Mi[(size_t)i * m + j] = M[(size_t)(i + 1) * nn + (j + 1)];
    }
  cholesky(Mi, m);  // Mi = L L^T
  // C = L^-1 K L^-T
  std::vector<double> X = Ki;  // solve L X = K  (columns)
  for (int col = 0; col < m; ++col)
    for (int i = 0; i < m; ++i) {
      double s = X[(size_t)i * m + col];
      for (int k = 0; k < i; ++k) s -= Mi[(size_t)i * m + k] * X[(size_t)k * m + col];
      X[(size_t)i * m + col] = s / Mi[(size_t)i * m + i];
    }
  std::vector<double> Cm((size_t)m * m);  // C = X L^-T  ->  solve L C^T = X^T
  for (int row = 0; row < m; ++row)
    for (int i = 0; i < m; ++i) {
      double s = X[(size_t)row * m + i];
      for (int k = 0; k < i; ++k) s -= Mi[(size_t)i * m + k] * Cm[(size_t)row * m + k];
      Cm[(size_t)row * m + i] = s / Mi[(size_t)i * m + i];
    }
  for (int i = 0; i < m; ++i)  // symmetrise rounding
    for (int j = i + 1; j < m; ++j) {
      const double v = 0.5 * (Cm[(size_t)i * m + j] + Cm[(size_t)j * m + i]);
      Cm[(size_t)i * m + j] = Cm[(size_t)j * m + i] = v;
    }
  std::vector<double> U;
  jacobi_eigen(Cm, m, lam, U);
  // S = L^-T U  (back substitution with L^T)
  S.assign((size_t)m * m, 0.0);
  for (int col = 0; col < m; ++col)
    for (int i = m - 1; i >= 0; --i) {
      double s = U[(size_t)i * m + col];
      for (int k = i + 1; k < m; ++k) s -= Mi[(size_t)k * m + i] * S[(size_t)k * m + col];
      S[(size_t)i * m + col] = s / Mi[(size_t)i * m + i];
    }
}

// t0 <- K_box^-1 t0 (interior vectors; t1 is scratch): the six 1D transforms
// and the diagonal scaling of the fast diagonalisation of the rectilinear
// stiffness built from the axes of tdfe_fdm_setup
tdfe_status fdm_passes(tdfe_ctx* c) {
  const int n1x = c->Nx - 2, n1y = c->Ny - 2, n1z = c->Nz - 2;
  const int64_t nd = c->n_dof;
  const double* Sx = c->fdmS;
  const double* Sy = Sx + (size_t)n1x * n1x;
  const double* Sz = Sy + (size_t)n1y * n1y;
  const double* lx = c->fdmL;
  const double* ly = lx + n1x;
  const double* lz = ly + n1y;
  const size_t nS = (size_t)n1x * n1x + (size_t)n1y * n1y + (size_t)n1z * n1z;
  auto pass = [&](const double* in, double* out, int axis, int trans, bool scale) -> tdfe_status {
    const int nax = axis == 0 ? n1x : (axis == 1 ? n1y : n1z);
    const int64_t nlines = nd / nax;
    const double* S = axis == 0 ? Sx : (axis == 1 ? Sy : Sz);
    const double* St = S + nS;  // transposed copy
    const double* sl = scale ? lx : nullptr;
    int mpt = (nax + FDM_G - 1) / FDM_G;
    for (int cand : {1, 2, 3, 4, 5, 6, 8})
      if (mpt <= cand) {
        mpt = cand;
        break;
      }
    const size_t shm_t = fdm_tile_lds(nax, mpt);
    const unsigned gt = (unsigned)((nlines + FDM_TB - 1) / FDM_TB);
    const double* Rm = trans ? S : St;
#define TDFE_FDM_TILE(M)                                                                                       \
  do {                                                                                                          \
    TDFE_HIP(c, hipFuncSetAttribute((const void*)fdm_tile_kernel<M>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                    (int)shm_t));                                                              \
    hipLaunchKernelGGL((fdm_tile_kernel<M>), dim3(gt), dim3(FDM_TB * FDM_G), shm_t, c->stream, in, out, Rm, n1x, \
                       n1y, n1z, axis, sl, ly, lz);                                                            \
  } while (0)
    if (shm_t > 160 * 1024 || mpt > 8)
      mpt = 1 << 30;  // matrix does not fit LDS: rocBLAS below
    if (mpt <= 1)
      TDFE_FDM_TILE(1);
    else if (mpt <= 2)
      TDFE_FDM_TILE(2);
    else if (mpt <= 3)
      TDFE_FDM_TILE(3);
    else if (mpt <= 4)
      TDFE_FDM_TILE(4);
    else if (mpt <= 5)
      TDFE_FDM_TILE(5);
    else if (mpt <= 6)
      TDFE_FDM_TILE(6);
    else if (mpt <= 8)
      TDFE_FDM_TILE(8);
#undef TDFE_FDM_TILE
    else {
      TDFE_TRY(fdm_blas_pass(c, in, out, S, axis, trans));
      if (sl) {
        hipLaunchKernelGGL(fdm_scale_kernel, dim3(nblk(nd)), dim3(EW), 0, c->stream, out, n1x, n1y, n1z, sl, ly, lz);
      }
    }
    TDFE_HIP(c, hipGetLastError());
    return TDFE_OK;
  };
  TDFE_TRY(pass(c->t0, c->t1, 0, 1, false));
  TDFE_TRY(pass(c->t1, c->t0, 1, 1, false));
  TDFE_TRY(pass(c->t0, c->t1, 2, 1, true));
  TDFE_TRY(pass(c->t1, c->t0, 2, 0, false));
  TDFE_TRY(pass(c->t0, c->t1, 1, 0, false));
  TDFE_TRY(pass(c->t1, c->t0, 0, 0, false));
  return TDFE_OK;
}

// box meshes: the exact Hartree solve, phi_interior = K^-1 (4 pi c - (K f))_interior
tdfe_status fdm_solve(tdfe_ctx* c, bool with_lift, double* phi_full) {
  const int64_t nd = c->n_dof;
  hipLaunchKernelGGL(gather_interior_kernel, dim3(nblk(nd)), dim3(EW), 0, c->stream, c->cload,
                     with_lift ? (const double*)c->lift : (const double*)nullptr, 4.0 * M_PI, c->t0, c->Nx, c->Ny, c->Nz);
  TDFE_TRY(fdm_passes(c));
  hipLaunchKernelGGL(scatter_interior_kernel, dim3(nblk(nd)), dim3(EW), 0, c->stream, c->t0, phi_full, c->Nx, c->Ny,
                     c->Nz);
  TDFE_HIP(c, hipGetLastError());
  c->last_poisson_iters = 0;
  return TDFE_OK;
}

// curved meshes: the PCG preconditioner z = K_box^-1 r on full-grid vectors
// (interior entries; the boundary entries of z are left as they are, zero)
tdfe_status fdm_precondition(tdfe_ctx* c, const double* r_full, double* z_full) {
  const int64_t nd = c->n_dof;
  hipLaunchKernelGGL(gather_interior_kernel, dim3(nblk(nd)), dim3(EW), 0, c->stream, r_full, (const double*)nullptr,
                     1.0, c->t0, c->Nx, c->Ny, c->Nz);
  TDFE_TRY(fdm_passes(c));
  hipLaunchKernelGGL(scatter_interior_kernel, dim3(nblk(nd)), dim3(EW), 0, c->stream, c->t0, z_full, c->Nx, c->Ny,
                     c->Nz);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

template <int N>
tdfe_status launch_density_n(tdfe_ctx* c, DensParams& P) {
  constexpr int CB = (N * N * 16 <= 1024 && N <= 6) ? 16 : ((N * N * 8 <= 1024) ? 8 : 4);
  hipLaunchKernelGGL((density_kernel<N, CB>), dim3((unsigned)c->n_cell), dim3(N * N * CB), 0, c->stream, P);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

template <int N>
tdfe_status launch_load_interp(tdfe_ctx* c, int which, const double* in, const double* rho, int flag, double* out) {
  if (which == 0) {
    constexpr int CPB = load_cpb(N);
    hipLaunchKernelGGL((load_kernel<N>), dim3((unsigned)((c->n_cell + CPB - 1) / CPB)), dim3(CPB * N * N), 0,
                       c->stream, in, c->wdet, c->tab, out, (int64_t)c->n_cell, c->ncx, c->ncy, c->p, c->Nx, c->Ny,
                       flag);
  } else {
    hipLaunchKernelGGL((interp_xc_kernel<N>), dim3((unsigned)c->n_cell), dim3(N * N), 0, c->stream, in, rho,
                       c->tab, out, in != nullptr ? 1 : 0, flag, c->ncx, c->ncy, c->p, c->Nx, c->Ny);
  }
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

#define TDFE_DISPATCH_N(FN, ...)                        \
  switch (c->n) {                                      \
    case 2: return FN<2>(__VA_ARGS__);                 \
    case 3: return FN<3>(__VA_ARGS__);                 \
    case 4: return FN<4>(__VA_ARGS__);                 \
    case 5: return FN<5>(__VA_ARGS__);                 \
    case 6: return FN<6>(__VA_ARGS__);                 \
    case 7: return FN<7>(__VA_ARGS__);                 \
    case 8: return FN<8>(__VA_ARGS__);                 \
    case 9: return FN<9>(__VA_ARGS__);                 \
  }                                                    \
  return tdfe_fail(c, TDFE_EINVAL, "unsupported order");

tdfe_status density_launch(tdfe_ctx* c, DensParams& P) { TDFE_DISPATCH_N(launch_density_n, c, P) }
tdfe_status load_launch(tdfe_ctx* c) { TDFE_DISPATCH_N(launch_load_interp, c, 0, c->rho, nullptr, 1, c->cload) }
tdfe_status interp_launch(tdfe_ctx* c, double* W) {
  TDFE_DISPATCH_N(launch_load_interp, c, 1, c->hartree ? c->phi : nullptr, c->rho, c->xc, W)
}
tdfe_status load_launch_f(tdfe_ctx* c, const double* f, int weighted) {
  TDFE_DISPATCH_N(launch_load_interp, c, 0, f, nullptr, weighted, c->cload)
}
tdfe_status interp_launch_f(tdfe_ctx* c, const double* phi, const double* rho, int xcmode, double* out) {
  TDFE_DISPATCH_N(launch_load_interp, c, 1, phi, rho, xcmode, out)
}

tdfe_status upload_occ(tdfe_ctx* c, int n_orb, double** dev) {
  // occupations live in the scalar block's tail
  double* occ = c->scal + (size_t)(8 * c->k_max + 32) * c->n_orb_max - c->n_orb_max;
  *dev = occ;
  // uploaded once per set of occupations and orbital count (an upload per
  // density evaluation would stall the stream for a host staging copy)
  if (c->occ_dev_ver == c->occ_ver && c->occ_dev_n == n_orb) return TDFE_OK;
  c->occ_dev_ver = c->occ_ver;
  c->occ_dev_n = n_orb;
  // persistent host copy: the asynchronous upload may still read it after return
  c->occ_host.assign(c->n_orb_max, 1.0);
  for (int o = 0; o < n_orb && o < (int)c->occ.size(); ++o) c->occ_host[o] = c->occ[o];
  TDFE_HIP(c, hipMemcpyAsync(occ, c->occ_host.data(), n_orb * sizeof(double), hipMemcpyHostToDevice, c->stream));
  *dev = occ;
  return TDFE_OK;
}

// ------------------------------------------------------------------------------------------------
// curved meshes: Hartree by Jacobi-preconditioned conjugate gradients on the interior nodes
// (K_00 phi_0 = 4 pi c_0 - (K f)_0, Eqs. Poisson, VHDiscretePoisson), warm-started from the
// previous solution.  Vectors are full-grid arrays with zero boundary entries so that the
// operator kernel's stiffness mode applies K directly; p^T K p comes from that kernel's own
// quadrature-point quadratic form.  Reductions are two-level in a fixed order.
// ------------------------------------------------------------------------------------------------
constexpr int PCG_BLOCKS = 512;
constexpr int PCG_DONE = 160, PCG_ITERS = 161, PCG_FAIL = 162;  // int slots in c->counters

__device__ __forceinline__ bool interior_node(int64_t idx, int Nx, int Ny, int Nz) {
  const int I = (int)(idx % Nx), J = (int)((idx / Nx) % Ny), K = (int)(idx / ((int64_t)Nx * Ny));
  return I > 0 && I < Nx - 1 && J > 0 && J < Ny - 1 && K > 0 && K < Nz - 1;
}

// diag(K) over all nodes: sum over cells and Gauss points of w detJ (grad_xi N)^T J^-1 J^-T (grad_xi N)
template <int N>
__global__ void __launch_bounds__(N* N* N) stiffness_diag_kernel(const double* corners, const double* tab,
                                                                  double* diag, int ncx, int ncy, int p, int Nx,
                                                                  int Ny) {
  constexpr int VOL = N * N * N;
  __shared__ double sG[VOL * 6];
  __shared__ double sB[N * N], sD[N * N];
  const int t = threadIdx.x;
  const int64_t cell = blockIdx.x;
  if (t < N * N) {
    sB[t] = tab[TAB_B + (t / N) * TDFE_MAXN + (t % N)];
    sD[t] = tab[TAB_D + (t / N) * TDFE_MAXN + (t % N)];
  }
  {
    const int a = t % N, b = (t / N) % N, cq = t / (N * N);
    const double xa = tab[TAB_ETA + a], xb = tab[TAB_ETA + b], xc = tab[TAB_ETA + cq];
    const double f[2][3] = {{0.5 * (1 - xa), 0.5 * (1 - xb), 0.5 * (1 - xc)},
                            {0.5 * (1 + xa), 0.5 * (1 + xb), 0.5 * (1 + xc)}};
    const double* C = corners + cell * 24;
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int vz = 0; vz < 2; ++vz)
      for (int vy = 0; vy < 2; ++vy)
        for (int vx = 0; vx < 2; ++vx) {
          const double* X3 = C + ((vz * 2 + vy) * 2 + vx) * 3;
          const double d0 = (vx ? 0.5 : -0.5) * f[vy][1] * f[vz][2];
          const double d1 = f[vx][0] * (vy ? 0.5 : -0.5) * f[vz][2];
          const double d2 = f[vx][0] * f[vy][1] * (vz ? 0.5 : -0.5);
          for (int d = 0; d < 3; ++d) {
            J[d][0] += X3[d] * d0;
            J[d][1] += X3[d] * d1;
            J[d][2] += X3[d] * d2;
          }
        }
    double A[3][3];  // adjugate rows: J^-1 = A / det
    A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
    const double s = tab[TAB_W3Q + t] / det;
    double* g = sG + t * 6;
    g[0] = s * (A[0][0] * A[0][0] + A[0][1] * A[0][1] + A[0][2] * A[0][2]);
    g[1] = s * (A[0][0] * A[1][0] + A[0][1] * A[1][1] + A[0][2] * A[1][2]);
    g[2] = s * (A[0][0] * A[2][0] + A[0][1] * A[2][1] + A[0][2] * A[2][2]);
    g[3] = s * (A[1][0] * A[1][0] + A[1][1] * A[1][1] + A[1][2] * A[1][2]);
    g[4] = s * (A[1][0] * A[2][0] + A[1][1] * A[2][1] + A[1][2] * A[2][2]);
    g[5] = s * (A[2][0] * A[2][0] + A[2][1] * A[2][1] + A[2][2] * A[2][2]);
  }
  __syncthreads();
  const int i = t % N, j = (t / N) % N, k = t / (N * N);
  double acc = 0.0;
  for (int cq = 0; cq < N; ++cq)
    for (int b = 0; b < N; ++b)
      for (int a = 0; a < N; ++a) {
        const double bi = sB[a * N + i], bj = sB[b * N + j], bk = sB[cq * N + k];
        const double g0 = sD[a * N + i] * bj * bk, g1 = bi * sD[b * N + j] * bk, g2 = bi * bj * sD[cq * N + k];
        const double* G = sG + (a + N * (b + N * cq)) * 6;
        acc += G[0] * g0 * g0 + G[3] * g1 * g1 + G[5] * g2 * g2 +
               2.0 * (G[1] * g0 * g1 + G[2] * g0 * g2 + G[4] * g1 * g2);
      }
  const int cx = (int)(cell % ncx), cy = (int)((cell / ncx) % ncy), cz = (int)(cell / ((int64_t)ncx * ncy));
  const int64_t node = (int64_t)(cx * p + i) + (int64_t)Nx * ((int64_t)(cy * p + j) + (int64_t)Ny * (cz * p + k));
  unsafeAtomicAdd(diag + node, acc);
}

// in place: d <- 1/d inside, 0 on the boundary
__global__ void invert_diag_kernel(double* d, int Nx, int Ny, int Nz) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)Nx * Ny * Nz) return;
  d[idx] = interior_node(idx, Nx, Ny, Nz) ? 1.0 / d[idx] : 0.0;
}

// b <- 4 pi c - lift inside, 0 on the boundary (in place on the load vector); x <- interior of phi
__global__ void pcg_rhs_kernel(double* b, const double* lift, const double* phi, double* x, int Nx, int Ny, int Nz) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)Nx * Ny * Nz) return;
  const int I = (int)(idx % Nx), J = (int)((idx / Nx) % Ny), K = (int)(idx / ((int64_t)Nx * Ny));
  const bool in = I > 0 && I < Nx - 1 && J > 0 && J < Ny - 1 && K > 0 && K < Nz - 1;
  if (in) {
    const int64_t d = (int64_t)(I - 1) + (int64_t)(Nx - 2) * ((int64_t)(J - 1) + (int64_t)(Ny - 2) * (K - 1));
    b[idx] = 4.0 * M_PI * b[idx] - lift[d];
    x[idx] = phi[idx];
  } else {
    b[idx] = 0.0;
    x[idx] = 0.0;
  }
}

__device__ void block_sum3(double v0, double v1, double v2, double* out) {
  __shared__ double sred[3][EW];
  const int t = threadIdx.x;
  sred[0][t] = v0;
  sred[1][t] = v1;
  sred[2][t] = v2;
  __syncthreads();
  for (int s = EW / 2; s > 0; s >>= 1) {
    if (t < s) {
      sred[0][t] += sred[0][t + s];
      sred[1][t] += sred[1][t + s];
      sred[2][t] += sred[2][t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = sred[0][0];
    out[1] = sred[1][0];
    out[2] = sred[2][0];
  }
}

// r = b - Ap (interior), Ap = 0; Jacobi (jacobi != 0): z = D^-1 r, p = z;
// partials of r.z (0 without Jacobi: the preconditioner pass fills it), r.r, b.b
__global__ void __launch_bounds__(EW) pcg_start_kernel(const double* b, double* r, double* z, double* pv, double* Ap,
                                                       const double* dinv, int jacobi, int64_t n, double* partial) {
  double rz = 0, rr = 0, bb = 0;
  for (int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x; i < n; i += (int64_t)gridDim.x * EW) {
    const double di = dinv[i];
    const double ri = di != 0.0 ? b[i] - Ap[i] : 0.0;  // dinv is 0 exactly on the boundary
    r[i] = ri;
    Ap[i] = 0.0;
    if (jacobi) {
      const double zi = di * ri;
      z[i] = zi;
      pv[i] = zi;
      rz += ri * zi;
    }
    rr += ri * ri;
    bb += b[i] * b[i];
  }
  block_sum3(rz, rr, bb, partial + blockIdx.x * 3);
}

// x += alpha p, r -= alpha Ap (interior), Ap = 0; Jacobi: z = D^-1 r;
// partials of r.z (0 without Jacobi), r.r
__global__ void __launch_bounds__(EW) pcg_update_kernel(double* x, double* r, double* z, const double* pv, double* Ap,
                                                        const double* dinv, int jacobi, const double* S, int64_t n,
                                                        double* partial, const int* done) {
  if (*done) return;
  const double alpha = S[3];
  double rz = 0, rr = 0;
  for (int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x; i < n; i += (int64_t)gridDim.x * EW) {
    const double di = dinv[i];
    const double pi = pv[i];
    x[i] += alpha * pi;
    const double ri = di != 0.0 ? r[i] - alpha * Ap[i] : 0.0;
    r[i] = ri;
    Ap[i] = 0.0;
    if (jacobi) {
      const double zi = di * ri;
      z[i] = zi;
      rz += ri * zi;
    }
    rr += ri * ri;
  }
  block_sum3(rz, rr, 0.0, partial + blockIdx.x * 3);
}

// the r.z slot of the update partials, after the preconditioner pass wrote z
// (same grid and stride as pcg_update_kernel, so the fixed-order sums match)
__global__ void __launch_bounds__(EW) pcg_rz_kernel(const double* r, const double* z, int64_t n, double* partial,
                                                    const int* done) {
  if (done && *done) return;
  double rz = 0;
  for (int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x; i < n; i += (int64_t)gridDim.x * EW) rz += r[i] * z[i];
  __shared__ double sred[EW];
  sred[threadIdx.x] = rz;
  __syncthreads();
  for (int s = EW / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sred[threadIdx.x] += sred[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x * 3] = sred[0];
}

// p = z + beta p
__global__ void pcg_direction_kernel(const double* z, double* pv, const double* S, int64_t n, const int* done) {
  if (*done) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  pv[i] = z[i] + S[4] * pv[i];
}

// mode 0 (start): S[0]=rz, S[1]=rr, S[2]=bb, done if converged
// mode 1 (alpha): S[5]=pAp from the operator partials [nb][1]; S[3] = rz / pAp
// mode 2 (beta):  rz_new, rr -> S[4] = rz_new / rz, S[0] = rz_new, S[1] = rr; iteration count, stop test
__device__ void pcg_scalars(int mode, double v0, double v1, double v2, double* S, int* flags, double tol, int maxit) {
  if (mode == 0) {
    S[0] = v0;
    S[1] = v1;
    S[2] = v2;
    flags[1] = 0;
    flags[2] = 0;
    flags[0] = (S[2] == 0.0 || sqrt(S[1]) <= tol * sqrt(S[2])) ? 1 : 0;
  } else if (mode == 1) {
    const double pAp = v0;
    S[5] = pAp;
    if (!(pAp > 0.0)) {
      flags[2] = 2;
      flags[0] = 1;
      return;
    }
    S[3] = S[0] / pAp;
  } else {
    const double rz = v0, rr = v1;
    S[4] = rz / S[0];
    S[0] = rz;
    S[1] = rr;
    flags[1] += 1;
    if (sqrt(rr) <= tol * sqrt(S[2])) {
      flags[0] = 1;
    } else if (flags[1] >= maxit) {
      flags[2] = 1;
      flags[0] = 1;
    }
  }
}

__global__ void __launch_bounds__(EW) pcg_scalar_kernel(const double* partial, int64_t nb, int stride, int mode,
                                                        double* S, int* flags, double tol, int maxit,
                                                        int* host_flag) {
  if (mode != 0 && flags[0]) return;
  __shared__ double sred[3][EW];
  const int t = threadIdx.x;
  double v[3] = {0, 0, 0};
  for (int64_t b = t; b < nb; b += EW)
    for (int u = 0; u < stride; ++u) v[u] += partial[b * stride + u];
  for (int u = 0; u < 3; ++u) sred[u][t] = v[u];
  __syncthreads();
  for (int s = EW / 2; s > 0; s >>= 1) {
    if (t < s)
      for (int u = 0; u < 3; ++u) sred[u][t] += sred[u][t + s];
    __syncthreads();
  }
  if (t != 0) return;
  pcg_scalars(mode, sred[0][0], sred[1][0], sred[2][0], S, flags, tol, maxit);
  if (flags[0]) {
    *host_flag = 1;  // pinned memory the host polls; cleared by the host before the solve
    __threadfence_system();
  }
}

// phi <- x inside (boundary values stay)
__global__ void pcg_store_kernel(const double* x, double* phi, int Nx, int Ny, int Nz) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)Nx * Ny * Nz) return;
  if (interior_node(idx, Nx, Ny, Nz)) phi[idx] = x[idx];
}

template <int N>
tdfe_status launch_stiffness_diag_n(tdfe_ctx* c) {
  hipLaunchKernelGGL((stiffness_diag_kernel<N>), dim3((unsigned)c->n_cell), dim3(N * N * N), 0, c->stream, c->corners,
                     c->tab, c->dinvK, c->ncx, c->ncy, c->p, c->Nx, c->Ny);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

tdfe_status stiffness_diag(tdfe_ctx* c) {
  TDFE_HIP(c, hipMemsetAsync(c->dinvK, 0, c->n_nodes * sizeof(double), c->stream));
  tdfe_status s;
  switch (c->n) {
    case 2: s = launch_stiffness_diag_n<2>(c); break;
    case 3: s = launch_stiffness_diag_n<3>(c); break;
    case 4: s = launch_stiffness_diag_n<4>(c); break;
    case 5: s = launch_stiffness_diag_n<5>(c); break;
    case 6: s = launch_stiffness_diag_n<6>(c); break;
    case 7: s = launch_stiffness_diag_n<7>(c); break;
    case 8: s = launch_stiffness_diag_n<8>(c); break;
    case 9: s = launch_stiffness_diag_n<9>(c); break;
    default: return tdfe_fail(c, TDFE_EINVAL, "unsupported order");
  }
  if (s != TDFE_OK) return s;
  hipLaunchKernelGGL(invert_diag_kernel, dim3(nblk(c->n_nodes)), dim3(EW), 0, c->stream, c->dinvK, c->Nx, c->Ny,
                     c->Nz);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

// solves for the interior of c->phi from the load vector in c->cload (overwritten)
tdfe_status pcg_solve(tdfe_ctx* c) {
  const int64_t nn = c->n_nodes;
  double* r = c->pcg;
  double* z = r + nn;
  double* pv = z + nn;
  double* Ap = pv + nn;
  double* x = Ap + nn;
  double* S = c->pcgs;
  int* flags = (int*)c->counters + PCG_DONE;
  // past the density/dipole partials (n_cell x 4 + 4), which are read after the solve
  double* part = c->partial + ((c->n_cell * 4 + 8 + 63) / 64) * 64;
  auto apply_K = [&](const double* in, bool energy, int64_t* groups) -> tdfe_status {
    ApplyArgs a{};
    a.x = in;
    a.y = Ap;
    a.ld = 1;
    a.cols = 1;
    a.kin = 1.0;
    a.lowdin = false;
    a.fullgrid = true;
    a.energy = energy ? part : nullptr;
    a.n_blocks_out = groups;
    a.done_flag = energy ? flags : nullptr;
    return tdfe_launch_apply(c, a);
  };
  // preconditioner: Jacobi (z = D^-1 r inside the update kernels) or the fast
  // diagonalisation of the rectilinear stand-in mesh (a pass of its own)
  const int jacobi = c->pcg_precond == TDFE_PCG_JACOBI ? 1 : 0;
  auto precondition = [&](const int* done) -> tdfe_status {
    if (jacobi) return TDFE_OK;
    TDFE_TRY(fdm_precondition(c, r, z));
    hipLaunchKernelGGL(pcg_rz_kernel, dim3(PCG_BLOCKS), dim3(EW), 0, c->stream, (const double*)r, (const double*)z, nn,
                       part, done);
    TDFE_HIP(c, hipGetLastError());
    return TDFE_OK;
  };
  hipLaunchKernelGGL(pcg_rhs_kernel, dim3(nblk(nn)), dim3(EW), 0, c->stream, c->cload, (const double*)c->lift,
                     (const double*)c->phi, x, c->Nx, c->Ny, c->Nz);
  TDFE_TRY(tdfe_zero(c, Ap, nn * sizeof(double)));
  if (!jacobi) TDFE_TRY(tdfe_zero(c, z, nn * sizeof(double)));  // boundary entries stay zero
  TDFE_TRY(apply_K(x, false, nullptr));
  hipLaunchKernelGGL(pcg_start_kernel, dim3(PCG_BLOCKS), dim3(EW), 0, c->stream, (const double*)c->cload, r, z, pv, Ap,
                     (const double*)c->dinvK, jacobi, nn, part);
  TDFE_TRY(precondition(nullptr));
  if (!jacobi) TDFE_HIP(c, hipMemcpyAsync(pv, z, nn * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  volatile int* hflag = c->poll + 40;  // nothing on the stream writes it now
  *hflag = 0;
  int* dflag = nullptr;
  TDFE_HIP(c, hipHostGetDevicePointer((void**)&dflag, (void*)(c->poll + 40), 0));
  hipLaunchKernelGGL(pcg_scalar_kernel, dim3(1), dim3(EW), 0, c->stream, (const double*)part, (int64_t)PCG_BLOCKS, 3,
                     0, S, flags, c->pcg_tol, c->pcg_maxit, dflag);
  TDFE_HIP(c, hipGetLastError());
  const int LOOK = 4, RING = TDFE_N_EVENTS;
  TDFE_TRY(tdfe_poll_events(c));
  TDFE_HIP(c, hipStreamSynchronize(c->stream));
  if (!*hflag) {
    for (int it = 1; it <= c->pcg_maxit; ++it) {
      int64_t groups = 0;
      TDFE_TRY(apply_K(pv, true, &groups));
      hipLaunchKernelGGL(pcg_scalar_kernel, dim3(1), dim3(EW), 0, c->stream, (const double*)part, groups, 1, 1, S,
                         flags, c->pcg_tol, c->pcg_maxit, dflag);
      hipLaunchKernelGGL(pcg_update_kernel, dim3(PCG_BLOCKS), dim3(EW), 0, c->stream, x, r, z, (const double*)pv, Ap,
                         (const double*)c->dinvK, jacobi, (const double*)S, nn, part, (const int*)flags);
      TDFE_TRY(precondition(flags));
      hipLaunchKernelGGL(pcg_scalar_kernel, dim3(1), dim3(EW), 0, c->stream, (const double*)part, (int64_t)PCG_BLOCKS,
                         3, 2, S, flags, c->pcg_tol, c->pcg_maxit, dflag);
      hipLaunchKernelGGL(pcg_direction_kernel, dim3(nblk(nn)), dim3(EW), 0, c->stream, (const double*)z, pv,
                         (const double*)S, nn, (const int*)flags);
      TDFE_HIP(c, hipGetLastError());
      TDFE_HIP(c, hipEventRecord(c->evs[it % RING], c->stream));
      if (it > LOOK) {
        TDFE_HIP(c, hipEventSynchronize(c->evs[(it - LOOK) % RING]));
        if (*hflag) break;
      }
    }
  }
  hipLaunchKernelGGL(pcg_store_kernel, dim3(nblk(nn)), dim3(EW), 0, c->stream, (const double*)x, c->phi, c->Nx, c->Ny,
                     c->Nz);
  TDFE_HIP(c, hipGetLastError());
  const void* hfl = nullptr;
  TDFE_TRY(tdfe_readback(c, flags, 3 * sizeof(int), 2048, &hfl));
  TDFE_HIP(c, hipStreamSynchronize(c->stream));
  int fl[3];
  for (int i = 0; i < 3; ++i) fl[i] = ((const volatile int*)hfl)[i];
  c->last_poisson_iters = fl[1];
  if (fl[2] == 2) return tdfe_fail(c, TDFE_ENONFINITE, "Hartree CG: p^T K p <= 0");
  if (fl[2] == 1 || !fl[0])
    return tdfe_fail(c, TDFE_ENOCONV, "Hartree CG did not reach %g in %d iterations", c->pcg_tol, c->pcg_maxit);
  return TDFE_OK;
}

}  // namespace

// density at the Gauss points into rho (device) and 4 partial sums per cell
tdfe_status tdfe_density_dev(tdfe_ctx* c, const void* psibar, int n_orb, double* rho, double* partial4) {
  if (c->octree) {
    const double* occ = nullptr;
    TDFE_TRY(upload_occ(c, n_orb, (double**)&occ));
    return tdfe_octree_density(c, (const double*)psibar, n_orb, occ, rho, partial4);
  }
  DensParams P{};
  P.psi = (const double*)psibar;
  P.cols = 2 * n_orb;
  TDFE_TRY(upload_occ(c, n_orb, (double**)&P.occ));
  P.minv = c->minv;
  P.tab = c->tab;
  P.wdet = c->wdet;
  P.xq = c->xq;
  P.rho = rho;
  P.partial = partial4;
  P.ncx = c->ncx;
  P.ncy = c->ncy;
  P.ncz = c->ncz;
  P.p = c->p;
  P.Nx = c->Nx;
  P.Ny = c->Ny;
  P.Nz = c->Nz;
  P.n_cell = c->n_cell;
  return density_launch(c, P);
}

// W = V_H[rho] + V_xc[rho] at the Gauss points for the orbitals psibar;
// mu/charge (host, may be null) receive the dipole and charge of rho
tdfe_status tdfe_scf_potential(tdfe_ctx* c, const void* psibar, int n_orb, double* W, double* mu, double* charge) {
  const void* hr = nullptr;
  TDFE_TRY(tdfe_scf_potential_async(c, psibar, n_orb, W, (mu || charge) ? &hr : nullptr));
  if (hr) {
    TDFE_HIP(c, hipStreamSynchronize(c->stream));
    const volatile double* h = (const volatile double*)hr;
    if (charge) *charge = h[0];
    if (mu) {
      mu[0] = h[1];
      mu[1] = h[2];
      mu[2] = h[3];
    }
  }
  return TDFE_OK;
}

tdfe_status tdfe_scf_potential_async(tdfe_ctx* c, const void* psibar, int n_orb, double* W, const void** host_red) {
  TDFE_TRY(tdfe_density_dev(c, psibar, n_orb, c->rho, c->partial));
  double* red = c->partial + c->n_cell * 4;
  hipLaunchKernelGGL(finalize4_kernel, dim3(4), dim3(256), 0, c->stream, c->partial, c->n_cell, red);
  TDFE_HIP(c, hipGetLastError());
  if (c->hartree) {
    TDFE_TRY(tdfe_zero(c, c->cload, c->n_nodes * sizeof(double)));
    TDFE_TRY(load_launch(c));
    if (c->box) {
      TDFE_TRY(fdm_solve(c, true, c->phi));
    } else {
      TDFE_TRY(pcg_solve(c));
    }
  }
  TDFE_TRY(interp_launch(c, W));
  if (host_red) {
    TDFE_TRY(tdfe_readback(c, red, 4 * sizeof(double), 2304, host_red));
  }
  return TDFE_OK;
}

tdfe_status tdfe_fdm_setup(tdfe_ctx* c) {
  std::vector<double> Sx, Sy, Sz, lx, ly, lz;
  fdm_axis(c, c->ax_x, Sx, lx);
  fdm_axis(c, c->ax_y, Sy, ly);
  fdm_axis(c, c->ax_z, Sz, lz);
  std::vector<double> S, L;
  S.insert(S.end(), Sx.begin(), Sx.end());
  S.insert(S.end(), Sy.begin(), Sy.end());
  S.insert(S.end(), Sz.begin(), Sz.end());
  for (const std::vector<double>* M : {&Sx, &Sy, &Sz}) {
    const int m = (int)std::lround(std::sqrt((double)M->size()));
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) S.push_back((*M)[(size_t)b * m + a]);
  }
  L.insert(L.end(), lx.begin(), lx.end());
  L.insert(L.end(), ly.begin(), ly.end());
  L.insert(L.end(), lz.begin(), lz.end());
  TDFE_HIP(c, hipMemcpy(c->fdmS, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice));
  TDFE_HIP(c, hipMemcpy(c->fdmL, L.data(), L.size() * sizeof(double), hipMemcpyHostToDevice));
  return TDFE_OK;
}

// lift = (K f)_interior with f the boundary data (interior zero)
tdfe_status tdfe_compute_lift(tdfe_ctx* c) {
  TDFE_TRY(tdfe_zero(c, c->cload, c->n_nodes * sizeof(double)));
  ApplyArgs a{};
  a.x = c->fb;
  a.y = c->cload;
  a.ld = 1;
  a.cols = 1;
  a.kin = 1.0;
  a.lowdin = false;
  a.fullgrid = true;
  TDFE_TRY(tdfe_launch_apply(c, a));
  hipLaunchKernelGGL(gather_interior_kernel, dim3(nblk(c->n_dof)), dim3(EW), 0, c->stream, c->cload, (const double*)nullptr,
                     1.0, c->lift, c->Nx, c->Ny, c->Nz);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

tdfe_status tdfe_load_vector(tdfe_ctx* c, const double* f, bool weighted) {
  TDFE_TRY(tdfe_zero(c, c->cload, c->n_nodes * sizeof(double)));
  return load_launch_f(c, f, weighted ? 1 : 0);
}

void tdfe_blas_destroy(tdfe_ctx* c) {
  if (c->blas) rocblas_destroy_handle((rocblas_handle)c->blas);
  c->blas = nullptr;
}

tdfe_status tdfe_fdm_solve_into(tdfe_ctx* c, bool with_lift, double* phi_full) {
  if (!c->box) return tdfe_fail(c, TDFE_EINVAL, "Hartree adjoint: needs a box mesh (exact inverse)");
  return fdm_solve(c, with_lift, phi_full);
}

tdfe_status tdfe_interp_field(tdfe_ctx* c, const double* phi_full, const double* rho, int xcmode, double* out) {
  return interp_launch_f(c, phi_full, rho, xcmode, out);
}

void tdfe_sym_eigen(const std::vector<double>& A, int n, std::vector<double>& lam, std::vector<double>& U) {
  jacobi_eigen(A, n, lam, U);
}

tdfe_status tdfe_assemble_vw(tdfe_ctx* c, const double* A, double ca, const double* B, double cb, double E) {
  const int64_t nqd = c->n_quad;
  float* v32 = !tdfe_fp32(c) ? nullptr : c->vw32;
  hipLaunchKernelGGL(assemble_vw_kernel, dim3(nblk(nqd)), dim3(EW), 0, c->stream, c->vext, c->xq, c->wdet, A, ca, B, cb,
                     (const double*)nullptr, 0.0, E * c->fdir[0], E * c->fdir[1], E * c->fdir[2], c->vw, v32, nqd);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

tdfe_status tdfe_occ_dev(tdfe_ctx* c, int n_orb, const double** dev) {
  double* d = nullptr;
  TDFE_TRY(upload_occ(c, n_orb, &d));
  *dev = d;
  return TDFE_OK;
}

extern "C" {

tdfe_status tdfe_set_midpoint(tdfe_ctx* c, const tdfe_midpoint_desc* m) {
  if (!c || !m) return TDFE_EINVAL;
  if (m->mode != TDFE_MIDPOINT_PC && m->mode != TDFE_MIDPOINT_SC)
    return tdfe_fail(c, TDFE_EINVAL, "set_midpoint: unknown mode");
  if (m->order != 1 && m->order != 2) return tdfe_fail(c, TDFE_EINVAL, "set_midpoint: order must be 1 or 2");
  if (m->mode == TDFE_MIDPOINT_SC && (!(m->sc_tol > 0.0) || !std::isfinite(m->sc_tol) || m->sc_maxit < 1))
    return tdfe_fail(c, TDFE_EINVAL, "set_midpoint: sc_tol > 0 and sc_maxit >= 1 required");
  c->mid_mode = m->mode;
  c->mid_order = m->order;
  if (m->mode == TDFE_MIDPOINT_SC) {
    c->sc_tol = m->sc_tol;
    c->sc_maxit = m->sc_maxit;
  }
  return TDFE_OK;
}

// rectilinear stand-in of a curved grid for the Hartree preconditioner: the
// mean vertex coordinate of every logical plane along each axis; if a mean
// sequence is not increasing (a folded map), a uniform one between its ends
static void stand_in_axes(tdfe_ctx* c) {
  const int nc[3] = {c->ncx, c->ncy, c->ncz};
  std::vector<double>* out[3] = {&c->ax_x, &c->ax_y, &c->ax_z};
  for (int d = 0; d < 3; ++d) {
    std::vector<double>& ax = *out[d];
    ax.assign(nc[d] + 1, 0.0);
    std::vector<double> cnt(nc[d] + 1, 0.0);
    for (int k = 0; k <= c->ncz; ++k)
      for (int j = 0; j <= c->ncy; ++j)
        for (int i = 0; i <= c->ncx; ++i) {
          const int m = d == 0 ? i : (d == 1 ? j : k);
          ax[m] += c->vertices[(((size_t)k * (c->ncy + 1) + j) * (c->ncx + 1) + i) * 3 + d];
          cnt[m] += 1.0;
        }
    for (int m = 0; m <= nc[d]; ++m) ax[m] /= cnt[m];
    bool inc = true;
    for (int m = 1; m <= nc[d]; ++m) inc = inc && ax[m] > ax[m - 1];
    if (!inc) {
      const double a = ax[0], b = ax[nc[d]] > a ? ax[nc[d]] : a + nc[d];
      for (int m = 0; m <= nc[d]; ++m) ax[m] = a + (b - a) * m / nc[d];
    }
  }
}

tdfe_status tdfe_set_scf(tdfe_ctx* c, const tdfe_scf_desc* s) {
  if (!c || !s) return TDFE_EINVAL;
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "set_scf before bind_workspace");
  if (s->xc < TDFE_XC_NONE || s->xc > TDFE_XC_XC) return tdfe_fail(c, TDFE_EINVAL, "set_scf: bad xc mode");
  if (s->n_nuclei < 0 || (s->n_nuclei > 0 && (!s->Z || !s->R))) return tdfe_fail(c, TDFE_EINVAL, "set_scf: nuclei");
  if (s->n_orb < 0 || s->n_orb > c->n_orb_max) return tdfe_fail(c, TDFE_EINVAL, "set_scf: n_orb");
  if (c->octree && (s->hartree || s->xc != TDFE_XC_NONE))
    return tdfe_fail(c, TDFE_EINVAL, "set_scf: octree meshes take no Hartree or exchange-correlation term");
  if (s->hartree && !c->box && !(s->pcg_tol > 0.0)) return tdfe_fail(c, TDFE_EINVAL, "set_scf: pcg_tol");
  if (s->pcg_precond != TDFE_PCG_FDM && s->pcg_precond != TDFE_PCG_JACOBI)
    return tdfe_fail(c, TDFE_EINVAL, "set_scf: pcg_precond");
  c->hartree = s->hartree ? 1 : 0;
  c->xc = s->xc;
  c->nucZ.assign(s->Z, s->Z + s->n_nuclei);
  c->nucR.assign(s->R, s->R + 3 * s->n_nuclei);
  c->occ.assign(s->n_orb, 1.0);
  ++c->occ_ver;
  if (s->occupation)
    for (int o = 0; o < s->n_orb; ++o) c->occ[o] = s->occupation[o];
  c->pcg_tol = s->pcg_tol;
  c->pcg_maxit = s->pcg_maxit;
  c->pcg_precond = s->pcg_precond;
  if (c->hartree) {
    std::vector<double> zr(4 * std::max(1, s->n_nuclei));
    for (int a = 0; a < s->n_nuclei; ++a) {
      zr[a * 4 + 0] = s->Z[a];
      zr[a * 4 + 1] = s->R[a * 3 + 0];
      zr[a * 4 + 2] = s->R[a * 3 + 1];
      zr[a * 4 + 3] = s->R[a * 3 + 2];
    }
    double* dzr = c->partial;  // staging
    TDFE_HIP(c, hipMemcpyAsync(dzr, zr.data(), zr.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(boundary_values_kernel, dim3(nblk(c->n_nodes)), dim3(EW), 0, c->stream, c->nodexyz_ptr,
                       (const double*)dzr, s->n_nuclei, c->fb, c->phi, c->Nx, c->Ny, c->Nz);
    TDFE_HIP(c, hipGetLastError());
    TDFE_TRY(tdfe_compute_lift(c));
    TDFE_HIP(c, hipStreamSynchronize(c->stream));
    const bool fdm = c->box || c->pcg_precond == TDFE_PCG_FDM;
    if (c->box) {
      TDFE_TRY(tdfe_fdm_setup(c));
    } else {
      TDFE_TRY(stiffness_diag(c));
      if (fdm) {
        stand_in_axes(c);
        TDFE_TRY(tdfe_fdm_setup(c));
      }
    }
    // axes of more than 128 interior nodes transform through rocBLAS: its
    // handle (and the device memory it takes) is made here, not in the step
    if (fdm && std::max(c->Nx, std::max(c->Ny, c->Nz)) - 2 > 128) TDFE_TRY(blas_ready(c));
  }
  c->have_scf = c->hartree || c->xc != TDFE_XC_NONE;
  c->scf_init = false;
  return TDFE_OK;
}

tdfe_status tdfe_scf_fields(tdfe_ctx* c, const void* dev_psibar, int n_orb, double* dev_phi, double* dev_w) {
  if (!c || !dev_psibar || (!dev_phi && !dev_w)) return TDFE_EINVAL;
  if (n_orb < 1 || n_orb > c->n_orb_max) return tdfe_fail(c, TDFE_EINVAL, "scf_fields: n_orb out of range");
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "scf_fields before bind_workspace");
  if (!c->have_scf) return tdfe_fail(c, TDFE_ESTATE, "scf_fields before set_scf");
  if (dev_phi && !c->hartree) return tdfe_fail(c, TDFE_EINVAL, "scf_fields: phi requested without Hartree");
  // W goes to the caller's array, or to the midpoint slot that every Magnus
  // step recomputes before reading it; the W history is not touched
  TDFE_TRY(tdfe_scf_potential(c, dev_psibar, n_orb, dev_w ? dev_w : c->wh, nullptr, nullptr));
  if (dev_phi)
    TDFE_HIP(c, hipMemcpyAsync(dev_phi, c->phi, (size_t)c->n_nodes * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
  TDFE_HIP(c, hipStreamSynchronize(c->stream));
  return TDFE_OK;
}

tdfe_status tdfe_density(tdfe_ctx* c, const void* dev_psibar, int n_orb, double* dev_rho_q) {
  if (!c || !dev_psibar || !dev_rho_q) return TDFE_EINVAL;
  if (n_orb < 1 || n_orb > c->n_orb_max) return tdfe_fail(c, TDFE_EINVAL, "density: n_orb out of range");
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "density before bind_workspace");
  return tdfe_density_dev(c, dev_psibar, n_orb, dev_rho_q, c->partial);
}

tdfe_status tdfe_dipole(tdfe_ctx* c, const void* dev_psibar, int n_orb, double* host_mu, double* host_charge) {
  if (!c || !dev_psibar || !host_mu) return TDFE_EINVAL;
  if (n_orb < 1 || n_orb > c->n_orb_max) return tdfe_fail(c, TDFE_EINVAL, "dipole: n_orb out of range");
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "dipole before bind_workspace");
  TDFE_TRY(tdfe_density_dev(c, dev_psibar, n_orb, c->rho, c->partial));
  double* red = c->partial + c->n_cell * 4;
  hipLaunchKernelGGL(finalize4_kernel, dim3(4), dim3(256), 0, c->stream, c->partial, c->n_cell, red);
  TDFE_HIP(c, hipGetLastError());
  const void* hr = nullptr;
  TDFE_TRY(tdfe_readback(c, red, 4 * sizeof(double), 2304, &hr));
  TDFE_HIP(c, hipStreamSynchronize(c->stream));
  double h[4];
  for (int i = 0; i < 4; ++i) h[i] = ((const volatile double*)hr)[i];
  host_mu[0] = h[1];
  host_mu[1] = h[2];
  host_mu[2] = h[3];
  if (host_charge) *host_charge = h[0];
  if (!std::isfinite(h[0])) return tdfe_fail(c, TDFE_ENONFINITE, "dipole: non-finite density");
  return TDFE_OK;
}

// batched steps (tdfe_propagate): the step ends without a synchronisation;
// its Lanczos results are folded into acc on the device and its {charge,
// mu} (when red_dst is set) copied to red_dst
struct StepBatch {
  double* acc;      // [8]: max k, sum k, max error estimate, not-converged flag, table-overflow flag,
                    // non-finite flag
  double* red_dst;  // [4] or null
};

static tdfe_status magnus_step_impl(tdfe_ctx* c, void* dev_psibar, int n_orb, double dt, double field_E, double tol,
                                    tdfe_step_report* rep, const StepBatch* batch) {
  if (!c || !dev_psibar) return TDFE_EINVAL;
  if (n_orb < 1 || n_orb > c->n_orb_max) return tdfe_fail(c, TDFE_EINVAL, "magnus_step: n_orb out of range");
  if (!(dt > 0.0) || !std::isfinite(dt) || !(tol > 0.0) || !std::isfinite(field_E))
    return tdfe_fail(c, TDFE_EINVAL, "magnus_step: dt, tol or field");
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "magnus_step before bind_workspace");
  if (!c->have_potential) return tdfe_fail(c, TDFE_ESTATE, "magnus_step before set_potential");
  const int64_t nqd = c->n_quad;
  float* v32 = !tdfe_fp32(c) ? nullptr : c->vw32;
  tdfe_step_report r{};
  // the Lanczos results of the step (Krylov dimensions, error estimates,
  // convergence) and the dipole stay on the device until one readback and one
  // stream synchronisation at the end of the step
  const bool defer = tdfe_lanczos_can_defer(c);
  const void *hpred = nullptr, *hcorr = nullptr, *hred = nullptr;
  tdfe_status st = TDFE_OK, s2 = TDFE_OK;
  double eh = 0.0;
  auto lanczos = [&](const void* in, void* out, double tau, int slot, int* kmax, int* ksum, double* emax) {
    if (defer) return tdfe_lanczos_run(c, c->vw, in, out, n_orb, tau, tol, nullptr, nullptr, nullptr, nullptr,
                                       nullptr, nullptr, slot);
    return tdfe_lanczos_run(c, c->vw, in, out, n_orb, tau, tol, nullptr, nullptr, kmax, ksum, emax);
  };
  if (!c->have_scf) {
    hipLaunchKernelGGL(assemble_vw_kernel, dim3(nblk(nqd)), dim3(EW), 0, c->stream, c->vext, c->xq, c->wdet,
                       (const double*)nullptr, 0.0, (const double*)nullptr, 0.0, (const double*)nullptr, 0.0,
                       field_E * c->fdir[0],
                       field_E * c->fdir[1], field_E * c->fdir[2], c->vw, v32, nqd);
    TDFE_HIP(c, hipGetLastError());
    s2 = lanczos(dev_psibar, dev_psibar, dt, 1, &r.k_corr_max, &r.k_corr_sum, &r.err_max);
    if (s2 != TDFE_OK && s2 != TDFE_ENOCONV) return s2;
    if (rep || (batch && batch->red_dst)) {
      TDFE_TRY(tdfe_density_dev(c, dev_psibar, n_orb, c->rho, c->partial));
      double* red = c->partial + c->n_cell * 4;
      hipLaunchKernelGGL(finalize4_kernel, dim3(4), dim3(256), 0, c->stream, c->partial, c->n_cell, red);
      TDFE_HIP(c, hipGetLastError());
      if (batch && batch->red_dst) {
        hipLaunchKernelGGL(copy4_kernel, dim3(1), dim3(64), 0, c->stream, (const double*)red, batch->red_dst);
        TDFE_HIP(c, hipGetLastError());
      }
      if (rep) TDFE_TRY(tdfe_readback(c, red, 4 * sizeof(double), 2304, &hred));
    }
  } else {
    if (!c->scf_init) {
      TDFE_TRY(tdfe_scf_potential(c, dev_psibar, n_orb, c->w1, nullptr, nullptr));
      TDFE_HIP(c, hipMemcpyAsync(c->w2, c->w1, nqd * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      TDFE_HIP(c, hipMemcpyAsync(c->w3, c->w1, nqd * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      c->scf_init = true;
    }
    const double Ex = field_E * c->fdir[0], Ey = field_E * c->fdir[1], Ez = field_E * c->fdir[2];
    double l[3];
    extrapolation_weights(c->mid_mode == TDFE_MIDPOINT_SC ? 0.5 : 0.25, c->mid_order, l);
    const double* w3 = c->mid_order >= 2 ? c->w3 : nullptr;
    if (c->mid_mode == TDFE_MIDPOINT_PC) {
      // predictor: W(t + dt/4) extrapolated from W_{n-1}, W_{n-2} (, W_{n-3})
      hipLaunchKernelGGL(assemble_vw_kernel, dim3(nblk(nqd)), dim3(EW), 0, c->stream, c->vext, c->xq, c->wdet,
                         (const double*)c->w1, l[0], (const double*)c->w2, l[1], w3, l[2], Ex, Ey, Ez, c->vw, v32,
                         nqd);
      TDFE_HIP(c, hipGetLastError());
      st = lanczos(dev_psibar, c->half, 0.5 * dt, 0, &r.k_pred_max, &r.k_pred_sum, &eh);
      if (st != TDFE_OK && st != TDFE_ENOCONV) return st;
      TDFE_TRY(tdfe_scf_potential_async(c, c->half, n_orb, c->wh, nullptr));
      // corrector with the midpoint potential
      hipLaunchKernelGGL(assemble_vw_kernel, dim3(nblk(nqd)), dim3(EW), 0, c->stream, c->vext, c->xq, c->wdet,
                         (const double*)c->wh, 1.0, (const double*)nullptr, 0.0, (const double*)nullptr, 0.0, Ex, Ey,
                         Ez, c->vw, v32, nqd);
      TDFE_HIP(c, hipGetLastError());
      s2 = lanczos(dev_psibar, dev_psibar, dt, 1, &r.k_corr_max, &r.k_corr_sum, &r.err_max);
      if (s2 != TDFE_OK && s2 != TDFE_ENOCONV) return s2;
      // history: W_{n-3} <- W_{n-2} <- W_{n-1} <- W[rho(psibar^n)]
      double* t = c->w3;
      c->w3 = c->w2;
      c->w2 = c->w1;
      c->w1 = t;
      TDFE_TRY(tdfe_scf_potential_async(c, dev_psibar, n_orb, c->w1, rep ? &hred : nullptr));
      if (batch && batch->red_dst) {
        hipLaunchKernelGGL(copy4_kernel, dim3(1), dim3(64), 0, c->stream, (const double*)(c->partial + c->n_cell * 4),
                           batch->red_dst);
        TDFE_HIP(c, hipGetLastError());
      }
    } else {
      // (i) W_mid extrapolated to t + dt/2; psibar^{n-1} kept in the half-step buffer
      hipLaunchKernelGGL(combine3_kernel, dim3(nblk(nqd)), dim3(EW), 0, c->stream, (const double*)c->w1, l[0],
                         (const double*)c->w2, l[1], w3, l[2], c->wh, nqd);
      TDFE_HIP(c, hipGetLastError());
      TDFE_HIP(c, hipMemcpyAsync(c->half, dev_psibar, (size_t)c->n_dof * n_orb * 2 * sizeof(double),
                                 hipMemcpyDeviceToDevice, c->stream));
      double change = 0.0;
      int it = 0;
      bool conv = false;
      while (it < c->sc_maxit) {
        // (ii) propagate psibar^{n-1} with W_mid, then W_n = W[rho(psibar^n)]
        hipLaunchKernelGGL(assemble_vw_kernel, dim3(nblk(nqd)), dim3(EW), 0, c->stream, c->vext, c->xq, c->wdet,
                           (const double*)c->wh, 1.0, (const double*)nullptr, 0.0, (const double*)nullptr, 0.0, Ex,
                           Ey, Ez, c->vw, v32, nqd);
        TDFE_HIP(c, hipGetLastError());
        int km = 0, ks = 0;
        double em = 0.0;
        s2 = tdfe_lanczos_run(c, c->vw, c->half, dev_psibar, n_orb, dt, tol, nullptr, nullptr, &km, &ks, &em);
        if (s2 != TDFE_OK && s2 != TDFE_ENOCONV) return s2;
        if (s2 == TDFE_ENOCONV) st = s2;
        r.k_corr_max = std::max(r.k_corr_max, km);
        r.k_corr_sum += ks;
        r.err_max = std::max(r.err_max, em);
        TDFE_TRY(tdfe_scf_potential_async(c, dev_psibar, n_orb, c->wn, rep ? &hred : nullptr));
        // (iii) W_mid <- (W_{n-1} + W_n)/2 and its largest change
        hipLaunchKernelGGL(midpoint_update_kernel, dim3(SC_BLOCKS), dim3(EW), 0, c->stream, (const double*)c->w1,
                           (const double*)c->wn, c->wh, nqd, c->scbuf);
        hipLaunchKernelGGL(max_final_kernel, dim3(1), dim3(64), 0, c->stream, (const double*)c->scbuf, SC_BLOCKS,
                           c->scbuf + SC_BLOCKS);
        TDFE_HIP(c, hipGetLastError());
        const void* hc = nullptr;
        TDFE_TRY(tdfe_readback(c, c->scbuf + SC_BLOCKS, sizeof(double), 3328, &hc));
        TDFE_HIP(c, hipStreamSynchronize(c->stream));
        change = *(const volatile double*)hc;
        ++it;
        // (iv) until the midpoint potential settles
        if (change <= c->sc_tol) {
          conv = true;
          break;
        }
      }
      double* t = c->w3;
      c->w3 = c->w2;
      c->w2 = c->w1;
      c->w1 = c->wn;
      c->wn = t;
      r.sc_iters = it;
      r.sc_change = change;
      if (!conv && st == TDFE_OK) {
        st = TDFE_ENOCONV;
        tdfe_fail(c, TDFE_ENOCONV, "magnus_step: self-consistent midpoint not converged in %d iterations (change %g)",
                  it, change);
      }
    }
  }
  const bool deferred = defer && !(c->have_scf && c->mid_mode == TDFE_MIDPOINT_SC);
  if (batch) {
    // tdfe_propagate batches only deferred predictor-corrector steps
    if (!deferred) return tdfe_fail(c, TDFE_EINVAL, "magnus batch: step mode cannot defer its results");
    if (c->have_scf)
      hipLaunchKernelGGL(accum_results_kernel, dim3(1), dim3(64), 0, c->stream,
                         (const double*)tdfe_lanczos_result_slot(c, 0), n_orb, c->n_orb_max, batch->acc);
    hipLaunchKernelGGL(accum_results_kernel, dim3(1), dim3(64), 0, c->stream,
                       (const double*)tdfe_lanczos_result_slot(c, 1), n_orb, c->n_orb_max, batch->acc);
    TDFE_HIP(c, hipGetLastError());
    return TDFE_OK;
  }
  if (deferred) {
    if (c->have_scf) TDFE_TRY(tdfe_lanczos_enqueue_results(c, 0, &hpred));
    TDFE_TRY(tdfe_lanczos_enqueue_results(c, 1, &hcorr));
  }
  TDFE_HIP(c, hipStreamSynchronize(c->stream));
  if (deferred) {
    if (hpred) {
      st = tdfe_lanczos_results(c, hpred, n_orb, tol, &r.k_pred_max, &r.k_pred_sum, &eh);
      if (st != TDFE_OK && st != TDFE_ENOCONV) return st;
    }
    s2 = tdfe_lanczos_results(c, hcorr, n_orb, tol, &r.k_corr_max, &r.k_corr_sum, &r.err_max);
    if (s2 != TDFE_OK && s2 != TDFE_ENOCONV) return s2;
  }
  if (s2 == TDFE_ENOCONV) st = s2;
  r.err_max = std::max(r.err_max, eh);
  if (hred) {
    const volatile double* h = (const volatile double*)hred;
    r.charge = h[0];
    r.mu[0] = h[1];
    r.mu[1] = h[2];
    r.mu[2] = h[3];
  }
  r.poisson_iters = c->last_poisson_iters;
  if (rep) {
    *rep = r;
    if (!std::isfinite(r.charge)) return tdfe_fail(c, TDFE_ENONFINITE, "magnus_step: non-finite density");
  }
  return st;
}

tdfe_status tdfe_magnus_step(tdfe_ctx* c, void* dev_psibar, int n_orb, double dt, double field_E, double tol,
                             tdfe_step_report* rep) {
  return magnus_step_impl(c, dev_psibar, n_orb, dt, field_E, tol, rep, nullptr);
}

tdfe_status tdfe_propagate(tdfe_ctx* c, void* dev_psibar, int n_orb, int n_steps, double dt, const double* host_E,
                           double tol, double* dev_mu, tdfe_step_report* rep) {
  if (!c || !dev_psibar) return TDFE_EINVAL;
  if (n_steps < 1) return tdfe_fail(c, TDFE_EINVAL, "propagate: n_steps < 1");
  if (host_E)
    for (int n = 0; n < n_steps; ++n)
      if (!std::isfinite(host_E[n])) return tdfe_fail(c, TDFE_EINVAL, "propagate: non-finite field amplitude");
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "propagate before bind_workspace");
  const bool batched = tdfe_lanczos_can_defer(c) && !(c->have_scf && c->mid_mode == TDFE_MIDPOINT_SC);
  if (!batched) {
    // modes that synchronise inside a step: one step at a time, totals on the host
    tdfe_step_report tot{}, r{};
    tdfe_status worst = TDFE_OK;
    for (int n = 0; n < n_steps; ++n) {
      const tdfe_status s = magnus_step_impl(c, dev_psibar, n_orb, dt, host_E ? host_E[n] : 0.0, tol, &r, nullptr);
      if (s != TDFE_OK && s != TDFE_ENOCONV) return s;
      if (s == TDFE_ENOCONV) worst = s;
      tot.k_pred_max = std::max(tot.k_pred_max, r.k_pred_max);
      tot.k_corr_max = std::max(tot.k_corr_max, r.k_corr_max);
      tot.k_pred_sum += r.k_pred_sum;
      tot.k_corr_sum += r.k_corr_sum;
      tot.err_max = std::max(tot.err_max, r.err_max);
      tot.sc_iters += r.sc_iters;
      tot.sc_change = std::max(tot.sc_change, r.sc_change);
      if (dev_mu) {
        const double v[4] = {r.charge, r.mu[0], r.mu[1], r.mu[2]};
        TDFE_HIP(c, hipMemcpyAsync(dev_mu + 4 * (size_t)n, v, sizeof(v), hipMemcpyHostToDevice, c->stream));
        TDFE_HIP(c, hipStreamSynchronize(c->stream));
      }
    }
    tot.poisson_iters = r.poisson_iters;
    tot.charge = r.charge;
    for (int k = 0; k < 3; ++k) tot.mu[k] = r.mu[k];
    if (rep) *rep = tot;
    return worst;
  }
  double* acc = c->scbuf + 320;
  TDFE_TRY(tdfe_zero(c, acc, 8 * sizeof(double)));
  for (int n = 0; n < n_steps; ++n) {
    StepBatch b{acc, dev_mu ? dev_mu + 4 * (size_t)n : (n == n_steps - 1 && rep ? acc + 8 : nullptr)};
    TDFE_TRY(magnus_step_impl(c, dev_psibar, n_orb, dt, host_E ? host_E[n] : 0.0, tol, nullptr, &b));
  }
  const void *ha = nullptr, *hm = nullptr;
  TDFE_TRY(tdfe_readback(c, acc, 8 * sizeof(double), 3584, &ha));
  if (rep) TDFE_TRY(tdfe_readback(c, dev_mu ? dev_mu + 4 * (size_t)(n_steps - 1) : acc + 8, 4 * sizeof(double), 3712, &hm));
  TDFE_HIP(c, hipStreamSynchronize(c->stream));
  const volatile double* a = (const volatile double*)ha;
  bool charge_finite = true;
  if (rep) {
    tdfe_step_report r{};
    // the predictor and corrector runs are folded together
    r.k_corr_max = (int)a[0];
    r.k_corr_sum = (int)a[1];
    r.err_max = a[2];
    r.poisson_iters = c->last_poisson_iters;
    const volatile double* m = (const volatile double*)hm;
    r.charge = m[0];
    r.mu[0] = m[1];
    r.mu[1] = m[2];
    r.mu[2] = m[3];
    *rep = r;
    charge_finite = std::isfinite(r.charge);
  }
  if (a[5] != 0.0) return tdfe_fail(c, TDFE_ENONFINITE, "propagate: non-finite norm or Lanczos coefficient");
  if (!charge_finite) return tdfe_fail(c, TDFE_ENONFINITE, "propagate: non-finite density");
  if (a[4] != 0.0) return tdfe_fail(c, TDFE_EINVAL, "small exponential: |tau| ||T|| too large for the Chebyshev table");
  if (a[3] != 0.0) return tdfe_fail(c, TDFE_ENOCONV, "propagate: a Lanczos run reached k_max=%d without eps <= %g",
                                    c->k_max, tol);
  return TDFE_OK;
}

}  // extern "C"
