// Nonlocal pseudopotential term in the Kleinman-Bylander form (Eq. VPSP).
//
// The term acts on phi as sum_p (int chi_p phi / D_p) chi_p with chi_p =
// u_p dV_p and D_p = int u_p dV_p u_p.  On the FE basis its Galerkin matrix is
// C^T diag(E) C with c_pj = int chi_p N_j (Gauss rule) and E_p = 1 / D_p; in
// the Loewdin form (Eq. TDKSMatVecStandard) the library stores
// Cbar = C M^-1/2 ([n_proj][n_dof], projector-major) and adds
//   Hbar x += Cbar^T diag(E) Cbar x
// after the local operator kernel of every Hamiltonian launch:
//   project   per-block partials of t = Cbar (cs x)     (cs: the launch's column scale)
//   finalize  t (fixed-order sum), E t, and the term's share of the quadratic form
//   add       y += Cbar^T (E t)
// These are tall-skinny contractions over the DoFs: one streaming pass over
// Cbar and x each, HBM-bound.
#include "tdfe_internal.h"

namespace {

constexpr int NL_BLOCKS = 256;    // blocks of the projection pass
constexpr int NL_THREADS = 256;
constexpr int NL_PCH = 16;        // projectors per register chunk

struct NlLayout {
  double* cbar;     // [n_proj][n_dof]
  float* cbar32;    // [n_proj][n_dof] (mixed contexts)
  double* E;        // [n_proj]
  double* part;     // [NL_BLOCKS][n_proj][TDFE_MAX_COLS]
  double* tE;       // [n_proj][TDFE_MAX_COLS]
  double* eP;       // [n_proj][TDFE_MAX_COLS]
  double* scratch;  // [n_quad] (set-up)
  double* red;      // [NL_BLOCKS + 8] (set-up)
  size_t bytes;
};

NlLayout nl_layout(const tdfe_ctx* c, int n_proj, char* base) {
  NlLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const size_t np = (size_t)n_proj;
  L.cbar = (double*)take(np * c->n_dof * sizeof(double));
  L.cbar32 = (float*)take(c->precision == TDFE_FP64 ? sizeof(float) : np * c->n_dof * sizeof(float));
  L.E = (double*)take(np * sizeof(double));
  L.part = (double*)take((size_t)NL_BLOCKS * np * TDFE_MAX_COLS * sizeof(double));
  L.tE = (double*)take(np * TDFE_MAX_COLS * sizeof(double));
  L.eP = (double*)take(np * TDFE_MAX_COLS * sizeof(double));
  L.scratch = (double*)take((size_t)c->n_quad * sizeof(double));
  L.red = (double*)take((NL_BLOCKS + 8) * sizeof(double));
  L.bytes = off + 256;
  return L;
}

// ---------------------------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------------------------
__global__ void nl_chi_kernel(const double* u, const double* dv, double* chi, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) chi[i] = u[i] * dv[i];
}

// partial sums of wdet chi u over the Gauss points (fixed order per block)
__global__ void nl_norm_partial_kernel(const double* wdet, const double* chi, const double* u, int64_t n,
                                       double* part) {
  __shared__ double s[NL_THREADS];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NL_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * NL_THREADS)
    acc += wdet[i] * chi[i] * u[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = NL_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// E_p = 1 / D_p from the block partials; a zero D_p is reported through *bad
__global__ void nl_norm_final_kernel(const double* part, int nb, double* E, int* bad) {
  if (threadIdx.x != 0) return;
  double D = 0.0;
  for (int b = 0; b < nb; ++b) D += part[b];
  if (!(D != 0.0) || !isfinite(D)) {
    *bad = 1;
    *E = 0.0;
  } else {
    *E = 1.0 / D;
  }
}

// Cbar_p(dof) = c_p(node(dof)) M^-1/2(dof), with an FP32 copy when requested
__global__ void nl_extract_kernel(const double* cload, const double* minv, double* cbar, float* cbar32, int Nx,
                                  int Ny, int64_t n_dof) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n_dof) return;
  const int64_t nxi = Nx - 2, nyi = Ny - 2;
  const int64_t I = d % nxi + 1, J = (d / nxi) % nyi + 1, K = d / (nxi * nyi) + 1;
  const double v = cload[I + (int64_t)Nx * (J + (int64_t)Ny * K)] * minv[d];
  cbar[d] = v;
  if (cbar32) cbar32[d] = (float)v;
}

// ---------------------------------------------------------------------------------------------
// apply
// ---------------------------------------------------------------------------------------------
// per-block partials of t[p][col] = sum_r Cbar[p][r] cs[col] x[r][col] for a
// chunk of NL_PCH projectors; thread t serves column t % CP of rows
// t / CP, t / CP + NL_THREADS / CP, ... of the block's row range
template <typename T, typename CT, int CP>
__global__ void __launch_bounds__(NL_THREADS)
    nl_project_kernel(const T* __restrict__ x, int ld, int cols, const double* __restrict__ colscale,
                      const CT* __restrict__ cbar, int64_t n_dof, int p0, int np, double* __restrict__ part,
                      int n_proj, const int* done) {
  constexpr int RG = NL_THREADS / CP;  // row groups per block
  __shared__ double s[NL_PCH][NL_THREADS];
  if (done && *done) return;
  const int t = threadIdx.x;
  const int col = t % CP, rg = t / CP;
  const bool cok = col < cols;
  const int64_t rows_per_block = (n_dof + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < n_dof ? r0 + rows_per_block : n_dof;
  double acc[NL_PCH];
#pragma unroll
  for (int q = 0; q < NL_PCH; ++q) acc[q] = 0.0;
  for (int64_t r = r0 + rg; r < r1; r += RG) {
    const double xv = cok ? (double)x[r * ld + col] : 0.0;
#pragma unroll
    for (int q = 0; q < NL_PCH; ++q)
      if (q < np) acc[q] += (double)cbar[(int64_t)(p0 + q) * n_dof + r] * xv;
  }
#pragma unroll
  for (int q = 0; q < NL_PCH; ++q) s[q][t] = acc[q];
  __syncthreads();
  // sum over the row groups (fixed order), one column per thread
  if (t < CP && cok) {
    const double cs = colscale ? colscale[t >> 1] : 1.0;
    for (int q = 0; q < np; ++q) {
      double v = 0.0;
      for (int g = 0; g < RG; ++g) v += s[q][g * CP + t];
      part[((int64_t)blockIdx.x * n_proj + p0 + q) * TDFE_MAX_COLS + t] = v * cs;
    }
  }
}

// t[p][col] = sum_b part[b][p][col]; tE = E t; eP = E t^2 (one block per projector)
__global__ void nl_finalize_kernel(const double* part, int nb, int n_proj, int cols, const double* E, double* tE,
                                   double* eP, const int* done) {
  if (done && *done) return;
  const int p = blockIdx.x, col = threadIdx.x;
  if (col >= cols) return;
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += part[((int64_t)b * n_proj + p) * TDFE_MAX_COLS + col];
  tE[p * TDFE_MAX_COLS + col] = E[p] * t;
  eP[p * TDFE_MAX_COLS + col] = E[p] * t * t;
}

// the term's share of the per-column quadratic form, as one more row of the
// operator kernel's block partials
__global__ void nl_energy_kernel(const double* eP, int n_proj, int cols, double* energy_row, const int* done) {
  if (done && *done) return;
  const int col = threadIdx.x;
  if (col >= cols) return;
  double e = 0.0;
  for (int p = 0; p < n_proj; ++p) e += eP[p * TDFE_MAX_COLS + col];
  energy_row[col] = e;
}

// y[r][col] += sum_p Cbar[p][r] tE[p][col]
template <typename T, typename CT>
__global__ void __launch_bounds__(NL_THREADS)
    nl_add_kernel(T* __restrict__ y, int ld, int cols, const CT* __restrict__ cbar, int64_t n_dof,
                  const double* __restrict__ tE, int n_proj, const int* done) {
  if (done && *done) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = idx / cols;
  const int col = (int)(idx % cols);
  if (r >= n_dof) return;
  double acc = 0.0;
  for (int p = 0; p < n_proj; ++p) acc += (double)cbar[(int64_t)p * n_dof + r] * tE[p * TDFE_MAX_COLS + col];
  y[r * ld + col] += (T)acc;
}

template <typename T, typename CT, int CP>
tdfe_status nl_project_launch(tdfe_ctx* c, const T* x, int ld, int cols, const double* colscale, const int* done,
                              const CT* cbar, const NlLayout& L) {
  for (int p0 = 0; p0 < c->n_proj; p0 += NL_PCH) {
    const int np = std::min(NL_PCH, c->n_proj - p0);
    hipLaunchKernelGGL((nl_project_kernel<T, CT, CP>), dim3(NL_BLOCKS), dim3(NL_THREADS), 0, c->stream, x, ld, cols,
                       colscale, cbar, c->n_dof, p0, np, L.part, c->n_proj, done);
    TDFE_HIP(c, hipGetLastError());
  }
  return TDFE_OK;
}

// columns [col0, col0 + cols) of the launch (cols <= TDFE_MAX_COLS, col0 even)
template <typename T, typename CT>
tdfe_status nl_apply_t(tdfe_ctx* c, const ApplyArgs& a, int col0, int cols, double* energy_row, const CT* cbar,
                       const NlLayout& L) {
  const T* x = (const T*)a.x + col0;
  T* y = (T*)a.y + col0;
  const double* cs = a.colscale ? a.colscale + col0 / 2 : nullptr;
  if (cols <= 16)
    TDFE_TRY((nl_project_launch<T, CT, 16>(c, x, a.ld, cols, cs, a.done_flag, cbar, L)));
  else if (cols <= 32)
    TDFE_TRY((nl_project_launch<T, CT, 32>(c, x, a.ld, cols, cs, a.done_flag, cbar, L)));
  else
    TDFE_TRY((nl_project_launch<T, CT, 64>(c, x, a.ld, cols, cs, a.done_flag, cbar, L)));
  hipLaunchKernelGGL(nl_finalize_kernel, dim3(c->n_proj), dim3(64), 0, c->stream, (const double*)L.part, NL_BLOCKS,
                     c->n_proj, cols, (const double*)L.E, L.tE, L.eP, a.done_flag);
  TDFE_HIP(c, hipGetLastError());
  if (energy_row) {
    hipLaunchKernelGGL(nl_energy_kernel, dim3(1), dim3(64), 0, c->stream, (const double*)L.eP, c->n_proj, cols,
                       energy_row, a.done_flag);
    TDFE_HIP(c, hipGetLastError());
  }
  const int64_t n = c->n_dof * cols;
  hipLaunchKernelGGL((nl_add_kernel<T, CT>), dim3((unsigned)((n + NL_THREADS - 1) / NL_THREADS)), dim3(NL_THREADS),
                     0, c->stream, y, a.ld, cols, cbar, c->n_dof, (const double*)L.tE, c->n_proj, a.done_flag);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

}  // namespace

tdfe_status tdfe_launch_nonlocal(tdfe_ctx* c, const ApplyArgs& a) {
  if (c->n_proj <= 0) return TDFE_OK;
  if (!a.lowdin || a.fullgrid) return tdfe_fail(c, TDFE_EINVAL, "nonlocal term: Loewdin DoF launches only");
  const NlLayout L = nl_layout(c, c->n_proj, (char*)c->nl_store);
  // the term's share of the quadratic form goes to one more row of the block partials
  double* erow = nullptr;
  if (a.energy && a.n_blocks_out) {
    erow = a.energy + *a.n_blocks_out * a.cols;
    *a.n_blocks_out += 1;
  }
  for (int col0 = 0; col0 < a.cols; col0 += TDFE_MAX_COLS) {
    const int cols = std::min(TDFE_MAX_COLS, a.cols - col0);
    double* er = erow ? erow + col0 : nullptr;
    if (a.fp32)
      TDFE_TRY((nl_apply_t<float, float>(c, a, col0, cols, er, L.cbar32, L)));
    else
      TDFE_TRY((nl_apply_t<double, double>(c, a, col0, cols, er, L.cbar, L)));
  }
  return TDFE_OK;
}

extern "C" {

tdfe_status tdfe_projector_query(const tdfe_ctx* c, int n_proj, size_t* bytes) {
  if (!c || !bytes) return TDFE_EINVAL;
  if (n_proj < 0 || n_proj > TDFE_MAX_PROJ) return TDFE_EINVAL;
  *bytes = n_proj == 0 ? 0 : nl_layout(c, n_proj, nullptr).bytes;
  return TDFE_OK;
}

tdfe_status tdfe_set_projectors(tdfe_ctx* c, int n_proj, const double* dev_u, const double* dev_dv, void* dev_store,
                                size_t store_bytes) {
  if (!c) return TDFE_EINVAL;
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "set_projectors before bind_workspace");
  if (n_proj < 0 || n_proj > TDFE_MAX_PROJ)
    return tdfe_fail(c, TDFE_EINVAL, "set_projectors: n_proj outside [0, %d]", TDFE_MAX_PROJ);
  if (n_proj == 0) {
    c->n_proj = 0;
    c->nl_store = nullptr;
    return TDFE_OK;
  }
  if (!dev_u || !dev_dv || !dev_store) return tdfe_fail(c, TDFE_EINVAL, "set_projectors: null pointer");
  if ((uintptr_t)dev_store % 256 != 0) return tdfe_fail(c, TDFE_EINVAL, "set_projectors: store not 256-byte aligned");
  const NlLayout L = nl_layout(c, n_proj, (char*)dev_store);
  if (store_bytes < L.bytes) return tdfe_fail(c, TDFE_ENOMEM, "set_projectors: store of %zu bytes, %zu needed",
                                              store_bytes, L.bytes);
  c->n_proj = 0;  // the term is off until its tables are complete
  const int64_t nq = c->n_quad;
  int* bad = (int*)c->counters + 210;
  TDFE_TRY(tdfe_zero(c, bad, sizeof(int)));
  for (int p = 0; p < n_proj; ++p) {
    const double* u = dev_u + (size_t)p * nq;
    const double* dv = dev_dv + (size_t)p * nq;
    hipLaunchKernelGGL(nl_chi_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, c->stream, u, dv, L.scratch,
                       nq);
    TDFE_HIP(c, hipGetLastError());
    // c_p on every node (Gauss rule, weights varpi detJ), then Cbar on the DoFs
    TDFE_TRY(tdfe_load_vector(c, L.scratch, true));
    hipLaunchKernelGGL(nl_extract_kernel, dim3((unsigned)((c->n_dof + 255) / 256)), dim3(256), 0, c->stream,
                       (const double*)c->cload, (const double*)c->minv, L.cbar + (size_t)p * c->n_dof,
                       c->precision == TDFE_FP64 ? nullptr : L.cbar32 + (size_t)p * c->n_dof, c->Nx, c->Ny,
                       c->n_dof);
    TDFE_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(nl_norm_partial_kernel, dim3(NL_BLOCKS), dim3(NL_THREADS), 0, c->stream,
                       (const double*)c->wdet, (const double*)L.scratch, u, nq, L.red);
    hipLaunchKernelGGL(nl_norm_final_kernel, dim3(1), dim3(64), 0, c->stream, (const double*)L.red, NL_BLOCKS,
                       L.E + p, bad);
    TDFE_HIP(c, hipGetLastError());
  }
  const void* hb = nullptr;
  TDFE_TRY(tdfe_readback(c, bad, sizeof(int), 3072, &hb));
  TDFE_HIP(c, hipStreamSynchronize(c->stream));
  if (*(const volatile int*)hb)
    return tdfe_fail(c, TDFE_EINVAL, "set_projectors: int u dV u is zero or not finite for a projector");
  c->nl_store = dev_store;
  c->n_proj = n_proj;
  return TDFE_OK;
}

}  // extern "C"
