// fe_mesh_setup, workspace binding, geometry and overlap (tdfe C ABI).
//
// Reference element (Sec. "Higher-order spectral finite-elements"): the
// nodes of an order-p element are the GLL points (end points and roots of
// P_p'), the overlap M uses the GLL rule (hence diagonal) and every other
// integral the Gauss-Legendre rule with nq = p + 1 points.  The 1D tables
// come from the constexpr rule of tdfe_rule1d.h (Newton iteration on the
// Legendre three-term recurrence, barycentric Lagrange formulas), evaluated
// here at run time; the per-point geometry and M are computed on the device.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>

#include "tdfe_cheb.h"
#include "tdfe_internal.h"
#include "tdfe_rule1d.h"

tdfe_status tdfe_fail(tdfe_ctx* c, tdfe_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

namespace {

// ----------------------------------------------------------------------------------------------
// device geometry kernels
// ----------------------------------------------------------------------------------------------
struct GeoParams {
  const double* corners;  // [n_cell][2][2][2][3]
  const double* tab;
  int n, nq, ncx, ncy, ncz, p, Nx, Ny, Nz;
  int64_t n_cell;
  double gll[TDFE_MAXN], wgll[TDFE_MAXN];
};

__device__ void trilinear(const double* C, double s0, double s1, double s2, double x[3], double J[3][3]) {
  const double f[2][3] = {{0.5 * (1 - s0), 0.5 * (1 - s1), 0.5 * (1 - s2)},
                          {0.5 * (1 + s0), 0.5 * (1 + s1), 0.5 * (1 + s2)}};
  for (int d = 0; d < 3; ++d) {
    x[d] = 0;
    J[d][0] = J[d][1] = J[d][2] = 0;
  }
  for (int vz = 0; vz < 2; ++vz)
    for (int vy = 0; vy < 2; ++vy)
      for (int vx = 0; vx < 2; ++vx) {
        const double* X3 = C + ((vz * 2 + vy) * 2 + vx) * 3;
        const double sx = vx ? 0.5 : -0.5, sy = vy ? 0.5 : -0.5, sz = vz ? 0.5 : -0.5;
        const double v = f[vx][0] * f[vy][1] * f[vz][2];
        const double d0 = sx * f[vy][1] * f[vz][2];
        const double d1 = f[vx][0] * sy * f[vz][2];
        const double d2 = f[vx][0] * f[vy][1] * sz;
        for (int d = 0; d < 3; ++d) {
          x[d] += X3[d] * v;
          J[d][0] += X3[d] * d0;
          J[d][1] += X3[d] * d1;
          J[d][2] += X3[d] * d2;
        }
      }
}

__device__ double det3(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// per Gauss point: coordinates and varpi_q det J_q; flags a non-positive Jacobian
__global__ void quad_geometry_kernel(GeoParams P, double* xq, double* wdet, int* bad) {
  const int nq3 = P.nq * P.nq * P.nq;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= P.n_cell * nq3) return;
  const int64_t e = idx / nq3;
  const int q = (int)(idx % nq3);
  const int a = q % P.nq, b = (q / P.nq) % P.nq, c = q / (P.nq * P.nq);
  double x[3], J[3][3];
  trilinear(P.corners + e * 24, P.tab[TAB_ETA + a], P.tab[TAB_ETA + b], P.tab[TAB_ETA + c], x, J);
  const double d = det3(J);
  if (!(d > 0.0)) atomicOr(bad, 1);
  xq[idx * 3 + 0] = x[0];
  xq[idx * 3 + 1] = x[1];
  xq[idx * 3 + 2] = x[2];
  wdet[idx] = P.tab[TAB_W3Q + q] * d;
}

// per global node: position, GLL-lumped overlap summed over the cells that
// contain it (fixed order), and the DoF outputs for interior nodes
__global__ void node_kernel(GeoParams P, double* nodexyz, double* mdiag, double* minv, float* minv32,
                            double* dofxyz, int* bad) {
  const int64_t nn = (int64_t)P.Nx * P.Ny * P.Nz;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  const int I = (int)(idx % P.Nx);
  const int J = (int)((idx / P.Nx) % P.Ny);
  const int K = (int)(idx / ((int64_t)P.Nx * P.Ny));
  int lo[3], hi[3];
  const int G[3] = {I, J, K};
  const int nc[3] = {P.ncx, P.ncy, P.ncz};
  for (int d = 0; d < 3; ++d) {
    hi[d] = G[d] / P.p;
    lo[d] = (G[d] % P.p == 0) ? hi[d] - 1 : hi[d];
    if (hi[d] > nc[d] - 1) hi[d] = nc[d] - 1;
    if (lo[d] < 0) lo[d] = 0;
  }
  double m = 0.0, x[3] = {0, 0, 0};
  bool first = true;
  for (int cz = lo[2]; cz <= hi[2]; ++cz)
    for (int cy = lo[1]; cy <= hi[1]; ++cy)
      for (int cx = lo[0]; cx <= hi[0]; ++cx) {
        const int i = I - cx * P.p, j = J - cy * P.p, k = K - cz * P.p;
        const int64_t e = cx + (int64_t)P.ncx * (cy + (int64_t)P.ncy * cz);
        double xx[3], JJ[3][3];
        trilinear(P.corners + e * 24, P.gll[i], P.gll[j], P.gll[k], xx, JJ);
        const double d = det3(JJ);
        if (!(d > 0.0)) atomicOr(bad, 1);
        m += P.wgll[i] * P.wgll[j] * P.wgll[k] * d;
        if (first) {
          x[0] = xx[0];
          x[1] = xx[1];
          x[2] = xx[2];
          first = false;
        }
      }
  nodexyz[idx * 3 + 0] = x[0];
  nodexyz[idx * 3 + 1] = x[1];
  nodexyz[idx * 3 + 2] = x[2];
  if (I > 0 && I < P.Nx - 1 && J > 0 && J < P.Ny - 1 && K > 0 && K < P.Nz - 1) {
    const int64_t dof = (I - 1) + (int64_t)(P.Nx - 2) * ((J - 1) + (int64_t)(P.Ny - 2) * (K - 1));
    mdiag[dof] = m;
    minv[dof] = 1.0 / sqrt(m);
    if (minv32) minv32[dof] = (float)(1.0 / sqrt(m));
    dofxyz[dof * 3 + 0] = x[0];
    dofxyz[dof * 3 + 1] = x[1];
    dofxyz[dof * 3 + 2] = x[2];
  }
}

__global__ void weight_potential_kernel(const double* v, const double* wdet, double* vw, float* vw32, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = v[i] * wdet[i];
  vw[i] = x;
  if (vw32) vw32[i] = (float)x;
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// workspace layout: a deterministic bump allocation used by both query and bind
// ------------------------------------------------------------------------------------------------
namespace {
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

size_t elem_bytes(const tdfe_ctx* c) { return !tdfe_fp32(c) ? 8 : 4; }

void carve(tdfe_ctx* c, char* base) {
  Carver k{base};
  const int64_t nd = c->n_dof, nqd = c->n_quad, nn = c->n_nodes, ne = c->n_cell;
  c->tab = k.take<double>(TAB_SIZE);
  c->mfma_tab = c->mfma ? k.take<double>(6 * 256) : nullptr;
  c->minv = k.take<double>(nd);
  c->mdiag = k.take<double>(nd);
  c->dofxyz = k.take<double>(3 * nd);
  double* nodexyz = k.take<double>(3 * nn);
  (void)nodexyz;
  c->m1x = k.take<double>(c->Nx);
  c->m1y = k.take<double>(c->Ny);
  c->m1z = k.take<double>(c->Nz);
  c->cellgeo = k.take<double>(4 * ne);
  c->corners = k.take<double>(24 * ne);
  c->xq = k.take<double>(3 * nqd);
  c->wdet = k.take<double>(nqd);
  c->vext = k.take<double>(nqd);
  c->vw = k.take<double>(nqd);
  c->vw32 = k.take<float>(nqd);
  c->w1 = k.take<double>(nqd);
  c->w2 = k.take<double>(nqd);
  c->w3 = k.take<double>(nqd);
  c->wn = k.take<double>(nqd);
  c->scbuf = k.take<double>(512);
  c->wh = k.take<double>(nqd);
  c->rho = k.take<double>(nqd);
  c->phi = k.take<double>(nn);
  c->cload = k.take<double>(nn);
  c->fb = k.take<double>(nn);
  c->lift = k.take<double>(nd);
  c->t0 = k.take<double>(nd);
  c->t1 = k.take<double>(nd);
  const int n1x = c->Nx - 2, n1y = c->Ny - 2, n1z = c->Nz - 2;
  c->fdmS = k.take<double>(2 * ((size_t)n1x * n1x + (size_t)n1y * n1y + (size_t)n1z * n1z));
  c->fdmL = k.take<double>((size_t)n1x + n1y + n1z);
  c->pcg = (c->box || c->octree) ? k.take<double>(1) : k.take<double>(5 * nn);
  c->dinvK = (c->box || c->octree) ? k.take<double>(1) : k.take<double>(nn);
  c->pcgs = k.take<double>(16);
  const int cols = 2 * std::max(c->chunk_orb, c->wide_orb);  // widest chunk's columns
  c->krylov = k.take<char>((size_t)(c->k_max + 1) * nd * 2 * c->chunk_orb * elem_bytes(c));
  c->hq = k.take<char>((size_t)nd * cols * elem_bytes(c));
  c->half = k.take<double>((size_t)nd * 2 * c->n_orb_max);
  // block partials of the operator kernels, plus rows appended after them (the nonlocal term's)
  c->n_partial = (std::max<int64_t>(ne, 4096) + 8) * std::max(cols, 8);
  c->partial = k.take<double>(c->n_partial);
  c->partial2 = k.take<double>(128 * TDFE_MAX_COLS);
  c->scal = k.take<double>((size_t)(8 * c->k_max + 32) * c->n_orb_max);
  c->jtab = k.take<double>((size_t)std::max({c->chunk_orb, c->wide_orb, 1}) * TDFE_JTAB_STRIDE);
  c->counters = k.take<unsigned>(256);
  // octree meshes: cell node lists, cube edges, C, the operator's slot codes and hanging rows, node work arrays
  if (c->octree) {
    c->oct_cn = k.take<int>(c->oct_cn_h.size());
    c->oct_s = k.take<double>(c->oct_s_h.size());
    c->oct_eptr = k.take<int>(c->oct_eptr_h.size());
    c->oct_ecol = k.take<int>(c->oct_ecol_h.size());
    c->oct_eval = k.take<double>(c->oct_eval_h.size());
    c->oct_cd = k.take<int>(c->oct_cd_h.size());
    c->oct_hv = k.take<int>(c->oct_hv_h.size());
    c->oct_mptr = k.take<int>(c->oct_mptr_h.size());
    c->oct_md = k.take<int>(c->oct_md_h.size());
    c->oct_mh = k.take<int>(c->oct_mh_h.size());
    c->oct_mv = k.take<double>(c->oct_mv_h.size());
    c->oct_xf = k.take<double>((size_t)nn * c->oct_w);
    c->oct_yf = k.take<double>((size_t)nn * c->oct_w);
  }
  // FP32 copy of M^-1/2 for the mixed path's operator (placed last)
  c->minv32 = !tdfe_fp32(c) ? k.take<float>(1) : k.take<float>(nd);
  c->ws_need = k.off + 256;
  // node coordinates live right after dofxyz; keep the pointer in the ctx via fb's neighbour
  c->nodexyz_ptr = nodexyz;
}
}  // namespace

namespace {

// reference element tables (the same constexpr rule the operator kernels
// evaluate at compile time)
void init_tables(tdfe_ctx* c) {
  const tdfe1d::Rule R = tdfe1d::make_rule(c->p);
  static_assert(tdfe1d::MAXN == TDFE_MAXN, "table stride");
  std::memcpy(c->xi, R.xi, sizeof c->xi);
  std::memcpy(c->w, R.w, sizeof c->w);
  std::memcpy(c->eta, R.eta, sizeof c->eta);
  std::memcpy(c->wq, R.wq, sizeof c->wq);
  std::memcpy(c->B, R.B, sizeof c->B);
  std::memcpy(c->D, R.D, sizeof c->D);
  std::memcpy(c->Dg, R.Dg, sizeof c->Dg);
}

void init_variant(tdfe_ctx* c) {
  const char* v = std::getenv("TDFE_APPLY_VARIANT");
  c->variant = 0;
  if (v && std::strcmp(v, "line") == 0) c->variant = TDFE_VARIANT_LINE;
  if (v && std::strcmp(v, "pair") == 0) c->variant = TDFE_VARIANT_PAIR;
  if (v && std::strcmp(v, "plane") == 0) c->variant = TDFE_VARIANT_PLANE;
}

// Krylov chunk: as many orbitals as fit in 60% of the device memory free at
// creation (about 170 GB on an idle 288 GB device; 128 GB if it cannot be queried)
void init_chunk(tdfe_ctx* c) {
  const size_t eb = !tdfe_fp32(c) ? 8 : 4;
  const double per_orb = (double)(c->k_max + 2) * (double)c->n_dof * 2.0 * (double)eb;
  double basis_bytes = 128e9;
  {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) basis_bytes = 0.6 * (double)free_b;
    else (void)hipGetLastError();
  }
  int chunk = (int)std::min<double>(c->n_orb_max, std::floor(basis_bytes / per_orb));
  if (chunk > TDFE_MAX_COLS / 2) chunk = TDFE_MAX_COLS / 2;
  // optional caps: TDFE_MAX_CHUNK_ORB on every chunk (tests use it to run
  // several chunks on small meshes), TDFE_BASIS_CHUNK_ORB on the basis memory
  // only, as on a device with less memory (soft-capped chunks stay possible)
  const char* vmax = std::getenv("TDFE_MAX_CHUNK_ORB");
  const int cap_all = vmax && std::atoi(vmax) > 0 ? std::atoi(vmax) : 0;
  const char* vbas = std::getenv("TDFE_BASIS_CHUNK_ORB");
  if (vbas && std::atoi(vbas) > 0) chunk = std::min(chunk, std::atoi(vbas));
  if (cap_all) chunk = std::min(chunk, cap_all);
  if (chunk < 1) chunk = 1;
  c->chunk_orb = chunk;
  // soft-capped chunks: every width whose cap keeps TDFE_SOFT_CAP_MIN vectors
  int wide = chunk;
  const int wlim = std::min(c->n_orb_max, TDFE_MAX_COLS / 2);
  for (int w = chunk + 1; w <= wlim; ++w)
    if (tdfe_soft_cap(c, w) >= TDFE_SOFT_CAP_MIN) wide = w;
  if (cap_all) wide = std::min(wide, cap_all);
  c->wide_orb = std::max(wide, chunk);
}

}  // namespace

tdfe_status tdfe_octree_configure(tdfe_ctx* c, const tdfe_octree_desc* d);

extern "C" {

tdfe_status tdfe_fe_mesh_setup(const tdfe_mesh_desc* d, void* hip_stream, tdfe_ctx** out) {
  if (!d || !out) return TDFE_EINVAL;
  *out = nullptr;
  if (d->p < 1 || d->p > 8) return TDFE_EINVAL;
  if (d->nq != d->p + 1) return TDFE_EINVAL;
  if (d->ncell[0] < 1 || d->ncell[1] < 1 || d->ncell[2] < 1) return TDFE_EINVAL;
  if (!d->vertices) return TDFE_EINVAL;
  if (d->n_orb_max < 1 || d->n_orb_max > 4096) return TDFE_EINVAL;
  if (d->k_max < 1 || d->k_max > 1024) return TDFE_EINVAL;
  if (d->precision < TDFE_FP64 || d->precision > TDFE_FP64_MFMA) return TDFE_EINVAL;
  const int64_t Nx = (int64_t)d->ncell[0] * d->p + 1, Ny = (int64_t)d->ncell[1] * d->p + 1,
                Nz = (int64_t)d->ncell[2] * d->p + 1;
  if (Nx < 3 || Ny < 3 || Nz < 3) return TDFE_EINVAL;  // no interior node
  if (Nx * Ny * Nz > ((int64_t)1 << 31)) return TDFE_EINVAL;
  for (int64_t i = 0; i < (d->ncell[0] + 1LL) * (d->ncell[1] + 1LL) * (d->ncell[2] + 1LL) * 3; ++i)
    if (!std::isfinite(d->vertices[i])) return TDFE_EINVAL;

  tdfe_ctx* c = new tdfe_ctx();
  c->p = d->p;
  c->n = d->p + 1;
  c->nq = d->nq;
  c->ncx = d->ncell[0];
  c->ncy = d->ncell[1];
  c->ncz = d->ncell[2];
  c->Nx = (int)Nx;
  c->Ny = (int)Ny;
  c->Nz = (int)Nz;
  c->n_cell = (int64_t)c->ncx * c->ncy * c->ncz;
  c->n_nodes = Nx * Ny * Nz;
  c->n_dof = (Nx - 2) * (Ny - 2) * (Nz - 2);
  c->n_quad = c->n_cell * c->nq * c->nq * c->nq;
  c->n_orb_max = d->n_orb_max;
  c->k_max = d->k_max;
  c->precision = d->precision;
  c->stream = (hipStream_t)hip_stream;
  const size_t nv = (size_t)(c->ncx + 1) * (c->ncy + 1) * (c->ncz + 1) * 3;
  c->vertices.assign(d->vertices, d->vertices + nv);

  init_tables(c);

  // rectilinear (box) detection: x depends only on the x index, etc.
  auto V = [&](int i, int j, int k, int dd) {
    return c->vertices[(((size_t)k * (c->ncy + 1) + j) * (c->ncx + 1) + i) * 3 + dd];
  };
  bool box = true;
  for (int k = 0; k <= c->ncz && box; ++k)
    for (int j = 0; j <= c->ncy && box; ++j)
      for (int i = 0; i <= c->ncx && box; ++i) {
        if (V(i, j, k, 0) != V(i, 0, 0, 0) || V(i, j, k, 1) != V(0, j, 0, 1) || V(i, j, k, 2) != V(0, 0, k, 2))
          box = false;
      }
  if (box) {
    for (int i = 0; i <= c->ncx; ++i) c->ax_x.push_back(V(i, 0, 0, 0));
    for (int j = 0; j <= c->ncy; ++j) c->ax_y.push_back(V(0, j, 0, 1));
    for (int k = 0; k <= c->ncz; ++k) c->ax_z.push_back(V(0, 0, k, 2));
    for (size_t i = 1; i < c->ax_x.size(); ++i)
      if (!(c->ax_x[i] > c->ax_x[i - 1])) box = false;
    for (size_t i = 1; i < c->ax_y.size(); ++i)
      if (!(c->ax_y[i] > c->ax_y[i - 1])) box = false;
    for (size_t i = 1; i < c->ax_z.size(); ++i)
      if (!(c->ax_z[i] > c->ax_z[i - 1])) box = false;
  }
  c->box = box;
  // matrix-core variants: box cells, p <= 7 (p <= 6 in FP64: three FP64 cell
  // arrays of 16 columns fill the 160 KB of LDS)
  c->mfma = c->precision == TDFE_FP32_MFMA || c->precision == TDFE_BF16_MFMA || c->precision == TDFE_FP64_MFMA;
  if (c->mfma && (!box || c->p > (c->precision == TDFE_FP64_MFMA ? 6 : 7))) {
    delete c;
    return TDFE_EINVAL;
  }
  init_variant(c);
  init_chunk(c);
  carve(c, nullptr);
  *out = c;
  return TDFE_OK;
}

tdfe_status tdfe_fe_octree_setup(const tdfe_octree_desc* d, void* hip_stream, tdfe_ctx** out) {
  if (!d || !out) return TDFE_EINVAL;
  *out = nullptr;
  if (d->p < 1 || d->p > 8) return TDFE_EINVAL;
  if (!(d->hi > d->lo) || !std::isfinite(d->lo) || !std::isfinite(d->hi)) return TDFE_EINVAL;
  if (d->n0 < 1 || d->n0 > 64 || d->max_level < 0 || d->max_level > 10) return TDFE_EINVAL;
  if (d->n_leaf < 1 || !d->leaves) return TDFE_EINVAL;
  if (d->n_orb_max < 1 || d->n_orb_max > 4096) return TDFE_EINVAL;
  if (d->k_max < 1 || d->k_max > 1024) return TDFE_EINVAL;
  if (d->precision != TDFE_FP64) return TDFE_EINVAL;
  tdfe_ctx* c = new tdfe_ctx();
  c->p = d->p;
  c->n = d->p + 1;
  c->nq = d->p + 1;
  c->octree = true;
  c->box = false;
  // the structured-grid fields keep the smallest valid values (their arrays
  // are not used on octree meshes)
  c->ncx = c->ncy = c->ncz = 1;
  c->Nx = c->Ny = c->Nz = 3;
  c->n_cell = d->n_leaf;
  c->n_quad = c->n_cell * c->nq * c->nq * c->nq;
  c->n_orb_max = d->n_orb_max;
  c->k_max = d->k_max;
  c->precision = d->precision;
  c->stream = (hipStream_t)hip_stream;
  init_tables(c);
  const tdfe_status st = tdfe_octree_configure(c, d);
  if (st != TDFE_OK) {
    delete c;
    return st;
  }
  init_variant(c);
  init_chunk(c);
  c->oct_w = std::min(TDFE_MAX_COLS, std::max(2 * c->chunk_orb, 2 * c->n_orb_max));
  carve(c, nullptr);
  *out = c;
  return TDFE_OK;
}

tdfe_status tdfe_query(const tdfe_ctx* c, int64_t* n_dof, int64_t* n_cell, int64_t* n_quad, size_t* ws) {
  if (!c) return TDFE_EINVAL;
  if (n_dof) *n_dof = c->n_dof;
  if (n_cell) *n_cell = c->n_cell;
  if (n_quad) *n_quad = c->n_quad;
  if (ws) *ws = c->ws_need;
  return TDFE_OK;
}

static tdfe_status finish_bind(tdfe_ctx* c) {
  // pinned poll buffer for the Lanczos convergence flags
  if (!c->poll) {
    TDFE_HIP(c, hipHostMalloc((void**)&c->poll, 4096 * sizeof(int), hipHostMallocDefault));
    std::memset(c->poll, 0, 4096 * sizeof(int));  // flags compare against generation numbers >= 1
  }
  c->bound = true;
  c->have_potential = false;
  c->have_scf = false;
  c->scf_init = false;
  return TDFE_OK;
}

tdfe_status tdfe_bind_workspace(tdfe_ctx* c, void* dev, size_t bytes) {
  if (!c) return TDFE_EINVAL;
  if (!dev) return tdfe_fail(c, TDFE_EINVAL, "bind_workspace: null buffer");
  if (((uintptr_t)dev) & 255) return tdfe_fail(c, TDFE_EINVAL, "bind_workspace: buffer not 256-byte aligned");
  if (bytes < c->ws_need)
    return tdfe_fail(c, TDFE_ENOMEM, "bind_workspace: %zu bytes < required %zu", bytes, c->ws_need);
  c->ws = (char*)dev;
  c->ws_bytes = bytes;
  carve(c, c->ws);
  c->occ_dev_ver = -1;  // device-side copies in the old workspace are gone

  // 1D tables
  std::vector<double> tab(TAB_SIZE, 0.0);
  for (int a = 0; a < TDFE_MAXN; ++a)
    for (int i = 0; i < TDFE_MAXN; ++i) {
      tab[TAB_B + a * TDFE_MAXN + i] = c->B[a * TDFE_MAXN + i];
      tab[TAB_D + a * TDFE_MAXN + i] = c->D[a * TDFE_MAXN + i];
      tab[TAB_DG + a * TDFE_MAXN + i] = c->Dg[a * TDFE_MAXN + i];
    }
  for (int a = 0; a < c->nq; ++a) {
    tab[TAB_ETA + a] = c->eta[a];
    tab[TAB_WQ + a] = c->wq[a];
  }
  for (int cc = 0; cc < c->nq; ++cc)
    for (int b = 0; b < c->nq; ++b)
      for (int a = 0; a < c->nq; ++a)
        tab[TAB_W3Q + a + c->nq * (b + c->nq * cc)] = c->wq[a] * c->wq[b] * c->wq[cc];
  TDFE_HIP(c, hipMemcpyAsync(c->tab, tab.data(), TAB_SIZE * sizeof(double), hipMemcpyHostToDevice, c->stream));
  std::vector<double> mt(c->mfma ? 6 * 256 : 0);  // (the stream is synchronised before the host copies go)
  if (c->mfma) {
    tdfe_mfma_tables(c->p, mt.data());
    TDFE_HIP(c, hipMemcpyAsync(c->mfma_tab, mt.data(), mt.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  }

  if (c->octree) {
    TDFE_TRY(tdfe_octree_bind(c));
    TDFE_HIP(c, hipMemsetAsync(c->counters, 0, 256 * sizeof(unsigned), c->stream));
    return finish_bind(c);
  }
  // cell corners (and per-cell box metric)
  std::vector<double> cor((size_t)c->n_cell * 24), geo((size_t)c->n_cell * 4);
  auto V = [&](int i, int j, int k, int dd) {
    return c->vertices[(((size_t)k * (c->ncy + 1) + j) * (c->ncx + 1) + i) * 3 + dd];
  };
  for (int cz = 0; cz < c->ncz; ++cz)
    for (int cy = 0; cy < c->ncy; ++cy)
      for (int cx = 0; cx < c->ncx; ++cx) {
        const size_t e = cx + (size_t)c->ncx * (cy + (size_t)c->ncy * cz);
        for (int vz = 0; vz < 2; ++vz)
          for (int vy = 0; vy < 2; ++vy)
            for (int vx = 0; vx < 2; ++vx)
              for (int dd = 0; dd < 3; ++dd)
                cor[e * 24 + ((vz * 2 + vy) * 2 + vx) * 3 + dd] = V(cx + vx, cy + vy, cz + vz, dd);
        if (c->box) {
          const double hx = c->ax_x[cx + 1] - c->ax_x[cx], hy = c->ax_y[cy + 1] - c->ax_y[cy],
                       hz = c->ax_z[cz + 1] - c->ax_z[cz];
          const double det = hx * hy * hz / 8.0;
          geo[e * 4 + 0] = det * 4.0 / (hx * hx);
          geo[e * 4 + 1] = det * 4.0 / (hy * hy);
          geo[e * 4 + 2] = det * 4.0 / (hz * hz);
          geo[e * 4 + 3] = det;
        }
      }
  // box meshes: the GLL-lumped overlap factorises, M(I,J,K) = mx[I] my[J] mz[K] with
  // m[I] = sum over the 1D cells containing node I of w_i h / 2
  std::vector<double> f1[3];
  if (c->box) {
    const std::vector<double>* axs[3] = {&c->ax_x, &c->ax_y, &c->ax_z};
    for (int d = 0; d < 3; ++d) {
      const auto& ax = *axs[d];
      const int nc = (int)ax.size() - 1;
      std::vector<double> m(nc * c->p + 1, 0.0);
      for (int e = 0; e < nc; ++e)
        for (int i = 0; i <= c->p; ++i) m[e * c->p + i] += c->w[i] * 0.5 * (ax[e + 1] - ax[e]);
      f1[d].resize(m.size());
      for (size_t i = 0; i < m.size(); ++i) f1[d][i] = 1.0 / std::sqrt(m[i]);
    }
    TDFE_HIP(c, hipMemcpyAsync(c->m1x, f1[0].data(), f1[0].size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    TDFE_HIP(c, hipMemcpyAsync(c->m1y, f1[1].data(), f1[1].size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    TDFE_HIP(c, hipMemcpyAsync(c->m1z, f1[2].data(), f1[2].size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  }
  TDFE_HIP(c, hipMemcpyAsync(c->corners, cor.data(), cor.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  TDFE_HIP(c, hipMemcpyAsync(c->cellgeo, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  TDFE_HIP(c, hipMemsetAsync(c->counters, 0, 256 * sizeof(unsigned), c->stream));

  GeoParams G{};
  G.corners = c->corners;
  G.tab = c->tab;
  G.n = c->n;
  G.nq = c->nq;
  G.ncx = c->ncx;
  G.ncy = c->ncy;
  G.ncz = c->ncz;
  G.p = c->p;
  G.Nx = c->Nx;
  G.Ny = c->Ny;
  G.Nz = c->Nz;
  G.n_cell = c->n_cell;
  for (int i = 0; i < c->n; ++i) {
    G.gll[i] = c->xi[i];
    G.wgll[i] = c->w[i];
  }
  int* bad = (int*)c->counters + 200;
  {
    const int64_t n = c->n_quad;
    hipLaunchKernelGGL(quad_geometry_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, G, c->xq,
                       c->wdet, bad);
    TDFE_HIP(c, hipGetLastError());
  }
  {
    const int64_t n = c->n_nodes;
    hipLaunchKernelGGL(node_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, G,
                       c->nodexyz_ptr, c->mdiag, c->minv, !tdfe_fp32(c) ? nullptr : c->minv32,
                       c->dofxyz, bad);
    TDFE_HIP(c, hipGetLastError());
  }
  int hbad = 0;
  TDFE_HIP(c, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  TDFE_HIP(c, hipStreamSynchronize(c->stream));
  if (hbad) return tdfe_fail(c, TDFE_EINVAL, "mesh has a non-positive Jacobian");
  return finish_bind(c);
}

tdfe_status tdfe_dof_coords(tdfe_ctx* c, double* dev_xyz) {
  if (!c || !dev_xyz) return TDFE_EINVAL;
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "dof_coords before bind_workspace");
  TDFE_HIP(c, hipMemcpyAsync(dev_xyz, c->dofxyz, c->n_dof * 3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return TDFE_OK;
}

tdfe_status tdfe_quad_coords(tdfe_ctx* c, double* dev_xyz) {
  if (!c || !dev_xyz) return TDFE_EINVAL;
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "quad_coords before bind_workspace");
  TDFE_HIP(c, hipMemcpyAsync(dev_xyz, c->xq, c->n_quad * 3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return TDFE_OK;
}

tdfe_status tdfe_mass_diag(tdfe_ctx* c, double* dev_m) {
  if (!c || !dev_m) return TDFE_EINVAL;
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "mass_diag before bind_workspace");
  TDFE_HIP(c, hipMemcpyAsync(dev_m, c->mdiag, c->n_dof * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return TDFE_OK;
}

tdfe_status tdfe_set_potential(tdfe_ctx* c, const double* dev_v) {
  if (!c || !dev_v) return TDFE_EINVAL;
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "set_potential before bind_workspace");
  TDFE_HIP(c, hipMemcpyAsync(c->vext, dev_v, c->n_quad * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  const int64_t n = c->n_quad;
  hipLaunchKernelGGL(weight_potential_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->vext,
                     c->wdet, c->vw, c->vw32, n);
  TDFE_HIP(c, hipGetLastError());
  c->have_potential = true;
  return TDFE_OK;
}

const char* tdfe_last_error(const tdfe_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

void tdfe_destroy(tdfe_ctx* c) {
  if (!c) return;
  // pending copies into the pinned poll buffer must land before it is freed
  if (c->bound) (void)hipStreamSynchronize(c->stream);
  for (int i = 0; i < c->n_evs; ++i) (void)hipEventDestroy(c->evs[i]);
  delete[] c->evs;
  tdfe_blas_destroy(c);
  if (c->poll) (void)hipHostFree(c->poll);
  delete c;
}

}  // extern "C"
