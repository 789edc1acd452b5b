// A priori element-size distribution (Sec. "Efficient spatio-temporal
// discretization", Eqs. OptimalMeshMin and OptimalMeshSize) and the graded
// rectilinear axes built from it.
//
//   h(r) = E g(r)^(-1/(p+3)),
//   g = sum over atoms of 2 Dbar^{p+1} phi + Dbar^{p+3} phi + Dbar^{p+1} V,
//   Dbar^k f = sum over multi-indices |l| = k of |D^l f|,
// with phi = (pi s^2)^(-3/4) exp(-|r-R|^2/(2 s^2)) the atom's orbital at both
// times of the bound, V = -Z exp(-|r-R|^2/(2 a^2)) its potential, and E from
// int dr / h^3 = N_elem.  For a Gaussian A exp(-|u|^2/2), u = (r - R)/s,
// D^l f = A (-1/s)^k prod_i He_{l_i}(u_i) exp(-|u|^2/2) (probabilists'
// Hermite polynomials), so Dbar^k f = |A| s^-k exp(-|u|^2/2)
// sum_{l1+l2+l3=k} prod_i |He_{l_i}(u_i)|.
//
// On the GPU: g at every point of a uniform S^3 sample grid (one thread per
// point), the trapezoid sum of g^{3/(p+3)} for E, and the largest g over every
// sample plane of each axis.  On the host: the 1D spacing h_a(s) = E (largest
// g over the plane)^(-1/(p+3)), its cumulative trapezoid integral of 1/h_a,
// the cell counts and the equidistributed vertices.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <set>
#include <vector>

#include "tdfe_internal.h"

// Scratch of tdfe_adaptive_axes_static (the allocation-free variant): one copy
// of this array per GPU, held until the process ends.  Host code never passes
// its name to a kernel or a copy (that is a host-side stand-in, not a device
// address): it uses the per-device address from hipGetSymbolAddress below.
static __device__ __align__(256) double scratch[TDFE_AXES_STATIC_BYTES / sizeof(double)];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// device address of `scratch` on the current device, looked up once per
// device with that device current; null on failure
void* static_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

constexpr int MAX_K = 11;  // p + 3 for p <= 8
constexpr int MT = 256;
constexpr int SUM_BLOCKS = 256;

struct AtomParams {
  double R[3];
  double Z, s, a;
};

// sum over l1 + l2 + l3 = k of |Hx[l1]| |Hy[l2]| |Hz[l3]|
__device__ double multi_sum(const double* Hx, const double* Hy, const double* Hz, int k) {
  double tot = 0.0;
  for (int l1 = 0; l1 <= k; ++l1)
    for (int l2 = 0; l2 <= k - l1; ++l2) tot += fabs(Hx[l1]) * fabs(Hy[l2]) * fabs(Hz[k - l1 - l2]);
  return tot;
}

// He_0 .. He_k at u: He_{n+1} = u He_n - n He_{n-1}
__device__ void hermite(double u, int k, double* H) {
  H[0] = 1.0;
  if (k >= 1) H[1] = u;
  for (int n = 1; n < k; ++n) H[n + 1] = u * H[n] - n * H[n - 1];
}

__device__ double dbar(const double* pt, const double* R, double s, double A, int k) {
  double Hx[MAX_K + 1], Hy[MAX_K + 1], Hz[MAX_K + 1];
  const double ux = (pt[0] - R[0]) / s, uy = (pt[1] - R[1]) / s, uz = (pt[2] - R[2]) / s;
  hermite(ux, k, Hx);
  hermite(uy, k, Hy);
  hermite(uz, k, Hz);
  return fabs(A) * pow(s, -k) * multi_sum(Hx, Hy, Hz, k) * exp(-0.5 * (ux * ux + uy * uy + uz * uz));
}

// g at one point: the sum over atoms above
__device__ double weight_at(const double* pt, const AtomParams* atoms, int n_atoms, int p) {
  double v = 0.0;
  for (int a = 0; a < n_atoms; ++a) {
    const AtomParams A = atoms[a];
    const double amp = pow(M_PI * A.s * A.s, -0.75);
    v += 2.0 * dbar(pt, A.R, A.s, amp, p + 1) + dbar(pt, A.R, A.s, amp, p + 3);
    v += dbar(pt, A.R, A.a, A.Z, p + 1);
  }
  return v;
}

// g at n given points (octree refinement)
__global__ void __launch_bounds__(MT)
    point_weight_kernel(const AtomParams* atoms, int n_atoms, int p, const double* pts, int64_t n, double* g) {
  const int64_t idx = (int64_t)blockIdx.x * MT + threadIdx.x;
  if (idx >= n) return;
  const double pt[3] = {pts[3 * idx], pts[3 * idx + 1], pts[3 * idx + 2]};
  g[idx] = weight_at(pt, atoms, n_atoms, p);
}

__global__ void __launch_bounds__(MT)
    size_weight_kernel(const AtomParams* atoms, int n_atoms, int p, double lo, double step, double hi, int S,
                       double* g) {
  const int64_t idx = (int64_t)blockIdx.x * MT + threadIdx.x;
  const int64_t n = (int64_t)S * S * S;
  if (idx >= n) return;
  const int k = (int)(idx % S), j = (int)((idx / S) % S), i = (int)(idx / ((int64_t)S * S));
  auto coord = [&](int m) { return m == S - 1 ? hi : lo + m * step; };
  const double pt[3] = {coord(i), coord(j), coord(k)};  // sample (i, j, k) = (x, y, z), z fastest
  g[idx] = weight_at(pt, atoms, n_atoms, p);
}

// partial[b] = sum over a grid-stride share of w_i w_j w_k g^{3/(p+3)} (trapezoid weights / step^3)
__global__ void __launch_bounds__(MT) count_partial_kernel(const double* g, int S, int p, double* partial) {
  __shared__ double s[MT];
  const int64_t n = (int64_t)S * S * S;
  double acc = 0.0;
  for (int64_t idx = (int64_t)blockIdx.x * MT + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * MT) {
    const int k = (int)(idx % S), j = (int)((idx / S) % S), i = (int)(idx / ((int64_t)S * S));
    const double w = (i == 0 || i == S - 1 ? 0.5 : 1.0) * (j == 0 || j == S - 1 ? 0.5 : 1.0) *
                     (k == 0 || k == S - 1 ? 0.5 : 1.0);
    acc += w * pow(g[idx], 3.0 / (p + 3));
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = MT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

// gmax[axis][m] = largest g over the sample plane m of the axis (block (m, axis))
__global__ void __launch_bounds__(MT) plane_max_kernel(const double* g, int S, double* gmax) {
  __shared__ double s[MT];
  const int m = blockIdx.x, axis = blockIdx.y;
  const int64_t plane = (int64_t)S * S;
  double v = 0.0;
  for (int64_t r = threadIdx.x; r < plane; r += MT) {
    const int u = (int)(r / S), w = (int)(r % S);
    int64_t idx;
    if (axis == 0)
      idx = ((int64_t)m * S + u) * S + w;
    else if (axis == 1)
      idx = ((int64_t)u * S + m) * S + w;
    else
      idx = ((int64_t)u * S + w) * S + m;
    v = fmax(v, g[idx]);
  }
  s[threadIdx.x] = v;
  __syncthreads();
  for (int w = MT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) gmax[axis * S + m] = s[0];
}

size_t scratch_need(int S) {
  return ((size_t)S * S * S + 3 * (size_t)S + SUM_BLOCKS + (size_t)TDFE_MAX_ATOMS_MESH * 8) * sizeof(double) + 1024;
}

bool desc_ok(const tdfe_adapt_desc* d) {
  if (!d || d->p < 1 || d->p > 8 || !(d->hi > d->lo) || !std::isfinite(d->lo) || !std::isfinite(d->hi)) return false;
  if (d->n_atoms < 1 || d->n_atoms > TDFE_MAX_ATOMS_MESH || !d->R || !d->Z || !d->s_orb || !d->a_pot) return false;
  if (!(d->n_elem >= 1.0) || !std::isfinite(d->n_elem) || d->samples < 3 || d->samples > 1024) return false;
  for (int a = 0; a < d->n_atoms; ++a) {
    if (!std::isfinite(d->R[3 * a]) || !std::isfinite(d->R[3 * a + 1]) || !std::isfinite(d->R[3 * a + 2])) return false;
    if (!std::isfinite(d->Z[a]) || !(d->s_orb[a] > 0.0) || !(d->a_pot[a] > 0.0)) return false;
  }
  return true;
}

}  // namespace

extern "C" {

tdfe_status tdfe_adaptive_axes_query(const tdfe_adapt_desc* d, size_t* bytes) {
  if (!desc_ok(d) || !bytes) return TDFE_EINVAL;
  *bytes = scratch_need(d->samples);
  return TDFE_OK;
}

}  // extern "C"

namespace {

// both entry points: every element of the scratch that is read is written
// earlier in the same call (g by one thread per sample, the partials and the
// plane maxima by one block each), so nothing needs clearing between calls
tdfe_status adaptive_axes_impl(const tdfe_adapt_desc* d, void* dev_scratch, hipStream_t st, int max_cells,
                               double* host_axes, int* host_ncell, double* host_E) {
  const int S = d->samples, p = d->p;
  double* g = (double*)dev_scratch;
  double* gmax = g + (size_t)S * S * S;
  double* partial = gmax + 3 * (size_t)S;
  AtomParams* atoms = (AtomParams*)(partial + SUM_BLOCKS);
  std::vector<AtomParams> ha(d->n_atoms);
  for (int a = 0; a < d->n_atoms; ++a) {
    for (int c = 0; c < 3; ++c) ha[a].R[c] = d->R[3 * a + c];
    ha[a].Z = d->Z[a];
    ha[a].s = d->s_orb[a];
    ha[a].a = d->a_pot[a];
  }
  const double step = (d->hi - d->lo) / (S - 1);
  const int64_t n = (int64_t)S * S * S;
  if (hipMemcpyAsync(atoms, ha.data(), ha.size() * sizeof(AtomParams), hipMemcpyHostToDevice, st) != hipSuccess)
    return TDFE_EDEVICE;
  hipLaunchKernelGGL(size_weight_kernel, dim3((unsigned)((n + MT - 1) / MT)), dim3(MT), 0, st,
                     (const AtomParams*)atoms, d->n_atoms, p, d->lo, step, d->hi, S, g);
  hipLaunchKernelGGL(count_partial_kernel, dim3(SUM_BLOCKS), dim3(MT), 0, st, (const double*)g, S, p, partial);
  hipLaunchKernelGGL(plane_max_kernel, dim3(S, 3), dim3(MT), 0, st, (const double*)g, S, gmax);
  if (hipGetLastError() != hipSuccess) return TDFE_EDEVICE;
  std::vector<double> hg(3 * (size_t)S), hp(SUM_BLOCKS);
  if (hipMemcpyAsync(hg.data(), gmax, hg.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(hp.data(), partial, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return TDFE_EDEVICE;
  double sum = 0.0;
  for (double v : hp) sum += v;
  // E^3 = (trapezoid integral of g^{3/(p+3)}) / N_elem
  const double E = std::cbrt(sum * step * step * step / d->n_elem);
  if (!(E > 0.0) || !std::isfinite(E)) return TDFE_EINVAL;
  // sample coordinates as numpy's linspace forms them
  std::vector<double> t(S);
  for (int m = 0; m < S; ++m) t[m] = d->lo + m * step;
  t[S - 1] = d->hi;
  std::vector<double> F[3];
  for (int a = 0; a < 3; ++a) {
    F[a].assign(S, 0.0);
    double acc = 0.0;
    for (int m = 0; m + 1 < S; ++m) {
      const double i0 = std::pow(hg[a * S + m], 1.0 / (p + 3)) / E, i1 = std::pow(hg[a * S + m + 1], 1.0 / (p + 3)) / E;
      acc += 0.5 * (i1 + i0) * (t[m + 1] - t[m]);
      F[a][m + 1] = acc;
    }
    if (!(acc > 0.0) || !std::isfinite(acc)) return TDFE_EINVAL;
  }
  const double c = std::cbrt(d->n_elem / (F[0][S - 1] * F[1][S - 1] * F[2][S - 1]));
  for (int a = 0; a < 3; ++a) {
    const int nc = std::max(1, (int)std::floor(c * F[a][S - 1] + 0.5));
    if (nc > max_cells) return TDFE_ENOMEM;
    host_ncell[a] = nc;
  }
  for (int a = 0; a < 3; ++a) {
    const int nc = host_ncell[a];
    const std::vector<double>& f = F[a];
    double* out = host_axes + (size_t)a * (max_cells + 1);
    for (int v = 0; v <= nc; ++v) {
      const double target = f[S - 1] * v / nc;
      // the sample interval holding the target, then linear inversion
      int jj = (int)(std::upper_bound(f.begin(), f.end(), target) - f.begin()) - 1;
      jj = std::min(std::max(jj, 0), S - 2);
      const double slope = (t[jj + 1] - t[jj]) / (f[jj + 1] - f[jj]);
      out[v] = slope * (target - f[jj]) + t[jj];
    }
    out[0] = d->lo;
    out[nc] = d->hi;
  }
  if (host_E) *host_E = E;
  return TDFE_OK;
}

}  // namespace

extern "C" {

tdfe_status tdfe_adaptive_axes(const tdfe_adapt_desc* d, void* dev_scratch, size_t scratch_bytes, void* hip_stream,
                               int max_cells, double* host_axes, int* host_ncell, double* host_E) {
  if (!desc_ok(d) || !dev_scratch || !host_axes || !host_ncell || max_cells < 1) return TDFE_EINVAL;
  if (scratch_bytes < scratch_need(d->samples) || (uintptr_t)dev_scratch % 256 != 0) return TDFE_ENOMEM;
  return adaptive_axes_impl(d, dev_scratch, (hipStream_t)hip_stream, max_cells, host_axes, host_ncell, host_E);
}

tdfe_status tdfe_adaptive_axes_static(const tdfe_adapt_desc* d, void* hip_stream, int max_cells, double* host_axes,
                                      int* host_ncell, double* host_E) {
  if (!desc_ok(d) || !host_axes || !host_ncell || max_cells < 1) return TDFE_EINVAL;
  if (scratch_need(d->samples) > TDFE_AXES_STATIC_BYTES) return TDFE_ENOMEM;
  void* ptr = static_scratch();
  if (!ptr) return TDFE_EDEVICE;
  return adaptive_axes_impl(d, ptr, (hipStream_t)hip_stream, max_cells, host_axes, host_ncell, host_E);
}

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// octree leaves following h(r): E from the samples^3 grid as above, g at the
// 27 sample points of every cube of a level on the GPU, split decisions and
// the 2:1 balance on the host
// ------------------------------------------------------------------------------------------------
namespace {

size_t octree_scratch_need(int S, int max_leaves) {
  const size_t pts = (size_t)TDFE_MAX_ATOMS_MESH * 8 * sizeof(double) + (size_t)max_leaves * 27 * 4 * sizeof(double) + 1024;
  return std::max(scratch_need(S), pts);
}

struct LeafKey {
  int q, i, j, k;
  bool operator<(const LeafKey& o) const {
    if (q != o.q) return q < o.q;
    if (i != o.i) return i < o.i;
    if (j != o.j) return j < o.j;
    return k < o.k;
  }
};

}  // namespace

extern "C" {

tdfe_status tdfe_octree_leaves_query(const tdfe_adapt_desc* d, int max_leaves, size_t* bytes) {
  if (!desc_ok(d) || !bytes || max_leaves < 1) return TDFE_EINVAL;
  *bytes = octree_scratch_need(d->samples, max_leaves);
  return TDFE_OK;
}

tdfe_status tdfe_octree_leaves(const tdfe_adapt_desc* d, int n0, int max_level, void* dev_scratch,
                               size_t scratch_bytes, void* hip_stream, int max_leaves, int* host_leaves,
                               int* host_n_leaf, double* host_E) {
  if (!desc_ok(d) || !dev_scratch || !host_leaves || !host_n_leaf || max_leaves < 1) return TDFE_EINVAL;
  if (n0 < 1 || n0 > 64 || max_level < 0 || max_level > 10) return TDFE_EINVAL;
  if (scratch_bytes < octree_scratch_need(d->samples, max_leaves) || (uintptr_t)dev_scratch % 256 != 0)
    return TDFE_ENOMEM;
  hipStream_t st = (hipStream_t)hip_stream;
  const int S = d->samples, p = d->p;
  std::vector<AtomParams> ha(d->n_atoms);
  for (int a = 0; a < d->n_atoms; ++a) {
    for (int c = 0; c < 3; ++c) ha[a].R[c] = d->R[3 * a + c];
    ha[a].Z = d->Z[a];
    ha[a].s = d->s_orb[a];
    ha[a].a = d->a_pot[a];
  }
  // E^3 = (trapezoid integral of g^{3/(p+3)} on the samples) / N_elem
  double E = 0.0;
  {
    double* g = (double*)dev_scratch;
    double* partial = g + (size_t)S * S * S + 3 * (size_t)S;
    AtomParams* atoms = (AtomParams*)(partial + SUM_BLOCKS);
    const double step = (d->hi - d->lo) / (S - 1);
    const int64_t n = (int64_t)S * S * S;
    if (hipMemcpyAsync(atoms, ha.data(), ha.size() * sizeof(AtomParams), hipMemcpyHostToDevice, st) != hipSuccess)
      return TDFE_EDEVICE;
    hipLaunchKernelGGL(size_weight_kernel, dim3((unsigned)((n + MT - 1) / MT)), dim3(MT), 0, st,
                       (const AtomParams*)atoms, d->n_atoms, p, d->lo, step, d->hi, S, g);
    hipLaunchKernelGGL(count_partial_kernel, dim3(SUM_BLOCKS), dim3(MT), 0, st, (const double*)g, S, p, partial);
    if (hipGetLastError() != hipSuccess) return TDFE_EDEVICE;
    std::vector<double> hp(SUM_BLOCKS);
    if (hipMemcpyAsync(hp.data(), partial, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return TDFE_EDEVICE;
    double sum = 0.0;
    for (double v : hp) sum += v;
    E = std::cbrt(sum * step * step * step / d->n_elem);
    if (!(E > 0.0) || !std::isfinite(E)) return TDFE_EINVAL;
  }
  // refinement, level by level
  AtomParams* atoms = (AtomParams*)dev_scratch;
  double* pts = (double*)dev_scratch + (size_t)TDFE_MAX_ATOMS_MESH * 8;
  double* gp = pts + (size_t)max_leaves * 27 * 3;
  if (hipMemcpyAsync(atoms, ha.data(), ha.size() * sizeof(AtomParams), hipMemcpyHostToDevice, st) != hipSuccess)
    return TDFE_EDEVICE;
  std::set<LeafKey> leaves;
  for (int i = 0; i < n0; ++i)
    for (int j = 0; j < n0; ++j)
      for (int k = 0; k < n0; ++k) leaves.insert({0, i, j, k});
  if ((int64_t)leaves.size() > max_leaves) return TDFE_ENOMEM;
  const double frac[3] = {0.0, 0.5, 1.0};
  auto split = [&](const LeafKey& c) {
    leaves.erase(c);
    for (int dd = 0; dd < 8; ++dd)
      leaves.insert({c.q + 1, 2 * c.i + (dd & 1), 2 * c.j + ((dd >> 1) & 1), 2 * c.k + (dd >> 2)});
  };
  for (int q = 0; q < max_level; ++q) {
    std::vector<LeafKey> cells;
    for (const auto& c : leaves)
      if (c.q == q) cells.push_back(c);
    if (cells.empty()) continue;
    const double s = (d->hi - d->lo) / (double)(n0 << q);
    std::vector<double> hpts(cells.size() * 27 * 3);
    for (size_t e = 0; e < cells.size(); ++e) {
      const double org[3] = {d->lo + s * cells[e].i, d->lo + s * cells[e].j, d->lo + s * cells[e].k};
      int m = 0;
      for (int fx = 0; fx < 3; ++fx)
        for (int fy = 0; fy < 3; ++fy)
          for (int fz = 0; fz < 3; ++fz, ++m) {
            hpts[(e * 27 + m) * 3 + 0] = org[0] + s * frac[fx];
            hpts[(e * 27 + m) * 3 + 1] = org[1] + s * frac[fy];
            hpts[(e * 27 + m) * 3 + 2] = org[2] + s * frac[fz];
          }
    }
    const int64_t np = (int64_t)cells.size() * 27;
    std::vector<double> hg(np);
    if (hipMemcpyAsync(pts, hpts.data(), hpts.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess)
      return TDFE_EDEVICE;
    hipLaunchKernelGGL(point_weight_kernel, dim3((unsigned)((np + MT - 1) / MT)), dim3(MT), 0, st,
                       (const AtomParams*)atoms, d->n_atoms, p, (const double*)pts, np, gp);
    if (hipGetLastError() != hipSuccess) return TDFE_EDEVICE;
    if (hipMemcpyAsync(hg.data(), gp, np * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return TDFE_EDEVICE;
    for (size_t e = 0; e < cells.size(); ++e) {
      double gmax = 0.0;
      for (int m = 0; m < 27; ++m) gmax = std::max(gmax, hg[e * 27 + m]);
      const double h = gmax > 0.0 ? E * std::pow(gmax, -1.0 / (p + 3)) : INFINITY;
      if (s > h) {
        if ((int64_t)leaves.size() + 7 > max_leaves) return TDFE_ENOMEM;
        split(cells[e]);
      }
    }
  }
  // 2:1 balance across faces, edges and corners
  while (true) {
    std::set<LeafKey> to_split;
    for (const auto& c : leaves) {
      if (c.q < 2) continue;
      const int nm = n0 << c.q;
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            if (!dx && !dy && !dz) continue;
            const int a = c.i + dx, b = c.j + dy, cc = c.k + dz;
            if (a < 0 || b < 0 || cc < 0 || a >= nm || b >= nm || cc >= nm) continue;
            for (int q = c.q - 2; q >= 0; --q) {
              const int sh = c.q - q;
              const LeafKey anc{q, a >> sh, b >> sh, cc >> sh};
              if (leaves.count(anc)) {
                to_split.insert(anc);
                break;
              }
            }
          }
    }
    if (to_split.empty()) break;
    if ((int64_t)leaves.size() + 7 * (int64_t)to_split.size() > max_leaves) return TDFE_ENOMEM;
    for (const auto& c : to_split) split(c);
  }
  int64_t m = 0;
  for (const auto& c : leaves) {
    host_leaves[4 * m + 0] = c.q;
    host_leaves[4 * m + 1] = c.i;
    host_leaves[4 * m + 2] = c.j;
    host_leaves[4 * m + 3] = c.k;
    ++m;
  }
  *host_n_leaf = (int)m;
  if (host_E) *host_E = E;
  return TDFE_OK;
}

}  // extern "C"
