// Octree meshes with hanging nodes (Sec. "Efficient spatio-temporal
// discretization": adaptive hexahedra that follow the element size
// h(r) = E g(r)^(-1/(p+3)) of Eq. OptimalMeshSize).
//
// Host (set-up): the GLL nodes of all leaves are merged by position; a node
// on the closed boundary of a leaf that does not own it takes that leaf's
// polynomial value there (tensor Lagrange interpolant of the leaf's nodes,
// non-zero only on its face or edge nodes), chains are substituted, masters
// on the domain boundary drop out.  C maps DoF values to every node.  The
// overlap is lumped by rows, M_d = sum_m C_md N_m with N_m the GLL-rule mass
// of node m, so that Hbar = M^-1/2 C^T H_nodes C M^-1/2 (Eq.
// TDKSMatVecStandard) keeps a diagonal M.
//
// Device (every operator application, Eq. DiscreteHamiltonian), with C
// split into its identity rows (DoF nodes) and the rows of hanging nodes:
//   hexpand  xh = C_h (cs M^-1/2 x)           one thread per (hanging node, column)
//   cells    per cube: gather DoF nodes from x (x cs M^-1/2), hanging nodes
//            from xh, boundary nodes 0; H_e; scatter-add DoF nodes onto y
//            (x M^-1/2), hanging nodes onto yh
//   hreduce  y += M^-1/2 C_h^T yh             one thread per (master DoF, column)
// The density expands every node (xf = C cs M^-1/2 x) and interpolates from xf.
// The cell kernel keeps the cube's values in LDS and runs one 1D contraction
// per thread and pass (x, y, z interpolation to the Gauss points, collocation
// derivatives there, the diagonal metric of a cube, transposed passes back);
// the quadratic form per column gives the Lanczos alpha as on other meshes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <unordered_map>
#include <unordered_set>

#include "tdfe_fold.h"
#include "tdfe_internal.h"

namespace {

// ------------------------------------------------------------------------------------------------
// host: merged nodes, constraints, lumped overlap
// ------------------------------------------------------------------------------------------------
struct K3 {
  int64_t x, y, z;
  bool operator==(const K3& o) const { return x == o.x && y == o.y && z == o.z; }
  bool operator<(const K3& o) const { return x != o.x ? x < o.x : (y != o.y ? y < o.y : z < o.z); }
};
struct K3Hash {
  size_t operator()(const K3& k) const {
    uint64_t h = (uint64_t)k.x * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)k.y + 0x7F4A7C159E3779B9ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)k.z + 0x94D049BB133111EBull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

// leaf (q, i, j, k) as one integer key (q <= 10, indices < 64 * 2^10)
inline uint64_t leaf_key(int q, int64_t i, int64_t j, int64_t k) {
  return ((uint64_t)q << 60) | ((uint64_t)i << 40) | ((uint64_t)j << 20) | (uint64_t)k;
}

// l_m(t) for the GLL nodes xi[0..n-1], product form
void lagrange_at(const double* xi, int n, double t, double* out) {
  for (int m = 0; m < n; ++m) {
    double v = 1.0;
    for (int r = 0; r < n; ++r)
      if (r != m) v *= (t - xi[r]) / (xi[m] - xi[r]);
    out[m] = v;
  }
}

constexpr double KEY_SCALE = 16777216.0;  // lattice positions are keyed at 2^-24 lattice units

tdfe_status build_octree(tdfe_ctx* c, const tdfe_octree_desc* d) {
  const int n = c->n, L = d->max_level;
  const int64_t top = (int64_t)d->n0 << L;  // lattice units per axis
  const int64_t nl = d->n_leaf;
  std::unordered_set<uint64_t> leafset;
  leafset.reserve((size_t)nl * 2);
  int64_t vol = 0;
  for (int64_t e = 0; e < nl; ++e) {
    const int* r = d->leaves + 4 * e;
    const int q = r[0];
    if (q < 0 || q > L) return tdfe_fail(c, TDFE_EINVAL, "octree: leaf %lld has level %d", (long long)e, q);
    const int64_t lim = (int64_t)d->n0 << q;
    for (int a = 1; a < 4; ++a)
      if (r[a] < 0 || r[a] >= lim) return tdfe_fail(c, TDFE_EINVAL, "octree: leaf %lld out of range", (long long)e);
    if (!leafset.insert(leaf_key(q, r[1], r[2], r[3])).second)
      return tdfe_fail(c, TDFE_EINVAL, "octree: leaf %lld repeated", (long long)e);
    vol += (int64_t)1 << (3 * (L - q));
  }
  for (int64_t e = 0; e < nl; ++e) {
    const int* r = d->leaves + 4 * e;
    for (int q = r[0] - 1; q >= 0; --q) {
      const int sh = r[0] - q;
      if (leafset.count(leaf_key(q, r[1] >> sh, r[2] >> sh, r[3] >> sh)))
        return tdfe_fail(c, TDFE_EINVAL, "octree: leaf %lld lies inside another leaf", (long long)e);
    }
  }
  if (vol != top * top * top) return tdfe_fail(c, TDFE_EINVAL, "octree: the leaves do not tile the domain");
  // balance: no neighbour (face, edge, corner) two or more levels coarser
  for (int64_t e = 0; e < nl; ++e) {
    const int* r = d->leaves + 4 * e;
    const int m = r[0];
    const int64_t nm = (int64_t)d->n0 << m;
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          if (!dx && !dy && !dz) continue;
          const int64_t a = r[1] + dx, b = r[2] + dy, cc = r[3] + dz;
          if (a < 0 || b < 0 || cc < 0 || a >= nm || b >= nm || cc >= nm) continue;
          for (int q = m - 2; q >= 0; --q) {
            const int sh = m - q;
            if (leafset.count(leaf_key(q, a >> sh, b >> sh, cc >> sh)))
              return tdfe_fail(c, TDFE_EINVAL, "octree: leaves %d levels apart share a boundary", m - q);
          }
        }
  }

  // merged nodes: lattice positions keyed at 2^-24 lattice units
  const int n3 = n * n * n;
  std::unordered_map<K3, int64_t, K3Hash> id;
  id.reserve((size_t)nl * n3);
  std::vector<K3> keys;
  std::vector<double> pos;  // lattice position of every node (from the first cell that has it)
  std::vector<int64_t> cn((size_t)nl * n3);
  std::vector<int> own_level;
  for (int64_t e = 0; e < nl; ++e) {
    const int* r = d->leaves + 4 * e;
    const double S = (double)((int64_t)1 << (L - r[0]));
    double loc[3][TDFE_MAXN];
    for (int a = 0; a < 3; ++a)
      for (int m = 0; m < n; ++m) loc[a][m] = (double)r[1 + a] * S + S * (1.0 + c->xi[m]) / 2.0;
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          const double P[3] = {loc[0][i], loc[1][j], loc[2][k]};
          const K3 kk{std::llround(P[0] * KEY_SCALE), std::llround(P[1] * KEY_SCALE), std::llround(P[2] * KEY_SCALE)};
          auto it = id.find(kk);
          int64_t v;
          if (it == id.end()) {
            v = (int64_t)keys.size();
            id.emplace(kk, v);
            keys.push_back(kk);
            pos.insert(pos.end(), P, P + 3);
            own_level.push_back(r[0]);
          } else {
            v = it->second;
            own_level[v] = std::max(own_level[v], r[0]);
          }
          cn[(size_t)e * n3 + (k * n + j) * n + i] = v;
        }
  }
  // node numbering by position (x slowest, z fastest)
  const int64_t nn = (int64_t)keys.size();
  if (nn > ((int64_t)1 << 31) - 2) return tdfe_fail(c, TDFE_EINVAL, "octree: too many nodes");
  std::vector<int64_t> order(nn);
  for (int64_t v = 0; v < nn; ++v) order[v] = v;
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return keys[a] < keys[b]; });
  std::vector<int64_t> rank(nn);
  for (int64_t r = 0; r < nn; ++r) rank[order[r]] = r;
  std::vector<double> npos(3 * (size_t)nn);
  std::vector<int> nlev(nn);
  std::vector<char> bnd(nn);
  const int64_t topkey = top * (int64_t)KEY_SCALE;
  for (int64_t v = 0; v < nn; ++v) {
    const int64_t r = rank[v];
    for (int a = 0; a < 3; ++a) npos[3 * r + a] = pos[3 * v + a];
    nlev[r] = own_level[v];
    const K3& k = keys[v];
    bnd[r] = (k.x == 0 || k.y == 0 || k.z == 0 || k.x == topkey || k.y == topkey || k.z == topkey) ? 1 : 0;
  }
  for (auto& v : cn) v = rank[v];
  std::vector<int64_t> leaf_of;  // leaf key -> cell index
  std::unordered_map<uint64_t, int64_t> cell_of;
  cell_of.reserve((size_t)nl * 2);
  for (int64_t e = 0; e < nl; ++e) {
    const int* r = d->leaves + 4 * e;
    cell_of.emplace(leaf_key(r[0], r[1], r[2], r[3]), e);
  }

  // raw constraints of hanging nodes: the first leaf (coarsest level first,
  // then the 8 candidate cells around the point) whose closed box holds the
  // node without owning it
  std::vector<std::vector<std::pair<int64_t, double>>> raw(nn);
  std::vector<char> hang(nn, 0);
  double lx[TDFE_MAXN], ly[TDFE_MAXN], lz[TDFE_MAXN];
  for (int64_t v = 0; v < nn; ++v) {
    if (bnd[v]) continue;
    const double* x = &npos[3 * v];
    bool found = false;
    for (int q = 0; q < nlev[v] && !found; ++q) {
      const double Sq = (double)((int64_t)1 << (L - q));
      const int64_t nq_ = (int64_t)d->n0 << q;
      int64_t lo_i[3], hi_i[3];
      for (int a = 0; a < 3; ++a) {
        lo_i[a] = (int64_t)std::floor((x[a] - 1e-7) / Sq);
        hi_i[a] = (int64_t)std::floor((x[a] + 1e-7) / Sq);
      }
      for (int combo = 0; combo < 8 && !found; ++combo) {
        int64_t ix[3];
        bool in = true;
        for (int a = 0; a < 3; ++a) {
          ix[a] = ((combo >> a) & 1) ? hi_i[a] : lo_i[a];
          if (ix[a] < 0 || ix[a] >= nq_) in = false;
        }
        if (!in) continue;
        auto it = cell_of.find(leaf_key(q, ix[0], ix[1], ix[2]));
        if (it == cell_of.end()) continue;
        double ref[3];
        bool owned = true, on_face = false;
        for (int a = 0; a < 3; ++a) {
          ref[a] = 2.0 * (x[a] - (double)ix[a] * Sq) / Sq - 1.0;
          double best = 1e300;
          for (int m = 0; m < n; ++m) best = std::min(best, std::fabs(c->xi[m] - ref[a]));
          if (best >= 1e-9) owned = false;
          if (std::fabs(ref[a]) == 1.0) on_face = true;
        }
        if (owned) continue;
        if (!on_face) return tdfe_fail(c, TDFE_EINVAL, "octree: a node lies inside a leaf that does not own it");
        lagrange_at(c->xi, n, ref[0], lx);
        lagrange_at(c->xi, n, ref[1], ly);
        lagrange_at(c->xi, n, ref[2], lz);
        const int64_t ce = it->second;
        // the oracle's order: (i, j, k) with k fastest
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
              const double wgt = lx[i] * ly[j] * lz[k];
              if (wgt != 0.0) raw[v].push_back({cn[(size_t)ce * n3 + (k * n + j) * n + i], wgt});
            }
        hang[v] = 1;
        found = true;
      }
    }
  }
  // DoFs: interior nodes that are not hanging, in node order
  std::vector<int64_t> dof_of(nn, -1);
  int64_t ndof = 0;
  for (int64_t v = 0; v < nn; ++v)
    if (!bnd[v] && !hang[v]) dof_of[v] = ndof++;
  if (ndof < 1) return tdfe_fail(c, TDFE_EINVAL, "octree: no degree of freedom");
  // substitute chains; boundary masters carry 0
  std::vector<std::map<int64_t, double>> res(nn);
  std::vector<char> done(nn, 0);
  std::function<const std::map<int64_t, double>&(int64_t)> expand = [&](int64_t v) -> const std::map<int64_t, double>& {
    if (done[v]) return res[v];
    std::map<int64_t, double> acc;
    for (const auto& mw : raw[v]) {
      if (bnd[mw.first]) continue;
      if (hang[mw.first]) {
        for (const auto& kv : expand(mw.first)) acc[kv.first] += mw.second * kv.second;
      } else {
        acc[dof_of[mw.first]] += mw.second;
      }
    }
    res[v] = std::move(acc);
    done[v] = 1;
    return res[v];
  };
  c->oct_eptr_h.assign(nn + 1, 0);
  c->oct_ecol_h.clear();
  c->oct_eval_h.clear();
  int64_t nh = 0;
  for (int64_t v = 0; v < nn; ++v) {
    if (dof_of[v] >= 0) {
      c->oct_ecol_h.push_back((int)dof_of[v]);
      c->oct_eval_h.push_back(1.0);
    } else if (hang[v]) {
      ++nh;
      for (const auto& kv : expand(v)) {
        c->oct_ecol_h.push_back((int)kv.first);
        c->oct_eval_h.push_back(kv.second);
      }
    }
    c->oct_eptr_h[v + 1] = (int)c->oct_ecol_h.size();
  }
  if ((int64_t)c->oct_ecol_h.size() > ((int64_t)1 << 31) - 2) return tdfe_fail(c, TDFE_EINVAL, "octree: C too large");
  // unconstrained GLL mass of every node, then the row-sum lumped overlap
  const double unit = (d->hi - d->lo) / (double)top;
  std::vector<double> Mn(nn, 0.0);
  c->oct_s_h.resize(nl);
  for (int64_t e = 0; e < nl; ++e) {
    const double s = (double)((int64_t)1 << (L - d->leaves[4 * e])) * unit;
    c->oct_s_h[e] = s;
    const double det = (s / 2.0) * (s / 2.0) * (s / 2.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k)
          Mn[cn[(size_t)e * n3 + (k * n + j) * n + i]] += c->w[i] * c->w[j] * c->w[k] * det;
  }
  c->oct_m_h.assign(ndof, 0.0);
  for (int64_t v = 0; v < nn; ++v)
    for (int j = c->oct_eptr_h[v]; j < c->oct_eptr_h[v + 1]; ++j) c->oct_m_h[c->oct_ecol_h[j]] += c->oct_eval_h[j] * Mn[v];
  for (int64_t dd = 0; dd < ndof; ++dd)
    if (!(c->oct_m_h[dd] > 0.0)) return tdfe_fail(c, TDFE_EINVAL, "octree: lumped overlap not positive");
  c->oct_dofxyz_h.assign(3 * (size_t)ndof, 0.0);
  for (int64_t v = 0; v < nn; ++v)
    if (dof_of[v] >= 0)
      for (int a = 0; a < 3; ++a) c->oct_dofxyz_h[3 * dof_of[v] + a] = d->lo + npos[3 * v + a] * unit;
  // Gauss points and weights of every cube
  const int nq = c->nq, nq3 = nq * nq * nq;
  c->oct_xq_h.assign((size_t)nl * nq3 * 3, 0.0);
  c->oct_wdet_h.assign((size_t)nl * nq3, 0.0);
  for (int64_t e = 0; e < nl; ++e) {
    const int* r = d->leaves + 4 * e;
    const double s = c->oct_s_h[e];
    const double det = (s / 2.0) * (s / 2.0) * (s / 2.0);
    const double o[3] = {d->lo + (double)r[1] * s, d->lo + (double)r[2] * s, d->lo + (double)r[3] * s};
    for (int cc = 0; cc < nq; ++cc)
      for (int b = 0; b < nq; ++b)
        for (int a = 0; a < nq; ++a) {
          const size_t g = (size_t)e * nq3 + a + nq * (b + nq * cc);
          c->oct_xq_h[3 * g + 0] = o[0] + s * (1.0 + c->eta[a]) / 2.0;
          c->oct_xq_h[3 * g + 1] = o[1] + s * (1.0 + c->eta[b]) / 2.0;
          c->oct_xq_h[3 * g + 2] = o[2] + s * (1.0 + c->eta[cc]) / 2.0;
          c->oct_wdet_h[g] = c->wq[a] * c->wq[b] * c->wq[cc] * det;
        }
  }
  c->oct_cn_h.resize(cn.size());
  for (size_t i = 0; i < cn.size(); ++i) c->oct_cn_h[i] = (int)cn[i];
  // the operator's slot codes and the hanging rows of C^T by master DoF
  std::vector<int64_t> hidx(nn, -1);
  c->oct_hv_h.clear();
  for (int64_t v = 0; v < nn; ++v)
    if (hang[v] && c->oct_eptr_h[v + 1] > c->oct_eptr_h[v]) {
      hidx[v] = (int64_t)c->oct_hv_h.size();
      c->oct_hv_h.push_back((int)v);
    }
  c->oct_cd_h.resize(cn.size());
  for (size_t i = 0; i < cn.size(); ++i) {
    const int64_t v = cn[i];
    c->oct_cd_h[i] = dof_of[v] >= 0 ? (int)dof_of[v] : (hidx[v] >= 0 ? (int)(-2 - hidx[v]) : -1);
  }
  {
    std::vector<int> cnt(ndof, 0);
    for (const int v : c->oct_hv_h)
      for (int j = c->oct_eptr_h[v]; j < c->oct_eptr_h[v + 1]; ++j) ++cnt[c->oct_ecol_h[j]];
    std::vector<int> slot(ndof, -1);
    c->oct_md_h.clear();
    c->oct_mptr_h.assign(1, 0);
    for (int64_t dd = 0; dd < ndof; ++dd)
      if (cnt[dd] > 0) {
        slot[dd] = (int)c->oct_md_h.size();
        c->oct_md_h.push_back((int)dd);
        c->oct_mptr_h.push_back(c->oct_mptr_h.back() + cnt[dd]);
      }
    c->oct_mh_h.assign(c->oct_mptr_h.back(), 0);
    c->oct_mv_h.assign(c->oct_mptr_h.back(), 0.0);
    std::vector<int> fill(c->oct_mptr_h.begin(), c->oct_mptr_h.end() - 1);
    for (size_t h = 0; h < c->oct_hv_h.size(); ++h) {
      const int v = c->oct_hv_h[h];
      for (int j = c->oct_eptr_h[v]; j < c->oct_eptr_h[v + 1]; ++j) {
        const int k = slot[c->oct_ecol_h[j]];
        c->oct_mh_h[fill[k]] = (int)h;
        c->oct_mv_h[fill[k]] = c->oct_eval_h[j];
        ++fill[k];
      }
    }
  }
  c->n_nodes = nn;
  c->n_dof = ndof;
  c->oct_hanging = nh;
  return TDFE_OK;
}

// ------------------------------------------------------------------------------------------------
// device kernels
// ------------------------------------------------------------------------------------------------
constexpr int EW = 256;

// xf[v][col] = sum_j C_vj (cs M^-1/2 x)_j; yf = 0
__global__ void __launch_bounds__(EW)
    oct_expand_kernel(const double* __restrict__ x, int ld, int cols, const double* colscale,
                      const double* __restrict__ minv, const int* __restrict__ eptr, const int* __restrict__ ecol,
                      const double* __restrict__ eval, int64_t nn, int W, double* __restrict__ xf,
                      double* __restrict__ yf, const int* done) {
  if (done && *done) return;
  const int64_t idx = (int64_t)blockIdx.x * EW + threadIdx.x;
  if (idx >= nn * cols) return;
  const int64_t v = idx / cols;
  const int col = (int)(idx % cols);
  double acc = 0.0;
  for (int j = eptr[v]; j < eptr[v + 1]; ++j) {
    const int dd = ecol[j];
    acc += eval[j] * (minv ? minv[dd] : 1.0) * x[(int64_t)dd * ld + col];
  }
  if (colscale) acc *= colscale[col >> 1];
  xf[v * W + col] = acc;
  if (yf) yf[v * W + col] = 0.0;
}

// the hanging nodes' values for the operator: xh[h][col] = sum_j C_vj (cs
// M^-1/2 x)_j for v = hv[h]; yh[h][col] = 0
__global__ void __launch_bounds__(EW)
    oct_hexpand_kernel(const double* __restrict__ x, int ld, int cols, const double* colscale,
                       const double* __restrict__ minv, const int* __restrict__ hv, const int* __restrict__ eptr,
                       const int* __restrict__ ecol, const double* __restrict__ eval, int64_t nh, int W,
                       double* __restrict__ xh, double* __restrict__ yh, const int* done) {
  if (done && *done) return;
  const int64_t idx = (int64_t)blockIdx.x * EW + threadIdx.x;
  if (idx >= nh * cols) return;
  const int64_t h = idx / cols;
  const int col = (int)(idx % cols);
  const int v = hv[h];
  // four independent partial sums keep four rows' loads in flight
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int j0 = eptr[v], j1 = eptr[v + 1];
  int j = j0;
  for (; j + 4 <= j1; j += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int dd = ecol[j + u];
      acc[u] += eval[j + u] * (minv ? minv[dd] : 1.0) * x[(int64_t)dd * ld + col];
    }
  }
  for (; j < j1; ++j) {
    const int dd = ecol[j];
    acc[0] += eval[j] * (minv ? minv[dd] : 1.0) * x[(int64_t)dd * ld + col];
  }
  double sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  if (colscale) sum *= colscale[col >> 1];
  xh[h * W + col] = sum;
  yh[h * W + col] = 0.0;
}

// y[d][col] += M^-1/2_d sum_h C_hd yh[h][col] over the master DoFs of hanging nodes
__global__ void __launch_bounds__(EW)
    oct_hreduce_kernel(double* __restrict__ y, int ld, int cols, const double* __restrict__ minv,
                       const int* __restrict__ mptr, const int* __restrict__ md, const int* __restrict__ mh,
                       const double* __restrict__ mv, int64_t nmd, int W, const double* __restrict__ yh,
                       const int* done) {
  if (done && *done) return;
  const int64_t idx = (int64_t)blockIdx.x * EW + threadIdx.x;
  if (idx >= nmd * cols) return;
  const int64_t k = idx / cols;
  const int col = (int)(idx % cols);
  // four independent partial sums keep four rows' loads in flight
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int j0 = mptr[k], j1 = mptr[k + 1];
  int j = j0;
  for (; j + 4 <= j1; j += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += mv[j + u] * yh[(int64_t)mh[j + u] * W + col];
  }
  for (; j < j1; ++j) acc[0] += mv[j] * yh[(int64_t)mh[j] * W + col];
  const int dd = md[k];
  y[(int64_t)dd * ld + col] += (minv ? minv[dd] : 1.0) * ((acc[0] + acc[1]) + (acc[2] + acc[3]));
}

// one 1D pass: the thread's line along axis AX of src, times the folded
// table F (symmetry S), into dst (added when ADD)
template <int N, int CB, int AX, int S, bool ADD>
__device__ __forceinline__ void line_pass(const double* src, double* dst, const Folded<double>& F, int line, int col) {
  const int u = line % N, w = line / N;
  auto at = [&](int m) {
    const int x = AX == 0 ? m : u;
    const int y = AX == 0 ? u : (AX == 1 ? m : w);
    const int z = AX == 2 ? m : w;
    return ((z * N + y) * N + x) * CB + col;
  };
  double in[N], out[N];
#pragma unroll
  for (int m = 0; m < N; ++m) in[m] = src[at(m)];
  eo<double, N, S>(F, in, out);
#pragma unroll
  for (int m = 0; m < N; ++m) {
    if constexpr (ADD)
      dst[at(m)] += out[m];
    else
      dst[at(m)] = out[m];
  }
}

struct OctCellParams {
  const double* x;         // DoF input, [n_dof][ld] from the launch's first column
  double* y;               // DoF output (accumulated), same layout
  int ld;
  const double* minv;      // M^-1/2 per DoF or null
  const double* colscale;  // per orbital of the launch or null
  const double* xh;        // hanging-node input [n_h][W]
  double* yh;              // hanging-node output [n_h][W]
  int W, cols, cols_total, col0, nchunks;
  const int* cd;      // [n_cell][n^3] slot codes
  const double* s;    // [n_cell]
  const double* vw;   // [n_cell][nq^3] or null
  double kin;
  double* energy;     // [n_cell][cols_total] or null
  const int* done;
  int64_t n_cell;
};

// yf += H_e xf_e for the columns of one block; quadratic form per column
template <int N, int CB>
__global__ void __launch_bounds__(N* N* CB) oct_cell_kernel(OctCellParams P) {
  constexpr int VOL = N * N * N;
  constexpr int T = N * N * CB;
  constexpr FoldSet<N> FS = make_foldset<N>();
  __shared__ double sQ[VOL * CB], sT[VOL * CB], sR[VOL * CB];
  __shared__ double sRed[T];
  if (P.done && *P.done) return;
  const int t = threadIdx.x;
  const int col = t % CB, line = t / CB;
  const int64_t cell = blockIdx.x / P.nchunks;
  const int chunk = blockIdx.x % P.nchunks;
  const int colg = chunk * CB + col;
  const bool ok = colg < P.cols;
  // the cube's slot codes and per-slot M^-1/2, staged once per block
  __shared__ int sCode[VOL];
  __shared__ double sM[VOL];
  for (int q = t; q < VOL; q += T) {
    const int cq = P.cd[cell * VOL + q];
    sCode[q] = cq;
    sM[q] = (cq >= 0 && P.minv) ? P.minv[cq] : 1.0;
  }
  __syncthreads();
  auto L = [&](int x, int y, int z) { return ((z * N + y) * N + x) * CB + col; };
  const int cg = ok ? colg : 0;
  // gather: the thread's x-line (y, z) = (line % N, line / N); DoFs straight
  // from the input (x M^-1/2 x column scale), hanging nodes from their
  // expanded values, boundary nodes 0
  {
    const int y = line % N, z = line / N;
    const double cs = P.colscale ? P.colscale[cg >> 1] : 1.0;
    double v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int q = sCode[(z * N + y) * N + i];
      double val = 0.0;
      if (q >= 0)
        val = P.x[(int64_t)q * P.ld + cg] * (sM[(z * N + y) * N + i] * cs);
      else if (q <= -2)
        val = P.xh[(int64_t)(-2 - q) * P.W + cg];
      v[i] = val;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) sQ[L(i, y, z)] = ok ? v[i] : 0.0;
  }
  __syncthreads();
  line_pass<N, CB, 0, 1, false>(sQ, sT, FS.B, line, col);
  __syncthreads();
  line_pass<N, CB, 1, 1, false>(sT, sQ, FS.B, line, col);
  __syncthreads();
  line_pass<N, CB, 2, 1, false>(sQ, sT, FS.B, line, col);  // sT: u at the Gauss points
  __syncthreads();
  const double half_s = 0.5 * P.s[cell];
  double energy = 0.0;
  // per direction: collocation derivative, flux kin w_q s/2 d_u, energy,
  // transposed derivative accumulated into sR
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    {
      const int u = line % N, w = line / N;
      double in[N], dv[N];
#pragma unroll
      for (int m = 0; m < N; ++m) {
        const int x = ax == 0 ? m : u, y = ax == 0 ? u : (ax == 1 ? m : w), z = ax == 2 ? m : w;
        in[m] = sT[L(x, y, z)];
      }
      eo<double, N, -1>(FS.G, in, dv);
#pragma unroll
      for (int m = 0; m < N; ++m) {
        const int x = ax == 0 ? m : u, y = ax == 0 ? u : (ax == 1 ? m : w), z = ax == 2 ? m : w;
        const double cq = P.kin * FS.wq[x] * FS.wq[y] * FS.wq[z] * half_s;
        const double f = cq * dv[m];
        energy += f * dv[m];
        sQ[L(x, y, z)] = f;
      }
    }
    __syncthreads();
    if (ax == 0) line_pass<N, CB, 0, -1, false>(sQ, sR, FS.Gt, line, col);
    if (ax == 1) line_pass<N, CB, 1, -1, true>(sQ, sR, FS.Gt, line, col);
    if (ax == 2) line_pass<N, CB, 2, -1, true>(sQ, sR, FS.Gt, line, col);
    __syncthreads();
  }
  // potential term on the thread's x-line of Gauss points
  if (P.vw) {
    const int y = line % N, z = line / N;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      const double uq = sT[L(a, y, z)];
      const double pot = P.vw[cell * VOL + a + N * (y + N * z)] * uq;
      energy += pot * uq;
      sR[L(a, y, z)] += pot;
    }
  }
  __syncthreads();
  line_pass<N, CB, 2, 1, false>(sR, sQ, FS.Bt, line, col);
  __syncthreads();
  line_pass<N, CB, 1, 1, false>(sQ, sT, FS.Bt, line, col);
  __syncthreads();
  {
    const int y = line % N, z = line / N;
    double in[N], out[N];
#pragma unroll
    for (int a = 0; a < N; ++a) in[a] = sT[L(a, y, z)];
    eo<double, N, 1>(FS.Bt, in, out);
    if (ok) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int q = sCode[(z * N + y) * N + i];
        if (q >= 0)
          unsafeAtomicAdd(P.y + (int64_t)q * P.ld + colg, out[i] * sM[(z * N + y) * N + i]);
        else if (q <= -2)
          unsafeAtomicAdd(P.yh + (int64_t)(-2 - q) * P.W + colg, out[i]);
      }
    }
  }
  if (P.energy) {
    sRed[t] = ok ? energy : 0.0;
    __syncthreads();
    if (t < CB && chunk * CB + t < P.cols) {
      double acc = 0.0;
      for (int l = 0; l < N * N; ++l) acc += sRed[l * CB + t];
      P.energy[cell * P.cols_total + P.col0 + chunk * CB + t] = acc;
    }
  }
}

struct OctDensParams {
  const double* xf;  // expanded orbitals (M^-1/2 applied), [n_nodes][W]
  int W, cols, col0;
  const int* cn;
  const double* occ;  // [n_orb] (indexed by global column / 2)
  const double* wdet;
  const double* xq;
  double* rho;
  double* partial;  // [n_cell][4] (last chunk only)
  int accumulate, last;
  int64_t n_cell;
};

// rho at the Gauss points from one chunk of columns, the 4 partial sums
// (charge, dipole) of the complete rho on the last chunk
template <int N, int CB>
__global__ void __launch_bounds__(N* N* CB) oct_density_kernel(OctDensParams P) {
  constexpr int VOL = N * N * N;
  constexpr int T = N * N * CB;
  constexpr FoldSet<N> FS = make_foldset<N>();
  __shared__ double sQ[VOL * CB], sT[VOL * CB];
  __shared__ double sRed[T * 4 > VOL ? T * 4 : VOL];
  const int t = threadIdx.x;
  const int col = t % CB, line = t / CB;
  const int64_t cell = blockIdx.x;
  const int* cnode = P.cn + cell * VOL;
  auto L = [&](int x, int y, int z) { return ((z * N + y) * N + x) * CB + col; };
  double racc[N];
#pragma unroll
  for (int a = 0; a < N; ++a) racc[a] = 0.0;
  for (int c0 = 0; c0 < P.cols; c0 += CB) {
    const int cg = c0 + col;
    const bool ok = cg < P.cols;
    {
      const int y = line % N, z = line / N;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const double v = P.xf[(int64_t)cnode[(z * N + y) * N + i] * P.W + (ok ? cg : 0)];
        sQ[L(i, y, z)] = ok ? v : 0.0;
      }
    }
    __syncthreads();
    line_pass<N, CB, 0, 1, false>(sQ, sT, FS.B, line, col);
    __syncthreads();
    line_pass<N, CB, 1, 1, false>(sT, sQ, FS.B, line, col);
    __syncthreads();
    {
      // z-line (x, y) of Gauss points
      const int x = line % N, y = line / N;
      double in[N], out[N];
#pragma unroll
      for (int m = 0; m < N; ++m) in[m] = sQ[L(x, y, m)];
      eo<double, N, 1>(FS.B, in, out);
      const double f = ok ? P.occ[(P.col0 + cg) >> 1] : 0.0;
#pragma unroll
      for (int m = 0; m < N; ++m) racc[m] += f * out[m] * out[m];
    }
    __syncthreads();
  }
  // sum over the column lanes
  {
    const int x = line % N, y = line / N;
#pragma unroll
    for (int m = 0; m < N; ++m) sQ[L(x, y, m)] = racc[m];
  }
  __syncthreads();
  for (int q = t; q < VOL; q += T) {
    double s = 0.0;
    for (int cc = 0; cc < CB; ++cc) s += sQ[q * CB + cc];
    const int64_t g = cell * VOL + q;
    const double r = (P.accumulate ? P.rho[g] : 0.0) + s;
    P.rho[g] = r;
  }
  if (!P.last) return;
  __syncthreads();  // every rho of the cell written by this block
  double vals[4] = {0, 0, 0, 0};
  for (int q = t; q < VOL; q += T) {
    const int64_t g = cell * VOL + q;
    const double wr = P.wdet[g] * P.rho[g];
    vals[0] += wr;
    vals[1] += wr * P.xq[3 * g + 0];
    vals[2] += wr * P.xq[3 * g + 1];
    vals[3] += wr * P.xq[3 * g + 2];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) sRed[t * 4 + v] = vals[v];
  __syncthreads();
  if (t < 4) {
    double acc = 0.0;
    for (int u = 0; u < T; ++u) acc += sRed[u * 4 + t];
    P.partial[cell * 4 + t] = acc;
  }
}

// columns per block and their LDS: three (two) cell arrays of CB columns
constexpr int oct_cb(int N) { return N <= 5 ? 16 : (N <= 7 ? 8 : 4); }

template <int N>
tdfe_status launch_cells(tdfe_ctx* c, OctCellParams& P) {
  constexpr int CB = oct_cb(N);
  static_assert(3 * N * N * N * CB * 8 + N * N * CB * 8 + N * N * N * 12 <= 160 * 1024, "LDS");
  P.nchunks = (P.cols + CB - 1) / CB;
  hipLaunchKernelGGL((oct_cell_kernel<N, CB>), dim3((unsigned)(c->n_cell * P.nchunks)), dim3(N * N * CB), 0,
                     c->stream, P);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

template <int N>
tdfe_status launch_dens(tdfe_ctx* c, OctDensParams& P) {
  constexpr int CB = oct_cb(N);
  hipLaunchKernelGGL((oct_density_kernel<N, CB>), dim3((unsigned)c->n_cell), dim3(N * N * CB), 0, c->stream, P);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

#define OCT_DISPATCH(fn, c, P)                     \
  switch ((c)->n) {                                \
    case 2: return fn<2>(c, P);                    \
    case 3: return fn<3>(c, P);                    \
    case 4: return fn<4>(c, P);                    \
    case 5: return fn<5>(c, P);                    \
    case 6: return fn<6>(c, P);                    \
    case 7: return fn<7>(c, P);                    \
    case 8: return fn<8>(c, P);                    \
    case 9: return fn<9>(c, P);                    \
  }                                                \
  return tdfe_fail(c, TDFE_EINVAL, "octree: unsupported order p=%d", (c)->p);

tdfe_status cells_launch(tdfe_ctx* c, OctCellParams& P) { OCT_DISPATCH(launch_cells, c, P) }
tdfe_status dens_launch(tdfe_ctx* c, OctDensParams& P) { OCT_DISPATCH(launch_dens, c, P) }

inline unsigned nblk(int64_t n) { return (unsigned)((n + EW - 1) / EW); }

}  // namespace

tdfe_status tdfe_launch_apply_octree(tdfe_ctx* c, const ApplyArgs& a) {
  if (a.fp32) return tdfe_fail(c, TDFE_EINVAL, "octree meshes run in FP64");
  if (a.fullgrid) return tdfe_fail(c, TDFE_EINVAL, "octree meshes: no full-grid operator");
  if (a.cols < 1) return tdfe_fail(c, TDFE_EINVAL, "apply: cols < 1");
  const int W = c->oct_w;
  const double* x = (const double*)a.x;
  double* y = (double*)a.y;
  if (a.n_blocks_out) *a.n_blocks_out = c->n_cell;
  const int64_t nh = (int64_t)c->oct_hv_h.size(), nmd = (int64_t)c->oct_md_h.size();
  const double* minv = a.lowdin ? (const double*)c->minv : (const double*)nullptr;
  for (int col0 = 0; col0 < a.cols; col0 += W) {
    const int cols = std::min(W, a.cols - col0);
    const double* cs = a.colscale ? a.colscale + col0 / 2 : (const double*)nullptr;
    if (nh > 0) {
      hipLaunchKernelGGL(oct_hexpand_kernel, dim3(nblk(nh * cols)), dim3(EW), 0, c->stream, x + col0, a.ld, cols, cs,
                         minv, (const int*)c->oct_hv, (const int*)c->oct_eptr, (const int*)c->oct_ecol,
                         (const double*)c->oct_eval, nh, W, c->oct_xf, c->oct_yf, a.done_flag);
      TDFE_HIP(c, hipGetLastError());
    }
    OctCellParams P{};
    P.x = x + col0;
    P.y = y + col0;
    P.ld = a.ld;
    P.minv = minv;
    P.colscale = cs;
    P.xh = c->oct_xf;
    P.yh = c->oct_yf;
    P.W = W;
    P.cols = cols;
    P.cols_total = a.cols;
    P.col0 = col0;
    P.cd = c->oct_cd;
    P.s = c->oct_s;
    P.vw = a.vw;
    P.kin = a.kin;
    P.energy = a.energy;
    P.done = a.done_flag;
    P.n_cell = c->n_cell;
    TDFE_TRY(cells_launch(c, P));
    if (nmd > 0) {
      hipLaunchKernelGGL(oct_hreduce_kernel, dim3(nblk(nmd * cols)), dim3(EW), 0, c->stream, y + col0, a.ld, cols,
                         minv, (const int*)c->oct_mptr, (const int*)c->oct_md, (const int*)c->oct_mh,
                         (const double*)c->oct_mv, nmd, W, (const double*)c->oct_yf, a.done_flag);
      TDFE_HIP(c, hipGetLastError());
    }
  }
  return TDFE_OK;
}

tdfe_status tdfe_octree_density(tdfe_ctx* c, const double* psibar, int n_orb, const double* occ, double* rho,
                                double* partial4) {
  const int W = c->oct_w;
  const int cols_all = 2 * n_orb;
  for (int col0 = 0; col0 < cols_all; col0 += W) {
    const int cols = std::min(W, cols_all - col0);
    hipLaunchKernelGGL(oct_expand_kernel, dim3(nblk(c->n_nodes * cols)), dim3(EW), 0, c->stream, psibar + col0,
                       cols_all, cols, (const double*)nullptr, (const double*)c->minv, (const int*)c->oct_eptr,
                       (const int*)c->oct_ecol, (const double*)c->oct_eval, c->n_nodes, W, c->oct_xf,
                       (double*)nullptr, (const int*)nullptr);
    TDFE_HIP(c, hipGetLastError());
    OctDensParams P{};
    P.xf = c->oct_xf;
    P.W = W;
    P.cols = cols;
    P.col0 = col0;
    P.cn = c->oct_cn;
    P.occ = occ;
    P.wdet = c->wdet;
    P.xq = c->xq;
    P.rho = rho;
    P.partial = partial4;
    P.accumulate = col0 > 0;
    P.last = col0 + W >= cols_all;
    P.n_cell = c->n_cell;
    TDFE_TRY(dens_launch(c, P));
  }
  return TDFE_OK;
}

tdfe_status tdfe_octree_bind(tdfe_ctx* c) {
  auto up = [&](void* dst, const void* src, size_t bytes) -> tdfe_status {
    if (bytes == 0) return TDFE_OK;
    TDFE_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    return TDFE_OK;
  };
  std::vector<double> minv(c->n_dof);
  for (int64_t dd = 0; dd < c->n_dof; ++dd) minv[dd] = 1.0 / std::sqrt(c->oct_m_h[dd]);
  TDFE_TRY(up(c->minv, minv.data(), minv.size() * sizeof(double)));
  TDFE_TRY(up(c->mdiag, c->oct_m_h.data(), c->oct_m_h.size() * sizeof(double)));
  TDFE_TRY(up(c->dofxyz, c->oct_dofxyz_h.data(), c->oct_dofxyz_h.size() * sizeof(double)));
  TDFE_TRY(up(c->xq, c->oct_xq_h.data(), c->oct_xq_h.size() * sizeof(double)));
  TDFE_TRY(up(c->wdet, c->oct_wdet_h.data(), c->oct_wdet_h.size() * sizeof(double)));
  TDFE_TRY(up(c->oct_cn, c->oct_cn_h.data(), c->oct_cn_h.size() * sizeof(int)));
  TDFE_TRY(up(c->oct_s, c->oct_s_h.data(), c->oct_s_h.size() * sizeof(double)));
  TDFE_TRY(up(c->oct_eptr, c->oct_eptr_h.data(), c->oct_eptr_h.size() * sizeof(int)));
  TDFE_TRY(up(c->oct_ecol, c->oct_ecol_h.data(), c->oct_ecol_h.size() * sizeof(int)));
  TDFE_TRY(up(c->oct_eval, c->oct_eval_h.data(), c->oct_eval_h.size() * sizeof(double)));
  TDFE_TRY(up(c->oct_cd, c->oct_cd_h.data(), c->oct_cd_h.size() * sizeof(int)));
  TDFE_TRY(up(c->oct_hv, c->oct_hv_h.data(), c->oct_hv_h.size() * sizeof(int)));
  TDFE_TRY(up(c->oct_mptr, c->oct_mptr_h.data(), c->oct_mptr_h.size() * sizeof(int)));
  TDFE_TRY(up(c->oct_md, c->oct_md_h.data(), c->oct_md_h.size() * sizeof(int)));
  TDFE_TRY(up(c->oct_mh, c->oct_mh_h.data(), c->oct_mh_h.size() * sizeof(int)));
  TDFE_TRY(up(c->oct_mv, c->oct_mv_h.data(), c->oct_mv_h.size() * sizeof(double)));
  // the host vectors stay: a later bind to another workspace uploads them again
  TDFE_HIP(c, hipStreamSynchronize(c->stream));
  return TDFE_OK;
}

// fills the configuration of an octree context (tdfe_setup.hip finishes it)
tdfe_status tdfe_octree_configure(tdfe_ctx* c, const tdfe_octree_desc* d) { return build_octree(c, d); }

extern "C" tdfe_status tdfe_octree_info(const tdfe_ctx* c, int64_t* n_nodes, int64_t* n_hanging, int64_t* nnz) {
  if (!c || !c->octree) return TDFE_EINVAL;
  if (n_nodes) *n_nodes = c->n_nodes;
  if (n_hanging) *n_hanging = c->oct_hanging;
  if (nnz) *nnz = (int64_t)c->oct_ecol_h.size();
  return TDFE_OK;
}
