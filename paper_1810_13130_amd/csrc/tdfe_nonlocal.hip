// Nonlocal pseudopotential term in the Kleinman-Bylander form (Eq. VPSP).
//
// The term acts on phi as sum_p (int chi_p phi / D_p) chi_p with chi_p =
// u_p dV_p and D_p = int u_p dV_p u_p.  On the FE basis its Galerkin matrix is
// C^T diag(E) C with c_pj = int chi_p N_j (Gauss rule) and E_p = 1 / D_p; in
// the Loewdin form (Eq. TDKSMatVecStandard) the library keeps
// Cbar = C M^-1/2 and adds
//   Hbar x += Cbar^T diag(E) Cbar x
// after the local operator kernel of every Hamiltonian launch.
//
// Projectors are compact around their atoms, so Cbar is stored per group of
// projectors (consecutive projectors whose supports nearly coincide, e.g. the
// s and p channels of one atom) on a box of the structured DoF grid: the
// smallest box holding every entry of magnitude above 2^-60 of the
// projector's largest entry.  The dropped entries change a projection by at
// most 2^-60 sqrt(n_dof) of |Cbar_p| |x| (below 1e-14 at 10^7 DoFs).
// Hot passes, both over the boxes only (one launch each for all groups):
//   project   per-block partials of t = Cbar (cs x)   (cs: the launch's column scale)
//   finalize  t (fixed-order sum over the group's blocks), E t, E t^2
//   add       y += Cbar^T (E t) line by line over the DoF lines crossed by
//             boxes; each (DoF, column) has one owner, which adds its groups in order
// Both are HBM-bound streaming passes (Cbar over the boxes; x over the boxes,
// y over the lines).
#include <algorithm>
#include <climits>

#include "tdfe_internal.h"

namespace {

constexpr int NL_THREADS = 256;
constexpr int NL_PCH = 16;           // projectors per group (register accumulators)
constexpr int NL_TARGET_BLOCKS = 4096;
constexpr int NL_SETUP_BLOCKS = 256;
constexpr double NL_DROP = 8.673617379884035e-19;  // 2^-60

struct NlGroup {
  int I0, J0, K0;   // first DoF of the box (0-based interior DoF coordinates)
  int nx, ny, nz;   // box extent
  int p0, np;       // projectors p0 .. p0 + np - 1
  int b0, nb;       // blocks b0 .. b0 + nb - 1 of the hot passes
  int lpb;          // box lines (x rows) per block
  int pad;
  int64_t off;      // element offset of the group's Cbar: [np][nz][ny][nx]
};

// the add pass: a segment of at most NL_SEG consecutive DoFs of a grid line
// (fixed J, K) crossed by group boxes; its groups are the line's entries
// lg[gs .. gs + gn)
constexpr int NL_SEG = 32;
struct NlSeg {
  int J, K, I0, I1, gs, gn;
};
// a group crossing a line: Cbar of projector p0 + q at DoF I of the line is
// cbar[cbase + q vol + I] for I0 <= I <= I1
struct NlLineGroup {
  int64_t cbase, vol;
  int I0, I1, p0, np;
};

struct NlLayout {
  double* cbar;     // packed groups (at most n_proj x n_dof)
  float* cbar32;    // the same in FP32 (mixed contexts)
  double* E;        // [n_proj]
  double* part;     // [max blocks][NL_PCH][TDFE_MAX_COLS]
  double* tE;       // [n_proj][TDFE_MAX_COLS]
  double* eP;       // [n_proj][TDFE_MAX_COLS]
  NlGroup* groups;  // [n_proj]
  int* pgrp;        // [n_proj] group of each projector
  int* blk2grp;     // [max blocks]
  int* box;         // [n_proj][6] set-up: I0, J0, K0, I1, J1, K1
  double* amax;     // [n_proj] set-up: largest |Cbar_p|
  double* chi;      // [n_quad] set-up
  double* dense;    // [n_dof] set-up: Cbar_p on every DoF
  double* red;      // [NL_SETUP_BLOCKS] set-up
  NlSeg* segs;      // [at most nyi nzi (nxi / NL_SEG + 1)] blocks of the add pass
  NlLineGroup* lg;  // [at most nyi nzi n_proj] groups crossing each line
  size_t bytes;
};

int nl_max_blocks(int n_proj) { return NL_TARGET_BLOCKS + n_proj; }

NlLayout nl_layout(const tdfe_ctx* c, int n_proj, char* base) {
  NlLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const size_t np = (size_t)n_proj, mb = (size_t)nl_max_blocks(n_proj);
  L.cbar = (double*)take(np * c->n_dof * sizeof(double));
  L.cbar32 = (float*)take(!tdfe_fp32(c) ? sizeof(float) : np * c->n_dof * sizeof(float));
  L.E = (double*)take(np * sizeof(double));
  L.part = (double*)take(mb * NL_PCH * TDFE_MAX_COLS * sizeof(double));
  L.tE = (double*)take(np * TDFE_MAX_COLS * sizeof(double));
  L.eP = (double*)take(np * TDFE_MAX_COLS * sizeof(double));
  L.groups = (NlGroup*)take(np * sizeof(NlGroup));
  L.pgrp = (int*)take(np * sizeof(int));
  L.blk2grp = (int*)take(mb * sizeof(int));
  L.box = (int*)take(np * 6 * sizeof(int));
  L.amax = (double*)take(np * sizeof(double));
  L.chi = (double*)take((size_t)c->n_quad * sizeof(double));
  L.dense = (double*)take((size_t)c->n_dof * sizeof(double));
  L.red = (double*)take(NL_SETUP_BLOCKS * sizeof(double));
  const size_t nlines = (size_t)(c->Ny - 2) * (c->Nz - 2);
  L.segs = (NlSeg*)take(nlines * ((size_t)(c->Nx - 2) / NL_SEG + 1) * sizeof(NlSeg));
  L.lg = (NlLineGroup*)take(nlines * np * sizeof(NlLineGroup));
  L.bytes = off + 256;
  return L;
}

// ---------------------------------------------------------------------------------------------
// set-up kernels
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

// E_p = 1 / D_p from the block partials; a zero or non-finite D_p sets *bad
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

// dense[d] = c_p(node(d)) M^-1/2(d)
__global__ void nl_extract_kernel(const double* cload, const double* minv, double* dense, int Nx, int Ny,
                                  int64_t n_dof) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n_dof) return;
  const int64_t nxi = Nx - 2, nyi = Ny - 2;
  const int64_t I = d % nxi + 1, J = (d / nxi) % nyi + 1, K = d / (nxi * nyi) + 1;
  dense[d] = cload[I + (int64_t)Nx * (J + (int64_t)Ny * K)] * minv[d];
}

// per-block max |v| (exact, order independent)
__global__ void nl_absmax_partial_kernel(const double* v, int64_t n, double* part) {
  __shared__ double s[NL_THREADS];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NL_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * NL_THREADS)
    m = fmax(m, fabs(v[i]));
  s[threadIdx.x] = m;
  __syncthreads();
  for (int w = NL_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// amax = max of the partials; the box starts empty (I0 > I1)
__global__ void nl_absmax_final_kernel(const double* part, int nb, double* amax, int* box, int nxi, int nyi,
                                       int nzi) {
  if (threadIdx.x != 0) return;
  double m = 0.0;
  for (int b = 0; b < nb; ++b) m = fmax(m, part[b]);
  *amax = m;
  box[0] = nxi;
  box[1] = nyi;
  box[2] = nzi;
  box[3] = -1;
  box[4] = -1;
  box[5] = -1;
}

// smallest DoF box holding every |v| > NL_DROP amax (integer min / max atomics)
__global__ void nl_box_kernel(const double* v, int64_t n_dof, int nxi, int nyi, const double* amax, int* box) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n_dof) return;
  if (!(fabs(v[d]) > NL_DROP * *amax)) return;
  const int I = (int)(d % nxi), J = (int)((d / nxi) % nyi), K = (int)(d / ((int64_t)nxi * nyi));
  atomicMin(box + 0, I);
  atomicMin(box + 1, J);
  atomicMin(box + 2, K);
  atomicMax(box + 3, I);
  atomicMax(box + 4, J);
  atomicMax(box + 5, K);
}

// dst[(k ny + j) nx + i] = dense[box DoF (i, j, k)] (FP32 copy alongside when requested)
__global__ void nl_pack_kernel(const double* dense, NlGroup G, int nxi, int nyi, double* dst, float* dst32) {
  const int64_t vol = (int64_t)G.nx * G.ny * G.nz;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= vol) return;
  const int i = (int)(e % G.nx), j = (int)((e / G.nx) % G.ny), k = (int)(e / ((int64_t)G.nx * G.ny));
  const double v = dense[(G.I0 + i) + (int64_t)nxi * ((G.J0 + j) + (int64_t)nyi * (G.K0 + k))];
  dst[e] = v;
  if (dst32) dst32[e] = (float)v;
}

// ---------------------------------------------------------------------------------------------
// hot kernels
// ---------------------------------------------------------------------------------------------
// Walk over the slots of a block: slot s covers x positions rg + RG sl of box
// line l0 + s / nslot (sl = s % nslot).  The walk is the same for every lane
// of the block, so its state lives in scalar registers.
struct SlotWalk {
  int sl, j, k;
  int64_t dline, eline;  // DoF of the line's first box entry; element offset of the line
  __device__ void start(const NlGroup& G, int l0, int nxi, int nyi) {
    sl = 0;
    j = l0 % G.ny;
    k = l0 / G.ny;
    dline = G.I0 + (int64_t)nxi * ((G.J0 + j) + (int64_t)nyi * (G.K0 + k));
    eline = (int64_t)l0 * G.nx;
  }
  __device__ void next(const NlGroup& G, int nslot, int nxi, int nyi) {
    if (++sl == nslot) {
      sl = 0;
      eline += G.nx;
      if (++j == G.ny) {
        j = 0;
        ++k;
        dline += (int64_t)nxi * (nyi - G.ny + 1);
      } else {
        dline += nxi;
      }
    }
  }
};

template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
};
template <>
struct Vec2<float> {
  using type = float2;
};

// block b serves box lines [l0, l1) of its group; thread t takes the column
// pair t % CPP (two real columns, one vector load) and the x positions
// t / CPP + RG sl of each line.  U slots are loaded before any is used
// (invalid slots read a valid address and contribute zero); projector
// indices past the group's np read the group's last projector and are
// discarded.  Lanes of a wave that share a column pair are summed by a fixed
// butterfly, then the four waves in order.
template <typename T, typename CT, int CP, int NP, int U>
__global__ void __launch_bounds__(NL_THREADS)
    nl_project_kernel(const T* __restrict__ x, int ld, int cols, const double* __restrict__ colscale,
                      const CT* __restrict__ cbar, const NlGroup* __restrict__ groups,
                      const int* __restrict__ blk2grp, int nxi, int nyi, double* __restrict__ part, const int* done) {
  using T2 = typename Vec2<T>::type;
  constexpr int CPP = CP / 2;
  constexpr int RG = NL_THREADS / CPP;
  constexpr int NW = NL_THREADS / 64;
  __shared__ double s[NP][2][NW][CPP];
  if (done && *done) return;
  const int b = blockIdx.x;
  const NlGroup G = groups[blk2grp[b]];
  const int t = threadIdx.x, pr = t % CPP, rg = t / CPP;
  const bool pok = 2 * pr < cols;
  const int prc = pok ? pr : 0;
  const int l0 = (b - G.b0) * G.lpb;
  const int l1 = min(l0 + G.lpb, G.ny * G.nz);
  const int nslot = (G.nx + RG - 1) / RG;
  const int S = (l1 - l0) * nslot;
  const int64_t vol = (int64_t)G.nx * G.ny * G.nz;
  const CT* cg = cbar + G.off;
  int64_t qoff[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) qoff[q] = (int64_t)min(q, G.np - 1) * vol;
  SlotWalk w;
  w.start(G, l0, nxi, nyi);
  const int64_t d0 = w.dline, e0 = w.eline;
  double acc[NP][2];
#pragma unroll
  for (int q = 0; q < NP; ++q) acc[q][0] = acc[q][1] = 0.0;
  for (int s0 = 0; s0 < S; s0 += U) {
    T2 xr[U];
    CT cr[U][NP];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = rg + RG * w.sl;
      const bool v = s0 + u < S && i < G.nx;
      ok[u] = v && pok;
      const int64_t d = v ? w.dline + i : d0;
      const int64_t e = v ? w.eline + i : e0;
      xr[u] = *(const T2*)(x + d * ld + 2 * prc);
#pragma unroll
      for (int q = 0; q < NP; ++q) cr[u][q] = cg[qoff[q] + e];
      w.next(G, nslot, nxi, nyi);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double x0 = ok[u] ? (double)xr[u].x : 0.0, x1 = ok[u] ? (double)xr[u].y : 0.0;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        acc[q][0] += (double)cr[u][q] * x0;
        acc[q][1] += (double)cr[u][q] * x1;
      }
    }
  }
  const int lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int q = 0; q < NP; ++q)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double v = acc[q][h];
      for (int off = CPP; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
      if (lane < CPP) s[q][h][wave][lane] = v;
    }
  __syncthreads();
  for (int idx = t; idx < NP * CP; idx += NL_THREADS) {
    const int q = idx / CP, cc = idx % CP;
    if (q < G.np && cc < cols) {
      double v = 0.0;
      for (int k = 0; k < NW; ++k) v += s[q][cc & 1][k][cc >> 1];
      const double cs = colscale ? colscale[cc >> 1] : 1.0;
      part[((int64_t)b * NL_PCH + q) * TDFE_MAX_COLS + cc] = v * cs;
    }
  }
}

// t[p][col] = sum over the group's blocks (slices of blocks per lane group,
// then the slices in order); tE = E t; eP = E t^2.  One block per projector.
__global__ void __launch_bounds__(NL_THREADS)
    nl_finalize_kernel(const double* __restrict__ part, const NlGroup* __restrict__ groups,
                       const int* __restrict__ pgrp, int cols, const double* __restrict__ E, double* tE, double* eP,
                       const int* done) {
  __shared__ double s[NL_THREADS];
  if (done && *done) return;
  const int p = blockIdx.x, t = threadIdx.x;
  const int cw = cols <= 16 ? 16 : cols <= 32 ? 32 : 64;
  const int nsl = NL_THREADS / cw;
  const int col = t % cw, sl = t / cw;
  const NlGroup G = groups[pgrp[p]];
  const int q = p - G.p0;
  double acc = 0.0;
  if (col < cols) {
    const double* pp = part + (int64_t)q * TDFE_MAX_COLS + col;
    int b = G.b0 + sl;
    const int b1 = G.b0 + G.nb;
    for (; b + 3 * nsl < b1; b += 4 * nsl) {
      const double v0 = pp[(int64_t)b * NL_PCH * TDFE_MAX_COLS];
      const double v1 = pp[(int64_t)(b + nsl) * NL_PCH * TDFE_MAX_COLS];
      const double v2 = pp[(int64_t)(b + 2 * nsl) * NL_PCH * TDFE_MAX_COLS];
      const double v3 = pp[(int64_t)(b + 3 * nsl) * NL_PCH * TDFE_MAX_COLS];
      acc += v0;
      acc += v1;
      acc += v2;
      acc += v3;
    }
    for (; b < b1; b += nsl) acc += pp[(int64_t)b * NL_PCH * TDFE_MAX_COLS];
  }
  s[t] = acc;
  __syncthreads();
  if (t < cols) {
    double v = 0.0;
    for (int k = 0; k < nsl; ++k) v += s[k * cw + t];
    tE[p * TDFE_MAX_COLS + t] = E[p] * v;
    eP[p * TDFE_MAX_COLS + t] = E[p] * v * v;
  }
}

// the term's share of the per-column quadratic form, as one more row of the
// operator kernel's block partials
__device__ __forceinline__ void nl_energy_row(const double* eP, int n_proj, int cols, double* energy_row) {
  const int col = threadIdx.x;
  if (col >= cols) return;
  double e = 0.0;
  for (int p = 0; p < n_proj; ++p) e += eP[p * TDFE_MAX_COLS + col];
  energy_row[col] = e;
}

__global__ void nl_energy_kernel(const double* eP, int n_proj, int cols, double* energy_row, const int* done) {
  if (done && *done) return;
  nl_energy_row(eP, n_proj, cols, energy_row);
}

// y[d][col] += sum over the groups g whose box holds d of
// sum_q Cbar_g[q][d] tE[p0_g + q][col].  Block b owns segment b; thread t
// takes the column pair t % CPP (one vector load and store) of DoFs
// t / CPP + RG u.  The C values of the segment and the E t rows of up to
// GS groups at a time are staged in LDS by the whole block (one global load
// per value instead of one per column lane), then each (DoF, column) adds
// the crossing groups in their stored order: no atomics, and the result does
// not depend on scheduling.  Block 0 also writes the energy row (all
// projections are final by now).
template <typename T, typename CT, int CP, int NP>
__global__ void __launch_bounds__(NL_THREADS)
    nl_add_kernel(T* __restrict__ y, int ld, int cols, const CT* __restrict__ cbar, const NlSeg* __restrict__ segs,
                  const NlLineGroup* __restrict__ lgs, int nxi, int nyi, const double* __restrict__ tE,
                  const double* __restrict__ eP, int n_proj, double* energy_row, const int* done) {
  using T2 = typename Vec2<T>::type;
  constexpr int CPP = CP / 2;
  constexpr int RG = NL_THREADS / CPP;
  constexpr int U = NL_SEG / RG;
  constexpr int GS = 16 / NP > 0 ? 16 / NP : 1;  // groups staged at a time
  static_assert(U >= 1 && U * RG == NL_SEG, "segment length must be a multiple of the DoF lanes");
  __shared__ double sC[GS][NP][NL_SEG];
  __shared__ double sT[GS][NP][CP];
  if (done && *done) return;
  const int b = blockIdx.x;
  if (b == 0 && energy_row) nl_energy_row(eP, n_proj, cols, energy_row);
  const int t = threadIdx.x, pr = t % CPP, rg = t / CPP;
  const bool pok = 2 * pr < cols;
  const NlSeg sg = segs[b];
  const int64_t dline = (int64_t)nxi * (sg.J + (int64_t)nyi * sg.K);
  T2 yv[U];
  double acc[U][2];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int I = min(sg.I0 + rg + RG * u, sg.I1);
    yv[u] = *(const T2*)(y + (dline + I) * ld + 2 * (pok ? pr : 0));
    acc[u][0] = acc[u][1] = 0.0;
  }
  for (int g0 = sg.gs; g0 < sg.gs + sg.gn; g0 += GS) {
    const int ng = min(GS, sg.gs + sg.gn - g0);
    for (int idx = t; idx < ng * NP * NL_SEG; idx += NL_THREADS) {
      const int gi = idx / (NP * NL_SEG), q = (idx / NL_SEG) % NP, i = idx % NL_SEG;
      const NlLineGroup g = lgs[g0 + gi];
      const int I = sg.I0 + i;
      const bool in = q < g.np && I <= sg.I1 && I >= g.I0 && I <= g.I1;
      sC[gi][q][i] = in ? (double)cbar[g.cbase + I + (int64_t)q * g.vol] : 0.0;
    }
    for (int idx = t; idx < ng * NP * CP; idx += NL_THREADS) {
      const int gi = idx / (NP * CP), q = (idx / CP) % NP, c = idx % CP;
      const NlLineGroup g = lgs[g0 + gi];
      sT[gi][q][c] = (q < g.np && c < cols) ? tE[(g.p0 + q) * TDFE_MAX_COLS + c] : 0.0;
    }
    __syncthreads();
    for (int gi = 0; gi < ng; ++gi) {
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const double t0 = sT[gi][q][2 * pr], t1 = sT[gi][q][2 * pr + 1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double cv = sC[gi][q][rg + RG * u];
          acc[u][0] += cv * t0;
          acc[u][1] += cv * t1;
        }
      }
    }
    __syncthreads();
  }
  if (!pok) return;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int I = sg.I0 + rg + RG * u;
    if (I <= sg.I1) {
      T2 o;
      o.x = yv[u].x + (T)acc[u][0];
      o.y = yv[u].y + (T)acc[u][1];
      *(T2*)(y + (dline + I) * ld + 2 * pr) = o;
    }
  }
}

template <typename T, typename CT, int CP, int NP>
tdfe_status nl_passes(tdfe_ctx* c, const T* x, T* y, int ld, int cols, const double* cs, const int* done,
                      double* energy_row, const CT* cbar, const NlLayout& L) {
  constexpr int U = NP >= 16 ? 1 : 16 / NP;
  const int nxi = c->Nx - 2, nyi = c->Ny - 2;
  if (c->nl_blocks > 0) {
    hipLaunchKernelGGL((nl_project_kernel<T, CT, CP, NP, U>), dim3(c->nl_blocks), dim3(NL_THREADS), 0, c->stream, x,
                       ld, cols, cs, cbar, (const NlGroup*)L.groups, (const int*)L.blk2grp, nxi, nyi, L.part, done);
    TDFE_HIP(c, hipGetLastError());
  }
  hipLaunchKernelGGL(nl_finalize_kernel, dim3(c->n_proj), dim3(NL_THREADS), 0, c->stream, (const double*)L.part,
                     (const NlGroup*)L.groups, (const int*)L.pgrp, cols, (const double*)L.E, L.tE, L.eP, done);
  TDFE_HIP(c, hipGetLastError());
  if (c->nl_add_blocks > 0) {
    hipLaunchKernelGGL((nl_add_kernel<T, CT, CP, NP>), dim3(c->nl_add_blocks), dim3(NL_THREADS), 0, c->stream, y,
                       ld, cols, cbar, (const NlSeg*)L.segs, (const NlLineGroup*)L.lg, nxi, nyi, (const double*)L.tE,
                       (const double*)L.eP, c->n_proj, energy_row, done);
    TDFE_HIP(c, hipGetLastError());
  } else if (energy_row) {
    hipLaunchKernelGGL(nl_energy_kernel, dim3(1), dim3(64), 0, c->stream, (const double*)L.eP, c->n_proj, cols,
                       energy_row, done);
    TDFE_HIP(c, hipGetLastError());
  }
  return TDFE_OK;
}

template <typename T, typename CT, int CP>
tdfe_status nl_passes_np(tdfe_ctx* c, const T* x, T* y, int ld, int cols, const double* cs, const int* done,
                         double* energy_row, const CT* cbar, const NlLayout& L) {
  if (c->nl_np_max <= 4) return nl_passes<T, CT, CP, 4>(c, x, y, ld, cols, cs, done, energy_row, cbar, L);
  if (c->nl_np_max <= 8) return nl_passes<T, CT, CP, 8>(c, x, y, ld, cols, cs, done, energy_row, cbar, L);
  return nl_passes<T, CT, CP, 16>(c, x, y, ld, cols, cs, done, energy_row, cbar, L);
}

// columns [col0, col0 + cols) of the launch (cols <= TDFE_MAX_COLS, col0 even)
template <typename T, typename CT>
tdfe_status nl_apply_t(tdfe_ctx* c, const ApplyArgs& a, int col0, int cols, double* energy_row, const CT* cbar,
                       const NlLayout& L) {
  const T* x = (const T*)a.x + col0;
  T* y = (T*)a.y + col0;
  const double* cs = a.colscale ? a.colscale + col0 / 2 : nullptr;
  if (cols <= 16) return nl_passes_np<T, CT, 16>(c, x, y, a.ld, cols, cs, a.done_flag, energy_row, cbar, L);
  if (cols <= 32) return nl_passes_np<T, CT, 32>(c, x, y, a.ld, cols, cs, a.done_flag, energy_row, cbar, L);
  return nl_passes_np<T, CT, 64>(c, x, y, a.ld, cols, cs, a.done_flag, energy_row, cbar, L);
}

// chi = u dV, the load vector c_p on every node, Cbar_p on every DoF (dense)
tdfe_status nl_dense_column(tdfe_ctx* c, const double* u, const double* dv, const NlLayout& L) {
  const int64_t nq = c->n_quad;
  hipLaunchKernelGGL(nl_chi_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, c->stream, u, dv, L.chi, nq);
  TDFE_HIP(c, hipGetLastError());
  TDFE_TRY(tdfe_load_vector(c, L.chi, true));
  hipLaunchKernelGGL(nl_extract_kernel, dim3((unsigned)((c->n_dof + 255) / 256)), dim3(256), 0, c->stream,
                     (const double*)c->cload, (const double*)c->minv, L.dense, c->Nx, c->Ny, c->n_dof);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

int64_t box_vol(const int* b) {
  if (b[3] < b[0]) return 0;
  return (int64_t)(b[3] - b[0] + 1) * (b[4] - b[1] + 1) * (b[5] - b[2] + 1);
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
  if (n_proj > 0 && (!dev_u || !dev_dv || !dev_store)) return tdfe_fail(c, TDFE_EINVAL, "set_projectors: null pointer");
  if (n_proj > 0 && c->octree) return tdfe_fail(c, TDFE_EINVAL, "set_projectors: not on octree meshes");
  if (n_proj > 0 && (uintptr_t)dev_store % 256 != 0)
    return tdfe_fail(c, TDFE_EINVAL, "set_projectors: store not 256-byte aligned");
  const NlLayout L = nl_layout(c, n_proj, (char*)dev_store);
  if (n_proj > 0 && store_bytes < L.bytes)
    return tdfe_fail(c, TDFE_ENOMEM, "set_projectors: store of %zu bytes, %zu needed", store_bytes, L.bytes);
  // the term is off until its tables are complete
  c->n_proj = 0;
  c->nl_store = nullptr;
  c->nl_blocks = 0;
  c->nl_groups = 0;
  c->nl_packed = 0;
  c->nl_box_dofs = 0;
  c->nl_lines = c->nl_add_blocks = 0;
  c->nl_line_dofs = 0;
  if (n_proj == 0) return TDFE_OK;
  const int64_t nq = c->n_quad, nd = c->n_dof;
  const int nxi = c->Nx - 2, nyi = c->Ny - 2, nzi = c->Nz - 2;
  const unsigned gd = (unsigned)((nd + 255) / 256);
  int* bad = (int*)c->counters + 210;
  TDFE_TRY(tdfe_zero(c, bad, sizeof(int)));

  // pass 1: D_p, the largest entry and the box of each projector
  for (int p = 0; p < n_proj; ++p) {
    const double* u = dev_u + (size_t)p * nq;
    TDFE_TRY(nl_dense_column(c, u, dev_dv + (size_t)p * nq, L));
    hipLaunchKernelGGL(nl_norm_partial_kernel, dim3(NL_SETUP_BLOCKS), dim3(NL_THREADS), 0, c->stream,
                       (const double*)c->wdet, (const double*)L.chi, u, nq, L.red);
    hipLaunchKernelGGL(nl_norm_final_kernel, dim3(1), dim3(64), 0, c->stream, (const double*)L.red,
                       NL_SETUP_BLOCKS, L.E + p, bad);
    hipLaunchKernelGGL(nl_absmax_partial_kernel, dim3(NL_SETUP_BLOCKS), dim3(NL_THREADS), 0, c->stream,
                       (const double*)L.dense, nd, L.red);
    hipLaunchKernelGGL(nl_absmax_final_kernel, dim3(1), dim3(64), 0, c->stream, (const double*)L.red,
                       NL_SETUP_BLOCKS, L.amax + p, L.box + 6 * p, nxi, nyi, nzi);
    hipLaunchKernelGGL(nl_box_kernel, dim3(gd), dim3(256), 0, c->stream, (const double*)L.dense, nd, nxi, nyi,
                       (const double*)(L.amax + p), L.box + 6 * p);
    TDFE_HIP(c, hipGetLastError());
  }
  std::vector<int> box((size_t)6 * n_proj);
  int hbad = 0;
  TDFE_HIP(c, hipMemcpyAsync(box.data(), L.box, box.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  TDFE_HIP(c, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  TDFE_HIP(c, hipStreamSynchronize(c->stream));
  if (hbad) return tdfe_fail(c, TDFE_EINVAL, "set_projectors: int u dV u is zero or not finite for a projector");

  // groups: consecutive projectors whose union box is at most 25% larger than the larger of the two
  std::vector<NlGroup> groups;
  std::vector<int> pgrp(n_proj);
  int gb[6] = {0, 0, 0, -1, -1, -1};
  for (int p = 0; p < n_proj; ++p) {
    const int* b = &box[(size_t)6 * p];
    bool join = false;
    int ub[6];
    if (!groups.empty() && groups.back().np < NL_PCH) {
      const int64_t vg = box_vol(gb), vb = box_vol(b);
      if (vb == 0) {
        join = true;
        std::copy(gb, gb + 6, ub);
      } else if (vg > 0) {
        for (int a = 0; a < 3; ++a) {
          ub[a] = std::min(gb[a], b[a]);
          ub[a + 3] = std::max(gb[a + 3], b[a + 3]);
        }
        join = 4 * box_vol(ub) <= 5 * std::max(vg, vb);
      }
    }
    if (join) {
      std::copy(ub, ub + 6, gb);
      groups.back().np += 1;
    } else {
      NlGroup g{};
      g.p0 = p;
      g.np = 1;
      groups.push_back(g);
      std::copy(b, b + 6, gb);
    }
    NlGroup& g = groups.back();
    if (box_vol(gb) > 0) {
      g.I0 = gb[0];
      g.J0 = gb[1];
      g.K0 = gb[2];
      g.nx = gb[3] - gb[0] + 1;
      g.ny = gb[4] - gb[1] + 1;
      g.nz = gb[5] - gb[2] + 1;
    } else {
      g.I0 = g.J0 = g.K0 = 0;
      g.nx = g.ny = g.nz = 0;
    }
    pgrp[p] = (int)groups.size() - 1;
  }
  // packed offsets and the block partition of the hot passes
  int64_t total = 0, off = 0;
  for (const NlGroup& g : groups) total += (int64_t)g.nx * g.ny * g.nz;
  const int64_t epb = std::max<int64_t>(256, (total + NL_TARGET_BLOCKS - 1) / NL_TARGET_BLOCKS);
  std::vector<int> blk2grp;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    NlGroup& g = groups[gi];
    g.off = off;
    off += (int64_t)g.np * g.nx * g.ny * g.nz;
    g.b0 = (int)blk2grp.size();
    if (g.nx > 0) {
      g.lpb = (int)std::max<int64_t>(1, (epb + g.nx - 1) / g.nx);
      g.nb = (g.ny * g.nz + g.lpb - 1) / g.lpb;
    } else {
      g.lpb = 1;
      g.nb = 0;
    }
    blk2grp.insert(blk2grp.end(), (size_t)g.nb, (int)gi);
  }
  if ((int64_t)blk2grp.size() > nl_max_blocks(n_proj) || off > (int64_t)n_proj * nd)
    return tdfe_fail(c, TDFE_EINVAL, "set_projectors: internal partition error");

  // pass 2: pack each projector's Cbar into its group box
  for (const NlGroup& g : groups) {
    const int64_t vol = (int64_t)g.nx * g.ny * g.nz;
    if (vol == 0) continue;
    for (int q = 0; q < g.np; ++q) {
      const int p = g.p0 + q;
      TDFE_TRY(nl_dense_column(c, dev_u + (size_t)p * nq, dev_dv + (size_t)p * nq, L));
      const int64_t o = g.off + q * vol;
      hipLaunchKernelGGL(nl_pack_kernel, dim3((unsigned)((vol + 255) / 256)), dim3(256), 0, c->stream,
                         (const double*)L.dense, g, nxi, nyi, L.cbar + o,
                         !tdfe_fp32(c) ? (float*)nullptr : L.cbar32 + o);
      TDFE_HIP(c, hipGetLastError());
    }
  }
  // the add pass: every grid line (J, K) crossed by a group box, its groups in
  // order, cut into segments of at most NL_SEG DoFs
  std::vector<NlSeg> segs;
  std::vector<NlLineGroup> lgs;
  int64_t line_elems = 0;
  int n_lines = 0;
  {
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {-1, -1, -1};
    for (const NlGroup& g : groups) {
      if (g.nx == 0) continue;
      lo[1] = std::min(lo[1], g.J0);
      lo[2] = std::min(lo[2], g.K0);
      hi[1] = std::max(hi[1], g.J0 + g.ny - 1);
      hi[2] = std::max(hi[2], g.K0 + g.nz - 1);
    }
    for (int K = lo[2]; K <= hi[2]; ++K)
      for (int J = lo[1]; J <= hi[1]; ++J) {
        const int gs = (int)lgs.size();
        int I_lo = INT_MAX, I_hi = -1;
        for (const NlGroup& g : groups) {
          if (g.nx == 0 || J < g.J0 || J >= g.J0 + g.ny || K < g.K0 || K >= g.K0 + g.nz) continue;
          NlLineGroup e{};
          e.vol = (int64_t)g.nx * g.ny * g.nz;
          e.cbase = g.off + ((int64_t)(K - g.K0) * g.ny + (J - g.J0)) * g.nx - g.I0;
          e.I0 = g.I0;
          e.I1 = g.I0 + g.nx - 1;
          e.p0 = g.p0;
          e.np = g.np;
          lgs.push_back(e);
          I_lo = std::min(I_lo, e.I0);
          I_hi = std::max(I_hi, e.I1);
        }
        const int gn = (int)lgs.size() - gs;
        if (gn == 0) continue;
        ++n_lines;
        line_elems += I_hi - I_lo + 1;
        for (int I = I_lo; I <= I_hi; I += NL_SEG) segs.push_back(NlSeg{J, K, I, std::min(I + NL_SEG - 1, I_hi), gs, gn});
      }
  }
  if ((int64_t)segs.size() > (int64_t)nyi * nzi * (nxi / NL_SEG + 1) || (int64_t)lgs.size() > (int64_t)nyi * nzi * n_proj)
    return tdfe_fail(c, TDFE_EINVAL, "set_projectors: internal line table error");
  if (!segs.empty()) {
    TDFE_HIP(c, hipMemcpyAsync(L.segs, segs.data(), segs.size() * sizeof(NlSeg), hipMemcpyHostToDevice, c->stream));
    TDFE_HIP(c, hipMemcpyAsync(L.lg, lgs.data(), lgs.size() * sizeof(NlLineGroup), hipMemcpyHostToDevice,
                               c->stream));
  }
  TDFE_HIP(c, hipMemcpyAsync(L.groups, groups.data(), groups.size() * sizeof(NlGroup), hipMemcpyHostToDevice,
                             c->stream));
  TDFE_HIP(c, hipMemcpyAsync(L.pgrp, pgrp.data(), pgrp.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
  if (!blk2grp.empty())
    TDFE_HIP(c, hipMemcpyAsync(L.blk2grp, blk2grp.data(), blk2grp.size() * sizeof(int), hipMemcpyHostToDevice,
                               c->stream));
  TDFE_HIP(c, hipStreamSynchronize(c->stream));
  c->nl_store = dev_store;
  c->nl_blocks = (int)blk2grp.size();
  c->nl_groups = (int)groups.size();
  c->nl_packed = off;
  c->nl_box_dofs = total;
  c->nl_lines = n_lines;
  c->nl_line_dofs = line_elems;
  c->nl_add_blocks = (int)segs.size();
  c->nl_np_max = 1;
  for (const NlGroup& g : groups) c->nl_np_max = std::max(c->nl_np_max, g.np);
  c->n_proj = n_proj;
  return TDFE_OK;
}

tdfe_status tdfe_projector_info(const tdfe_ctx* c, int* n_groups, int64_t* stored, int64_t* box_dofs,
                                int64_t* line_dofs) {
  if (!c || !n_groups || !stored || !box_dofs || !line_dofs) return TDFE_EINVAL;
  *n_groups = c->nl_groups;
  *stored = c->nl_packed;
  *box_dofs = c->nl_box_dofs;
  *line_dofs = c->nl_line_dofs;
  return TDFE_OK;
}

}  // extern "C"
