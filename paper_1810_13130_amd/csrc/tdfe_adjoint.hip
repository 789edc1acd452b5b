// Gradient of the final dipole mu_z(t_N) with respect to the per-step field
// amplitudes E_n of the predictor-corrector Magnus scheme (reverse mode).
//
// The forward map is the step of the Magnus ABI with V_field = -E_n z on
// step n (Eq. VField; -E_n (d . r) for a field direction d other than z, and
// then z below reads d . r), the second-order Magnus propagator (Eq. Magnus2) and
// the predictor-corrector midpoint potential (Sec. on the midpoint
// Hamiltonian):
//   V_P = V_ext - E_n z + 1.25 W_n - 0.25 W_{n-1}       (W_{-1} := W_0)
//   phi = exp(-i dt/2 Hbar(V_P)) psi^n,  V_C = V_ext - E_n z + W[rho(phi)]
//   psi^{n+1} = exp(-i dt Hbar(V_C)) psi^n,  W_{n+1} = W[rho(psi^{n+1})]
//   L = mu_z(psi^N) = sum_q varpi_q detJ_q z_q rho_q.
// Cotangents are taken for the real inner product Re<a, b>.
//
// Exponential: for z = exp(-i tau Hbar) x with cotangent zb,
//   xb = exp(+i tau Hbar) zb  (a Lanczos run with -tau), and
//   Vb_q = Re[-i tau varpi_q detJ_q sum_alpha int_0^1 conj(y_q(s)) u_q(s) ds]
//   with u(s) = exp(-i s tau Hbar) x, y(s) = exp(i (1-s) tau Hbar) zb.
// Both curves live in the Krylov spaces the two Lanczos runs build:
//   u(s) = ||x|| Q_x exp(-i s tau T_x) e_1, y(s) = ||zb|| Q_z exp(i (1-s) tau T_z) e_1,
// so the s-integral reduces to a small matrix per orbital,
//   C = ||zb|| ||x|| U_z diag(U_z[0,:]) G diag(U_x[0,:]) U_x^T,
//   G_ab = exp(-i tau (th_a + th_b)/2) sinc(tau (th_b - th_a)/2)
// (T = U diag(th) U^T; G is the divided difference of exp(-i tau .)), and
//   Vb_q = tau varpi_q detJ_q Im[ sum_alpha sum_jl conj(A_qj) C_jl B_ql ]
// with A = I M^-1/2 Q_z and B = I M^-1/2 Q_x at the Gauss points.
// Density: psib_alpha = 2 f_alpha M^-1/2 I^T (rhob . I M^-1/2 psibar_alpha), the
// operator kernel with the kinetic term switched off and 2 rhob as potential.
// W = V_H + V_x: rhob = f_x(rho) Wb + varpi detJ . I K00^-1 (4 pi I^T Wb).
// dL/dE_n = -sum_q (Vb_P + Vb_C)_q z_q.
//
// States are checkpointed every `checkpoint_every` steps; each segment is
// recomputed once and its steps are reversed from its stored states.
#include <algorithm>
#include <cmath>
#include <system_error>
#include <atomic>
#include <thread>
#include <vector>

#include "tdfe_internal.h"

namespace {

constexpr int EW = 256;
constexpr int RED_BLOCKS = 512;
constexpr int KT = 8;  // rows of C per register tile in the bilinear kernel

inline unsigned nblk(int64_t n, int b = EW) { return (unsigned)((n + b - 1) / b); }

// -------------------------------------------------------------------------------------------
// Krylov basis q_j = s_j w_j of every orbital -> Gauss points (complex), I M^-1/2 q_j
//   out[((o * ks + j) * n_quad + q)] = (re, im)
// -------------------------------------------------------------------------------------------
struct BasisParams {
  const void* W;
  int64_t vstride;  // elements between basis vectors
  int C;            // 2 Nc columns
  int Nc;
  const double* scale;  // [j][Nc]
  const int* kconv;     // [Nc]
  const double* minv;
  const double* tab;
  double2* out;
  int64_t n_quad;
  int ks;
  int ncx, ncy, p, Nx, Ny, Nz;
};

template <typename T, int N, int CB>
__global__ void __launch_bounds__(N* N* CB) basis_quad_kernel(BasisParams P) {
  constexpr int VOL = N * N * N;
  constexpr int NT = N * N * CB;
  __shared__ double sU[VOL * CB];
  __shared__ double sB[N * N];
  const int t = threadIdx.x;
  const int col = t % CB, line = t / CB;
  const int64_t cell = blockIdx.x;
  const int j = blockIdx.y;
  const T* Wj = (const T*)P.W + (int64_t)j * P.vstride;
  for (int i = t; i < N * N; i += NT) sB[i] = P.tab[TAB_B + (i / N) * TDFE_MAXN + (i % N)];
  const int cx = (int)(cell % P.ncx), cy = (int)((cell / P.ncx) % P.ncy), cz = (int)(cell / ((int64_t)P.ncx * P.ncy));
  __syncthreads();
  auto L = [&](int z, int y, int x) { return ((z * N + y) * N + x) * CB + col; };
  for (int c0 = 0; c0 < P.C; c0 += CB) {
    const int cg = c0 + col;
    const bool ok = cg < P.C && j < P.kconv[cg >> 1];
    const double sj = ok ? P.scale[(size_t)j * P.Nc + (cg >> 1)] : 0.0;
    double r1[N];
    {
      const int i = line % N, jj = line / N;
      const int I = cx * P.p + i, J = cy * P.p + jj;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const int K = cz * P.p + k;
        double v = 0.0;
        if (ok && I > 0 && I < P.Nx - 1 && J > 0 && J < P.Ny - 1 && K > 0 && K < P.Nz - 1) {
          const int64_t d =
              (int64_t)(I - 1) + (int64_t)(P.Nx - 2) * ((int64_t)(J - 1) + (int64_t)(P.Ny - 2) * (K - 1));
          v = (double)Wj[d * P.C + cg] * P.minv[d] * sj;
        }
        r1[k] = v;
      }
#pragma unroll
      for (int c = 0; c < N; ++c) {
        double s = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) s += sB[c * N + k] * r1[k];
        sU[L(c, jj, i)] = s;
      }
    }
    __syncthreads();
    {
      const int i = line % N, c = line / N;
#pragma unroll
      for (int jj = 0; jj < N; ++jj) r1[jj] = sU[L(c, jj, i)];
#pragma unroll
      for (int b = 0; b < N; ++b) {
        double s = 0;
#pragma unroll
        for (int jj = 0; jj < N; ++jj) s += sB[b * N + jj] * r1[jj];
        sU[L(c, b, i)] = s;
      }
    }
    __syncthreads();
    {
      const int b = line % N, c = line / N;
#pragma unroll
      for (int i = 0; i < N; ++i) r1[i] = sU[L(c, b, i)];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        double s = 0;
#pragma unroll
        for (int i = 0; i < N; ++i) s += sB[a * N + i] * r1[i];
        sU[L(c, b, a)] = s;  // this thread's own line
      }
    }
    __syncthreads();
    // coalesced store: one (re, im) pair per thread
    for (int idx = t; idx < VOL * (CB / 2); idx += NT) {
      const int pr = idx / VOL, q = idx % VOL;
      const int cp = c0 + 2 * pr;
      if (cp < P.C) {
        const int o = cp >> 1;
        if (j < P.kconv[o])
          P.out[((int64_t)o * P.ks + j) * P.n_quad + cell * VOL + q] =
              make_double2(sU[q * CB + 2 * pr], sU[q * CB + 2 * pr + 1]);
      }
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------------------------------------
// Vb_q (+)= tau varpi_q detJ_q Im[ sum_o sum_{j<kz} conj(A_qj) sum_{l<kx} C_jl B_ql ]
// Cm rows are padded with zeros to a multiple of KT
// -------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(EW)
    bilinear_kernel(const double2* __restrict__ A, const double2* __restrict__ B, const double2* __restrict__ Cm,
                    const int* __restrict__ kz, const int* __restrict__ kx, int Nc, int ks, int64_t n_quad, double tau,
                    const double* __restrict__ wdet, double* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_quad) return;
  double ar = 0.0, ai = 0.0;
  for (int o = 0; o < Nc; ++o) {
    const int kzo = kz[o], kxo = kx[o];
    const double2* Ao = A + (int64_t)o * ks * n_quad + q;
    const double2* Bo = B + (int64_t)o * ks * n_quad + q;
    const double2* Co = Cm + (int64_t)o * ks * ks;
    for (int jt = 0; jt < kzo; jt += KT) {
      double tr[KT], ti[KT];
#pragma unroll
      for (int u = 0; u < KT; ++u) tr[u] = ti[u] = 0.0;
      for (int l = 0; l < kxo; ++l) {
        const double2 b = Bo[(int64_t)l * n_quad];
#pragma unroll
        for (int u = 0; u < KT; ++u) {
          const double2 cc = Co[(jt + u) * ks + l];
          tr[u] += cc.x * b.x - cc.y * b.y;
          ti[u] += cc.x * b.y + cc.y * b.x;
        }
      }
#pragma unroll
      for (int u = 0; u < KT; ++u) {
        if (jt + u < kzo) {
          const double2 a = Ao[(int64_t)(jt + u) * n_quad];
          // conj(a) * t
          ar += a.x * tr[u] + a.y * ti[u];
          ai += a.x * ti[u] - a.y * tr[u];
        }
      }
    }
  }
  out[q] = tau * ai * wdet[q];
}

// -------------------------------------------------------------------------------------------
// small elementwise kernels
// -------------------------------------------------------------------------------------------
// out = s (f_x(rho) Wb + [wdet vh])
__global__ void w_adjoint_kernel(const double* Wb, const double* rho, const double* wdet, const double* vh, int xc,
                                 double s, double* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  if (xc == TDFE_XC_X) {
    const double r = rho[i];
    if (r > 1e-30) v = -(1.0 / 3.0) * cbrt(3.0 / M_PI) * pow(r, -2.0 / 3.0) * Wb[i];
  }
  if (vh) v += wdet[i] * vh[i];
  out[i] = s * v;
}

// out = 2 wdet z (twice the cotangent of rho for L = mu_z)
__global__ void dipole_cotangent_kernel(const double* wdet, const double* xq, double* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = 2.0 * wdet[i] * xq[i * 3 + 2];
}

// Wb_a += ca v ; Wb_b += cb v   (a may equal b)
__global__ void wbar_update_kernel(const double* v, double* wa, double ca, double* wb, double cb, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = v[i];
  wa[i] += ca * x;
  wb[i] += cb * x;
}

__global__ void add_kernel(const double* a, const double* b, double* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = a[i] + b[i];
}

// partial[b] = sum over this block's grid-stride range of (v1 + v2) (d . r), d the field direction
__global__ void __launch_bounds__(EW) zdot_kernel(const double* v1, const double* v2, const double* xq, int64_t n,
                                                  double dx, double dy, double dz, double* partial) {
  __shared__ double sred[EW];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x; i < n; i += (int64_t)gridDim.x * EW)
    acc += ((v1 ? v1[i] : 0.0) + (v2 ? v2[i] : 0.0)) * (dx * xq[i * 3] + dy * xq[i * 3 + 1] + dz * xq[i * 3 + 2]);
  sred[threadIdx.x] = acc;
  __syncthreads();
  for (int s = EW / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sred[threadIdx.x] += sred[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sred[0];
}

// out[0] = -sum(partial)  (fixed order)
__global__ void __launch_bounds__(EW) neg_sum_kernel(const double* partial, int nb, double* out) {
  __shared__ double sred[EW];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += EW) acc += partial[b];
  sred[threadIdx.x] = acc;
  __syncthreads();
  for (int s = EW / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sred[threadIdx.x] += sred[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = -sred[0];
}

// -------------------------------------------------------------------------------------------
// host side
// -------------------------------------------------------------------------------------------
size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct GradLayout {
  int S = 0, Cseg = 0, ks = 0;
  size_t state = 0, quad = 0, qbasis = 0;
  size_t o_ckpt = 0, o_seg = 0, o_cur = 0, o_nxt = 0, o_phi = 0, o_tmp = 0, o_lam = 0, o_lamh = 0, o_xbc = 0;
  size_t o_W = 0, o_q = 0, o_full = 0, o_qx_p = 0, o_qx_c = 0, o_qz = 0, o_cm = 0, o_k = 0, o_de = 0, o_part = 0;
  size_t total = 0;
};
enum QuadSlot { Q_WH = 0, Q_VBC, Q_VBP, Q_RHOH, Q_RHO1, Q_RB, Q_VH, Q_WB0, Q_WB1, Q_WB2, Q_COUNT };

GradLayout layout(const tdfe_ctx* c, int n_orb, int n_steps, int ckpt, int ks) {
  GradLayout g;
  g.Cseg = std::min(ckpt, n_steps);
  g.S = (n_steps + g.Cseg - 1) / g.Cseg;
  g.ks = ks;
  g.state = al256((size_t)c->n_dof * 2 * n_orb * sizeof(double));
  g.quad = al256((size_t)c->n_quad * sizeof(double));
  g.qbasis = al256((size_t)n_orb * ks * c->n_quad * 2 * sizeof(double));
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t r = o;
    o += al256(b);
    return r;
  };
  g.o_ckpt = take(g.state * g.S);
  g.o_seg = take(g.state * (g.Cseg + 1));
  g.o_cur = take(g.state);
  g.o_nxt = take(g.state);
  g.o_phi = take(g.state);
  g.o_tmp = take(g.state);
  g.o_lam = take(g.state);
  g.o_lamh = take(g.state);
  g.o_xbc = take(g.state);
  g.o_W = take(g.quad * n_steps);
  g.o_q = take(g.quad * Q_COUNT);
  g.o_full = take((size_t)c->n_nodes * sizeof(double));
  g.o_qx_p = take(g.qbasis);
  g.o_qx_c = take(g.qbasis);
  g.o_qz = take(g.qbasis);
  g.o_cm = take((size_t)n_orb * ks * ks * 2 * sizeof(double));
  g.o_k = take((size_t)2 * n_orb * sizeof(int));
  g.o_de = take((size_t)n_steps * sizeof(double));
  g.o_part = take((size_t)RED_BLOCKS * sizeof(double));
  g.total = o;
  return g;
}

// what one Lanczos run leaves for the adjoint: its tridiagonal matrices and
// its basis at the Gauss points
struct KrylovRecord {
  double2* quad = nullptr;  // [Nc][ks][n_quad]
  std::vector<double> alpha, beta, nrm;  // alpha/beta [j][Nc]
  std::vector<int> k;
};

struct CaptureHook : LanczosHook {
  KrylovRecord* rec = nullptr;
  int ks = 0;
  tdfe_status after_loop(tdfe_ctx* c, const void* W, int64_t vstride, int Nc, int o0, const double* scale,
                         const int* kconv, const double* alpha, const double* beta, const double* nrm, int k_enq,
                         bool fp32) override;
};

template <typename T, int N>
tdfe_status launch_basis_n(tdfe_ctx* c, BasisParams& P, int kq) {
  constexpr int CB = N <= 4 ? 8 : 4;
  hipLaunchKernelGGL((basis_quad_kernel<T, N, CB>), dim3((unsigned)c->n_cell, (unsigned)kq), dim3(N * N * CB), 0,
                     c->stream, P);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

template <typename T>
tdfe_status launch_basis(tdfe_ctx* c, BasisParams& P, int kq) {
  switch (c->n) {
    case 2: return launch_basis_n<T, 2>(c, P, kq);
    case 3: return launch_basis_n<T, 3>(c, P, kq);
    case 4: return launch_basis_n<T, 4>(c, P, kq);
    case 5: return launch_basis_n<T, 5>(c, P, kq);
    case 6: return launch_basis_n<T, 6>(c, P, kq);
    case 7: return launch_basis_n<T, 7>(c, P, kq);
    case 8: return launch_basis_n<T, 8>(c, P, kq);
    case 9: return launch_basis_n<T, 9>(c, P, kq);
  }
  return tdfe_fail(c, TDFE_EINVAL, "unsupported order");
}

tdfe_status CaptureHook::after_loop(tdfe_ctx* c, const void* W, int64_t vstride, int Nc, int o0, const double* scale,
                                    const int* kconv, const double* alpha, const double* beta, const double* nrm,
                                    int k_enq, bool fp32) {
  if (o0 != 0) return tdfe_fail(c, TDFE_EINVAL, "gradient: orbitals must fit one Lanczos chunk");
  KrylovRecord& r = *rec;
  r.k.assign(Nc, 0);
  r.nrm.assign(Nc, 0.0);
  TDFE_HIP(c, hipMemcpyAsync(r.k.data(), kconv, Nc * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  TDFE_HIP(c, hipMemcpyAsync(r.nrm.data(), nrm, Nc * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  TDFE_HIP(c, hipStreamSynchronize(c->stream));
  int kq = 0;
  for (int o = 0; o < Nc; ++o) kq = std::max(kq, r.k[o]);
  if (kq > ks)
    return tdfe_fail(c, TDFE_EINVAL, "gradient: a Lanczos run needed %d basis vectors, the workspace holds %d", kq,
                     ks);
  r.alpha.assign((size_t)std::max(kq, 1) * Nc, 0.0);
  r.beta.assign((size_t)std::max(kq, 1) * Nc, 0.0);
  if (kq > 0) {
    TDFE_HIP(c, hipMemcpyAsync(r.alpha.data(), alpha, (size_t)kq * Nc * sizeof(double), hipMemcpyDeviceToHost,
                               c->stream));
    TDFE_HIP(c, hipMemcpyAsync(r.beta.data(), beta, (size_t)kq * Nc * sizeof(double), hipMemcpyDeviceToHost,
                               c->stream));
    BasisParams P{};
    P.W = W;
    P.vstride = vstride;
    P.C = 2 * Nc;
    P.Nc = Nc;
    P.scale = scale;
    P.kconv = kconv;
    P.minv = c->minv;
    P.tab = c->tab;
    P.out = r.quad;
    P.n_quad = c->n_quad;
    P.ks = ks;
    P.ncx = c->ncx;
    P.ncy = c->ncy;
    P.p = c->p;
    P.Nx = c->Nx;
    P.Ny = c->Ny;
    P.Nz = c->Nz;
    TDFE_TRY(fp32 ? launch_basis<float>(c, P, kq) : launch_basis<double>(c, P, kq));
    TDFE_HIP(c, hipStreamSynchronize(c->stream));
  }
  (void)k_enq;
  return TDFE_OK;
}

// C for every orbital from the forward (x) and adjoint (z) Krylov records
// returns false if a host allocation failed (in the caller or on a worker
// thread); every started thread has been joined by then
bool small_matrix_impl(const KrylovRecord& X, const KrylovRecord& Z, int Nc, int ks, double tau,
                       std::vector<double>& Cm, std::vector<int>& kk) {
  Cm.assign((size_t)Nc * ks * ks * 2, 0.0);
  kk.assign(2 * Nc, 0);
  auto eig = [&](const KrylovRecord& R, int o, std::vector<double>& th, std::vector<double>& U) {
    const int k = R.k[o];
    std::vector<double> T((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) {
      T[(size_t)j * k + j] = R.alpha[(size_t)j * Nc + o];
      if (j + 1 < k) T[(size_t)j * k + j + 1] = T[(size_t)(j + 1) * k + j] = R.beta[(size_t)j * Nc + o];
    }
    tdfe_sym_eigen(T, k, th, U);
  };
  // orbitals are independent (disjoint output blocks): spread them over a
  // few host threads, the device waits for this step
  auto one = [&](int o) {
    const int kx = X.k[o], kz = Z.k[o];
    if (kx == 0 || kz == 0 || !(X.nrm[o] > 0.0) || !(Z.nrm[o] > 0.0)) return;
    kk[o] = kz;
    kk[Nc + o] = kx;
    std::vector<double> thx, Ux, thz, Uz;
    eig(X, o, thx, Ux);
    eig(Z, o, thz, Uz);
    // M_ab = cz_a G_ab cx_b
    std::vector<double> Mr((size_t)kz * kx), Mi((size_t)kz * kx);
    for (int a = 0; a < kz; ++a)
      for (int b = 0; b < kx; ++b) {
        const double h = 0.5 * tau * (thx[b] - thz[a]);
        const double sinc = std::fabs(h) < 1e-8 ? 1.0 - h * h / 6.0 : std::sin(h) / h;
        const double ph = -0.5 * tau * (thz[a] + thx[b]);
        const double w = Uz[a] * Ux[b] * sinc;  // first rows: U[0 * k + a]
        Mr[(size_t)a * kx + b] = w * std::cos(ph);
        Mi[(size_t)a * kx + b] = w * std::sin(ph);
      }
    // C = nz nx Uz M Ux^T
    const double nn = Z.nrm[o] * X.nrm[o];
    std::vector<double> Tr((size_t)kz * kx, 0.0), Ti((size_t)kz * kx, 0.0);  // Uz M
    for (int j = 0; j < kz; ++j)
      for (int a = 0; a < kz; ++a) {
        const double u = Uz[(size_t)j * kz + a];
        for (int b = 0; b < kx; ++b) {
          Tr[(size_t)j * kx + b] += u * Mr[(size_t)a * kx + b];
          Ti[(size_t)j * kx + b] += u * Mi[(size_t)a * kx + b];
        }
      }
    double* Co = Cm.data() + (size_t)o * ks * ks * 2;
    for (int j = 0; j < kz; ++j)
      for (int l = 0; l < kx; ++l) {
        double sr = 0.0, si = 0.0;
        for (int b = 0; b < kx; ++b) {
          const double u = Ux[(size_t)l * kx + b];
          sr += Tr[(size_t)j * kx + b] * u;
          si += Ti[(size_t)j * kx + b] * u;
        }
        Co[((size_t)j * ks + l) * 2 + 0] = nn * sr;
        Co[((size_t)j * ks + l) * 2 + 1] = nn * si;
      }
  };
  const int nt = std::max(1, std::min({Nc, 8, (int)std::thread::hardware_concurrency()}));
  if (nt == 1) {
    for (int o = 0; o < Nc; ++o) one(o);
    return true;
  }
  std::atomic<bool> failed{false};
  auto share = [&](int w) {
    try {
      for (int o = w; o < Nc; o += nt) one(o);
    } catch (...) {
      failed = true;
    }
  };
  std::vector<std::thread> pool;
  int started = 1;  // workers 1..started-1 run; the caller takes the rest
  try {
    pool.reserve(nt - 1);
    for (int w = 1; w < nt; ++w, ++started) pool.emplace_back(share, w);
  } catch (...) {
    // no more threads (or no room for their handles): the orbitals of
    // unstarted workers run here
  }
  share(0);
  for (int w = started; w < nt; ++w) share(w);
  for (auto& th : pool) th.join();
  return !failed;
}

bool small_matrix(const KrylovRecord& X, const KrylovRecord& Z, int Nc, int ks, double tau, std::vector<double>& Cm,
                  std::vector<int>& kk) {
  try {
    return small_matrix_impl(X, Z, Nc, ks, tau, Cm, kk);
  } catch (...) {
    return false;
  }
}

struct Grad {
  tdfe_ctx* c;
  GradLayout g;
  char* base;
  int n_orb, N;
  double dt, tol;
  const double* E;
  const double* occ = nullptr;
  KrylovRecord XP, XC, Zr;
  CaptureHook hook;
  std::vector<double> Cm_host;
  std::vector<int> kk_host;

  double* state(size_t off, int i = 0) { return (double*)(base + off + (size_t)i * g.state); }
  double* quad(int slot) { return (double*)(base + g.o_q + (size_t)slot * g.quad); }
  double* Wk(int k) { return (double*)(base + g.o_W + (size_t)std::max(k, 0) * g.quad); }
  double* wbar(int k) { return quad(Q_WB0 + (std::max(k, 0) % 3)); }

  tdfe_status lanczos(const void* in, void* out, double tau, KrylovRecord* rec) {
    hook.rec = rec;
    hook.ks = g.ks;
    int kmax = 0, ksum = 0;
    double emax = 0.0;
    return tdfe_lanczos_run(c, c->vw, in, out, n_orb, tau, tol, nullptr, nullptr, &kmax, &ksum, &emax,
                            rec ? &hook : nullptr);
  }

  // one forward step psi_in -> psi_out; phi_out receives the predictor state,
  // Wnew (may be null) W[rho(psi_out)]; records capture the two Krylov runs
  tdfe_status step(int n, const double* psi_in, double* psi_out, double* phi_out, double* Wnew, KrylovRecord* rp,
                   KrylovRecord* rc) {
    if (!c->have_scf) {
      TDFE_TRY(tdfe_assemble_vw(c, nullptr, 0.0, nullptr, 0.0, E[n]));
      return lanczos(psi_in, psi_out, dt, rc);
    }
    TDFE_TRY(tdfe_assemble_vw(c, Wk(n), 1.25, Wk(n - 1), -0.25, E[n]));
    TDFE_TRY(lanczos(psi_in, phi_out, 0.5 * dt, rp));
    TDFE_TRY(tdfe_scf_potential(c, phi_out, n_orb, quad(Q_WH), nullptr, nullptr));
    TDFE_HIP(c, hipMemcpyAsync(quad(Q_RHOH), c->rho, c->n_quad * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    TDFE_TRY(tdfe_assemble_vw(c, quad(Q_WH), 1.0, nullptr, 0.0, E[n]));
    TDFE_TRY(lanczos(psi_in, psi_out, dt, rc));
    if (Wnew) TDFE_TRY(tdfe_scf_potential(c, psi_out, n_orb, Wnew, nullptr, nullptr));
    return TDFE_OK;
  }

  // y += psib = 2 f M^-1/2 I^T (rhob . I M^-1/2 psi)  with vw2 = 2 rhob
  tdfe_status density_adjoint(const double* psi, const double* vw2, double* y) {
    ApplyArgs a{};
    a.x = psi;
    a.y = y;
    a.ld = 2 * n_orb;
    a.cols = 2 * n_orb;
    a.colscale = occ;
    a.kin = 0.0;
    a.vw = vw2;
    a.lowdin = true;
    a.fp32 = false;
    return tdfe_launch_apply(c, a);
  }

  // out = 2 rhob for a cotangent Wb of W[rho] at density rho
  tdfe_status w_adjoint(const double* Wb, const double* rho, double* out) {
    const double* vh = nullptr;
    if (c->hartree) {
      TDFE_TRY(tdfe_load_vector(c, Wb, false));
      double* full = (double*)(base + g.o_full);
      TDFE_TRY(tdfe_fdm_solve_into(c, false, full));
      TDFE_TRY(tdfe_interp_field(c, full, nullptr, TDFE_XC_NONE, quad(Q_VH)));
      vh = quad(Q_VH);
    }
    hipLaunchKernelGGL(w_adjoint_kernel, dim3(nblk(c->n_quad)), dim3(EW), 0, c->stream, Wb, rho, c->wdet, vh, c->xc,
                       2.0, out, c->n_quad);
    TDFE_HIP(c, hipGetLastError());
    return TDFE_OK;
  }

  // Vb for the exponential recorded in X (forward) and Zr (adjoint run with -tau)
  tdfe_status potential_cotangent(const KrylovRecord& X, double tau, double* Vb) {
    if (!small_matrix(X, Zr, n_orb, g.ks, tau, Cm_host, kk_host))
      return tdfe_fail(c, TDFE_ENOMEM, "gradient: host allocation failed in the small-matrix step");
    double* Cm = (double*)(base + g.o_cm);
    int* kk = (int*)(base + g.o_k);
    TDFE_HIP(c, hipMemcpyAsync(Cm, Cm_host.data(), Cm_host.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    TDFE_HIP(c, hipMemcpyAsync(kk, kk_host.data(), kk_host.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(bilinear_kernel, dim3(nblk(c->n_quad)), dim3(EW), 0, c->stream, (const double2*)Zr.quad,
                       (const double2*)X.quad, (const double2*)Cm, (const int*)kk, (const int*)(kk + n_orb), n_orb,
                       g.ks, c->n_quad, tau, c->wdet, Vb);
    TDFE_HIP(c, hipGetLastError());
    // the host vectors are reused by the next call
    TDFE_HIP(c, hipStreamSynchronize(c->stream));
    return TDFE_OK;
  }

  tdfe_status field_grad(int n, const double* v1, const double* v2) {
    double* part = (double*)(base + g.o_part);
    hipLaunchKernelGGL(zdot_kernel, dim3(RED_BLOCKS), dim3(EW), 0, c->stream, v1, v2, c->xq, c->n_quad,
                       c->fdir[0], c->fdir[1], c->fdir[2], part);
    hipLaunchKernelGGL(neg_sum_kernel, dim3(1), dim3(EW), 0, c->stream, (const double*)part, RED_BLOCKS,
                       (double*)(base + g.o_de) + n);
    TDFE_HIP(c, hipGetLastError());
    return TDFE_OK;
  }

  tdfe_status zero(void* p, size_t b) {
    TDFE_HIP(c, hipMemsetAsync(p, 0, b, c->stream));
    return TDFE_OK;
  }

  tdfe_status copy(void* dst, const void* src, size_t b) {
    TDFE_HIP(c, hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToDevice, c->stream));
    return TDFE_OK;
  }

  // reverse of step n; lam holds the cotangent of psi^{n+1} on entry and of psi^n on exit
  tdfe_status reverse_step(int n, const double* psi_n, const double* psi_n1) {
    const size_t sb = (size_t)c->n_dof * 2 * n_orb * sizeof(double);
    const int64_t nq = c->n_quad;
    double* lam = state(g.o_lam);
    double* lamh = state(g.o_lamh);
    double* xbc = state(g.o_xbc);
    double* phi = state(g.o_phi);
    double* tmp = state(g.o_tmp);
    // recompute the step with the Krylov records
    TDFE_TRY(step(n, psi_n, tmp, phi, nullptr, &XP, &XC));
    // pending W cotangent of psi^{n+1}
    if (c->have_scf && n + 1 <= N - 1) {
      TDFE_TRY(tdfe_density_dev(c, psi_n1, n_orb, quad(Q_RHO1), c->partial));
      TDFE_TRY(w_adjoint(wbar(n + 1), quad(Q_RHO1), quad(Q_RB)));
      TDFE_TRY(density_adjoint(psi_n1, quad(Q_RB), lam));
      TDFE_TRY(zero(wbar(n + 1), nq * sizeof(double)));
    }
    // corrector: potential V_C is in c->vw after step()
    TDFE_TRY(lanczos(lam, xbc, -dt, &Zr));
    TDFE_TRY(potential_cotangent(XC, dt, quad(Q_VBC)));
    if (!c->have_scf) {
      TDFE_TRY(field_grad(n, quad(Q_VBC), nullptr));
      return copy(lam, xbc, sb);
    }
    // midpoint W of phi -> phi's cotangent -> predictor
    TDFE_TRY(w_adjoint(quad(Q_VBC), quad(Q_RHOH), quad(Q_RB)));
    TDFE_TRY(zero(lamh, sb));
    TDFE_TRY(density_adjoint(phi, quad(Q_RB), lamh));
    TDFE_TRY(tdfe_assemble_vw(c, Wk(n), 1.25, Wk(n - 1), -0.25, E[n]));
    TDFE_TRY(lanczos(lamh, lamh, -0.5 * dt, &Zr));
    TDFE_TRY(potential_cotangent(XP, 0.5 * dt, quad(Q_VBP)));
    TDFE_TRY(field_grad(n, quad(Q_VBC), quad(Q_VBP)));
    // W_n enters V_P with 1.25, W_{n-1} with -0.25
    hipLaunchKernelGGL(wbar_update_kernel, dim3(nblk(nq)), dim3(EW), 0, c->stream, (const double*)quad(Q_VBP),
                       wbar(n), 1.25, wbar(n - 1), -0.25, nq);
    hipLaunchKernelGGL(add_kernel, dim3(nblk((int64_t)c->n_dof * 2 * n_orb)), dim3(EW), 0, c->stream,
                       (const double*)xbc, (const double*)lamh, lam, (int64_t)c->n_dof * 2 * n_orb);
    TDFE_HIP(c, hipGetLastError());
    return TDFE_OK;
  }

  tdfe_status run(const void* psi0, double* L, double* grad) {
    const size_t sb = (size_t)c->n_dof * 2 * n_orb * sizeof(double);
    const int64_t nq = c->n_quad;
    XP.quad = (double2*)(base + g.o_qx_p);
    XC.quad = (double2*)(base + g.o_qx_c);
    Zr.quad = (double2*)(base + g.o_qz);
    TDFE_TRY(tdfe_occ_dev(c, n_orb, &occ));
    TDFE_TRY(zero(base + g.o_full, (size_t)c->n_nodes * sizeof(double)));
    for (int i = 0; i < 3; ++i) TDFE_TRY(zero(quad(Q_WB0 + i), nq * sizeof(double)));
    TDFE_TRY(zero(base + g.o_de, (size_t)N * sizeof(double)));
    // forward sweep: checkpoints, the W history and the last segment's states
    const int last0 = (g.S - 1) * g.Cseg;
    double* cur = state(g.o_cur);
    double* nxt = state(g.o_nxt);
    TDFE_TRY(copy(cur, psi0, sb));
    if (c->have_scf) TDFE_TRY(tdfe_scf_potential(c, cur, n_orb, Wk(0), nullptr, nullptr));
    for (int n = 0; n < N; ++n) {
      if (n % g.Cseg == 0) TDFE_TRY(copy(state(g.o_ckpt, n / g.Cseg), cur, sb));
      if (n >= last0) TDFE_TRY(copy(state(g.o_seg, n - last0), cur, sb));
      TDFE_TRY(step(n, cur, nxt, state(g.o_phi), (c->have_scf && n + 1 < N) ? Wk(n + 1) : nullptr, nullptr,
                    nullptr));
      std::swap(cur, nxt);
    }
    TDFE_TRY(copy(state(g.o_seg, N - last0), cur, sb));
    double mu[3], ch;
    TDFE_TRY(tdfe_dipole(c, cur, n_orb, mu, &ch));
    *L = mu[2];
    // cotangent of psi^N
    TDFE_TRY(zero(state(g.o_lam), sb));
    hipLaunchKernelGGL(dipole_cotangent_kernel, dim3(nblk(nq)), dim3(EW), 0, c->stream, c->wdet, c->xq, quad(Q_RB),
                       nq);
    TDFE_HIP(c, hipGetLastError());
    TDFE_TRY(density_adjoint(cur, quad(Q_RB), state(g.o_lam)));
    // reverse sweep, one segment at a time
    for (int s = g.S - 1; s >= 0; --s) {
      const int n0 = s * g.Cseg, n1 = std::min(N, n0 + g.Cseg);
      if (s < g.S - 1) {
        TDFE_TRY(copy(state(g.o_seg, 0), state(g.o_ckpt, s), sb));
        for (int n = n0; n < n1; ++n)
          TDFE_TRY(step(n, state(g.o_seg, n - n0), state(g.o_seg, n - n0 + 1), state(g.o_phi), nullptr, nullptr,
                        nullptr));
      }
      for (int n = n1 - 1; n >= n0; --n)
        TDFE_TRY(reverse_step(n, state(g.o_seg, n - n0), state(g.o_seg, n - n0 + 1)));
    }
    TDFE_HIP(c, hipMemcpyAsync(grad, base + g.o_de, (size_t)N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    // leave the operator potential as set_potential defined it
    TDFE_TRY(tdfe_assemble_vw(c, nullptr, 0.0, nullptr, 0.0, 0.0));
    TDFE_HIP(c, hipStreamSynchronize(c->stream));
    for (int n = 0; n < N; ++n)
      if (!std::isfinite(grad[n])) return tdfe_fail(c, TDFE_ENONFINITE, "gradient: non-finite value at step %d", n);
    return TDFE_OK;
  }
};

tdfe_status grad_checks(tdfe_ctx* c, int n_orb, int n_steps, int ckpt, int k_store) {
  if (!c) return TDFE_EINVAL;
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "gradient before bind_workspace");
  if (c->octree) return tdfe_fail(c, TDFE_EINVAL, "gradient: not on octree meshes");
  if (n_orb < 1 || n_orb > c->n_orb_max) return tdfe_fail(c, TDFE_EINVAL, "gradient: n_orb out of range");
  if (n_orb > c->chunk_orb) return tdfe_fail(c, TDFE_EINVAL, "gradient: orbitals must fit one Lanczos chunk");
  if (n_steps < 1 || ckpt < 1) return tdfe_fail(c, TDFE_EINVAL, "gradient: n_steps and checkpoint_every must be >= 1");
  if (k_store < 1 || k_store > c->k_max || k_store % 8 != 0)
    return tdfe_fail(c, TDFE_EINVAL, "gradient: k_store must be a multiple of 8 in [8, k_max]");
  return TDFE_OK;
}

}  // namespace

extern "C" {

tdfe_status tdfe_gradient_query(tdfe_ctx* c, int n_orb, int n_steps, int checkpoint_every, int k_store,
                                size_t* bytes) {
  if (!bytes) return TDFE_EINVAL;
  TDFE_TRY(grad_checks(c, n_orb, n_steps, checkpoint_every, k_store));
  *bytes = layout(c, n_orb, n_steps, checkpoint_every, k_store).total;
  return TDFE_OK;
}

tdfe_status tdfe_dipole_gradient(tdfe_ctx* c, const void* dev_psibar0, int n_orb, int n_steps, const double* host_E,
                                 double dt, double tol, int checkpoint_every, int k_store, void* dev_work,
                                 size_t work_bytes, double* host_L, double* host_grad) {
  if (!c || !dev_psibar0 || !host_E || !dev_work || !host_L || !host_grad) return TDFE_EINVAL;
  TDFE_TRY(grad_checks(c, n_orb, n_steps, checkpoint_every, k_store));
  if (!c->have_potential) return tdfe_fail(c, TDFE_ESTATE, "gradient before set_potential");
  if (!(dt > 0.0) || !std::isfinite(dt) || !(tol > 0.0)) return tdfe_fail(c, TDFE_EINVAL, "gradient: dt or tol");
  for (int n = 0; n < n_steps; ++n)
    if (!std::isfinite(host_E[n])) return tdfe_fail(c, TDFE_EINVAL, "gradient: non-finite field amplitude");
  if (c->xc == TDFE_XC_XC)
    return tdfe_fail(c, TDFE_EINVAL, "gradient: the exchange-correlation kernel is available for LDA exchange only");
  if (c->hartree && !c->box) return tdfe_fail(c, TDFE_EINVAL, "gradient: Hartree needs a box mesh");
  if (c->mid_mode != TDFE_MIDPOINT_PC || c->mid_order != 1)
    return tdfe_fail(c, TDFE_EINVAL, "gradient: the predictor-corrector midpoint with linear extrapolation only");
  Grad G;
  G.c = c;
  G.g = layout(c, n_orb, n_steps, checkpoint_every, k_store);
  if (work_bytes < G.g.total) return tdfe_fail(c, TDFE_EINVAL, "gradient: workspace too small (%zu < %zu)", work_bytes,
                                               G.g.total);
  if (((uintptr_t)dev_work & 255) != 0) return tdfe_fail(c, TDFE_EINVAL, "gradient: workspace must be 256-byte aligned");
  G.base = (char*)dev_work;
  G.n_orb = n_orb;
  G.N = n_steps;
  G.dt = dt;
  G.tol = tol;
  G.E = host_E;
  return G.run(dev_psibar0, host_L, host_grad);
}

}  // extern "C"
