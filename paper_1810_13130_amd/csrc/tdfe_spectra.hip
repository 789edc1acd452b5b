// Excitations and observables of a real-time run (Sec. on the numerical
// studies, the table of simulation parameters, Eq. VField):
//   * the direction d of the external field, V_field = -E_n (d . r);
//   * the delta kick psibar <- exp(-i kappa d . r) psibar at the DoF nodes;
//   * field shapes: the weak Gaussian pulse and the sin^2-enveloped laser;
//   * the absorption spectrum S(w) = (2w / 3 pi) Tr Im alpha(w) with a
//     Gaussian window on the induced dipole, and the dipole power spectrum
//     P(w) = Im int e^{-iwt} d^2 mu / dt^2 dt.
// The spectra are direct quadratures over the dipole samples: one block per
// frequency, each lane summing a strided share of the samples, combined in a
// fixed order (the result does not depend on scheduling).
#include <cmath>

#include "tdfe_internal.h"

namespace {

constexpr int SP_THREADS = 256;

// fixed-order block sum of NV values per lane; results valid in lane 0
template <int NV>
__device__ void block_sum(double (&v)[NV]) {
  __shared__ double s[NV][SP_THREADS];
#pragma unroll
  for (int k = 0; k < NV; ++k) s[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = SP_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = s[k][0];
}

__device__ __forceinline__ double trap_weight(int n, int n0, int n1) { return (n == n0 || n == n1) ? 0.5 : 1.0; }

// For each direction a: mu~_a(w) = sum_n tw_n e^{i w t_n} e^{-alpha t_n^2} (mu_a(t_n) - mu_a(t_0)) dt,
// E~_a(w) = sum_n tw_n e^{i w t_n} E_a(t_n) dt (or -kappa for a kick exp(-i kappa r_a)),
// S(w) = (2 w / 3 pi) sum_a Im(mu~_a / E~_a)
__global__ void __launch_bounds__(SP_THREADS)
    absorption_kernel(const double* __restrict__ mu, const double* __restrict__ field, int n_t, double dt,
                      double kappa, double alpha, const double* __restrict__ omega, double* __restrict__ S) {
  const double w = omega[blockIdx.x];
  double v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = 0.0;
  for (int n = threadIdx.x; n < n_t; n += SP_THREADS) {
    const double t = n * dt;
    double sn, cn;
    sincos(w * t, &sn, &cn);
    const double tw = trap_weight(n, 0, n_t - 1) * dt;
    const double g = tw * exp(-alpha * t * t);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double m = (mu[(int64_t)a * n_t + n] - mu[(int64_t)a * n_t]) * g;
      v[4 * a + 0] += m * cn;
      v[4 * a + 1] += m * sn;
      if (field) {
        const double e = field[(int64_t)a * n_t + n] * tw;
        v[4 * a + 2] += e * cn;
        v[4 * a + 3] += e * sn;
      }
    }
  }
  block_sum(v);
  if (threadIdx.x != 0) return;
  double acc = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double mr = v[4 * a], mi = v[4 * a + 1];
    const double er = field ? v[4 * a + 2] : -kappa, ei = field ? v[4 * a + 3] : 0.0;
    // Im(m / e) = (mi er - mr ei) / |e|^2
    acc += (mi * er - mr * ei) / (er * er + ei * ei);
  }
  S[blockIdx.x] = 2.0 * w / (3.0 * M_PI) * acc;
}

// P(w) = Im sum_{n=1}^{N-2} tw_n e^{-i w t_n} (mu_{n+1} - 2 mu_n + mu_{n-1}) / dt^2 dt
__global__ void __launch_bounds__(SP_THREADS)
    power_kernel(const double* __restrict__ mu, int n_t, double dt, const double* __restrict__ omega,
                 double* __restrict__ P) {
  const double w = omega[blockIdx.x];
  double v[1] = {0.0};
  for (int n = 1 + threadIdx.x; n < n_t - 1; n += SP_THREADS) {
    const double acc2 = (mu[n + 1] - 2.0 * mu[n] + mu[n - 1]) / (dt * dt);
    const double tw = trap_weight(n, 1, n_t - 2) * dt;
    v[0] += -sin(w * (n * dt)) * acc2 * tw;
  }
  block_sum(v);
  if (threadIdx.x == 0) P[blockIdx.x] = v[0];
}

// psibar[j][alpha] *= exp(-i kappa d . r_j)
__global__ void kick_kernel(double* psibar, int n_orb, const double* dofxyz, double kx, double ky, double kz,
                            int64_t n_dof) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_dof * n_orb) return;
  const int64_t j = idx / n_orb;
  const double ph = kx * dofxyz[j * 3] + ky * dofxyz[j * 3 + 1] + kz * dofxyz[j * 3 + 2];
  double s, c;
  sincos(ph, &s, &c);
  const double re = psibar[2 * idx], im = psibar[2 * idx + 1];
  // (re + i im)(c - i s)
  psibar[2 * idx] = re * c + im * s;
  psibar[2 * idx + 1] = im * c - re * s;
}

bool finite3(const double* d) { return std::isfinite(d[0]) && std::isfinite(d[1]) && std::isfinite(d[2]); }

}  // namespace

extern "C" {

tdfe_status tdfe_set_field_direction(tdfe_ctx* c, const double* dir) {
  if (!c || !dir) return TDFE_EINVAL;
  if (!finite3(dir) || (dir[0] == 0.0 && dir[1] == 0.0 && dir[2] == 0.0))
    return tdfe_fail(c, TDFE_EINVAL, "set_field_direction: zero or non-finite direction");
  for (int k = 0; k < 3; ++k) c->fdir[k] = dir[k];
  return TDFE_OK;
}

tdfe_status tdfe_kick(tdfe_ctx* c, void* dev_psibar, int n_orb, double kappa) {
  if (!c || !dev_psibar) return TDFE_EINVAL;
  if (n_orb < 1 || n_orb > c->n_orb_max) return tdfe_fail(c, TDFE_EINVAL, "kick: n_orb out of range");
  if (!std::isfinite(kappa)) return tdfe_fail(c, TDFE_EINVAL, "kick: non-finite kappa");
  if (!c->bound) return tdfe_fail(c, TDFE_ESTATE, "kick before bind_workspace");
  const int64_t n = c->n_dof * n_orb;
  hipLaunchKernelGGL(kick_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, (double*)dev_psibar,
                     n_orb, (const double*)c->dofxyz, kappa * c->fdir[0], kappa * c->fdir[1], kappa * c->fdir[2],
                     c->n_dof);
  TDFE_HIP(c, hipGetLastError());
  return TDFE_OK;
}

tdfe_status tdfe_field_samples(int shape, const double* params, int n, const double* t, double* out) {
  if (!params || !t || !out || n < 0) return TDFE_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(params[k])) return TDFE_EINVAL;
  if (shape == TDFE_FIELD_GAUSSIAN) {
    const double kap = params[0], t0 = params[1], w = params[2];
    if (!(w > 0.0)) return TDFE_EINVAL;
    for (int i = 0; i < n; ++i) {
      const double u = (t[i] - t0) / w;
      out[i] = kap * std::exp(-u * u);
    }
    return TDFE_OK;
  }
  if (shape == TDFE_FIELD_SIN2) {
    const double kap = params[0], om = params[1], T = params[2];
    if (!(T > 0.0)) return TDFE_EINVAL;
    for (int i = 0; i < n; ++i) {
      if (t[i] < 0.0 || t[i] > T) {
        out[i] = 0.0;
        continue;
      }
      const double s = std::sin(M_PI * t[i] / T);
      out[i] = kap * s * s * std::sin(om * t[i]);
    }
    return TDFE_OK;
  }
  return TDFE_EINVAL;
}

tdfe_status tdfe_absorption_spectrum(const double* dev_mu, const double* dev_field, int n_t, double dt,
                                     double kappa, double alpha, const double* dev_omega, int n_omega,
                                     double* dev_S, void* hip_stream) {
  if (!dev_mu || !dev_omega || !dev_S || n_t < 2 || n_omega < 0) return TDFE_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt) || !(alpha >= 0.0) || !std::isfinite(alpha)) return TDFE_EINVAL;
  if (!dev_field && (!(kappa != 0.0) || !std::isfinite(kappa))) return TDFE_EINVAL;
  if (n_omega == 0) return TDFE_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(absorption_kernel, dim3(n_omega), dim3(SP_THREADS), 0, st, dev_mu, dev_field, n_t, dt, kappa,
                     alpha, dev_omega, dev_S);
  return hipGetLastError() == hipSuccess ? TDFE_OK : TDFE_EDEVICE;
}

tdfe_status tdfe_power_spectrum(const double* dev_mu, int n_t, double dt, const double* dev_omega, int n_omega,
                                double* dev_P, void* hip_stream) {
  if (!dev_mu || !dev_omega || !dev_P || n_t < 3 || n_omega < 0) return TDFE_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt)) return TDFE_EINVAL;
  if (n_omega == 0) return TDFE_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(power_kernel, dim3(n_omega), dim3(SP_THREADS), 0, st, dev_mu, n_t, dt, dev_omega, dev_P);
  return hipGetLastError() == hipSuccess ? TDFE_OK : TDFE_EDEVICE;
}

}  // extern "C"
