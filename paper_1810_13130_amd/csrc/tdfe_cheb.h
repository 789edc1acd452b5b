// Chebyshev evaluation of y = exp(-i s T) e_1 for a real symmetric tridiagonal
// T (k x k; diagonal sa[0..k), off-diagonal sb[0..k-1)), on one workgroup of
// TDFE_CHEB_THREADS lanes: Gershgorin interval [c - r, c + r], Jacobi-Anger
// coefficients 2 (-i sgn(s))^m J_m(|s| r), Bessel values by Miller's backward
// recurrence normalised with J_0 + 2 sum J_2m = 1, and the three-term
// recurrence v_{m+1} = 2 X v_m - v_{m-1}, X = (T - c)/r, v_0 = e_1, rows across
// lanes.  cheb_expm_e1 and cheb_expm_e1_wave run on a one-wavefront
// workgroup and use its barriers; cheb_expm_e1_wave_gtab involves one
// wavefront of a larger workgroup only.  Every path reads its Bessel
// coefficients from a per-orbital table in global memory.
#pragma once
#include <hip/hip_runtime.h>

#define TDFE_CHEB_THREADS 64
// largest Bessel table: |s| r up to about 6.5e4 (the all-electron-like
// workload's smallest cells reach a few 1e4 at its dt)
#define TDFE_MAX_BESSEL 65536
#define TDFE_KCAP 1024
// per-orbital Bessel table in global memory (every evaluation path): the
// table plus two register chunks of padding for the look-ahead load
#define TDFE_JTAB_STRIDE (TDFE_MAX_BESSEL + 2 + 2 * TDFE_CHEB_THREADS)

struct ChebLds {
  double yr[TDFE_KCAP], yi[TDFE_KCAP];
  double red[3 * TDFE_CHEB_THREADS];
  double inv;  // normalisation of the Bessel table
  int M;
};

// Bessel values J_0..J_M(z) into J (by the calling lane); returns M, -1 if z
// exceeds the table, or -2 if z is not finite (an Inf in T).  z is bounded
// before it is converted to an integer, so no term count can overflow.
// Miller's backward recurrence runs in registers (the table is only written);
// the values are left unnormalised and *inv receives 1 / (J_0 + 2 sum J_2m),
// which callers apply to the Chebyshev coefficients.
#define TDFE_CHEB_NONFINITE (-2)
__device__ inline int cheb_bessel(double z, double* J, double* inv) {
  int M = 0;
  *inv = 1.0;
  if (isnan(z) || isinf(z)) return TDFE_CHEB_NONFINITE;
  if (z > 2.0 * TDFE_MAX_BESSEL) return -1;
  if (z > 1e-300) {
    M = (int)ceil(z + 10.0 * cbrt(z) + 20.0);
    int ms = M + 20 + (int)(2.0 * sqrt((double)M));
    ms += ms & 1;
    if (ms + 1 > TDFE_MAX_BESSEL) return -1;
    double jp = 0.0, jc = 1e-300;  // J_{m+1}, J_m
    J[ms + 1] = jp;
    J[ms] = jc;
    double even = jc;  // sum of J_2m for 2m >= 2 (ms is even)
    const double tz = 2.0 / z;
    for (int m = ms; m > 0; --m) {
      const double jm1 = (m * tz) * jc - jp;
      J[m - 1] = jm1;
      if (((m - 1) & 1) == 0 && m - 1 > 0) even += jm1;
      jp = jc;
      jc = jm1;
      if (fabs(jm1) > 1e250) {  // rescale what has been produced so far
        for (int q = m - 1; q <= ms + 1; ++q) J[q] *= 1e-250;
        jp *= 1e-250;
        jc *= 1e-250;
        even *= 1e-250;
      }
    }
    *inv = 1.0 / (jc + 2.0 * even);  // jc = J_0
  } else {
    J[0] = 1.0;
    *inv = 1.0;
  }
  return M;
}

// whole-wavefront neighbour exchange by DPP row shifts (the value of lane t-1,
// resp. t+1; 0 at the ends): no LDS traffic
__device__ __forceinline__ double lane_prev(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);  // wave_shr:1
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_next(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);  // wave_shl:1
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_read(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Same result for k <= TDFE_CHEB_THREADS, one row per lane of a single
// wavefront: the Chebyshev vectors stay in registers and the tridiagonal
// neighbours come from DPP lane shifts, so a term costs no LDS round trip.
// Lane j returns row j of y in (yr, yi) (zero for j >= k).  J is the
// orbital's global table of TDFE_JTAB_STRIDE entries, Ms / invs LDS scalars;
// every lane keeps 64 consecutive coefficients in one register and each term
// takes its own by a lane read.
__device__ inline int cheb_expm_e1_wave(int k, const double* sa, const double* sb, double s, double* J, int* Ms,
                                        double* invs, double& yr, double& yi, double* amax) {
  const int t = threadIdx.x;
  const bool row = t < k;
  const double a = row ? sa[t] : 0.0;
  const double bl = (row && t > 0) ? sb[t - 1] : 0.0;
  const double br = (row && t < k - 1) ? sb[t] : 0.0;
  double lo = row ? a - fabs(bl) - fabs(br) : 1e300;
  double hi = row ? a + fabs(bl) + fabs(br) : -1e300;
  double am = row ? fabs(a) : 0.0;
  for (int off = TDFE_CHEB_THREADS / 2; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off));
    hi = fmax(hi, __shfl_xor(hi, off));
    am = fmax(am, __shfl_xor(am, off));
  }
  *amax = am;
  const double cc = 0.5 * (lo + hi), rr = 0.5 * (hi - lo);
  const double z = fabs(s) * rr;
  if (t == 0) *Ms = cheb_bessel(z, J, invs);
  // lane 0's table stores complete and are visible to every lane's loads
  __threadfence();
  __syncthreads();
  const int M = *Ms;
  const double jn = *invs;
  yr = 0.0;
  yi = 0.0;
  if (M < 0) return M;
  const double sgn = s >= 0.0 ? 1.0 : -1.0;
  const double invr = rr > 0.0 ? 1.0 / rr : 0.0;
  const double ac = row ? a - cc : 0.0;
  double jr = J[t];
  double jnx = J[TDFE_CHEB_THREADS + t];
  double vp = (t == 0) ? 1.0 : 0.0;
  yr = jn * lane_read(jr, 0) * vp;
  if (M >= 1) {
    double left = lane_prev(vp), right = lane_next(vp);
    double vc = (ac * vp + bl * left + br * right) * invr;
    yi += -2.0 * sgn * jn * lane_read(jr, 1) * vc;
    for (int mm = 2; mm <= M; ++mm) {
      if ((mm & (TDFE_CHEB_THREADS - 1)) == 0) {
        jr = jnx;
        jnx = J[mm + TDFE_CHEB_THREADS + t];  // < TDFE_JTAB_STRIDE since mm <= M < TDFE_MAX_BESSEL
      }
      left = lane_prev(vc);
      right = lane_next(vc);
      const double w = ac * vc + bl * left + br * right;
      const double vn = 2.0 * w * invr - vp;
      vp = vc;
      vc = vn;
      const double cj = 2.0 * jn * lane_read(jr, mm & (TDFE_CHEB_THREADS - 1));
      const int ph = mm & 3;  // (-i sgn)^m : 1, -i sgn, -1, +i sgn
      if (ph == 0) yr += cj * vn;
      else if (ph == 1) yi -= sgn * cj * vn;
      else if (ph == 2) yr -= cj * vn;
      else yi += sgn * cj * vn;
    }
  }
  const double pr = cos(s * cc), pim = -sin(s * cc);
  const double a0 = yr, b0 = yi;
  yr = a0 * pr - b0 * pim;
  yi = a0 * pim + b0 * pr;
  return M;
}

// The same series as cheb_expm_e1_wave, with the same arithmetic in the same
// order, for a wavefront that has no LDS to spare (it runs inside a streaming
// kernel): the Bessel values go to a global table Jg of TDFE_JTAB_STRIDE
// doubles owned by the calling wavefront, every lane then holds 64
// consecutive entries in one register (the next 64 loaded one chunk ahead),
// and each term takes its coefficient by a lane read.  Called by one full
// wavefront (lanes 0..63, all active, no other wavefront of the workgroup
// involved).  a, bl, br: row t of T (diagonal, left and right off-diagonal;
// zero for rows t >= k).  Returns M, -1 if |s| r exceeds the table, or
// TDFE_CHEB_NONFINITE.
__device__ inline int cheb_expm_e1_wave_gtab(int k, double a, double bl, double br, double s, double* Jg,
                                             double& yr, double& yi, double* amax) {
  const int t = threadIdx.x;
  const bool row = t < k;
  double lo = row ? a - fabs(bl) - fabs(br) : 1e300;
  double hi = row ? a + fabs(bl) + fabs(br) : -1e300;
  double am = row ? fabs(a) : 0.0;
  for (int off = TDFE_CHEB_THREADS / 2; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off));
    hi = fmax(hi, __shfl_xor(hi, off));
    am = fmax(am, __shfl_xor(am, off));
  }
  *amax = am;
  const double cc = 0.5 * (lo + hi), rr = 0.5 * (hi - lo);
  const double z = fabs(s) * rr;
  int m0 = 0;
  double inv0 = 0.0;
  if (t == 0) m0 = cheb_bessel(z, Jg, &inv0);
  // lane 0's table stores complete and are visible to every lane's loads
  __threadfence();
  const int M = __builtin_amdgcn_readfirstlane(m0);
  const double jn = lane_read(inv0, 0);
  yr = 0.0;
  yi = 0.0;
  if (M < 0) return M;
  const double sgn = s >= 0.0 ? 1.0 : -1.0;
  const double invr = rr > 0.0 ? 1.0 / rr : 0.0;
  const double ac = row ? a - cc : 0.0;
  double jr = Jg[t];
  double jnx = Jg[TDFE_CHEB_THREADS + t];
  double vp = (t == 0) ? 1.0 : 0.0;
  yr = jn * lane_read(jr, 0) * vp;
  if (M >= 1) {
    double left = lane_prev(vp), right = lane_next(vp);
    double vc = (ac * vp + bl * left + br * right) * invr;
    yi += -2.0 * sgn * jn * lane_read(jr, 1) * vc;
    for (int mm = 2; mm <= M; ++mm) {
      if ((mm & (TDFE_CHEB_THREADS - 1)) == 0) {
        jr = jnx;
        jnx = Jg[mm + TDFE_CHEB_THREADS + t];  // < TDFE_JTAB_STRIDE since mm <= M < TDFE_MAX_BESSEL
      }
      left = lane_prev(vc);
      right = lane_next(vc);
      const double w = ac * vc + bl * left + br * right;
      const double vn = 2.0 * w * invr - vp;
      vp = vc;
      vc = vn;
      const double cj = 2.0 * jn * lane_read(jr, mm & (TDFE_CHEB_THREADS - 1));
      const int ph = mm & 3;  // (-i sgn)^m : 1, -i sgn, -1, +i sgn
      if (ph == 0) yr += cj * vn;
      else if (ph == 1) yi -= sgn * cj * vn;
      else if (ph == 2) yr -= cj * vn;
      else yi += sgn * cj * vn;
    }
  }
  const double pr = cos(s * cc), pim = -sin(s * cc);
  const double a0 = yr, b0 = yi;
  yr = a0 * pr - b0 * pim;
  yi = a0 * pim + b0 * pr;
  return M;
}

// Same function for k > TDFE_CHEB_THREADS: R consecutive rows per lane of one
// wavefront (lane t holds rows R t .. R t + R - 1), the Chebyshev vectors in
// registers, the neighbours across lanes by DPP shifts, so that a term costs
// no LDS round trip or barrier.  sa / sb: diagonal and off-diagonal (any
// memory the wavefront can read); row R t + r of y is returned in yr[r],
// yi[r] (zero past k).
template <int R>
__device__ inline int cheb_expm_e1_rows(int k, const double* sa, const double* sb, double s, double* Jg,
                                        double (&yr)[R], double (&yi)[R], double* amax) {
  const int t = threadIdx.x;
  double a[R], bl[R], br[R];
  double lo = 1e300, hi = -1e300, am = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = R * t + r;
    const bool row = j < k;
    a[r] = row ? sa[j] : 0.0;
    bl[r] = (row && j > 0) ? sb[j - 1] : 0.0;
    br[r] = (row && j < k - 1) ? sb[j] : 0.0;
    if (row) {
      lo = fmin(lo, a[r] - fabs(bl[r]) - fabs(br[r]));
      hi = fmax(hi, a[r] + fabs(bl[r]) + fabs(br[r]));
      am = fmax(am, fabs(a[r]));
    }
  }
  for (int off = TDFE_CHEB_THREADS / 2; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off));
    hi = fmax(hi, __shfl_xor(hi, off));
    am = fmax(am, __shfl_xor(am, off));
  }
  *amax = am;
  const double cc = 0.5 * (lo + hi), rr = 0.5 * (hi - lo);
  const double z = fabs(s) * rr;
  int m0 = 0;
  double inv0 = 0.0;
  if (t == 0) m0 = cheb_bessel(z, Jg, &inv0);
  // lane 0's table stores complete and are visible to every lane's loads
  __threadfence();
  const int M = __builtin_amdgcn_readfirstlane(m0);
  const double jn = lane_read(inv0, 0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    yr[r] = 0.0;
    yi[r] = 0.0;
  }
  if (M < 0) return M;
  const double sgn = s >= 0.0 ? 1.0 : -1.0;
  const double invr = rr > 0.0 ? 1.0 / rr : 0.0;
  double ac[R], vp[R], vc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    ac[r] = (R * t + r < k) ? a[r] - cc : 0.0;
    vp[r] = (t == 0 && r == 0) ? 1.0 : 0.0;
  }
  double jr = Jg[t];
  double jnx = Jg[TDFE_CHEB_THREADS + t];
  yr[0] = jn * lane_read(jr, 0) * vp[0];
  if (M >= 1) {
    {
      const double left = lane_prev(vp[R - 1]), right = lane_next(vp[0]);
      const double J1 = lane_read(jr, 1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double l = r > 0 ? vp[r - 1] : left, rt = r < R - 1 ? vp[r + 1] : right;
        vc[r] = (ac[r] * vp[r] + bl[r] * l + br[r] * rt) * invr;
        yi[r] += -2.0 * sgn * jn * J1 * vc[r];
      }
    }
    for (int mm = 2; mm <= M; ++mm) {
      if ((mm & (TDFE_CHEB_THREADS - 1)) == 0) {
        jr = jnx;
        jnx = Jg[mm + TDFE_CHEB_THREADS + t];  // < TDFE_JTAB_STRIDE since mm <= M < TDFE_MAX_BESSEL
      }
      const double left = lane_prev(vc[R - 1]), right = lane_next(vc[0]);
      double vn[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double l = r > 0 ? vc[r - 1] : left, rt = r < R - 1 ? vc[r + 1] : right;
        const double w = ac[r] * vc[r] + bl[r] * l + br[r] * rt;
        vn[r] = 2.0 * w * invr - vp[r];
      }
      const double cj = 2.0 * jn * lane_read(jr, mm & (TDFE_CHEB_THREADS - 1));
      const int ph = mm & 3;  // (-i sgn)^m : 1, -i sgn, -1, +i sgn
#pragma unroll
      for (int r = 0; r < R; ++r) {
        vp[r] = vc[r];
        vc[r] = vn[r];
        if (ph == 0) yr[r] += cj * vn[r];
        else if (ph == 1) yi[r] -= sgn * cj * vn[r];
        else if (ph == 2) yr[r] -= cj * vn[r];
        else yi[r] += sgn * cj * vn[r];
      }
    }
  }
  const double pr = cos(s * cc), pim = -sin(s * cc);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double a0 = yr[r], b0 = yi[r];
    yr[r] = a0 * pr - b0 * pim;
    yi[r] = a0 * pim + b0 * pr;
  }
  return M;
}

template <int R>
__device__ inline int cheb_rows_lds(int k, const double* sa, const double* sb, double s, ChebLds& L, double* Jg,
                                    double* amax) {
  double yr[R], yi[R];
  const int M = cheb_expm_e1_rows<R>(k, sa, sb, s, Jg, yr, yi, amax);
  const int t = threadIdx.x;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = R * t + r;
    if (j < k) {
      L.yr[j] = yr[r];
      L.yi[j] = yi[r];
    }
  }
  __syncthreads();
  return M;
}

// y = exp(-i s T) e_1 for TDFE_CHEB_THREADS < k <= TDFE_KCAP on one
// wavefront, left in L.yr / L.yi (rows per lane by k: 2, 3, 4, 8 or 16)
__device__ inline int cheb_expm_e1(int k, const double* sa, const double* sb, double s, ChebLds& L, double* Jg,
                                   double* amax) {
  if (k <= 2 * TDFE_CHEB_THREADS) return cheb_rows_lds<2>(k, sa, sb, s, L, Jg, amax);
  if (k <= 3 * TDFE_CHEB_THREADS) return cheb_rows_lds<3>(k, sa, sb, s, L, Jg, amax);
  if (k <= 4 * TDFE_CHEB_THREADS) return cheb_rows_lds<4>(k, sa, sb, s, L, Jg, amax);
  if (k <= 8 * TDFE_CHEB_THREADS) return cheb_rows_lds<8>(k, sa, sb, s, L, Jg, amax);
  return cheb_rows_lds<16>(k, sa, sb, s, L, Jg, amax);
}
