"""Excitations and spectra of a real-time run (oracle).

* Field shapes of the table of simulation parameters: a weak Gaussian pulse
  E(t) = kappa exp(-(t - t0)^2 / w^2) and a strong laser
  E(t) = kappa sin^2(pi t / T) sin(omega t) on [0, T] (0 outside).
* The delta kick that starts a linear-response run: psibar is multiplied at
  every DoF node by exp(-i kappa d . r).  In V_field = -E (d . r) (Eq. VField)
  it is the impulse of E(t) = -kappa delta(t).
* Absorption spectrum (dipole strength function):
  S(w) = (2 w / 3 pi) Tr Im alpha(w) with alpha_aa(w) = mu~_a(w) / E~_a(w),
  mu~ the Fourier transform of the induced dipole mu(t) - mu(0) under the
  Gaussian window exp(-alpha t^2), E~ that of the exciting field.
* Dipole power spectrum of a strong-field run:
  P(w) = Im int_0^T exp(-i w t) mu''(t) dt.

Readings (the printed formulas are garbled in places):
* the Gaussian pulse's exponent carries a minus sign (as printed it grows
  without bound), and the laser envelope is sin^2(pi t / T) (the printed
  form lacks t);
* integrals over time are trapezoid sums over the dipole samples t_n = n dt;
  the window multiplies the induced dipole only; a kick gives E~ = -kappa;
* mu'' is the central second difference, so the power spectrum's quadrature
  runs over the interior samples n = 1 .. N - 2.

This module is test infrastructure: only tests/, the package smoke check and
the benchmark's CPU baseline use it.
"""
import numpy as np


def field_gaussian(t, kappa, t0, w):
    t = np.asarray(t, dtype=np.float64)
    return kappa * np.exp(-(((t - t0) / w) ** 2))


def field_sin2(t, kappa, omega, T):
    t = np.asarray(t, dtype=np.float64)
    inside = (t >= 0.0) & (t <= T)
    return np.where(inside, kappa * np.sin(np.pi * t / T) ** 2 * np.sin(omega * t), 0.0)


def kick(psibar, dof_xyz, kappa, direction=(0.0, 0.0, 1.0)):
    """psibar (n_dof, n_orb) times exp(-i kappa d . r_j) row by row."""
    phase = np.asarray(dof_xyz) @ np.asarray(direction, dtype=np.float64)
    return np.asarray(psibar) * np.exp(-1j * kappa * phase)[:, None]


def trapezoid_weights(n):
    c = np.ones(n)
    c[0] = c[-1] = 0.5
    return c


def fourier(f, dt, omegas, alpha=0.0, sign=1):
    """sum_n c_n exp(sign i w t_n) exp(-alpha t_n^2) f_n dt for each w."""
    f = np.asarray(f, dtype=np.float64)
    t = dt * np.arange(f.shape[-1])
    g = trapezoid_weights(f.shape[-1]) * np.exp(-alpha * t * t) * dt
    ph = np.exp(sign * 1j * np.outer(np.asarray(omegas, dtype=np.float64), t))
    return ph @ (g * f)


def absorption_spectrum(mu, dt, omegas, alpha, kappa=None, field=None):
    """S(w) from mu (3, n_t): row a is the a-component of the dipole of the run
    excited along axis a.  Either kappa (delta kick exp(-i kappa r_a)) or
    field (3, n_t), the exciting field samples of each run."""
    mu = np.asarray(mu, dtype=np.float64)
    omegas = np.asarray(omegas, dtype=np.float64)
    tr = np.zeros(omegas.shape)
    for a in range(3):
        m = fourier(mu[a] - mu[a, 0], dt, omegas, alpha)
        e = -kappa * np.ones_like(m) if field is None else fourier(np.asarray(field)[a], dt, omegas, 0.0)
        tr += np.imag(m / e)
    return 2.0 * omegas / (3.0 * np.pi) * tr


def power_spectrum(mu, dt, omegas):
    """P(w) = Im sum over the interior samples of exp(-i w t) mu'' dt."""
    mu = np.asarray(mu, dtype=np.float64)
    acc = (mu[2:] - 2.0 * mu[1:-1] + mu[:-2]) / dt ** 2
    t = dt * np.arange(1, mu.shape[0] - 1)
    c = trapezoid_weights(acc.shape[0]) * dt
    ph = np.exp(-1j * np.outer(np.asarray(omegas, dtype=np.float64), t))
    return np.imag(ph @ (c * acc))
