"""Pins of the oracle's excitations and spectra (CPU only).

* Windowed Fourier sums against closed forms: a damped sine (the induced
  dipole of one oscillator after a kick) gives the absorption spectrum
  (2w/3pi) 3 f (1/4) sqrt(pi/alpha) [exp(-(W-w)^2/4alpha) - exp(-(W+w)^2/4alpha)];
  the Gaussian pulse transforms to kappa w sqrt(pi) exp(i w t0 - w^2 w_p^2 / 4).
* The power spectrum of mu = sin(W t) is W^2 int sin(w t) sin(W t) dt over
  the interior interval, in closed form (central differences and the
  trapezoid sum are second order in dt).
* Pulse integrals: int E = kappa w sqrt(pi) (Gaussian); the sin^2 laser over
  five optical cycles has no zero-frequency part and vanishes at both ends.
* The sum rule: int S dw equals the oscillator strength of the response.
* The kick on the harmonic trap: the dipole after the kick follows
  -kappa sin(t) (Ehrenfest; the trap frequency is 1) and its absorption peak
  sits at the trap frequency.
"""
import numpy as np
import pytest

import workloads as W
from oracle import spectra as sp
from oracle.magnus import State, System, magnus_step
from oracle.mesh import Mesh


def _windowed_sine_S(w, W0, f, alpha):
    return 2 * w / (3 * np.pi) * 3 * f * 0.25 * np.sqrt(np.pi / alpha) * (
        np.exp(-((W0 - w) ** 2) / (4 * alpha)) - np.exp(-((W0 + w) ** 2) / (4 * alpha)))


def test_kick_absorption_of_one_oscillator_in_closed_form():
    dt, T, alpha, kappa, W0, f = 0.01, 100.0, 0.005, 1e-3, 0.7, 0.4
    t = dt * np.arange(int(round(T / dt)) + 1)
    mu = np.stack([-kappa * f * np.sin(W0 * t)] * 3) + np.array([[0.3], [-0.2], [0.1]])
    w = np.linspace(0.05, 2.0, 40)
    S = sp.absorption_spectrum(mu, dt, w, alpha, kappa=kappa)
    ref = _windowed_sine_S(w, W0, f, alpha)
    assert np.abs(S - ref).max() < 1e-9 * np.abs(ref).max()
    # sum rule: a kick response -kappa (f_osc / W) sin(W t) has oscillator
    # strength f_osc = f W, and int S dw = f_osc whatever the window
    wf = np.linspace(1e-4, 6.0, 6001)
    Sf = sp.absorption_spectrum(mu[:, :4001], dt, wf, alpha, kappa=kappa)  # T = 40: window e^-8
    assert abs(np.trapezoid(Sf, wf) - f * W0) < 2e-3 * f * W0


def test_field_samples_path_matches_kick_path_for_an_impulse():
    """A field sampled as a one-sample spike of trapezoid area -kappa at t = 0
    (value -2 kappa / dt, end weight 1/2) has E~ = -kappa at every w: the
    field path must then reproduce the kick path."""
    dt, alpha, kappa = 0.02, 0.01, 2e-3
    t = dt * np.arange(2001)
    mu = np.stack([np.sin(0.9 * t), 0.5 * np.sin(1.3 * t), np.cos(0.4 * t) - 1.0]) * 1e-4
    field = np.zeros_like(mu)
    field[:, 0] = -2.0 * kappa / dt
    w = np.linspace(0.1, 2.0, 25)
    a = sp.absorption_spectrum(mu, dt, w, alpha, kappa=kappa)
    b = sp.absorption_spectrum(mu, dt, w, alpha, field=field)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


def test_gaussian_pulse_transform_and_integral():
    kappa, t0, wp, dt = 2e-5, 3.0, 0.2, 0.005
    t = dt * np.arange(int(20.0 / dt) + 1)
    E = sp.field_gaussian(t, kappa, t0, wp)
    w = np.linspace(0.0, 8.0, 33)
    ref = kappa * wp * np.sqrt(np.pi) * np.exp(1j * w * t0 - w ** 2 * wp ** 2 / 4)
    got = sp.fourier(E, dt, w)
    assert np.abs(got - ref).max() < 1e-12 * kappa
    assert E.max() == pytest.approx(kappa, rel=1e-12)  # peak at t0 (a sample)
    assert abs(np.trapezoid(E, t) - kappa * wp * np.sqrt(np.pi)) < 1e-14


def test_sin2_laser_has_no_dc_part_and_vanishes_at_the_ends():
    kappa, om = 0.01, 0.03
    T = 5 * 2 * np.pi / om
    t = np.linspace(0.0, T, 200001)
    E = sp.field_sin2(t, kappa, om, T)
    assert abs(np.trapezoid(E, t)) < 1e-9 * kappa * T
    assert abs(E[0]) < 1e-30 and abs(E[-1]) < 1e-15 * kappa
    assert sp.field_sin2(np.array([-1.0, T + 1.0]), kappa, om, T).tolist() == [0.0, 0.0]
    # envelope maximum at T/2: |E| <= kappa sin^2(pi t / T)
    assert np.all(np.abs(E) <= kappa * np.sin(np.pi * t / T) ** 2 + 1e-18)


def test_power_spectrum_of_a_sine_in_closed_form():
    dt, W0 = 0.005, 1.1
    n = 4001
    t = dt * np.arange(n)
    mu = np.sin(W0 * t)
    w = np.array([0.3, 0.9, 1.7, 3.3])
    a, b = dt, dt * (n - 2)

    def prim(x):
        return 0.5 * (np.sin((w - W0) * x) / (w - W0) - np.sin((w + W0) * x) / (w + W0))

    ref = W0 ** 2 * (prim(b) - prim(a))
    got = sp.power_spectrum(mu, dt, w)
    assert np.abs(got - ref).max() < 1e-4 * np.abs(ref).max()


def test_kicked_harmonic_trap_dipole_and_spectrum():
    """Harmonic trap (V = r^2/2, frequency 1): the nodal ground-state Gaussian
    kicked along z has mu_z(t) ~ -kappa sin(t) (Ehrenfest) to the
    discretisation error, and the absorption peak sits at w = 1."""
    from oracle import scf
    cfg = W.scaled(W.CONFIGS[1], ncell=(4, 4, 4), p=6)
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    vq = W.external_potential(cfg, m.quad_xyz)
    psi0 = np.abs(W.initial_psibar(cfg, m.dof_xyz, m.M)).astype(np.complex128)  # real Gaussian, no momentum
    kappa = 1e-2
    sysm = System(m, vq, tol=1e-12)
    st = State(sysm, sp.kick(psi0, m.dof_xyz, kappa))
    mu0 = scf.dipole(m, scf.density(m, psi0))[2]
    dt, nsteps = 0.1, 63  # one period
    mu = [scf.dipole(m, scf.density(m, st.psibar))[2] - mu0]
    for _ in range(nsteps):
        mu.append(magnus_step(sysm, st, dt)["dipole"][2] - mu0)
    mu = np.array(mu)
    t = dt * np.arange(nsteps + 1)
    assert abs(mu[0]) < 1e-14
    assert np.abs(mu + kappa * np.sin(t)).max() < 3e-2 * kappa  # 2% phase drift of the discrete trap at t = 2 pi
    # absorption from the same series for all three axes (the trap is isotropic)
    w = np.linspace(0.2, 2.0, 91)
    S = sp.absorption_spectrum(np.stack([mu] * 3), dt, w, 0.0, kappa=kappa)
    assert abs(w[np.argmax(S)] - 1.0) < 0.05 and S.max() > 0
