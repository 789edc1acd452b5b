"""Pins of the oracle's adaptive Lanczos exponential (CPU only).

Against the dense exponential (eigh of the assembled Hbar), scipy's
expm_multiply, exact invariants of a unitary propagator, and the
eigenvector / happy-breakdown special case.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.sparse.linalg import LinearOperator, expm_multiply

import workloads as W
from oracle import lanczos, operators as op
from oracle.mesh import Mesh


@pytest.fixture(scope="module")
def cfg1():
    cfg = W.CONFIGS[1]
    m = Mesh(cfg.p, cfg.ncell, W.box_vertices(cfg.lo, cfg.hi, cfg.ncell), cfg.nq)
    vq = W.external_potential(cfg, m.quad_xyz)
    Hb = op.dense_Hbar(m, vq)
    th, V = np.linalg.eigh(Hb)
    psi = W.initial_psibar(cfg, m.dof_xyz, m.M)
    return m, vq, Hb, th, V, psi


def _dense_exp(th, V, tau, x):
    c = V.T @ x
    ph = np.exp(-1j * tau * th)
    return V @ (ph[:, None] * c if c.ndim == 2 else ph * c)


def test_tridiagonal_exponential_matches_expm():
    rng = np.random.default_rng(0)
    a = rng.normal(size=9) * 3
    b = np.abs(rng.normal(size=8)) + 0.1
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    y = lanczos.tridiag_expm_e1(a, b, 0.7)
    np.testing.assert_allclose(y, sla.expm(-0.7j * T)[:, 0], atol=1e-13)


def test_lanczos_matches_dense_exponential(cfg1):
    m, vq, Hb, th, V, psi = cfg1
    tau = W.CONFIGS[1].dt
    z, ks, errs = lanczos.lanczos_expm(lambda x: op.apply_Hbar(m, vq, x), psi, tau, 1e-12)
    ref = _dense_exp(th, V, tau, psi)
    assert np.abs(z - ref).max() < 1e-10 * np.abs(ref).max()
    assert errs[0] <= 1e-12 and 2 < ks[0] < 60


def test_error_estimate_bounds_true_error(cfg1):
    m, vq, Hb, th, V, psi = cfg1
    rng = np.random.default_rng(3)
    x = rng.normal(size=m.n_dof) + 1j * rng.normal(size=m.n_dof)
    x /= np.linalg.norm(x)
    for tol in (1e-4, 1e-7, 1e-10):
        z, ks, errs = lanczos.lanczos_expm(lambda v: Hb @ v, x, 0.1, tol)
        true = np.linalg.norm(z[:, 0] - _dense_exp(th, V, 0.1, x))
        assert true <= 10 * tol


def test_unitarity_energy_and_reversibility(cfg1):
    m, vq, Hb, th, V, psi = cfg1
    f = lambda x: op.apply_Hbar(m, vq, x)
    z, _, _ = lanczos.lanczos_expm(f, psi, 0.4, 1e-12)
    assert abs(np.linalg.norm(z) - np.linalg.norm(psi)) < 1e-11
    e0 = np.vdot(psi[:, 0], f(psi[:, 0])).real
    e1 = np.vdot(z[:, 0], f(z[:, 0])).real
    assert abs(e1 - e0) < 1e-10 * abs(e0)
    back, _, _ = lanczos.lanczos_expm(f, z, -0.4, 1e-12)
    assert np.abs(back - psi).max() < 1e-10


def test_eigenvector_phase_and_happy_breakdown(cfg1):
    m, vq, Hb, th, V, psi = cfg1
    v = V[:, 2].astype(np.complex128)
    z, k, eps, info = lanczos.lanczos_expm_vec(lambda x: Hb @ x, v, 1.3, 1e-12)
    assert k <= 2
    np.testing.assert_allclose(z, np.exp(-1.3j * th[2]) * v, atol=1e-12)


def test_matches_scipy_expm_multiply():
    cfg = W.scaled(W.CONFIGS[2], ncell=(5, 5, 5), p=4)
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    vq = W.external_potential(cfg, m.quad_xyz)
    psi = W.initial_psibar(cfg, m.dof_xyz, m.M)[:, :2]
    z, ks, _ = lanczos.lanczos_expm(lambda x: op.apply_Hbar(m, vq, x), psi, 0.05, 1e-12)
    A = LinearOperator((m.n_dof, m.n_dof), matvec=lambda x: -0.05j * op.apply_Hbar(m, vq, x),
                       rmatvec=lambda x: 0.05j * op.apply_Hbar(m, vq, x),
                       matmat=lambda x: -0.05j * op.apply_Hbar(m, vq, x), dtype=np.complex128)
    ref = expm_multiply(A, psi, traceA=-0.05j * 0.0)
    assert np.abs(z - ref).max() < 1e-9


def test_not_converged_is_reported(cfg1):
    m, vq, Hb, th, V, psi = cfg1
    with pytest.raises(lanczos.NotConverged):
        lanczos.lanczos_expm(lambda x: Hb @ x, psi, 0.5, 1e-14, k_max=3)
