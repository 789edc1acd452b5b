"""Pins of the oracle's gradient dL/dE_n (CPU only): central finite
differences of the forward scheme and the second-order Taylor remainder.
The forward scheme uses exact (dense) exponentials on a tiny mesh."""
import numpy as np
import pytest

import workloads as W
from oracle.adjoint import DenseAdjointSystem
from oracle.mesh import Mesh


def _system(scf_on):
    cfg = W.scaled(W.CONFIGS[5], ncell=(3, 3, 3), p=3, n_orb=2)
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    vq = W.external_potential(cfg, m.quad_xyz)
    Z, R = W.atoms(cfg)
    s = DenseAdjointSystem(m, vq, Z, R, xc="x" if scf_on else "none", hartree=scf_on)
    psi0 = W.initial_psibar(cfg, m.dof_xyz, m.M)
    return cfg, s, psi0


@pytest.mark.parametrize("scf_on", [False, True])
def test_gradient_matches_central_differences(scf_on):
    cfg, s, psi0 = _system(scf_on)
    E = W.field_amplitudes(4) * 50.0  # a visible response on the tiny mesh
    L, g = s.gradient(psi0, E, cfg.dt)
    h = 1e-4
    for n in range(len(E)):
        ep, em = E.copy(), E.copy()
        ep[n] += h
        em[n] -= h
        fd = (s.forward(psi0, ep, cfg.dt)[0] - s.forward(psi0, em, cfg.dt)[0]) / (2 * h)
        assert abs(fd - g[n]) <= 1e-6 * np.abs(g).max() + 1e-12, (n, fd, g[n])


def test_taylor_remainder_is_second_order():
    cfg, s, psi0 = _system(True)
    E = W.field_amplitudes(3) * 50.0
    L0, g = s.gradient(psi0, E, cfg.dt)
    d = np.random.default_rng(7).normal(size=len(E))
    r = []
    for eps in (1e-2, 5e-3):
        r.append(abs(s.forward(psi0, E + eps * d, cfg.dt)[0] - L0 - eps * (g @ d)))
    assert 3.0 < r[0] / r[1] < 5.0
