"""Pins of the oracle's Kleinman-Bylander nonlocal term (Eq. VPSP; CPU only).

* A constant projector (u = dV = 1): c_j = int N_j by the Gauss rule equals the
  GLL-lumped overlap M_jj (both rules integrate N_j exactly on box and on
  trilinear cells), and D = int 1 is the domain volume.
* Gaussian projectors well inside the domain: sum_j c_j over all nodes is
  int chi (partition of unity) and D = int u^2 dV, both in closed form.
* Sylvester's law of inertia: the dense term has exactly as many positive
  (negative) eigenvalues as there are positive (negative) 1/D_p, the rest
  zero; and it is symmetric.
* The matrix-free action equals the dense matrix.
"""
import numpy as np
import pytest

import workloads as W
from oracle import nonlocal_kb as nl
from oracle import scf
from oracle.mesh import Mesh


def _box(p, ncell, lo=-1.0, hi=1.0):
    return Mesh(p, ncell, W.box_vertices(lo, hi, ncell))


def _graded(p=3, ncell=(3, 3, 3)):
    cfg = W.scaled(W.CONFIGS[3], ncell=ncell, p=p)
    return Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)


@pytest.mark.parametrize("which", ["box", "graded"])
def test_constant_projector_gives_lumped_overlap_and_volume(which):
    m = _box(3, (2, 3, 2)) if which == "box" else _graded()
    ones = np.ones((1, m.n_cell, m.nq ** 3))
    C, E = nl.kb_matrix(m, ones, ones)
    assert np.abs(C[0] - m.M).max() < 1e-13 * m.M.max()
    vol = float(np.sum(m.volume_weights))
    if which == "box":
        assert abs(vol - 8.0) < 1e-13
    assert abs(1.0 / E[0] - vol) < 1e-12 * vol


def test_gaussian_projector_integrals_in_closed_form():
    m = _box(6, (10, 10, 10), lo=-8.0, hi=8.0)  # h = 1.6: quadrature error ~1e-8
    xq = m.quad_xyz.reshape(m.n_cell, -1, 3)
    su, rc, A = 1.1, 0.9, -1.3
    r2 = np.sum(xq ** 2, axis=-1)
    u = np.exp(-r2 / (2 * su ** 2))
    dv = A * np.exp(-r2 / (2 * rc ** 2))
    C, E = nl.kb_matrix(m, u[None], dv[None])
    # chi = A exp(-r^2 / (2 s^2)), 1/s^2 = 1/su^2 + 1/rc^2
    s2 = 1.0 / (1.0 / su ** 2 + 1.0 / rc ** 2)
    exact_chi = A * (2 * np.pi * s2) ** 1.5
    full = scf.load_vector(m, u * dv)
    assert abs(full.sum() - exact_chi) < 1e-7 * abs(exact_chi)
    assert abs(C[0].sum() - exact_chi) < 1e-7 * abs(exact_chi)  # boundary nodes carry ~exp(-20)
    # D = A int exp(-r^2 (2/su^2 + 1/rc^2) / 2)
    t2 = 1.0 / (2.0 / su ** 2 + 1.0 / rc ** 2)
    exact_D = A * (2 * np.pi * t2) ** 1.5
    assert abs(1.0 / E[0] - exact_D) < 1e-7 * abs(exact_D)


def test_dense_term_inertia_and_symmetry():
    cfg = W.scaled(W.CONFIGS[2], ncell=(3, 3, 3), p=3)
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    u, dv = W.kb_projector_values(cfg, m.quad_xyz.reshape(m.n_cell, -1, 3))
    C, E = nl.kb_matrix(m, u, dv)
    V = nl.dense_nonlocal_bar(m, C, E)
    assert np.abs(V - V.T).max() < 1e-14 * np.abs(V).max()
    lam = np.linalg.eigvalsh(V)
    tiny = 1e-10 * np.abs(lam).max()
    assert int(np.sum(lam > tiny)) == int(np.sum(E > 0))
    assert int(np.sum(lam < -tiny)) == int(np.sum(E < 0))


def test_matrix_free_equals_dense():
    cfg = W.scaled(W.CONFIGS[2], ncell=(2, 3, 2), p=3)
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    u, dv = W.kb_projector_values(cfg, m.quad_xyz.reshape(m.n_cell, -1, 3))
    C, E = nl.kb_matrix(m, u, dv)
    x = W.random_block(m.n_dof, 3, 5)
    y = nl.apply_nonlocal_bar(m, C, E, x)
    assert np.abs(y - nl.dense_nonlocal_bar(m, C, E) @ x).max() < 1e-13 * np.abs(y).max()
