"""Pins of the oracle's discrete operators (CPU only).

Closed-form integrals of polynomials, constants in the kernel of K,
equality of the matrix-free and the dense-assembled operator, symmetry, and
the Dirichlet Laplacian spectrum of a cube.
"""
import numpy as np
import pytest

import workloads as W
from oracle import operators as op
from oracle.mesh import Mesh


def _box(p, ncell, lo=(0.0, 0.0, -1.0), hi=(1.0, 2.0, 1.0)):
    ncx, ncy, ncz = ncell
    xs = np.linspace(lo[0], hi[0], ncx + 1)
    ys = np.linspace(lo[1], hi[1], ncy + 1)
    zs = np.linspace(lo[2], hi[2], ncz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return Mesh(p, ncell, np.stack([X, Y, Z], axis=-1))


def _graded(p=3, ncell=(4, 4, 4)):
    cfg = W.scaled(W.CONFIGS[3], ncell=ncell, p=p)
    return Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)


def test_stiffness_energy_of_polynomial():
    # u = x^2 y + z^3 on [0,1]x[0,2]x[-1,1]: int |grad u|^2 = 64/9 + 4/5 + 36/5 = 136/9
    m = _box(3, (2, 2, 2))
    x, y, z = m.node_xyz.T
    u = x ** 2 * y + z ** 3
    assert abs(u @ op.apply_K(m, u) - 136.0 / 9.0) < 1e-12


def test_H_kinetic_half_and_mass_term():
    # u vanishing on the boundary: u = x(1-x) y(2-y) (1-z^2), degree 2 per direction
    m = _box(3, (2, 2, 2))
    x, y, z = m.dof_xyz.T
    u = x * (1 - x) * y * (2 - y) * (1 - z * z)
    # int |grad u|^2 and int u^2 in closed form (separable products of 1D integrals)
    ix = {"ff": 1 / 30, "dd": 1 / 3}            # f = x(1-x) on [0,1]
    iy = {"ff": 16 / 15, "dd": 8 / 3}           # f = y(2-y) on [0,2]
    iz = {"ff": 16 / 15, "dd": 8 / 3}           # f = 1-z^2 on [-1,1]
    grad2 = ix["dd"] * iy["ff"] * iz["ff"] + ix["ff"] * iy["dd"] * iz["ff"] + ix["ff"] * iy["ff"] * iz["dd"]
    mass = ix["ff"] * iy["ff"] * iz["ff"]
    h0 = u @ op.apply_H(m, None, u)
    assert abs(h0 - 0.5 * grad2) < 1e-13
    c = 2.7
    vq = np.full((m.n_cell, m.nq ** 3), c)
    assert abs(u @ op.apply_H(m, vq, u) - h0 - c * mass) < 1e-13


def test_constants_in_kernel_of_K():
    for m in (_box(4, (2, 1, 3)), _graded()):
        assert np.abs(op.apply_K(m, np.ones(m.n_nodes))).max() < 1e-11


def test_linear_energy_on_curved_mesh():
    # u = a . x is trilinear in the reference coordinates of every cell, so it is
    # represented exactly; int |grad u|^2 = |a|^2 vol exactly with Gauss quadrature
    m = _graded()
    a = np.array([0.3, -1.1, 0.7])
    u = m.node_xyz @ a
    vol = m.volume_weights.sum()
    assert abs(u @ op.apply_K(m, u) - (a @ a) * vol) < 1e-9 * vol


@pytest.mark.parametrize("which", ["box", "graded"])
def test_matrix_free_equals_dense(which):
    m = _box(3, (2, 2, 2)) if which == "box" else _graded(2, (3, 3, 3))
    vq = W.random_potential(m.n_cell, m.nq ** 3, 7)
    Hb = op.dense_Hbar(m, vq)
    u = W.random_block(m.n_dof, 3, 11)
    y = op.apply_Hbar(m, vq, u)
    assert np.abs(Hb @ u - y).max() < 1e-13 * np.abs(y).max()
    assert np.abs(Hb - Hb.T).max() < 1e-13 * np.abs(Hb).max()
    K = op.dense_K(m)
    un = W.random_block(m.n_nodes, 1, 3).real[:, 0]
    assert np.abs(K @ un - op.apply_K(m, un)).max() < 1e-12 * np.abs(K).max()


def test_hbar_symmetric_matrix_free():
    m = _graded(3, (3, 3, 3))
    vq = W.random_potential(m.n_cell, m.nq ** 3, 5)
    u = W.random_block(m.n_dof, 1, 1)[:, 0]
    v = W.random_block(m.n_dof, 1, 2)[:, 0]
    a = np.vdot(u, op.apply_Hbar(m, vq, v))
    b = np.vdot(op.apply_Hbar(m, vq, u), v)
    assert abs(a - b) < 1e-12 * abs(a)


def test_dirichlet_cube_spectrum_converges():
    # V = 0 on a cube of side L with psi = 0 on the boundary: continuum
    # eigenvalues (pi^2 / 2L^2)(n1^2 + n2^2 + n3^2)
    L = 2.0
    exact = np.pi ** 2 / (2 * L * L) * np.array([3, 6, 6, 6])
    errs = []
    for p in (2, 4, 6):
        m = _box(p, (2, 2, 2), lo=(0, 0, 0), hi=(L, L, L))
        ev = np.linalg.eigvalsh(op.dense_Hbar(m, None))[:4]
        errs.append(np.abs(ev - exact).max() / exact[0])
    # spectral convergence in the order p
    assert errs[2] < 1e-5 and errs[1] < errs[0] / 100 and errs[2] < errs[1] / 100


def test_harmonic_ground_state_converges():
    # V = |r|^2 / 2: continuum ground-state energy 3/2
    from scipy.sparse.linalg import LinearOperator, eigsh
    errs = []
    for nc in (4, 6):
        v = W.box_vertices(-8.0, 8.0, (nc, nc, nc))
        m = Mesh(4, (nc, nc, nc), v)
        vq = 0.5 * np.sum(m.quad_xyz ** 2, axis=-1)
        A = LinearOperator((m.n_dof, m.n_dof), matvec=lambda x: op.apply_Hbar(m, vq, x), dtype=np.float64)
        e0 = eigsh(A, k=1, which="SA", tol=1e-10)[0][0]
        errs.append(abs(e0 - 1.5))
    assert errs[0] < 3e-2 and errs[1] < errs[0] / 4
