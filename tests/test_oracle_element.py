"""Pins of the oracle's reference element and mesh (CPU only).

Each check compares against something the oracle does not compute itself:
closed-form GLL values, polynomial exactness, partition of unity, exact
volumes.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fe
from oracle.mesh import Mesh


def test_gll_p4_closed_form():
    # Lobatto rule with 5 points: nodes {0, +-sqrt(3/7), +-1}, weights {32/45, 49/90, 1/10}
    x, w = fe.gll_rule(4)
    s = np.sqrt(3.0 / 7.0)
    np.testing.assert_allclose(x, [-1, -s, 0, s, 1], atol=1e-15)
    np.testing.assert_allclose(w, [0.1, 49 / 90, 32 / 45, 49 / 90, 0.1], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_gll_exactness(p):
    # n = p+1 Lobatto points integrate x^m exactly for m <= 2p - 1
    x, w = fe.gll_rule(p)
    assert abs(w.sum() - 2.0) < 1e-14
    for m in range(0, 2 * p):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(w @ x ** m - exact) < 1e-13
    # and not for 2p (the rule is not Gauss)
    m = 2 * p
    assert abs(w @ x ** m - 2.0 / (m + 1)) > 1e-6


@pytest.mark.parametrize("nq", [2, 5, 8])
def test_gauss_exactness(nq):
    x, w = fe.gauss_rule(nq)
    for m in range(0, 2 * nq):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(w @ x ** m - exact) < 1e-13


@pytest.mark.parametrize("p", [1, 3, 5, 7])
def test_lagrange_tables(p):
    ref = fe.RefElement(p)
    Lv, _ = fe.lagrange(ref.xi, ref.xi)
    np.testing.assert_allclose(Lv, np.eye(p + 1), atol=1e-13)
    # partition of unity and its derivative
    np.testing.assert_allclose(ref.B.sum(axis=1), 1.0, atol=1e-13)
    np.testing.assert_allclose(ref.D.sum(axis=1), 0.0, atol=1e-11)
    # D maps GLL samples of a degree-p polynomial to its exact derivative
    c = np.arange(1, p + 2) * 0.3 - 1.0
    poly = np.polynomial.Polynomial(c)
    np.testing.assert_allclose(ref.B @ poly(ref.xi), poly(ref.eta), atol=1e-12)
    np.testing.assert_allclose(ref.D @ poly(ref.xi), poly.deriv()(ref.eta), atol=1e-10)


def _box(p, ncell, lo=(0.0, 0.0, -1.0), hi=(1.0, 2.0, 1.0)):
    ncx, ncy, ncz = ncell
    xs = np.linspace(lo[0], hi[0], ncx + 1)
    ys = np.linspace(lo[1], hi[1], ncy + 1)
    zs = np.linspace(lo[2], hi[2], ncz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return Mesh(p, ncell, np.stack([X, Y, Z], axis=-1))


def test_mass_sums_to_volume_box():
    m = _box(3, (2, 3, 2))
    assert abs(m.M_nodes.sum() - 4.0) < 1e-13
    assert np.all(m.M_nodes > 0)
    # DoF count and numbering
    assert m.n_dof == (2 * 3 - 1) * (3 * 3 - 1) * (2 * 3 - 1)
    xyz = m.dof_xyz
    assert np.all(np.diff(xyz[:m.Nx - 2, 0]) > 0)  # x fastest


def test_mass_and_gauss_volume_agree_graded():
    cfg = W.scaled(W.CONFIGS[3], ncell=(5, 5, 5), p=3)
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    vol_gll = m.M_nodes.sum()
    vol_gauss = m.volume_weights.sum()
    # det J of a trilinear map has degree <= 2 per direction: both rules are exact
    assert abs(vol_gll - vol_gauss) < 1e-11 * vol_gauss
    assert abs(vol_gauss - 32.0 ** 3) < 1e-9 * 32.0 ** 3  # map fixes the domain boundary? (checked)


def test_graded_mesh_positive():
    cfg = W.CONFIGS[3]
    V = W.vertices(cfg)
    e = np.linalg.norm(np.diff(V, axis=2), axis=-1)
    assert e.min() < 0.5 and e.max() > 1.0
