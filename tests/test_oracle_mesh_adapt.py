"""Pins of the oracle's a priori element-size distribution (CPU only).

* Dbar^k of a Gaussian at its centre in closed form: only even multi-indices
  survive, |He_2m(0)| = (2m-1)!!, so Dbar^2 = 3 |A| / s^2 and
  Dbar^4 = 12 |A| / s^4; away from the centre, Dbar^1 and Dbar^2 against
  central finite differences of the function itself.
* E meets the element-count constraint: int dr / h^3 = N_elem by an
  independent Gauss-Legendre rule.
* Optimality (Euler-Lagrange of Eq. OptimalMeshMin): feasible perturbations
  of h (rescaled to the same element count) never lower the objective
  int h^p g; the printed exponent read as -1/p + 3 does.
* The graded axes: symmetric about a centred atom, finest at the atom,
  about N_elem cells in total.
"""
import numpy as np

from oracle import mesh_adapt as ma

ATOM = [((0.3, -0.2, 0.1), 3.0, 0.8, 0.5)]


def test_dbar_gaussian_at_the_centre_in_closed_form():
    R, s, A = np.array([0.1, 0.2, -0.3]), 0.7, -2.0
    pt = R[None, :]
    assert abs(ma.dbar_gaussian(pt, R, s, A, 2)[0] - 3 * abs(A) / s ** 2) < 1e-12
    assert abs(ma.dbar_gaussian(pt, R, s, A, 4)[0] - 12 * abs(A) / s ** 4) < 1e-10
    assert abs(ma.dbar_gaussian(pt, R, s, A, 3)[0]) < 1e-12  # every order-3 index has an odd part


def test_dbar_gaussian_against_finite_differences():
    R, s, A = np.array([0.0, 0.0, 0.0]), 0.9, 1.7
    f = lambda x: A * np.exp(-np.sum((x - R) ** 2) / (2 * s * s))
    x0 = np.array([0.35, -0.5, 0.2])
    h = 1e-4
    e = np.eye(3)
    d1 = sum(abs((f(x0 + h * e[i]) - f(x0 - h * e[i])) / (2 * h)) for i in range(3))
    assert abs(ma.dbar_gaussian(x0[None], R, s, A, 1)[0] - d1) < 1e-7
    h = 1e-3
    d2 = 0.0
    for i in range(3):
        for j in range(i, 3):
            dij = (f(x0 + h * e[i] + h * e[j]) - f(x0 + h * e[i] - h * e[j]) - f(x0 - h * e[i] + h * e[j])
                   + f(x0 - h * e[i] - h * e[j])) / (4 * h * h)
            d2 += abs(dij)
    assert abs(ma.dbar_gaussian(x0[None], R, s, A, 2)[0] - d2) < 1e-5


def test_constant_meets_the_element_count():
    lo, hi, p, N, S = -4.0, 4.0, 4, 2000.0, 65
    t, g, E = ma.element_size(lo, hi, p, ATOM, N, S)
    x, w = np.polynomial.legendre.leggauss(48)
    x = lo + (hi - lo) * (x + 1) / 2
    w = w * (hi - lo) / 2
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    q = ma.size_weight(np.stack([X, Y, Z], -1), p, ATOM) ** (-1.0 / (p + 3))
    count = np.einsum("i,j,k,ijk->", w, w, w, (E * q) ** -3.0)
    assert abs(count - N) < 2e-2 * N


def _objective(h, g, W, p):
    return np.sum(W * h ** p * g)


def test_size_distribution_is_optimal_for_its_element_count():
    lo, hi, p, N, S = -4.0, 4.0, 5, 3000.0, 33
    t, pts = ma.sample_points(lo, hi, S)
    g = ma.size_weight(pts, p, ATOM)
    dx = t[1] - t[0]
    W = np.full((S, S, S), dx ** 3)
    rescale = lambda h: h * (np.sum(W / h ** 3) / N) ** (1.0 / 3.0)
    h_opt = rescale(g ** (-1.0 / (p + 3)))
    J0 = _objective(h_opt, g, W, p)
    rng = np.random.default_rng(7)
    for _ in range(20):
        phi = rng.normal(size=g.shape)
        h = rescale(h_opt * np.exp(0.05 * phi))
        assert _objective(h, g, W, p) >= J0 * (1 - 1e-12)
    wrong = rescale(g ** (-1.0 / p + 3.0))
    assert _objective(wrong, g, W, p) > 1.01 * J0


def test_graded_axes_symmetry_and_count():
    atoms = [((0.0, 0.0, 0.0), 3.0, 0.8, 0.5)]
    axes, E = ma.graded_axes(-6.0, 6.0, 4, atoms, 1000.0, 97)
    for ax in axes:
        assert np.abs(ax + ax[::-1]).max() < 1e-12       # symmetric about the atom
        d = np.diff(ax)
        assert np.all(d > 0)
        mid = len(d) // 2
        assert d[mid] < 0.5 * d[0]                        # finest at the atom
    assert np.abs(axes[0] - axes[1]).max() < 1e-12 and np.abs(axes[0] - axes[2]).max() < 1e-12
    n = np.prod([len(a) - 1 for a in axes])
    assert 0.7 * 1000 < n < 1.4 * 1000
