"""A priori element-size distribution and a graded rectilinear mesh (oracle).

Sec. "Efficient spatio-temporal discretization": minimising the bound on the
dipole error at a fixed number of elements (Eq. OptimalMeshMin) gives the
element size (Eq. OptimalMeshSize)
    h(r) = E g(r)^(-1/(p+3)),
    g = sum_alpha (2 Dbar^{p+1} psi_alpha + Dbar^{p+3} psi_alpha) + Dbar^{p+1} V_H + Dbar^{p+1} V_N,
    Dbar^k f = sum over multi-indices |l| = k of |D^l f|,
with E fixed by int dr / h^3 = N_elem.  The fields are atomic ground-state
stand-ins.

Readings:
* the printed exponent "-1/p+3" is -1/(p+3) (the Euler-Lagrange equation of
  Eq. OptimalMeshMin);
* atomic fields: per atom one normalised Gaussian orbital
  (pi s^2)^(-3/4) exp(-|r-R|^2/(2 s^2)) at both times s_1, s_2, and the
  atom's Gaussian potential -Z exp(-|r-R|^2/(2 a^2)) for V_N; V_H is left
  out (for a neutral atom it cancels the long-range part of V_N, and the
  synthetic V_N is already short-ranged);
* the mesh is rectilinear (hexahedra without hanging nodes, so the GLL mass
  matrix stays diagonal): along each axis the spacing follows
  h_a(s) = min of h over the plane through s, sampled on a uniform grid of
  S^3 points, and the vertices equidistribute int ds / h_a(s) (trapezoid
  rule, linear inversion); the cell counts n_a = max(1, round(c I_a)),
  I_a = int ds / h_a, with c^3 prod I_a = N_elem (halves rounded up).  This keeps the optimal
  coarsening rate away from the atoms, as the paper's conforming hexahedral
  meshes do, at the cost of refining whole slabs.

This module is test infrastructure: only tests/, the package smoke check and
the benchmark's CPU baseline use it.
"""
import numpy as np
from numpy.polynomial import hermite_e as He


def _hermite_abs(u, kmax):
    """|He_k(u)| for k = 0..kmax (probabilists' Hermite polynomials)."""
    return np.stack([np.abs(He.hermeval(u, [0] * k + [1])) for k in range(kmax + 1)])


def dbar_gaussian(pts, R, s, A, k):
    """Dbar^k of A exp(-|r-R|^2/(2 s^2)) at pts (..., 3): the sum over l1+l2+l3 = k
    of |A| s^-k prod_i |He_{l_i}(u_i)| exp(-|u|^2/2), u = (r-R)/s."""
    u = (np.asarray(pts) - np.asarray(R)) / s
    H = [_hermite_abs(u[..., i], k) for i in range(3)]
    tot = np.zeros(u.shape[:-1])
    for l1 in range(k + 1):
        for l2 in range(k + 1 - l1):
            l3 = k - l1 - l2
            tot = tot + H[0][l1] * H[1][l2] * H[2][l3]
    return abs(A) * s ** (-k) * tot * np.exp(-0.5 * np.sum(u * u, axis=-1))


def size_weight(pts, p, atoms):
    """g(r) for atoms = [(R, Z, s_orbital, a_potential), ...]."""
    g = np.zeros(np.asarray(pts).shape[:-1])
    for R, Z, s, a in atoms:
        A = (np.pi * s * s) ** -0.75
        g = g + 2 * dbar_gaussian(pts, R, s, A, p + 1) + dbar_gaussian(pts, R, s, A, p + 3)
        g = g + dbar_gaussian(pts, R, a, Z, p + 1)
    return g


def sample_points(lo, hi, S):
    t = np.linspace(lo, hi, S)
    X, Y, Zc = np.meshgrid(t, t, t, indexing="ij")
    return t, np.stack([X, Y, Zc], axis=-1)


def element_size(lo, hi, p, atoms, n_elem, S):
    """(t, g, E) on the S^3 sample grid: h = E g^(-1/(p+3)) (infinite where
    g = 0, e.g. at the centre of an atom for odd derivative orders), E from
    int dr / h^3 = n_elem by the trapezoid rule on the samples."""
    t, pts = sample_points(lo, hi, S)
    g = size_weight(pts, p, atoms)
    w = np.full(S, t[1] - t[0])
    w[0] = w[-1] = 0.5 * (t[1] - t[0])
    W3 = w[:, None, None] * w[None, :, None] * w[None, None, :]
    E = (np.sum(W3 * g ** (3.0 / (p + 3))) / n_elem) ** (1.0 / 3.0)
    return t, g, E


def graded_axes(lo, hi, p, atoms, n_elem, S):
    """Vertex coordinates along x, y, z of the graded rectilinear mesh; the
    smallest h over a plane is E (largest g over it)^(-1/(p+3))."""
    t, g, E = element_size(lo, hi, p, atoms, n_elem, S)
    gmax = [g.max(axis=(1, 2)), g.max(axis=(0, 2)), g.max(axis=(0, 1))]
    F = []
    for gm in gmax:
        inv_h = gm ** (1.0 / (p + 3)) / E
        f = np.concatenate([[0.0], np.cumsum(0.5 * (inv_h[1:] + inv_h[:-1]) * np.diff(t))])
        F.append(f)
    I = np.array([f[-1] for f in F])
    c = (n_elem / np.prod(I)) ** (1.0 / 3.0)
    axes = []
    for f in F:
        n = max(1, int(np.floor(c * f[-1] + 0.5)))
        targets = f[-1] * np.arange(n + 1) / n
        x = np.interp(targets, f, t)
        x[0], x[-1] = lo, hi
        axes.append(x)
    return axes, E
