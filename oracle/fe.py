"""Reference element of the spectral finite elements (oracle, test-only).

Sec. "Higher-order spectral finite-elements": the nodes of an order-p element
are the Gauss-Legendre-Lobatto (GLL) points, i.e. the roots of P_p' together
with the two end points; the GLL rule is used only for the overlap matrix and
Gauss-Legendre quadrature for every other integral.
"""
import numpy as np
from numpy.polynomial import legendre as L


def gll_rule(p):
    """GLL nodes and weights of order p on [-1, 1].

    Nodes: -1, the p-1 roots of P_p', +1 (spectral FE section).
    Weights: w_i = 2 / (p (p+1) P_p(x_i)^2), the standard Lobatto weights.
    """
    if p < 1:
        raise ValueError("order p must be >= 1")
    cp = np.zeros(p + 1)
    cp[p] = 1.0
    if p == 1:
        x = np.array([-1.0, 1.0])
    else:
        inner = np.sort(np.real(L.legroots(L.legder(cp))))
        # polish the library roots with Newton on P_p'
        d1 = L.legder(cp)
        d2 = L.legder(cp, 2)
        for _ in range(3):
            inner = inner - L.legval(inner, d1) / L.legval(inner, d2)
        x = np.concatenate(([-1.0], inner, [1.0]))
    w = 2.0 / (p * (p + 1) * L.legval(x, cp) ** 2)
    return x, w


def gauss_rule(nq):
    """Gauss-Legendre points and weights (numpy's library rule)."""
    return L.leggauss(nq)


def lagrange(nodes, x):
    """Lagrange basis on ``nodes`` evaluated at points ``x``.

    Returns (Lv, Ld) with Lv[a, i] = l_i(x_a) and Ld[a, i] = l_i'(x_a), from
    the product definition l_i(x) = prod_{m != i} (x - xi_m)/(xi_i - xi_m).
    Plain loops: the sizes are at most 9 x 9.
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    Lv = np.ones((len(x), n))
    Ld = np.zeros((len(x), n))
    for i in range(n):
        for m in range(n):
            if m != i:
                Lv[:, i] *= (x - nodes[m]) / (nodes[i] - nodes[m])
        for l in range(n):
            if l == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[l]))
            for m in range(n):
                if m != i and m != l:
                    term *= (x - nodes[m]) / (nodes[i] - nodes[m])
            Ld[:, i] += term
    return Lv, Ld


class RefElement:
    """1D tables of an order-p spectral element with nq Gauss points.

    B[a, i] = l_i(eta_a), D[a, i] = l_i'(eta_a) with l_i the GLL Lagrange
    basis and eta_a the Gauss points.
    """

    def __init__(self, p, nq=None):
        self.p = int(p)
        self.n = self.p + 1
        self.nq = self.n if nq is None else int(nq)
        self.xi, self.w = gll_rule(self.p)
        self.eta, self.wq = gauss_rule(self.nq)
        self.B, self.D = lagrange(self.xi, self.eta)
