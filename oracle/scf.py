"""Density, dipole, Hartree and exchange-correlation pieces (oracle).

* density rho = sum_alpha f_alpha |psi_alpha|^2 (Sec. "Time-dependent
  Kohn-Sham Equations"), evaluated from psi^h = sum_j N_j psi^j at the Gauss
  points, psi = M^-1/2 psibar (Eq. TDKSMatVecStandard);
* dipole mu = int r rho^h (Sec. "Optimal discretization", the dipole moment
  as the observable; electronic part only, Gauss quadrature);
* Hartree potential by the discrete Poisson problem K phi_H = 4 pi c with
  c_j = int rho^h N_j and phi_H = f on the boundary, f = sum_I Z_I/|r - R_I|
  interpolated at the boundary nodes (Eqs. Poisson, VHDiscretePoisson and the
  appendix's q_j / f^h construction);
* ALDA exchange-correlation in the Ceperley-Alder form (Sec. "Time-dependent
  Kohn-Sham Equations"), here the Perdew-Zunger 1981 parametrisation.

Readings: occupations f_alpha = 1 per listed orbital unless given; the
Poisson system is solved by Jacobi-preconditioned conjugate gradients to a
relative residual tolerance, warm-started from the previous solution (the
paper does not name its solver).
"""
import numpy as np


def quad_values(mesh, u_dof_or_nodes, nodes=False):
    """Interpolate nodal FE coefficients to the Gauss points: (e, a, b, c, ...)."""
    if nodes:
        u_nodes = u_dof_or_nodes
    else:
        u_nodes = mesh.nodes_from_dofs(u_dof_or_nodes)
    B = mesh.ref.B
    return np.einsum("ai,bj,ck,eijk...->eabc...", B, B, B, u_nodes[mesh.cell_nodes], optimize=True)


def density(mesh, psibar, occ=None):
    """rho at the Gauss points, (n_cell, nq^3) with x fastest."""
    psibar = np.asarray(psibar)
    if psibar.ndim == 1:
        psibar = psibar[:, None]
    occ = np.ones(psibar.shape[1]) if occ is None else np.asarray(occ, dtype=np.float64)
    psi = mesh.m_inv_sqrt[:, None] * psibar
    pq = quad_values(mesh, psi)
    rho = np.einsum("eabcn,n->eabc", np.abs(pq) ** 2, occ)
    return mesh.from_cell_quad(rho)


def charge(mesh, rho):
    return float(np.sum(mesh.volume_weights * mesh.to_cell_quad(rho)))


def dipole(mesh, rho):
    """mu_d = sum_q varpi_q detJ_q x_{q,d} rho_q (electronic, +int r rho)."""
    w = mesh.volume_weights * mesh.to_cell_quad(rho)
    return np.einsum("eabc,eabcd->d", w, mesh.xq)


def load_vector(mesh, fq):
    """c_j = int f N_j for every node j (boundary included); fq (n_cell, nq^3)."""
    B = mesh.ref.B
    g = mesh.volume_weights * mesh.to_cell_quad(fq)
    ce = np.einsum("ai,bj,ck,eabc->eijk", B, B, B, g, optimize=True)
    out = np.zeros(mesh.n_nodes)
    np.add.at(out, mesh.cell_nodes.reshape(-1), ce.reshape(-1))
    return out


def stiffness_diagonal(mesh):
    """diag(K) over all nodes, K_jj = sum_e int grad N_j . grad N_j."""
    B, D = mesh.ref.B, mesh.ref.D
    wdet = mesh.volume_weights
    G = mesh.Ginvq
    tabs = (B, D)
    de = 0.0
    for d in range(3):
        for k in range(3):
            t = [tabs[int(d == ax)] * tabs[int(k == ax)] for ax in range(3)]
            de = de + np.einsum("eabc,ai,bj,ck->eijk", wdet * G[..., d, k], t[0], t[1], t[2], optimize=True)
    out = np.zeros(mesh.n_nodes)
    np.add.at(out, mesh.cell_nodes.reshape(-1), de.reshape(-1))
    return out


def boundary_values(mesh, Z, R):
    """f(x_j) = sum_I Z_I / |x_j - R_I| at the boundary nodes, 0 elsewhere."""
    f = np.zeros(mesh.n_nodes)
    xb = mesh.node_xyz[mesh.is_boundary]
    acc = np.zeros(len(xb))
    for z, r in zip(Z, R):
        acc += z / np.linalg.norm(xb - np.asarray(r)[None, :], axis=1)
    f[mesh.is_boundary] = acc
    return f


def pcg(apply_A, b, x0, diag, tol, maxit):
    """Jacobi-preconditioned CG on the interior unknowns; stop at ||r|| <= tol ||b||."""
    x = x0.copy()
    r = b - apply_A(x)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0, 0.0
    if np.linalg.norm(r) <= tol * bn:
        return x, 0, np.linalg.norm(r) / bn
    z = r / diag
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        Ap = apply_A(p)
        a = rz / (p @ Ap)
        x = x + a * p
        r = r - a * Ap
        res = np.linalg.norm(r) / bn
        if res <= tol:
            return x, it, res
        z = r / diag
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    raise RuntimeError(f"PCG did not converge in {maxit} iterations (res={res:.3e})")


class Hartree:
    """Discrete Hartree solve with the boundary lifting f^h (appendix)."""

    def __init__(self, mesh, Z, R, tol=1e-13, maxit=5000):
        from .operators import apply_K
        self.mesh = mesh
        self.apply_K = apply_K
        self.fb = boundary_values(mesh, Z, R)
        self.interior = ~mesh.is_boundary
        self.diag = stiffness_diagonal(mesh)[self.interior]
        self.lift = apply_K(mesh, self.fb)[self.interior]
        self.tol, self.maxit = tol, maxit
        self.phi0 = np.zeros(int(self.interior.sum()))
        self.last_iters = 0

    def _A(self, x):
        u = np.zeros(self.mesh.n_nodes)
        u[self.interior] = x
        return self.apply_K(self.mesh, u)[self.interior]

    def solve(self, rho):
        """phi_H over all nodes and V_H at the Gauss points (n_cell, nq^3)."""
        c = load_vector(self.mesh, rho)[self.interior]
        b = 4.0 * np.pi * c - self.lift
        x, it, _ = pcg(self._A, b, self.phi0, self.diag, self.tol, self.maxit)
        self.phi0 = x
        self.last_iters = it
        phi = self.fb.copy()
        phi[self.interior] = x
        vq = quad_values(self.mesh, phi, nodes=True)
        return phi, self.mesh.from_cell_quad(vq)


# --- exchange-correlation (ALDA) -------------------------------------------
_PZ_GAMMA, _PZ_B1, _PZ_B2 = -0.1423, 1.0529, 0.3334
_PZ_A, _PZ_B, _PZ_C, _PZ_D = 0.0311, -0.048, 0.0020, -0.0116


def exchange_potential(rho):
    """V_x = -(3 rho / pi)^(1/3) (LDA exchange, unpolarised)."""
    rho = np.maximum(np.asarray(rho, dtype=np.float64), 0.0)
    return -np.cbrt(3.0 * rho / np.pi)


def exchange_energy_density(rho):
    """eps_x = -3/4 (3/pi)^(1/3) rho^(1/3)."""
    rho = np.maximum(np.asarray(rho, dtype=np.float64), 0.0)
    return -0.75 * np.cbrt(3.0 / np.pi) * np.cbrt(rho)


def pz_eps_c(rs):
    """Perdew-Zunger 1981 correlation energy per electron, unpolarised."""
    rs = np.asarray(rs, dtype=np.float64)
    hi = _PZ_GAMMA / (1.0 + _PZ_B1 * np.sqrt(rs) + _PZ_B2 * rs)
    lo = _PZ_A * np.log(rs) + _PZ_B + _PZ_C * rs * np.log(rs) + _PZ_D * rs
    return np.where(rs >= 1.0, hi, lo)


def pz_deps_c(rs):
    """d eps_c / d r_s, differentiated branch by branch."""
    rs = np.asarray(rs, dtype=np.float64)
    den = 1.0 + _PZ_B1 * np.sqrt(rs) + _PZ_B2 * rs
    hi = -_PZ_GAMMA * (0.5 * _PZ_B1 / np.sqrt(rs) + _PZ_B2) / den ** 2
    lo = _PZ_A / rs + _PZ_C * (np.log(rs) + 1.0) + _PZ_D
    return np.where(rs >= 1.0, hi, lo)


def correlation_potential(rho):
    """V_c = eps_c - (r_s / 3) d eps_c / d r_s, r_s = (3 / (4 pi rho))^(1/3); 0 where rho = 0."""
    rho = np.asarray(rho, dtype=np.float64)
    out = np.zeros_like(rho)
    m = rho > 1e-300
    rs = np.cbrt(3.0 / (4.0 * np.pi * rho[m]))
    out[m] = pz_eps_c(rs) - rs / 3.0 * pz_deps_c(rs)
    return out


def xc_potential(rho, mode):
    """mode: 'none', 'x' (exchange only) or 'xc' (exchange + PZ81 correlation)."""
    if mode == "none":
        return np.zeros_like(np.asarray(rho, dtype=np.float64))
    v = exchange_potential(rho)
    if mode == "xc":
        v = v + correlation_potential(rho)
    elif mode != "x":
        raise ValueError(mode)
    return v
