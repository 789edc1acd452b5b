"""Nonlocal pseudopotential term in the Kleinman-Bylander form (oracle).

Eq. VPSP: the nonlocal part acts on phi as a sum over atoms I and channels
(l, m) of  (int chi_p phi / D_p) chi_p  with chi_p = u_p dV_p (the pseudo-atomic
function times its channel's short-range potential) and
D_p = int u_p dV_p u_p.  Its Galerkin matrix on the FE basis is
    (V_nl)_jk = sum_p c_pj c_pk / D_p,   c_pj = int chi_p N_j,
with every integral evaluated by the Gauss rule of the Hamiltonian (spectral
FE section).  In the Loewdin form (Eq. TDKSMatVecStandard) the term added
to Hbar is  M^-1/2 C^T diag(1/D) C M^-1/2.

Readings: u_p and dV_p are given by their values at the Gauss points (the
paper gives them as tabulated functions); D_p uses the same quadrature.
This module is test infrastructure: only tests/, the package smoke check and
the benchmark's CPU baseline use it.
"""
import numpy as np

from . import scf


def kb_matrix(mesh, uq, dvq):
    """(C, E): C (n_proj, n_dof) with c_pj = int u_p dV_p N_j on the interior
    DoFs, E (n_proj) = 1 / int u_p dV_p u_p.  uq, dvq: (n_proj, n_cell, nq^3)."""
    uq = np.asarray(uq)
    dvq = np.asarray(dvq)
    n_proj = uq.shape[0]
    C = np.zeros((n_proj, mesh.n_dof))
    E = np.zeros(n_proj)
    for p in range(n_proj):
        chi = uq[p] * dvq[p]
        C[p] = scf.load_vector(mesh, chi)[mesh.dof_nodes]
        E[p] = 1.0 / np.sum(mesh.volume_weights * mesh.to_cell_quad(chi * uq[p]))
    return C, E


def apply_nonlocal_bar(mesh, C, E, psibar):
    """M^-1/2 C^T diag(E) C M^-1/2 psibar."""
    s = mesh.m_inv_sqrt.reshape((-1,) + (1,) * (psibar.ndim - 1))
    t = np.tensordot(C, s * psibar, axes=(1, 0))
    return s * np.tensordot(C, E.reshape((-1,) + (1,) * (psibar.ndim - 1)) * t, axes=(0, 0))


def dense_nonlocal_bar(mesh, C, E):
    """The same term as a dense (n_dof, n_dof) matrix (tiny meshes)."""
    Cb = C * mesh.m_inv_sqrt[None, :]
    return Cb.T @ (E[:, None] * Cb)
