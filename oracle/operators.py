"""Discrete Hamiltonian, stiffness and the Loewdin-transformed Hbar (oracle).

Eq. DiscreteHamiltonian:
    H_jk = 1/2 int grad N_j . grad N_k + int V N_j N_k,
integrated with Gauss quadrature (spectral FE section: Gauss rule for every
integral except the overlap).  Eq. TDKSMatVecStandard: Hbar = M^-1/2 H M^-1/2
with M the diagonal GLL overlap.  Eq. VHDiscretePoisson: K_jk = int grad N_j
. grad N_k.

Two independent evaluations are given: a matrix-free cell-by-cell one
(``apply_H``, ``apply_K``), and a dense assembly for tiny meshes
(``dense_H``, ``dense_K``) used to pin the former.
"""
import numpy as np


def _cell_values(mesh, u_nodes):
    """Gather node values to cells: (e, i, j, k, ...)."""
    return u_nodes[mesh.cell_nodes]


def _cell_operator(mesh, u_e, vq, kin):
    """Local action y_e = H_e u_e for every cell.

    vq: potential at the Gauss points, (e, a, b, c), or None.
    kin: coefficient of the gradient term (1/2 for H, 1 for K).
    Value and reference gradient at the Gauss points are
    (B x B x B) u, (D x B x B) u, (B x D x B) u, (B x B x D) u; the physical
    gradient product uses G = J^-1 J^-T; the test functions are applied with
    the transposed tables.
    """
    B, D = mesh.ref.B, mesh.ref.D
    es = "ai,bj,ck,eijk...->eabc..."
    val = np.einsum(es, B, B, B, u_e, optimize=True)
    g = [np.einsum(es, D, B, B, u_e, optimize=True),
         np.einsum(es, B, D, B, u_e, optimize=True),
         np.einsum(es, B, B, D, u_e, optimize=True)]
    wdet = mesh.volume_weights  # (e, a, b, c)
    extra = (None,) * (u_e.ndim - 4)
    G = mesh.Ginvq
    flux = []
    for d in range(3):
        f = sum(G[..., d, k][(...,) + extra] * g[k] for k in range(3))
        flux.append(kin * wdet[(...,) + extra] * f)
    et = "ai,bj,ck,eabc...->eijk..."
    y = (np.einsum(et, D, B, B, flux[0], optimize=True)
         + np.einsum(et, B, D, B, flux[1], optimize=True)
         + np.einsum(et, B, B, D, flux[2], optimize=True))
    if vq is not None:
        y = y + np.einsum(et, B, B, B, (wdet * vq)[(...,) + extra] * val, optimize=True)
    return y


def _assemble(mesh, y_e):
    out = np.zeros((mesh.n_nodes,) + y_e.shape[4:], dtype=y_e.dtype)
    np.add.at(out, mesh.cell_nodes.reshape(-1), y_e.reshape((-1,) + y_e.shape[4:]))
    return out


def apply_H(mesh, vq, u):
    """(H u) on the DoFs; u: (n_dof, ...) FE coefficients (real or complex).
    The mesh maps DoF values to node values (``nodes_from_dofs``: placement,
    or the hanging-node constraints of an octree mesh) and back (its
    transpose).

    vq: potential at the Gauss points in the (n_cell, nq^3) layout with the x
    index fastest, or None for the kinetic part alone.
    """
    u_nodes = mesh.nodes_from_dofs(u)
    v = None if vq is None else mesh.to_cell_quad(vq)
    y = _cell_operator(mesh, _cell_values(mesh, u_nodes), v, 0.5)
    return mesh.dofs_from_nodes(_assemble(mesh, y))


def apply_Hbar(mesh, vq, psibar):
    """Hbar psibar = M^-1/2 H M^-1/2 psibar (Eq. TDKSMatVecStandard)."""
    s = mesh.m_inv_sqrt.reshape((-1,) + (1,) * (psibar.ndim - 1))
    return s * apply_H(mesh, vq, s * psibar)


def apply_K(mesh, u_nodes):
    """K u over ALL nodes (boundary rows included); u_nodes: (n_nodes, ...)."""
    y = _cell_operator(mesh, _cell_values(mesh, u_nodes), None, 1.0)
    return _assemble(mesh, y)


# ---------------------------------------------------------------------------
# dense assembly for tiny meshes (independent pin of the matrix-free action)
# ---------------------------------------------------------------------------
def _element_tables(mesh):
    """Phi[q, a] = N_a(x_q) and dPhi[d][q, a] = dN_a/dxi_d on the reference cell.

    Point index q and node index a both run with the z index slowest, the same
    ordering as a C-order reshape of (x, y, z) arrays.
    """
    B, D = mesh.ref.B, mesh.ref.D
    Phi = np.kron(np.kron(B, B), B)  # rows (a,b,c), cols (i,j,k), x slowest
    dX = np.kron(np.kron(D, B), B)
    dY = np.kron(np.kron(B, D), B)
    dZ = np.kron(np.kron(B, B), D)
    return Phi, (dX, dY, dZ)


def _dense(mesh, vq, kin):
    Phi, dP = _element_tables(mesh)
    nn = mesh.n_nodes
    A = np.zeros((nn, nn))
    wdet = mesh.volume_weights.reshape(mesh.n_cell, -1)
    G = mesh.Ginvq.reshape(mesh.n_cell, -1, 3, 3)
    v = None if vq is None else mesh.to_cell_quad(vq).reshape(mesh.n_cell, -1)
    for e in range(mesh.n_cell):
        Ae = np.zeros((Phi.shape[1], Phi.shape[1]))
        for d in range(3):
            for k in range(3):
                Ae += kin * dP[d].T @ ((wdet[e] * G[e, :, d, k])[:, None] * dP[k])
        if v is not None:
            Ae += Phi.T @ ((wdet[e] * v[e])[:, None] * Phi)
        ids = mesh.cell_nodes[e].reshape(-1)
        A[np.ix_(ids, ids)] += Ae
    return A


def dense_H(mesh, vq):
    """Dense H restricted to the DoFs (tiny meshes only)."""
    A = _dense(mesh, vq, 0.5)
    if hasattr(mesh, "C"):  # hanging-node constraints: C^T A C
        C = mesh.C.toarray()
        return C.T @ A @ C
    return A[np.ix_(mesh.dof_nodes, mesh.dof_nodes)]


def dense_Hbar(mesh, vq):
    s = mesh.m_inv_sqrt
    return s[:, None] * dense_H(mesh, vq) * s[None, :]


def dense_K(mesh):
    """Dense stiffness over all nodes (tiny meshes only)."""
    return _dense(mesh, None, 1.0)
