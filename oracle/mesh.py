"""Hexahedral spectral-FE mesh, Dirichlet DoFs and the GLL overlap (oracle).

Follows Sec. "Semi-discrete solution" (Eq. PsiExpansion: order-p FE basis,
psi^h = 0 on the boundary) and Sec. "Higher-order spectral finite-elements"
(GLL quadrature for M, which makes M diagonal).

Mesh reading (the paper builds adaptive hexahedral meshes, Sec. "Optimal
discretization"; hanging nodes are never discussed): a structured logical
grid of ncx x ncy x ncz cells whose corners are given by a vertex array;
each cell is the trilinear image of [-1,1]^3.  Trilinear maps agree on shared
faces, so the global GLL nodes are well defined and M stays diagonal.
"""
import numpy as np

from .fe import RefElement


def _trilinear_shape(s):
    """phi_0, phi_1 of one direction and their derivatives at points s."""
    s = np.asarray(s, dtype=np.float64)
    phi = np.stack([(1.0 - s) / 2.0, (1.0 + s) / 2.0], axis=-1)
    dphi = np.stack([np.full_like(s, -0.5), np.full_like(s, 0.5)], axis=-1)
    return phi, dphi


class Mesh:
    """Order-p hexahedral mesh on a structured logical grid.

    vertices: array (ncz+1, ncy+1, ncx+1, 3) or flat ((ncx+1)(ncy+1)(ncz+1), 3)
    with x fastest.  Cells are numbered e = cx + ncx (cy + ncy cz); global
    nodes (I, J, K), I in [0, ncx p], are numbered I + Nx (J + Ny K); DoFs are
    the interior nodes, numbered lexicographically with x fastest.
    """

    def __init__(self, p, ncell, vertices, nq=None):
        self.ref = RefElement(p, nq)
        self.p, self.n, self.nq = self.ref.p, self.ref.n, self.ref.nq
        ncx, ncy, ncz = (int(c) for c in ncell)
        self.ncell = (ncx, ncy, ncz)
        self.n_cell = ncx * ncy * ncz
        V = np.asarray(vertices, dtype=np.float64).reshape(ncz + 1, ncy + 1, ncx + 1, 3)
        self.vertices = V
        p, n, nq = self.p, self.n, self.nq
        self.Nx, self.Ny, self.Nz = ncx * p + 1, ncy * p + 1, ncz * p + 1
        self.n_nodes = self.Nx * self.Ny * self.Nz

        # corners of each cell: (e, c, b, a, 3) for z,y,x corner offsets
        cz, cy, cx = np.meshgrid(np.arange(ncz), np.arange(ncy), np.arange(ncx), indexing="ij")
        cz, cy, cx = cz.ravel(), cy.ravel(), cx.ravel()
        corners = np.empty((self.n_cell, 2, 2, 2, 3))
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    corners[:, c, b, a, :] = V[cz + c, cy + b, cx + a, :]
        self.corners = corners
        self.cell_index = (cx, cy, cz)

        # global node ids of every cell node, local order (i, j, k) = (x, y, z)
        li = np.arange(n)
        I = cx[:, None, None, None] * p + li[None, :, None, None]
        J = cy[:, None, None, None] * p + li[None, None, :, None]
        K = cz[:, None, None, None] * p + li[None, None, None, :]
        self.cell_nodes = (I + self.Nx * (J + self.Ny * K)).astype(np.int64)

        # interior nodes are the DoFs (homogeneous Dirichlet, Eq. PsiExpansion)
        gI, gJ, gK = np.meshgrid(np.arange(self.Nx), np.arange(self.Ny), np.arange(self.Nz), indexing="ij")
        interior = ((gI > 0) & (gI < self.Nx - 1) & (gJ > 0) & (gJ < self.Ny - 1)
                    & (gK > 0) & (gK < self.Nz - 1))
        node_id = (gI + self.Nx * (gJ + self.Ny * gK))
        # lexicographic, x fastest: sort by node id
        ids = np.sort(node_id[interior].ravel())
        self.dof_nodes = ids
        self.n_dof = len(ids)
        self.node_to_dof = -np.ones(self.n_nodes, dtype=np.int64)
        self.node_to_dof[ids] = np.arange(self.n_dof)
        self.is_boundary = self.node_to_dof < 0

        # geometry at the Gauss points and at the GLL nodes
        self.xq, self.detJq, self.Ginvq = self._geometry(self.ref.eta)
        xn, self.detJn, _ = self._geometry(self.ref.xi)
        self.node_xyz = np.zeros((self.n_nodes, 3))
        self.node_xyz[self.cell_nodes.reshape(-1)] = xn.reshape(-1, 3)
        if np.any(self.detJq <= 0.0) or np.any(self.detJn <= 0.0):
            raise ValueError("mesh has a non-positive Jacobian")

        # GLL quadrature weight of every node of the reference cell
        w = self.ref.w
        self.w3n = w[:, None, None] * w[None, :, None] * w[None, None, :]
        wq = self.ref.wq
        self.w3q = wq[:, None, None] * wq[None, :, None] * wq[None, None, :]
        # diagonal overlap: M_jj = sum_e w_i w_j w_k detJ_e(node)
        Mn = np.zeros(self.n_nodes)
        np.add.at(Mn, self.cell_nodes.reshape(-1), (self.w3n[None] * self.detJn).reshape(-1))
        self.M_nodes = Mn
        self.M = Mn[self.dof_nodes]
        self.m_inv_sqrt = 1.0 / np.sqrt(self.M)
        self.m_sqrt = np.sqrt(self.M)

    def _geometry(self, pts):
        """Positions, det J and J^-1 J^-T of every cell at the tensor points pts^3.

        J[d, k] = dx_d / dxi_k of the trilinear map; the gradient of a function
        is J^-T grad_xi, so grad N . grad u = grad_xi N^T (J^-1 J^-T) grad_xi u.
        Arrays are indexed (e, a, b, c) with a along x, b along y, c along z.
        """
        phi, dphi = _trilinear_shape(pts)
        C = self.corners  # (e, cz, cy, cx, 3)
        x = np.einsum("ezyxd,ax,by,cz->eabcd", C, phi, phi, phi)
        Jx = np.einsum("ezyxd,ax,by,cz->eabcd", C, dphi, phi, phi)
        Jy = np.einsum("ezyxd,ax,by,cz->eabcd", C, phi, dphi, phi)
        Jz = np.einsum("ezyxd,ax,by,cz->eabcd", C, phi, phi, dphi)
        J = np.stack([Jx, Jy, Jz], axis=-1)  # (..., d, k)
        det = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        Ginv = np.einsum("...ij,...kj->...ik", Jinv, Jinv)
        return x, det, Ginv

    # -- convenience -----------------------------------------------------
    def nodes_from_dofs(self, u):
        """Values at every node from DoF values (boundary nodes 0)."""
        u = np.asarray(u)
        out = np.zeros((self.n_nodes,) + u.shape[1:], dtype=u.dtype)
        out[self.dof_nodes] = u
        return out

    def dofs_from_nodes(self, y):
        """Rows of a node array that belong to DoFs."""
        return np.asarray(y)[self.dof_nodes]

    @property
    def dof_xyz(self):
        return self.node_xyz[self.dof_nodes]

    @property
    def quad_xyz(self):
        """Gauss point coordinates, (n_cell, nq^3, 3), point order a + nq (b + nq c)."""
        x = self.xq.transpose(0, 3, 2, 1, 4)  # (e, c, b, a, d): a fastest
        return x.reshape(self.n_cell, self.nq ** 3, 3)

    def to_cell_quad(self, v):
        """(n_cell, nq^3) with a fastest -> (e, a, b, c)."""
        nq = self.nq
        return np.asarray(v).reshape(self.n_cell, nq, nq, nq).transpose(0, 3, 2, 1)

    def from_cell_quad(self, v):
        """(e, a, b, c) -> (n_cell, nq^3) with a fastest."""
        return np.asarray(v).transpose(0, 3, 2, 1).reshape(self.n_cell, -1)

    @property
    def volume_weights(self):
        """varpi_q det J_q at every Gauss point, layout (e, a, b, c)."""
        return self.w3q[None] * self.detJq

