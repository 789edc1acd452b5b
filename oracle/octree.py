"""Octree meshes with hanging nodes from the a priori element size (oracle).

Sec. "Efficient spatio-temporal discretization": the element size that
minimises the bound on the dipole error at a fixed element count (Eqs.
OptimalMeshMin, OptimalMeshSize) is h(r) = E g(r)^(-1/(p+3)), with g and E as
in ``oracle.mesh_adapt``.  The paper meshes the molecule with adaptive
hexahedra that follow h(r); it does not describe how the meshes are made
conforming, nor the overlap matrix on them.  Readings taken here:

* refinement: [lo, hi]^3 starts as n0^3 cubes; a cube of edge s is split into
  its 8 octants while s > h_cell = E (largest g over the cube's 27 sample
  points: corners, edge and face midpoints, centre)^(-1/(p+3)), at most
  max_level times;
* balance: leaves that share a face, an edge or a corner differ by at most one
  level (the coarser one is split until this holds);
* continuity: a GLL node of a leaf that lies on the closed boundary of another
  leaf without being one of that leaf's nodes (a hanging node) takes the value
  of that leaf's polynomial there, u(x) = sum_m N_m(x) u_m over the leaf's
  nodes (only its face or edge nodes are non-zero on its boundary); chains are
  resolved by substitution, and masters on the domain boundary (homogeneous
  Dirichlet data) drop out.  The remaining interior nodes are the DoFs and C
  maps DoF values to the values at every node;
* overlap: with N_m the GLL-quadrature mass of node m in the unconstrained
  space (diagonal), the constrained overlap C^T diag(N) C is not diagonal; its
  row sums M_d = sum_m C_md N_m are used (they keep the GLL quadrature of every
  function of the constrained space exact: sum_d M_d f_d = sum_m N_m f(x_m)),
  so that Hbar = M^-1/2 C^T H_nodes C M^-1/2 keeps the form of Eq.
  TDKSMatVecStandard.

The class below exposes the attributes the oracle's operator, density and
dipole functions use (``cell_nodes``, ``ref``, ``volume_weights``, ...), with
``nodes_from_dofs`` applying C and ``dofs_from_nodes`` its transpose.

This module is test infrastructure: only tests/, the package smoke check and
the benchmark's CPU baseline use it.
"""
import numpy as np
import scipy.sparse as sp

from .fe import RefElement, lagrange
from .mesh_adapt import element_size, size_weight

_OFFS = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1) if (dx, dy, dz) != (0, 0, 0)]


def _is_leaf_map(leaves, n0, L):
    """Boolean arrays per level: leaf[q][i, j, k]."""
    maps = [np.zeros((n0 << q,) * 3, dtype=bool) for q in range(L + 1)]
    for (q, i, j, k) in leaves:
        maps[q][i, j, k] = True
    return maps


def octree_leaves(lo, hi, n0, p, atoms, n_elem, max_level, S):
    """Leaves (level, i, j, k) of the balanced octree and the constant E.

    Cell (q, i, j, k) is the cube of edge (hi - lo) / (n0 2^q) whose lowest
    corner is lo + (i, j, k) times that edge."""
    _, _, E = element_size(lo, hi, p, atoms, n_elem, S)
    leaves = {(0, i, j, k) for i in range(n0) for j in range(n0) for k in range(n0)}
    t3 = np.array([0.0, 0.5, 1.0])
    frac = np.stack(np.meshgrid(t3, t3, t3, indexing="ij"), axis=-1).reshape(-1, 3)
    for q in range(max_level):
        cells = sorted(c for c in leaves if c[0] == q)
        if not cells:
            continue
        s = (hi - lo) / (n0 << q)
        org = lo + s * np.array([c[1:] for c in cells], dtype=np.float64)
        pts = org[:, None, :] + s * frac[None, :, :]
        gmax = size_weight(pts, p, atoms).max(axis=1)
        with np.errstate(divide="ignore"):
            h = E * gmax ** (-1.0 / (p + 3))
        for c, hc in zip(cells, h):
            if s > hc:
                leaves.discard(c)
                _, i, j, k = c
                for d in range(8):
                    leaves.add((q + 1, 2 * i + (d & 1), 2 * j + ((d >> 1) & 1), 2 * k + (d >> 2)))
    # 2:1 balance over faces, edges and corners
    while True:
        maps = _is_leaf_map(leaves, n0, max_level)
        split = set()
        for (m, i, j, k) in leaves:
            if m < 2:
                continue
            nm = n0 << m
            for dx, dy, dz in _OFFS:
                a, b, c = i + dx, j + dy, k + dz
                if not (0 <= a < nm and 0 <= b < nm and 0 <= c < nm):
                    continue
                for q in range(m - 2, -1, -1):  # a leaf two or more levels coarser?
                    sh = m - q
                    if maps[q][a >> sh, b >> sh, c >> sh]:
                        split.add((q, a >> sh, b >> sh, c >> sh))
                        break
        if not split:
            break
        for (q, i, j, k) in split:
            leaves.discard((q, i, j, k))
            for d in range(8):
                leaves.add((q + 1, 2 * i + (d & 1), 2 * j + ((d >> 1) & 1), 2 * k + (d >> 2)))
    return sorted(leaves), E


class OctreeMesh:
    """Order-p spectral elements on the leaves of an octree over [lo, hi]^3.

    leaves: (level, i, j, k) tuples (``octree_leaves``); cells are numbered in
    the given order.  Nodes are the distinct GLL nodes of all leaves, numbered
    by their position (x slowest, z fastest); DoFs are the interior nodes that
    are not hanging, in node order."""

    def __init__(self, p, lo, hi, n0, max_level, leaves):
        self.ref = RefElement(p)
        self.p, self.n, self.nq = self.ref.p, self.ref.n, self.ref.nq
        n, L = self.n, max_level
        self.lo, self.hi, self.n0, self.max_level = lo, hi, n0, L
        lv = np.array(leaves, dtype=np.int64).reshape(-1, 4)
        self.leaves = lv
        self.n_cell = len(lv)
        unit = (hi - lo) / (n0 << L)  # lattice unit of the finest level
        size = (1 << (L - lv[:, 0])).astype(np.float64)  # edge in lattice units
        origin = lv[:, 1:] * size[:, None]
        self.cell_size = size * unit
        self.cell_origin = lo + origin * unit
        xi = self.ref.xi
        # node positions in lattice units, (e, i, j, k, 3)
        loc = size[:, None] * (1.0 + xi[None, :]) / 2.0  # (e, n)
        P = np.empty((self.n_cell, n, n, n, 3))
        P[..., 0] = origin[:, 0, None, None, None] + loc[:, :, None, None]
        P[..., 1] = origin[:, 1, None, None, None] + loc[:, None, :, None]
        P[..., 2] = origin[:, 2, None, None, None] + loc[:, None, None, :]
        keys = np.round(P.reshape(-1, 3) * 2.0 ** 24).astype(np.int64)
        ukeys, inv = np.unique(keys, axis=0, return_inverse=True)
        self.n_nodes = len(ukeys)
        self.cell_nodes = inv.reshape(self.n_cell, n, n, n).astype(np.int64)
        # positions from the cells' own formula (identical for every cell
        # sharing a node), not from the rounded keys
        node_lat = np.empty((self.n_nodes, 3))
        node_lat[inv] = P.reshape(-1, 3)
        self.node_xyz = lo + node_lat * unit
        top = float(n0 << L)
        self.is_boundary = np.any((ukeys == 0) | (ukeys == int(round(top * 2.0 ** 24))), axis=1)

        # unconstrained GLL mass of every node: sum over the cells owning it
        w = self.ref.w
        w3n = w[:, None, None] * w[None, :, None] * w[None, None, :]
        detn = (self.cell_size / 2.0) ** 3
        Mn = np.zeros(self.n_nodes)
        np.add.at(Mn, self.cell_nodes.reshape(-1), (w3n[None] * detn[:, None, None, None]).reshape(-1))
        self.M_nodes = Mn

        # hanging nodes: on the closed box of a leaf that does not own them
        owner_level = np.full(self.n_nodes, -1, dtype=np.int64)
        np.maximum.at(owner_level, self.cell_nodes.reshape(-1), np.repeat(lv[:, 0], n ** 3))
        maps = _is_leaf_map([tuple(r) for r in lv], n0, L)
        leaf_id = [dict() for _ in range(L + 1)]
        for e, (q, i, j, k) in enumerate(lv):
            leaf_id[q][(i, j, k)] = e
        raw = {}
        cand = np.nonzero(~self.is_boundary)[0]
        for q in range(L):
            sz = float(1 << (L - q))
            nodes_q = cand[owner_level[cand] > q]
            if len(nodes_q) == 0:
                continue
            x = node_lat[nodes_q]
            eps = 1e-7
            lo_idx = np.floor((x - eps) / sz).astype(np.int64)
            hi_idx = np.floor((x + eps) / sz).astype(np.int64)
            nq_ = n0 << q
            for combo in range(8):
                idx = np.where(np.array([(combo >> a) & 1 for a in range(3)])[None, :] == 1, hi_idx, lo_idx)
                ok = np.all((idx >= 0) & (idx < nq_), axis=1)
                ok[ok] = maps[q][idx[ok, 0], idx[ok, 1], idx[ok, 2]]
                for t in np.nonzero(ok)[0]:
                    node = int(nodes_q[t])
                    if node in raw:
                        continue
                    e = leaf_id[q][tuple(int(v) for v in idx[t])]
                    ref = 2.0 * (x[t] - idx[t] * sz) / sz - 1.0  # reference coordinates in the leaf
                    owned = all(np.min(np.abs(xi - r)) < 1e-9 for r in ref)
                    if owned:
                        continue
                    if not np.any(np.abs(ref) == 1.0):
                        raise AssertionError("node inside a leaf that does not own it")
                    lx = lagrange(xi, ref[0:1])[0][0]
                    ly = lagrange(xi, ref[1:2])[0][0]
                    lz = lagrange(xi, ref[2:3])[0][0]
                    W = lx[:, None, None] * ly[None, :, None] * lz[None, None, :]
                    nz = np.nonzero(W)
                    raw[node] = list(zip(self.cell_nodes[e][nz].tolist(), W[nz].tolist()))
        self.hanging = np.zeros(self.n_nodes, dtype=bool)
        self.hanging[list(raw)] = True
        # resolve chains; boundary masters carry 0
        resolved = {}

        def expand(node):
            if node in resolved:
                return resolved[node]
            acc = {}
            for m, wt in raw[node]:
                if self.is_boundary[m]:
                    continue
                if m in raw:
                    for mm, ww in expand(m).items():
                        acc[mm] = acc.get(mm, 0.0) + wt * ww
                else:
                    acc[m] = acc.get(m, 0.0) + wt
            resolved[node] = acc
            return acc

        free = ~self.is_boundary & ~self.hanging
        self.dof_nodes = np.nonzero(free)[0]
        self.n_dof = len(self.dof_nodes)
        self.node_to_dof = -np.ones(self.n_nodes, dtype=np.int64)
        self.node_to_dof[self.dof_nodes] = np.arange(self.n_dof)
        rows, cols, vals = list(self.dof_nodes), list(range(self.n_dof)), [1.0] * self.n_dof
        for node in raw:
            for m, wt in expand(node).items():
                rows.append(node)
                cols.append(int(self.node_to_dof[m]))
                vals.append(wt)
        self.C = sp.csr_matrix((vals, (rows, cols)), shape=(self.n_nodes, self.n_dof))
        self.M = self.C.T @ self.M_nodes
        if np.any(self.M <= 0.0):
            raise ValueError("lumped overlap is not positive")
        self.m_inv_sqrt = 1.0 / np.sqrt(self.M)
        self.m_sqrt = np.sqrt(self.M)

        # geometry at the Gauss points (cubes: J = s/2 I)
        eta = self.ref.eta
        nqq = self.nq
        s = self.cell_size
        self.xq = np.empty((self.n_cell, nqq, nqq, nqq, 3))
        lq = s[:, None] * (1.0 + eta[None, :]) / 2.0
        o = self.cell_origin
        self.xq[..., 0] = o[:, 0, None, None, None] + lq[:, :, None, None]
        self.xq[..., 1] = o[:, 1, None, None, None] + lq[:, None, :, None]
        self.xq[..., 2] = o[:, 2, None, None, None] + lq[:, None, None, :]
        self.detJq = np.broadcast_to(((s / 2.0) ** 3)[:, None, None, None], (self.n_cell, nqq, nqq, nqq)).copy()
        g = (2.0 / s) ** 2
        self.Ginvq = np.zeros((self.n_cell, nqq, nqq, nqq, 3, 3))
        for d in range(3):
            self.Ginvq[..., d, d] = g[:, None, None, None]
        wq = self.ref.wq
        self.w3q = wq[:, None, None] * wq[None, :, None] * wq[None, None, :]

    # -- the interface the oracle's operators and density use -----------------
    def nodes_from_dofs(self, u):
        """Values at every node (hanging ones interpolated, boundary 0)."""
        u = np.asarray(u)
        return (self.C @ u.reshape(self.n_dof, -1)).reshape((self.n_nodes,) + u.shape[1:])

    def dofs_from_nodes(self, y):
        """C^T y: node contributions gathered onto the DoFs."""
        y = np.asarray(y)
        return (self.C.T @ y.reshape(self.n_nodes, -1)).reshape((self.n_dof,) + y.shape[1:])

    @property
    def dof_xyz(self):
        return self.node_xyz[self.dof_nodes]

    @property
    def quad_xyz(self):
        """Gauss point coordinates, (n_cell, nq^3, 3), point order a + nq (b + nq c)."""
        return self.xq.transpose(0, 3, 2, 1, 4).reshape(self.n_cell, self.nq ** 3, 3)

    def to_cell_quad(self, v):
        nq = self.nq
        return np.asarray(v).reshape(self.n_cell, nq, nq, nq).transpose(0, 3, 2, 1)

    def from_cell_quad(self, v):
        return np.asarray(v).transpose(0, 3, 2, 1).reshape(self.n_cell, -1)

    @property
    def volume_weights(self):
        return self.w3q[None] * self.detJq
