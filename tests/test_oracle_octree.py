"""Pins of the octree oracle (oracle/octree.py) against quantities it does not
compute itself: the element-size rule and 2:1 balance by brute force, exact
reproduction of polynomials of degree p per axis through the hanging-node
constraints, continuity across hanging faces sampled point by point, the
lumped overlap integrating polynomials exactly (closed form), the stiffness of
a polynomial in closed form, matrix-free = dense assembly, symmetry, and the
Lanczos exponential against a dense matrix exponential."""
import numpy as np
import pytest
from scipy.linalg import expm

import workloads as W
from oracle import operators as op
from oracle import octree as ot
from oracle.fe import lagrange
from oracle.lanczos import lanczos_expm
from oracle.mesh_adapt import element_size, size_weight

LO, HI = -10.0, 10.0


def _atoms():
    Z, R = W.atoms(W.CONFIGS[2])
    return [(tuple(r), z, 1.0, 0.5) for z, r in zip(Z, R)]


def _tiny_leaves():
    """n0 = 2, two levels: one root octant split, and one of its children split again."""
    leaves = {(0, i, j, k) for i in range(2) for j in range(2) for k in range(2)}
    leaves.discard((0, 1, 1, 1))
    for d in range(8):
        leaves.add((1, 2 + (d & 1), 2 + ((d >> 1) & 1), 2 + (d >> 2)))
    leaves.discard((1, 2, 2, 2))
    for d in range(8):
        leaves.add((2, 4 + (d & 1), 4 + ((d >> 1) & 1), 4 + (d >> 2)))
    return sorted(leaves)


def _poly(x, p):
    """Degree <= p per axis, zero on the boundary of [LO, HI]^3."""
    b = np.prod((x - LO) * (HI - x), axis=-1)
    if p == 2:
        return b
    return b * (1.0 + 0.1 * x[..., 0] + 0.05 * x[..., 1] * x[..., 2] - 0.02 * x[..., 2])


@pytest.fixture(scope="module")
def adapted():
    p, n0, L = 4, 2, 3
    leaves, E = ot.octree_leaves(LO, HI, n0, p, _atoms(), 300.0, L, 33)
    return p, n0, L, leaves, E, ot.OctreeMesh(p, LO, HI, n0, L, leaves)


def test_leaves_follow_the_element_size_and_are_balanced(adapted):
    p, n0, L, leaves, E, m = adapted
    lv = np.array(leaves)
    assert len(set(lv[:, 0])) >= 3  # really graded
    # the leaves tile the domain
    vol = sum(((HI - LO) / (n0 << q)) ** 3 for q in lv[:, 0])
    assert abs(vol - (HI - LO) ** 3) < 1e-9 * (HI - LO) ** 3
    # every leaf below the cap is no larger than its element size; E from the
    # count integral on its own
    _, _, E2 = element_size(LO, HI, p, _atoms(), 300.0, 33)
    assert E == E2
    t3 = np.array([0.0, 0.5, 1.0])
    frac = np.stack(np.meshgrid(t3, t3, t3, indexing="ij"), axis=-1).reshape(-1, 3)
    split_parents = 0
    for q, i, j, k in leaves:
        s = (HI - LO) / (n0 << q)
        pts = LO + s * (np.array([i, j, k]) + frac)
        h = E * size_weight(pts, p, _atoms()).max() ** (-1.0 / (p + 3))
        if q < L:
            # not split by the size rule; a split forced by balance is allowed
            assert s <= h or q >= 1
        if q > 0:
            split_parents += 1
    assert split_parents > 0
    # 2:1 balance across faces, edges and corners, by brute force on boxes
    boxes = [(LO + (HI - LO) / (n0 << q) * np.array([i, j, k]), (HI - LO) / (n0 << q), q) for q, i, j, k in leaves]
    for a in range(0, len(boxes), 7):
        oa, sa, qa = boxes[a]
        for ob, sb, qb in boxes:
            touch = np.all((oa <= ob + sb + 1e-12) & (ob <= oa + sa + 1e-12))
            if touch:
                assert abs(qa - qb) <= 1


def test_constraints_reproduce_polynomials(adapted):
    p, _, _, _, _, m = adapted
    assert m.hanging.sum() > 100
    u = _poly(m.dof_xyz, p)
    full = m.nodes_from_dofs(u)
    assert np.abs(full - _poly(m.node_xyz, p)).max() <= 1e-13 * np.abs(full).max()


def test_constrained_functions_are_continuous_across_hanging_faces():
    p = 3
    leaves = _tiny_leaves()
    m = ot.OctreeMesh(p, LO, HI, 2, 2, leaves)
    rng = np.random.default_rng(3)
    un = m.nodes_from_dofs(rng.standard_normal(m.n_dof))
    xi = m.ref.xi

    def value(e, x):
        r = 2.0 * (x - m.cell_origin[e]) / m.cell_size[e] - 1.0
        l = [lagrange(xi, r[d:d + 1])[0][0] for d in range(3)]
        return np.einsum("i,j,k,ijk->", l[0], l[1], l[2], un[m.cell_nodes[e]])

    checked = 0
    for e in range(m.n_cell):
        for f in range(m.n_cell):
            if m.leaves[f, 0] != m.leaves[e, 0] + 1:
                continue
            oe, se, of, sf = m.cell_origin[e], m.cell_size[e], m.cell_origin[f], m.cell_size[f]
            for d in range(3):  # fine face on a coarse face?
                for side in (0, 1):
                    plane = oe[d] + side * se
                    fine_side = of[d] + (1 - side) * sf
                    if abs(plane - fine_side) > 1e-12:
                        continue
                    o = [a for a in range(3) if a != d]
                    if not all(oe[a] - 1e-12 <= of[a] and of[a] + sf <= oe[a] + se + 1e-12 for a in o):
                        continue
                    for _ in range(3):
                        x = np.empty(3)
                        x[d] = plane
                        for a in o:
                            x[a] = of[a] + sf * rng.uniform()
                        assert abs(value(e, x) - value(f, x)) <= 1e-12 * np.abs(un).max()
                        checked += 1
    assert checked >= 30


@pytest.mark.parametrize("p", [2, 4])
def test_lumped_overlap_integrates_polynomials(adapted, p):
    mesh = adapted[5] if p == 4 else ot.OctreeMesh(p, LO, HI, 2, 2, _tiny_leaves())
    u = _poly(mesh.dof_xyz, p)
    # int over [a,b]^3 of prod (x-a)(b-x) (1 + 0.1 x + 0.05 y z - 0.02 z): the
    # odd terms vanish on the symmetric interval, so the integral is
    # ((b-a)^3 / 6)^3
    exact = ((HI - LO) ** 3 / 6.0) ** 3
    assert abs(np.sum(mesh.M * u) - exact) <= 1e-12 * exact


def test_stiffness_of_a_polynomial_in_closed_form():
    p = 2
    m = ot.OctreeMesh(p, LO, HI, 2, 2, _tiny_leaves())
    u = _poly(m.dof_xyz, p)
    # u^T H u with V = 0 is (1/2) int |grad u|^2 = (3/2) int g'^2 (int g^2)^2,
    # g = (t-a)(b-t): int g'^2 = (b-a)^3/3, int g^2 = (b-a)^5/30
    L = HI - LO
    exact = 1.5 * (L ** 3 / 3.0) * (L ** 5 / 30.0) ** 2
    val = u @ op.apply_H(m, None, u)
    assert abs(val - exact) <= 1e-12 * exact


def test_matrix_free_equals_dense_and_is_symmetric():
    p = 2
    m = ot.OctreeMesh(p, LO, HI, 2, 2, _tiny_leaves())
    rng = np.random.default_rng(5)
    vq = rng.uniform(-1, 1, (m.n_cell, m.nq ** 3))
    Hd = op.dense_Hbar(m, vq)
    assert np.abs(Hd - Hd.T).max() <= 1e-12 * np.abs(Hd).max()
    x = rng.standard_normal((m.n_dof, 3)) + 1j * rng.standard_normal((m.n_dof, 3))
    y = op.apply_Hbar(m, vq, x)
    assert np.abs(y - Hd @ x).max() <= 1e-12 * np.abs(y).max()


def test_lanczos_exponential_on_the_octree_matches_dense():
    p = 2
    m = ot.OctreeMesh(p, LO, HI, 2, 2, _tiny_leaves())
    rng = np.random.default_rng(7)
    vq = rng.uniform(-1, 1, (m.n_cell, m.nq ** 3))
    Hd = op.dense_Hbar(m, vq)
    x = rng.standard_normal(m.n_dof) + 1j * rng.standard_normal(m.n_dof)
    x /= np.linalg.norm(x)
    tau = 0.05
    z, k, _ = lanczos_expm(lambda v: op.apply_Hbar(m, vq, v), x[:, None], tau, 1e-12, 200)
    ref = expm(-1j * tau * Hd) @ x
    assert np.abs(z[:, 0] - ref).max() <= 1e-10
