"""Host side of the octree meshes (no GPU needed): tdfe_fe_octree_setup builds
the merged nodes, the hanging-node constraints and the lumped overlap on the
host, so its counts -- nodes, hanging nodes, non-zeros of C, DoFs, cells --
are compared with the oracle's OctreeMesh, and descriptions that do not
describe a balanced tiling of the domain are refused before any device work."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import octree as ot

LO, HI = -10.0, 10.0


def _atoms():
    Z, R = W.atoms(W.CONFIGS[2])
    return [(tuple(r), z, 1.0, 0.5) for z, r in zip(Z, R)]


def balanced_tiny_leaves():
    """n0 = 2: the root octant at the far corner split, and its far-corner
    child split again (every leaf within one level of its neighbours)."""
    leaves = {(0, i, j, k) for i in range(2) for j in range(2) for k in range(2)}
    leaves.discard((0, 1, 1, 1))
    for d in range(8):
        leaves.add((1, 2 + (d & 1), 2 + ((d >> 1) & 1), 2 + (d >> 2)))
    leaves.discard((1, 3, 3, 3))
    for d in range(8):
        leaves.add((2, 6 + (d & 1), 6 + ((d >> 1) & 1), 6 + (d >> 2)))
    return sorted(leaves)


@pytest.fixture(scope="module")
def lib():
    from paper_1810_13130_amd import tdfe
    return tdfe.load()


def _setup(lib, p, n0, L, leaves, precision=0):
    from paper_1810_13130_amd import tdfe
    lv = np.ascontiguousarray(np.array(leaves, dtype=np.int32).reshape(-1, 4))
    d = tdfe.OctreeDesc()
    d.p, d.lo, d.hi, d.n0, d.max_level = p, LO, HI, n0, L
    d.n_leaf, d.leaves = len(lv), lv.ctypes.data_as(tdfe._IP)
    d.n_orb_max, d.k_max, d.precision = 2, 16, precision
    h = ctypes.c_void_p()
    s = lib.tdfe_fe_octree_setup(ctypes.byref(d), None, ctypes.byref(h))
    return s, h


@pytest.mark.parametrize("case", ["adapted_p3", "tiny_p2", "tiny_p5"])
def test_host_builder_counts_match_oracle(lib, case):
    if case == "adapted_p3":
        p, n0, L = 3, 2, 2
        leaves, _ = ot.octree_leaves(LO, HI, n0, p, _atoms(), 200.0, L, 33)
    else:
        p, n0, L = (2 if case == "tiny_p2" else 5), 2, 2
        leaves = balanced_tiny_leaves()
    m = ot.OctreeMesh(p, LO, HI, n0, L, leaves)
    s, h = _setup(lib, p, n0, L, leaves)
    assert s == 0
    nn, nh, nz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert lib.tdfe_octree_info(h, ctypes.byref(nn), ctypes.byref(nh), ctypes.byref(nz)) == 0
    nd, nc, nq, ws = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
    assert lib.tdfe_query(h, ctypes.byref(nd), ctypes.byref(nc), ctypes.byref(nq), ctypes.byref(ws)) == 0
    assert (nn.value, nh.value, nz.value) == (m.n_nodes, int(m.hanging.sum()), m.C.nnz)
    assert (nd.value, nc.value, nq.value) == (m.n_dof, m.n_cell, m.n_cell * (p + 1) ** 3)
    assert m.hanging.sum() > 0
    lib.tdfe_destroy(h)


def test_unbalanced_overlapping_or_incomplete_leaves_are_refused(lib):
    good = balanced_tiny_leaves()
    s, h = _setup(lib, 2, 2, 2, good)
    assert s == 0
    lib.tdfe_destroy(h)
    # a level-2 leaf next to a level-0 leaf
    unbalanced = [c for c in good if c != (1, 2, 2, 2)] + [(2, 4 + (d & 1), 4 + ((d >> 1) & 1), 4 + (d >> 2))
                                                           for d in range(8)]
    assert _setup(lib, 2, 2, 2, unbalanced)[0] == -1
    assert _setup(lib, 2, 2, 2, good[:-1])[0] == -1                    # a gap
    assert _setup(lib, 2, 2, 2, good + [good[0]])[0] == -1             # a repeated leaf
    assert _setup(lib, 2, 2, 2, good + [(0, 1, 1, 1)])[0] == -1        # a leaf inside another
    assert _setup(lib, 2, 2, 2, [(0, 0, 0, 2)] + good[1:])[0] == -1    # out of range
    assert _setup(lib, 2, 2, 1, good)[0] == -1                         # level above max_level
    assert _setup(lib, 2, 2, 2, good, precision=1)[0] == -1            # FP64 only
