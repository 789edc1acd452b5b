"""GPU parity of the two box-cell operator kernels at even n = p + 1.

The lane-pair kernel (two lanes per plane) is the FP64 default at even n; the
plane kernel is the FP32 default and serves every odd n.  TDFE_APPLY_VARIANT
(read at context creation) selects either one for both precisions.  Each odd
order p = 1, 3, 5, 7 is checked against the FP64 oracle on a small box mesh
with an uneven cell count per axis and an orbital count that selects a
different column-block width (ragged chunks included), in FP64 (1e-12) and in
FP32 storage (2e-6), for both kernels; the Lanczos exponential exercises the
kernels' per-column quadratic form (the Lanczos alpha); and the benchmark
workload's full-size operator is compared across the kernels and with the
oracle.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_context, oracle_mesh, rel
from oracle import lanczos, operators as op

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
MIXED = 1

ORBS = {1: 1, 3: 5, 5: 9, 7: 2}


def _box(p, n_orb, ncell=(3, 2, 2)):
    return W.scaled(W.CONFIGS[2], ncell=ncell, p=p, n_orb=n_orb)


@pytest.mark.parametrize("variant", ["pair", "plane"])
@pytest.mark.parametrize("p", sorted(ORBS))
def test_box_operator_fp64(p, variant, monkeypatch):
    monkeypatch.setenv("TDFE_APPLY_VARIANT", variant)
    n_orb = ORBS[p]
    cfg = _box(p, n_orb)
    ctx = gpu_context(cfg, n_orb=n_orb, k_max=4)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, n_orb, 400 + p)
    y = ctx.apply_H(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel(y, op.apply_Hbar(m, vq, x)) < 1e-12


@pytest.mark.parametrize("variant", ["pair", "plane"])
@pytest.mark.parametrize("p", sorted(ORBS))
def test_box_operator_fp32(p, variant, monkeypatch):
    monkeypatch.setenv("TDFE_APPLY_VARIANT", variant)
    n_orb = ORBS[p]
    cfg = _box(p, n_orb)
    ctx = gpu_context(cfg, n_orb=n_orb, k_max=4, precision=MIXED)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, n_orb, 500 + p)
    xg = torch.from_numpy(x).to(torch.complex64).cuda()
    y = torch.zeros_like(xg)
    ctx.apply_H_add_f32(xg, y)
    assert rel(y.cpu().numpy(), op.apply_Hbar(m, vq, x)) < 2e-6


@pytest.mark.parametrize("variant", ["pair", "plane"])
def test_box_lanczos_matches_oracle(variant, monkeypatch):
    monkeypatch.setenv("TDFE_APPLY_VARIANT", variant)
    cfg = W.scaled(W.CONFIGS[2], ncell=(4, 4, 4), p=5, n_orb=3)
    ctx = gpu_context(cfg, n_orb=3)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, 3, 9)
    x /= np.linalg.norm(x, axis=0)
    g = torch.from_numpy(x).cuda()
    ks, _ = ctx.lanczos_expm(g, 0.05, 1e-12)
    z, kref, _ = lanczos.lanczos_expm(lambda v: op.apply_Hbar(m, vq, v), x, 0.05, 1e-12)
    assert rel(g.cpu().numpy(), z) < 1e-10
    assert all(abs(a - b) <= 1 for a, b in zip(ks, kref))


def test_box_kernels_agree_on_full_size_benchmark_operator(monkeypatch):
    cfg = W.CONFIGS[2]
    m, vq = oracle_mesh(cfg)
    x = torch.from_numpy(W.random_block(m.n_dof, cfg.n_orb, 7)).cuda()
    y_default = gpu_context(cfg, k_max=4).apply_H(x).cpu().numpy()
    monkeypatch.setenv("TDFE_APPLY_VARIANT", "plane")
    y_plane = gpu_context(cfg, k_max=4).apply_H(x).cpu().numpy()
    assert rel(y_default, y_plane) < 1e-13
    assert rel(y_default, op.apply_Hbar(m, vq, x.cpu().numpy())) < 1e-12


ODD_N_ORBS = {2: 3, 4: 2, 6: 1, 8: 1}


@pytest.mark.parametrize("p", sorted(ODD_N_ORBS))
def test_box_kernels_at_odd_n_on_non_uniform_axes(p):
    """Rectilinear cells of unequal widths (the metric and the separable
    M^-1/2 factors differ per cell and per node line) at every odd n = p + 1,
    FP64 and FP32, against the oracle."""
    from paper_1810_13130_amd import tdfe
    n_orb = ODD_N_ORBS[p]
    cfg = _box(p, n_orb)
    axes = [cfg.lo + (cfg.hi - cfg.lo) * np.linspace(0.0, 1.0, n + 1) ** e for n, e in ((3, 1.3), (2, 0.8), (2, 1.0))]
    axes[2] = np.array([cfg.lo, cfg.lo + 0.3 * (cfg.hi - cfg.lo), cfg.hi])
    verts = tdfe.rectilinear_vertices(*axes)
    ncell = (3, 2, 2)
    from oracle.mesh import Mesh
    m = Mesh(p, ncell, verts, p + 1)
    vq = W.external_potential(cfg, m.quad_xyz)
    x = W.random_block(m.n_dof, n_orb, 600 + p)
    ref = op.apply_Hbar(m, vq, x)
    for prec in (0, MIXED):
        ctx = tdfe.Context(p, ncell, verts, n_orb_max=n_orb, k_max=4, precision=prec)
        xq = ctx.quad_coords().cpu().numpy()
        ctx.set_potential(torch.from_numpy(W.external_potential(cfg, xq).reshape(ctx.n_cell, -1)).cuda())
        if prec == 0:
            y = ctx.apply_H(torch.from_numpy(x).cuda()).cpu().numpy()
            assert rel(y, ref) < 1e-12
        else:
            xg = torch.from_numpy(x).to(torch.complex64).cuda()
            y = torch.zeros_like(xg)
            ctx.apply_H_add_f32(xg, y)
            assert rel(y.cpu().numpy(), ref) < 2e-6
        ctx.close()
