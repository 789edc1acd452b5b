"""GPU parity of the operator on trilinear (curved) cells, every supported order.

The curved-cell operator has three kernels for two or more real columns at
orders p <= 7 -- lane pairs sharing a plane (the FP64 default), plane
ownership (the FP32 default) -- and the line-ownership kernel (one column,
p = 8, or on request).  Each order is checked in both of the first two
kernels against the FP64 oracle on a small graded mesh with an uneven cell
count per axis and an orbital count that selects a different column-block
width (ragged column chunks included), in FP64 (1e-12) and in FP32 storage
(2e-6, 1e-5 at p >= 7); the kernels are compared with each other; and one
predictor-corrector SCF step at p = 6 runs the one-column stiffness products
(full node grid, no M^-1/2) of the CG Hartree solve.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_context, gpu_initial_state, oracle_mesh, rel
from oracle import operators as op
from oracle.magnus import State, System, magnus_step

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
MIXED = 1

# order -> orbitals (2 real columns each): column blocks of 2, 4, 8 and 16,
# and 18 columns = one full block of 16 plus a ragged block
ORBS = {1: 1, 2: 2, 3: 3, 4: 5, 5: 9, 6: 3, 7: 2, 8: 1}


def _graded(p, n_orb, ncell=(2, 3, 2)):
    return W.scaled(W.CONFIGS[3], ncell=ncell, p=p, n_orb=n_orb)


@pytest.mark.parametrize("variant", ["pair", "plane"])
@pytest.mark.parametrize("p", sorted(ORBS))
def test_curved_operator_fp64_every_order(p, variant, monkeypatch):
    monkeypatch.setenv("TDFE_APPLY_VARIANT", variant)
    n_orb = ORBS[p]
    cfg = _graded(p, n_orb)
    ctx = gpu_context(cfg, n_orb=n_orb, k_max=4)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, n_orb, 100 + p)
    y = ctx.apply_H(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel(y, op.apply_Hbar(m, vq, x)) < 1e-12


@pytest.mark.parametrize("variant", ["pair", "plane"])
@pytest.mark.parametrize("p", sorted(ORBS))
def test_curved_operator_fp32_every_order(p, variant, monkeypatch):
    monkeypatch.setenv("TDFE_APPLY_VARIANT", variant)
    n_orb = ORBS[p]
    cfg = _graded(p, n_orb)
    ctx = gpu_context(cfg, n_orb=n_orb, k_max=4, precision=MIXED)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, n_orb, 200 + p)
    xg = torch.from_numpy(x).to(torch.complex64).cuda()
    y = torch.zeros_like(xg)
    ctx.apply_H_add_f32(xg, y)
    assert rel(y.cpu().numpy(), op.apply_Hbar(m, vq, x)) < (1e-5 if p >= 7 else 2e-6)


@pytest.mark.parametrize("p", [3, 6])
def test_pair_plane_and_line_kernels_agree_on_curved_cells(p, monkeypatch):
    cfg = _graded(p, 5)
    x = torch.from_numpy(W.random_block(_n_dof(cfg), 5, 300 + p)).cuda()
    monkeypatch.setenv("TDFE_APPLY_VARIANT", "plane")
    y_plane = gpu_context(cfg, n_orb=5, k_max=4).apply_H(x).cpu().numpy()
    monkeypatch.setenv("TDFE_APPLY_VARIANT", "pair")
    y_pair = gpu_context(cfg, n_orb=5, k_max=4).apply_H(x).cpu().numpy()
    monkeypatch.setenv("TDFE_APPLY_VARIANT", "line")
    y_line = gpu_context(cfg, n_orb=5, k_max=4).apply_H(x).cpu().numpy()
    assert rel(y_plane, y_line) < 1e-13
    assert rel(y_pair, y_line) < 1e-13


def _n_dof(cfg):
    nx, ny, nz = cfg.ncell
    return (nx * cfg.p - 1) * (ny * cfg.p - 1) * (nz * cfg.p - 1)


def test_scf_step_on_curved_cells_at_p6_matches_oracle():
    cfg = W.scaled(W.CONFIGS[3], ncell=(2, 2, 2), p=6, n_orb=2)
    ctx = gpu_context(cfg, n_orb=2)
    Z, R = W.atoms(cfg)
    ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=2, pcg_tol=1e-14, pcg_maxit=5000)
    g = gpu_initial_state(ctx, cfg)
    m, vq = oracle_mesh(cfg)
    sysm = System(m, vq, hartree=True, xc="x", Z=Z, R=R, tol=1e-12, pcg_tol=1e-14)
    st = State(sysm, W.initial_psibar(cfg, m.dof_xyz, m.M))
    rep = ctx.magnus_step(g, cfg.dt, 0.0, 1e-12)
    ref = magnus_step(sysm, st, cfg.dt)
    assert rep["poisson_iters"] > 0
    assert np.abs(rep["mu"] - ref["dipole"]).max() < 1e-10 * np.abs(ref["dipole"]).max()
    assert abs(rep["charge"] - ref["charge"]) < 1e-10 * abs(ref["charge"])
    assert rel(g.cpu().numpy(), st.psibar) < 1e-10


def test_pair_and_plane_agree_at_the_graded_launch_shape(monkeypatch):
    """The graded molecule's full mesh (31^3 cells, p = 6) at the FP64 step's
    launch shape (a Krylov chunk of 8 orbitals = 16 real columns): the
    lane-pair and the plane kernel agree to rounding."""
    cfg = W.scaled(W.CONFIGS[3], n_orb=8)
    x = None
    out = {}
    for variant in ("pair", "plane"):
        monkeypatch.setenv("TDFE_APPLY_VARIANT", variant)
        ctx = gpu_context(cfg, n_orb=8, k_max=4)
        if x is None:
            x = torch.from_numpy(W.random_block(ctx.n_dof, 8, 77)).cuda()
        out[variant] = ctx.apply_H(x).cpu().numpy()
        ctx.close()
    assert rel(out["pair"], out["plane"]) < 1e-13
