"""Mixed-precision path (FP32 operator and Krylov storage, FP64 recurrence
scalars, small exponential and master orbitals) against the FP64 oracle.

The bar is the dipole: relative error <= 1e-5 (max over the trajectory of
|mu_mixed - mu_ref| divided by max |mu_ref|); orbital errors are reported at
FP32 level (~1e-6 relative).
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_context, gpu_initial_state, oracle_mesh, rel
from oracle import lanczos, operators as op
from oracle.magnus import State, System, magnus_step

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
MIXED = 1


def _cfg2_small(n_orb=3, nc=4, p=4):
    return W.scaled(W.CONFIGS[2], ncell=(nc, nc, nc), p=p, n_orb=n_orb)


@pytest.mark.parametrize("which", ["box", "graded"])
def test_fp32_operator_matches_oracle(which):
    cfg = _cfg2_small(3) if which == "box" else W.scaled(W.CONFIGS[3], ncell=(3, 3, 3), p=3, n_orb=3)
    ctx = gpu_context(cfg, n_orb=3, precision=MIXED)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, 3, 42)
    xg = torch.from_numpy(x).to(torch.complex64).cuda()
    y = torch.zeros_like(xg)
    ctx.apply_H_add_f32(xg, y)
    ref = op.apply_Hbar(m, vq, x)
    assert rel(y.cpu().numpy(), ref) < 2e-6


def test_mixed_lanczos_matches_oracle():
    cfg = _cfg2_small(3)
    ctx = gpu_context(cfg, n_orb=3, precision=MIXED)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, 3, 9)
    x /= np.linalg.norm(x, axis=0)
    g = torch.from_numpy(x).cuda()
    ks, _ = ctx.lanczos_expm(g, 0.05, 1e-10)
    z, kref, _ = lanczos.lanczos_expm(lambda v: op.apply_Hbar(m, vq, v), x, 0.05, 1e-10)
    assert rel(g.cpu().numpy(), z) < 2e-6


def test_mixed_magnus_dipole_within_1e5():
    cfg = _cfg2_small(n_orb=3)
    ctx = gpu_context(cfg, n_orb=3, precision=MIXED)
    Z, R = W.atoms(cfg)
    ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=3)
    g = gpu_initial_state(ctx, cfg)
    m, vq = oracle_mesh(cfg)
    sysm = System(m, vq, hartree=True, xc="x", Z=Z, R=R, tol=1e-10, pcg_tol=1e-14)
    st = State(sysm, W.initial_psibar(cfg, m.dof_xyz, m.M))
    mu_g, mu_r = [], []
    for n in range(10):
        mu_g.append(ctx.magnus_step(g, cfg.dt, 0.0, 1e-10)["mu"])
        mu_r.append(magnus_step(sysm, st, cfg.dt)["dipole"])
    mu_g, mu_r = np.array(mu_g), np.array(mu_r)
    err = np.abs(mu_g - mu_r).max() / np.abs(mu_r).max()
    assert err < 1e-5, err
    assert rel(g.cpu().numpy(), st.psibar) < 1e-5
