"""Matrix-core variants of the box-cell operator (precisions FP64_MFMA,
FP32_MFMA, BF16_MFMA) against the oracle.

Bounds, from the arithmetic of each engine:
* FP64 products: the FP64 operator bar of every other parity test (1e-12);
* FP32 products: the mixed path's operator bar (2e-6, a few FP32 roundings
  through the seven sweeps);
* split BF16: a head and a remainder of 8 significand bits each keep about 16
  bits of every operand, and the dropped remainder x remainder term is
  2^-16 of a product: about 1.5e-5 per contraction, seven contractions deep
  on the longest path, so 1e-4 relative to the largest output.

Cases cover one column block exactly (8 orbitals = 16 real columns), fewer
columns than a block, several blocks with a ragged last one, every order the
variants support, and the early-exit flag path through the Lanczos loop.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_context, gpu_initial_state, oracle_mesh, rel
from oracle import lanczos, operators as op
from oracle.magnus import State, System, magnus_step

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_MFMA, BF16_MFMA, FP64_MFMA = 2, 3, 4
NAMES = {FP32_MFMA: "fp32", BF16_MFMA: "bf16x3", FP64_MFMA: "fp64"}
TOL = {FP64_MFMA: 1e-12, FP32_MFMA: 2e-6, BF16_MFMA: 1e-4}


def _cfg(p, nc, n_orb):
    return W.scaled(W.CONFIGS[2], ncell=(nc, nc, nc), p=p, n_orb=n_orb)


def _apply(ctx, prec, x):
    if prec == FP64_MFMA:
        return ctx.apply_H(torch.from_numpy(x).cuda()).cpu().numpy()
    xg = torch.from_numpy(x).to(torch.complex64).cuda()
    y = torch.zeros_like(xg)
    ctx.apply_H_add_f32(xg, y)
    return y.cpu().numpy()


@pytest.mark.parametrize("prec", [FP64_MFMA, FP32_MFMA, BF16_MFMA], ids=lambda v: NAMES[v])
@pytest.mark.parametrize("p,nc,n_orb", [(5, 4, 8), (5, 3, 11), (3, 5, 1), (6, 3, 3), (1, 4, 2), (2, 3, 5), (4, 3, 9),
                                        (7, 2, 2)])
def test_mfma_operator_matches_oracle(prec, p, nc, n_orb):
    if prec == FP64_MFMA and p > 6:
        pytest.skip("FP64 matrix-core variant: p <= 6")
    cfg = _cfg(p, nc, n_orb)
    print(f"[mfma-apply] {NAMES[prec]} p={p} {nc}^3 cells {n_orb} orbitals", flush=True)
    ctx = gpu_context(cfg, n_orb=n_orb, precision=prec)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, n_orb, 40 + n_orb)
    err = rel(_apply(ctx, prec, x), op.apply_Hbar(m, vq, x))
    print(f"[mfma-apply] relative error {err:.3e}", flush=True)
    assert err < TOL[prec]
    ctx.close()


@pytest.mark.parametrize("prec", [FP64_MFMA, FP32_MFMA], ids=lambda v: NAMES[v])
def test_mfma_lanczos_matches_oracle(prec):
    cfg = _cfg(4, 4, 3)
    ctx = gpu_context(cfg, n_orb=3, precision=prec)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, 3, 9)
    x /= np.linalg.norm(x, axis=0)
    g = torch.from_numpy(x).cuda()
    ks, _ = ctx.lanczos_expm(g, 0.05, 1e-10)
    z, kref, _ = lanczos.lanczos_expm(lambda v: op.apply_Hbar(m, vq, v), x, 0.05, 1e-10)
    print(f"[mfma-lanczos] {NAMES[prec]} k {list(ks)} vs {list(kref)}", flush=True)
    err = rel(g.cpu().numpy(), z)
    assert err < (1e-10 if prec == FP64_MFMA else 2e-6), err
    if prec == FP64_MFMA:
        assert np.abs(np.array(ks) - np.array(kref)).max() <= 1
    ctx.close()


@pytest.mark.parametrize("prec", [FP64_MFMA, FP32_MFMA], ids=lambda v: NAMES[v])
def test_mfma_magnus_steps_match_oracle(prec):
    cfg = _cfg(4, 4, 3)
    ctx = gpu_context(cfg, n_orb=3, precision=prec)
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
    print(f"[mfma-magnus] {NAMES[prec]} dipole error {err:.3e}", flush=True)
    # FP64: the FP64 Magnus bar; FP32: the mixed path's dipole bar
    assert err < (1e-10 if prec == FP64_MFMA else 1e-5), err
    ctx.close()


def test_bf16_split_magnus_dipole_error_is_reported():
    """The split-BF16 engine in a full step: the dipole error against the
    oracle is printed for the record; the run must stay finite, keep the
    charge and the orbitals' norms (the propagator stays unitary whatever
    the operator's rounding: the Lanczos exponential of a symmetric matrix)."""
    cfg = _cfg(4, 4, 3)
    ctx = gpu_context(cfg, n_orb=3, precision=BF16_MFMA)
    Z, R = W.atoms(cfg)
    ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=3)
    g = gpu_initial_state(ctx, cfg)
    m, vq = oracle_mesh(cfg)
    sysm = System(m, vq, hartree=True, xc="x", Z=Z, R=R, tol=1e-10, pcg_tol=1e-14)
    st = State(sysm, W.initial_psibar(cfg, m.dof_xyz, m.M))
    mu_g, mu_r = [], []
    for n in range(10):
        rep = ctx.magnus_step(g, cfg.dt, 0.0, 1e-10)
        ref = magnus_step(sysm, st, cfg.dt)
        mu_g.append(rep["mu"])
        mu_r.append(ref["dipole"])
        assert abs(rep["charge"] - ref["charge"]) < 1e-5 * abs(ref["charge"])
    mu_g, mu_r = np.array(mu_g), np.array(mu_r)
    err = np.abs(mu_g - mu_r).max() / np.abs(mu_r).max()
    print(f"[mfma-magnus] bf16x3 dipole error {err:.3e}", flush=True)
    assert np.isfinite(err)
    G = g.cpu().numpy().conj().T @ g.cpu().numpy()
    assert np.abs(G - np.eye(3)).max() < 1e-5
    ctx.close()


def test_mfma_operators_at_the_benchmark_workload():
    """The launch the engine benchmark times: 16^3 box cells, p = 5, 8 orbitals
    (493,039 DoFs), every engine against one oracle application."""
    cfg = W.CONFIGS[2]
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, cfg.n_orb, 7)
    ref = op.apply_Hbar(m, vq, x)
    for prec in (FP64_MFMA, FP32_MFMA, BF16_MFMA):
        ctx = gpu_context(cfg, precision=prec)
        err = rel(_apply(ctx, prec, x), ref)
        print(f"[mfma-full] {NAMES[prec]} relative error {err:.3e}", flush=True)
        assert err < TOL[prec]
        ctx.close()
