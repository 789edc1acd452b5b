"""Soft-capped Krylov chunks (wider chunks in the basis memory of narrower
ones, Eq. AdaptiveLanczos's per-orbital dimension unchanged) against the
oracle and against runs in plain chunks.

The basis memory is capped at one orbital (TDFE_BASIS_CHUNK_ORB=1, as on a
device that holds one orbital's basis at k_max = 100); four orbitals then
run in chunks of two with a cap of (100 + 1) / 2 - 1 = 49 vectors once an
exponential has shown its Krylov dimension.  On this mesh (4^3 box cells,
p = 4) the oracle needs k = 9 at tau = 0.05 and k = 56 at tau = 6: the
second exceeds the cap, so the chunk restarts at k_max.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_context, oracle_mesh, rel
from oracle import lanczos, operators as op

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K_MAX = 100


def _cfg():
    return W.scaled(W.CONFIGS[2], ncell=(4, 4, 4), p=4, n_orb=4)


def _block(m, seed=9):
    x = W.random_block(m.n_dof, 4, seed)
    return x / np.linalg.norm(x, axis=0)


# FP64: tolerance 1e-12 (k = 9, then 56 at tau = 6), against the oracle.
# Mixed: the FP32 basis stops at its floor 16 2^-24 (the oracle needs k = 5
# at that tolerance, and 66 at tau = 10); tau = 0.05 is compared with the
# oracle at the mixed path's 2e-6.  At tau = 10 each of the k iterations
# stores a basis vector rounded to FP32 and may stop at the floor, so the
# bar is k 16 2^-24 (6e-5 at k = 66) against the oracle and against the same
# exponential in a context of plain one-orbital chunks (the launches the
# restart runs; there only the order of the atomic additions differs)
@pytest.mark.parametrize("mixed", [False, True])
def test_soft_chunk_widens_after_first_exponential_and_restarts_past_cap(monkeypatch, mixed):
    from paper_1810_13130_amd import tdfe
    monkeypatch.setenv("TDFE_BASIS_CHUNK_ORB", "1")
    cfg = _cfg()
    ctx = gpu_context(cfg, n_orb=4, k_max=K_MAX, precision=tdfe.MIXED_FP32 if mixed else tdfe.FP64)
    m, vq = oracle_mesh(cfg)
    x = _block(m)
    tol, bar, tau_big = (1e-10, 2e-6, 10.0) if mixed else (1e-12, 1e-10, 6.0)
    ref = lambda tau: lanczos.lanczos_expm(lambda v: op.apply_Hbar(m, vq, v), x, tau, tol)
    assert ctx.krylov_chunk(4) == 1
    assert ctx.krylov_soft_chunk(4) == (1, K_MAX)  # no exponential yet
    # 1: plain one-orbital chunks
    g = torch.from_numpy(x).cuda()
    ks, _ = ctx.lanczos_expm(g, 0.05, tol)
    z, kref, _ = ref(0.05)
    assert rel(g.cpu().numpy(), z) < bar and max(ks) <= 16
    if not mixed:
        assert max(ks) == max(kref) == 9
    # 2: two-orbital chunks capped at 49 (at least 32 and twice k)
    assert ctx.krylov_soft_chunk(4) == (2, 49)
    g = torch.from_numpy(x).cuda()
    ks2, errs = ctx.lanczos_expm(g, 0.05, tol)
    assert rel(g.cpu().numpy(), z) < bar and all(abs(a - b) <= 1 for a, b in zip(ks2, ks))
    if not mixed:
        assert all(abs(a - b) <= 1 for a, b in zip(ks2, kref)) and max(errs) <= 1e-12
    # 3: k beyond the cap of 49: every chunk restarts at k_max, same result
    g = torch.from_numpy(x).cuda()
    ks, errs = ctx.lanczos_expm(g, tau_big, tol)
    assert min(ks) > 49
    zb, krefb, _ = ref(tau_big)
    bar_big = max(ks) * 16 * 2.0**-24 if mixed else bar
    assert rel(g.cpu().numpy(), zb) < bar_big
    if not mixed:
        assert all(abs(a - b) <= 1 for a, b in zip(ks, krefb)) and max(errs) <= 1e-12
    # twice that k is more than k_max: back to one-orbital chunks
    assert ctx.krylov_soft_chunk(4) == (1, K_MAX)
    ctx.close()
    if mixed:
        monkeypatch.setenv("TDFE_MAX_CHUNK_ORB", "1")
        plain = gpu_context(cfg, n_orb=4, k_max=K_MAX, precision=tdfe.MIXED_FP32)
        gp = torch.from_numpy(x).cuda()
        ksp, _ = plain.lanczos_expm(gp, tau_big, tol)
        assert plain.krylov_soft_chunk(4) == (1, K_MAX)
        assert all(abs(a - b) <= 1 for a, b in zip(ks, ksp))
        assert rel(g.cpu().numpy(), gp.cpu().numpy()) < bar_big
        plain.close()


@pytest.mark.parametrize("steps,warm", [(1, True), (3, True), (3, False)])
def test_soft_chunk_magnus_and_propagate_match_plain_chunks(monkeypatch, steps, warm):
    """magnus_step and propagate (both keep the Lanczos results on the
    device until the step ends) with soft-capped chunks against the same
    steps in one chunk.  warm: a short exponential first, so that the steps
    widen at once, and each restarts (tau = dt = 6, k = 56 > 49); cold: the
    first exponential of the context reads its Krylov dimensions back (k = 9
    at dt = 0.05) and the next steps run two-orbital chunks capped at 49."""
    cfg = _cfg()
    m, _ = oracle_mesh(cfg)
    x = _block(m, seed=21)
    dt = 6.0 if warm else 0.05
    out = []
    for basis in ("1", None):
        if basis:
            monkeypatch.setenv("TDFE_BASIS_CHUNK_ORB", basis)
        else:
            monkeypatch.delenv("TDFE_BASIS_CHUNK_ORB", raising=False)
        ctx = gpu_context(cfg, n_orb=4, k_max=K_MAX)
        if warm:
            w = torch.from_numpy(x).cuda()
            ctx.lanczos_expm(w, 0.01, 1e-12)
            if basis:
                assert ctx.krylov_soft_chunk(4)[0] > 1
        g = torch.from_numpy(x).cuda()
        if steps == 1:
            rep = ctx.magnus_step(g, dt, 0.0, 1e-12)
            mu = np.asarray(rep["mu"])
        else:
            rec, _ = ctx.propagate(g, steps, dt, tol=1e-12)
            mu = rec.cpu().numpy() if hasattr(rec, "cpu") else np.asarray(rec)
        if basis and not warm:
            assert ctx.krylov_soft_chunk(4) == (2, 49)
        out.append((g.cpu().numpy(), mu))
        ctx.close()
    (g1, mu1), (g2, mu2) = out
    assert rel(g1, g2) < 1e-12
    assert np.abs(mu1 - mu2).max() <= 1e-12 * max(1.0, np.abs(mu2).max())
