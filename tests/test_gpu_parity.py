"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Tolerance: 1e-10 relative for FP64 results (the FP64 target), tighter where
the operation is a fixed sequence of FP64 sums (operator apply, geometry:
1e-12).  Cases span several cells, an odd number of orbitals (ragged column
chunks), curved (trilinear) cells, and the full-size 16^3, p = 5, 8-orbital
operator of the benchmark workload.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_context, gpu_initial_state, oracle_mesh, rel
from oracle import lanczos, operators as op, scf
from oracle.magnus import State, System, magnus_step

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _cfg2_small(n_orb=3, nc=4, p=4):
    return W.scaled(W.CONFIGS[2], ncell=(nc, nc, nc), p=p, n_orb=n_orb)


def _cfg3_small(n_orb=3, nc=3, p=3):
    return W.scaled(W.CONFIGS[3], ncell=(nc, nc, nc), p=p, n_orb=n_orb)


@pytest.mark.parametrize("which", ["cfg1", "cfg2_small", "cfg3_small"])
def test_geometry_and_mass(which):
    cfg = {"cfg1": W.CONFIGS[1], "cfg2_small": _cfg2_small(), "cfg3_small": _cfg3_small()}[which]
    ctx = gpu_context(cfg, n_orb=1)
    m, _ = oracle_mesh(cfg)
    assert ctx.n_dof == m.n_dof and ctx.n_cell == m.n_cell
    assert rel(ctx.mass_diag().cpu().numpy(), m.M) < 1e-13
    assert np.abs(ctx.dof_coords().cpu().numpy() - m.dof_xyz).max() < 1e-12
    assert np.abs(ctx.quad_coords().cpu().numpy() - m.quad_xyz).max() < 1e-12


@pytest.mark.parametrize("which,n_orb", [("cfg1", 1), ("cfg2_small", 3), ("cfg2_small", 8), ("cfg3_small", 3),
                                         ("cfg3_small", 5)])
def test_apply_H_matches_oracle(which, n_orb):
    cfg = {"cfg1": W.CONFIGS[1], "cfg2_small": _cfg2_small(n_orb), "cfg3_small": _cfg3_small(n_orb)}[which]
    ctx = gpu_context(cfg, n_orb=n_orb)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, n_orb, 42)
    y = ctx.apply_H(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = op.apply_Hbar(m, vq, x)
    assert rel(y, ref) < 1e-12


def test_apply_H_full_size_benchmark_workload():
    cfg = W.CONFIGS[2]
    ctx = gpu_context(cfg)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, cfg.n_orb, 7)
    y = ctx.apply_H(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = op.apply_Hbar(m, vq, x)
    assert rel(y, ref) < 1e-12


def test_density_and_dipole_match_oracle():
    cfg = _cfg2_small(n_orb=3)
    ctx = gpu_context(cfg, n_orb=3)
    m, _ = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, 3, 5)
    rho = ctx.density(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = scf.density(m, x)
    assert rel(rho, ref) < 1e-12
    mu, ch = ctx.dipole(torch.from_numpy(x).cuda())
    assert abs(ch - scf.charge(m, ref)) < 1e-12 * abs(ch)
    assert np.abs(mu - scf.dipole(m, ref)).max() < 1e-12 * np.abs(mu).max()


# the last three: tau |T| large enough that the Chebyshev series of the small
# exponential runs past one 64-term register chunk (about 70, 100 and 150
# terms), converging at k = 42 and 63 (the in-update evaluation) and k = 102
# (the stop-test kernel's own evaluation beyond k = 64)
@pytest.mark.parametrize("which,n_orb,tau", [("cfg1", 1, 0.05), ("cfg2_small", 3, 0.05), ("cfg2_small", 3, -0.025),
                                             ("cfg3_small", 2, 0.05), ("cfg1", 1, 0.5), ("cfg1", 1, 1.0),
                                             ("cfg1", 2, -2.0)])
def test_lanczos_expm_matches_oracle(which, n_orb, tau):
    cfg = {"cfg1": W.CONFIGS[1], "cfg2_small": _cfg2_small(n_orb), "cfg3_small": _cfg3_small(n_orb)}[which]
    ctx = gpu_context(cfg, n_orb=n_orb)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, n_orb, 9)
    x /= np.linalg.norm(x, axis=0)
    g = torch.from_numpy(x).cuda()
    ks, errs = ctx.lanczos_expm(g, tau, 1e-12)
    z, kref, _ = lanczos.lanczos_expm(lambda v: op.apply_Hbar(m, vq, v), x, tau, 1e-12)
    assert rel(g.cpu().numpy(), z) < 1e-10
    assert all(abs(a - b) <= 1 for a, b in zip(ks, kref))
    assert max(errs) <= 1e-12


def test_lanczos_zero_orbital_and_ragged_block():
    cfg = _cfg2_small(n_orb=3)
    ctx = gpu_context(cfg, n_orb=3)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, 3, 1)
    x[:, 1] = 0.0
    g = torch.from_numpy(x).cuda()
    ks, _ = ctx.lanczos_expm(g, 0.05, 1e-12)
    out = g.cpu().numpy()
    assert ks[1] == 0 and np.abs(out[:, 1]).max() == 0.0
    z, _, _ = lanczos.lanczos_expm(lambda v: op.apply_Hbar(m, vq, v), x[:, [0, 2]], 0.05, 1e-12)
    assert rel(out[:, [0, 2]], z) < 1e-10


def test_lanczos_tau_zero_is_identity():
    cfg = _cfg2_small(n_orb=2, nc=3, p=3)
    ctx = gpu_context(cfg, n_orb=2)
    m, _ = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, 2, 3)
    g = torch.from_numpy(x).cuda()
    ks, errs = ctx.lanczos_expm(g, 0.0, 1e-12)
    assert ks == [1, 1] and max(errs) == 0.0
    assert rel(g.cpu().numpy(), x) < 1e-14


def test_lanczos_eigenvector_stops_at_k1():
    """A discrete eigenvector of Hbar: happy breakdown (or eps_1 below tol) at
    k = 1 and the exact phase exp(-i tau lambda)."""
    cfg = _cfg2_small(n_orb=1, nc=3, p=3)
    ctx = gpu_context(cfg, n_orb=1)
    m, vq = oracle_mesh(cfg)
    lam, U = np.linalg.eigh(op.dense_Hbar(m, vq))
    for idx in (0, 7):
        v = U[:, idx].astype(np.complex128)[:, None]
        g = torch.from_numpy(np.ascontiguousarray(v)).cuda()
        tau = 0.3
        ks, _ = ctx.lanczos_expm(g, tau, 1e-12)
        assert ks == [1]
        assert rel(g.cpu().numpy(), np.exp(-1j * tau * lam[idx]) * v) < 1e-11


@pytest.mark.slow
def test_graded_full_size_operator_matches_oracle():
    """Curved cells at the graded workload's full size (31^3 cells, p = 6,
    6,331,625 DoFs), two orbitals, every output compared with the oracle."""
    cfg = W.scaled(W.CONFIGS[3], n_orb=2)
    ctx = gpu_context(cfg, n_orb=2, k_max=4)
    m, vq = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, 2, 11)
    y = ctx.apply_H(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel(y, op.apply_Hbar(m, vq, x)) < 1e-12


def test_lanczos_not_converged_reports_enoconv():
    from paper_1810_13130_amd import tdfe
    cfg = W.CONFIGS[1]
    ctx = gpu_context(cfg, n_orb=1, k_max=3)
    x = gpu_initial_state(ctx, cfg)
    with pytest.raises(tdfe.TdfeError) as e:
        ctx.lanczos_expm(x, 0.5, 1e-14)
    assert e.value.status == tdfe.ENOCONV


@pytest.mark.parametrize("scf", [False, True])
def test_magnus_step_reports_enoconv(scf):
    """The step collects the Lanczos status at its end (one synchronisation):
    a Krylov cap too small for the tolerance is reported as ENOCONV, with and
    without the predictor-corrector SCF path, and a capped step leaves a
    finite state that the next normal step can continue from."""
    from paper_1810_13130_amd import tdfe
    cfg = _cfg2_small(n_orb=2)
    ctx = gpu_context(cfg, n_orb=2, k_max=3)
    if scf:
        Z, R = W.atoms(cfg)
        ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=2)
    g = gpu_initial_state(ctx, cfg)
    with pytest.raises(tdfe.TdfeError) as e:
        ctx.magnus_step(g, cfg.dt, 0.0, 1e-14)
    assert e.value.status == tdfe.ENOCONV
    assert torch.isfinite(torch.view_as_real(g)).all()


def test_magnus_step_capped_runs_match_across_chunkings(monkeypatch):
    """Krylov runs that end at k_max leave their convergence flag write for
    the next run to ignore: three one-orbital chunks per run (each stopping
    at k_max) must give exactly the state of one three-orbital chunk."""
    from paper_1810_13130_amd import tdfe
    cfg = _cfg2_small(n_orb=3)
    out = []
    for cap in (None, "1"):
        if cap:
            monkeypatch.setenv("TDFE_MAX_CHUNK_ORB", cap)
        ctx = gpu_context(cfg, n_orb=3, k_max=4)
        Z, R = W.atoms(cfg)
        ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=3)
        g = gpu_initial_state(ctx, cfg)
        for _ in range(2):
            with pytest.raises(tdfe.TdfeError) as e:
                ctx.magnus_step(g, cfg.dt, 0.0, 1e-14)
            assert e.value.status == tdfe.ENOCONV
        out.append(g.cpu().numpy())
    assert np.abs(out[0] - out[1]).max() <= 1e-12 * np.abs(out[0]).max()


def test_magnus_harmonic_trap_20_steps():
    cfg = W.CONFIGS[1]
    ctx = gpu_context(cfg, n_orb=1)
    g = gpu_initial_state(ctx, cfg)
    m, vq = oracle_mesh(cfg)
    sysm = System(m, vq, tol=1e-12)
    st = State(sysm, W.initial_psibar(cfg, m.dof_xyz, m.M))
    for n in range(cfg.steps):
        rep = ctx.magnus_step(g, cfg.dt, 0.0, 1e-12)
        ref = magnus_step(sysm, st, cfg.dt)
        assert np.abs(rep["mu"] - ref["dipole"]).max() < 1e-10
    assert rel(g.cpu().numpy(), st.psibar) < 1e-10
    assert abs(np.linalg.norm(g.cpu().numpy()) - 1.0) < 1e-10


@pytest.mark.parametrize("n_orb", [2, 3])
def test_magnus_scf_predictor_corrector_matches_oracle(n_orb):
    cfg = _cfg2_small(n_orb=n_orb)
    ctx = gpu_context(cfg, n_orb=n_orb)
    Z, R = W.atoms(cfg)
    ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=n_orb)
    g = gpu_initial_state(ctx, cfg)
    m, vq = oracle_mesh(cfg)
    sysm = System(m, vq, hartree=True, xc="x", Z=Z, R=R, tol=1e-12, pcg_tol=1e-14)
    st = State(sysm, W.initial_psibar(cfg, m.dof_xyz, m.M))
    for n in range(4):
        rep = ctx.magnus_step(g, cfg.dt, 0.0, 1e-12)
        ref = magnus_step(sysm, st, cfg.dt)
        assert np.abs(rep["mu"] - ref["dipole"]).max() < 1e-10 * np.abs(ref["dipole"]).max()
        assert abs(rep["charge"] - ref["charge"]) < 1e-10 * abs(ref["charge"])
    assert rel(g.cpu().numpy(), st.psibar) < 1e-10


@pytest.mark.parametrize("precond", ["fdm", "jacobi"])
@pytest.mark.parametrize("xc", ["x", "xc"])
def test_magnus_scf_on_graded_mesh_matches_oracle(xc, precond):
    """Curved (trilinear) cells: Hartree by the GPU's CG (preconditioned by the
    rectilinear stand-in's fast diagonalisation, or Jacobi as the oracle),
    exchange or exchange + PZ81 correlation, predictor-corrector steps."""
    from paper_1810_13130_amd import tdfe
    cfg = _cfg3_small(n_orb=3)
    ctx = gpu_context(cfg, n_orb=3)
    Z, R = W.atoms(cfg)
    ctx.set_scf(hartree=True, xc={"x": 1, "xc": 2}[xc], Z=Z, R=R, n_orb=3, pcg_tol=1e-14, pcg_maxit=5000,
                pcg_precond={"fdm": tdfe.PCG_FDM, "jacobi": tdfe.PCG_JACOBI}[precond])
    g = gpu_initial_state(ctx, cfg)
    m, vq = oracle_mesh(cfg)
    sysm = System(m, vq, hartree=True, xc=xc, Z=Z, R=R, tol=1e-12, pcg_tol=1e-14)
    st = State(sysm, W.initial_psibar(cfg, m.dof_xyz, m.M))
    for n in range(3):
        rep = ctx.magnus_step(g, cfg.dt, 0.0, 1e-12)
        ref = magnus_step(sysm, st, cfg.dt)
        assert rep["poisson_iters"] > 0
        assert np.abs(rep["mu"] - ref["dipole"]).max() < 1e-10 * np.abs(ref["dipole"]).max()
        assert abs(rep["charge"] - ref["charge"]) < 1e-10 * abs(ref["charge"])
    assert rel(g.cpu().numpy(), st.psibar) < 1e-10


@pytest.mark.parametrize("precond", ["fdm", "jacobi"])
def test_pcg_not_converging_is_reported(precond):
    from paper_1810_13130_amd import tdfe
    cfg = _cfg3_small(n_orb=2)
    ctx = gpu_context(cfg, n_orb=2)
    Z, R = W.atoms(cfg)
    ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=2, pcg_tol=1e-14, pcg_maxit=1,
                pcg_precond={"fdm": tdfe.PCG_FDM, "jacobi": tdfe.PCG_JACOBI}[precond])
    g = gpu_initial_state(ctx, cfg)
    with pytest.raises(tdfe.TdfeError) as e:
        ctx.magnus_step(g, cfg.dt, 0.0, 1e-12)
    assert e.value.status == tdfe.ENOCONV and "CG" in str(e.value)


def test_magnus_with_field_matches_oracle():
    cfg = _cfg2_small(n_orb=2)
    ctx = gpu_context(cfg, n_orb=2)
    Z, R = W.atoms(cfg)
    ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=2)
    g = gpu_initial_state(ctx, cfg)
    m, vq = oracle_mesh(cfg)
    sysm = System(m, vq, hartree=True, xc="x", Z=Z, R=R, tol=1e-12, pcg_tol=1e-14)
    st = State(sysm, W.initial_psibar(cfg, m.dof_xyz, m.M))
    E = W.field_amplitudes(3)
    for n in range(3):
        rep = ctx.magnus_step(g, cfg.dt, float(E[n]), 1e-12)
        ref = magnus_step(sysm, st, cfg.dt, E=float(E[n]))
        assert np.abs(rep["mu"] - ref["dipole"]).max() < 1e-10 * np.abs(ref["dipole"]).max()
    assert rel(g.cpu().numpy(), st.psibar) < 1e-10


def test_full_size_lanczos_samples_match_oracle():
    """The benchmark mesh (16^3 cells, p = 5) and launch configuration (all 8
    orbitals in one Krylov chunk, FP64 lane-pair operator, tau = dt): two of
    the eight propagated orbitals against the oracle's own Lanczos runs."""
    cfg = W.CONFIGS[2]
    ctx = gpu_context(cfg)
    g = gpu_initial_state(ctx, cfg)
    ks, errs = ctx.lanczos_expm(g, cfg.dt, cfg.tol)
    m, vq = oracle_mesh(cfg)
    x = W.initial_psibar(cfg, m.dof_xyz, m.M)
    cols = [0, 5]
    z, kref, _ = lanczos.lanczos_expm(lambda v: op.apply_Hbar(m, vq, v), x[:, cols], cfg.dt, cfg.tol)
    assert rel(g.cpu().numpy()[:, cols], z) < 1e-10
    assert all(abs(ks[c] - k) <= 1 for c, k in zip(cols, kref))
    assert max(errs) <= cfg.tol
    ctx.close()


def test_full_size_step_conserves_norm_and_charge():
    cfg = W.CONFIGS[2]
    ctx = gpu_context(cfg)
    Z, R = W.atoms(cfg)
    ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=cfg.n_orb)
    g = gpu_initial_state(ctx, cfg)
    n0 = torch.linalg.norm(g, dim=0).cpu().numpy()
    for _ in range(2):
        rep = ctx.magnus_step(g, cfg.dt, 0.0, 1e-10)
    n1 = torch.linalg.norm(g, dim=0).cpu().numpy()
    assert np.abs(n1 - n0).max() < 1e-9
    assert abs(rep["charge"] - cfg.n_orb) < 1e-6  # 8 electrons, discretisation of the GLL vs Gauss norm
    gram = (g.conj().T @ g).cpu().numpy()
    assert np.abs(gram - np.eye(cfg.n_orb)).max() < 1e-9
