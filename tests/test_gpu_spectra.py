"""GPU parity of the excitations and spectra against the CPU oracle
(oracle.spectra, pinned by test_oracle_spectra).

* the delta kick along a general direction, element by element (1e-14);
* Magnus steps under a field along x and along a general direction, with and
  without SCF terms (dipole 1e-10 relative, orbitals 1e-10);
* the absorption and power spectrum kernels on analytic and seeded series
  (1e-12 relative), kick and field-sample forms;
* end to end: the harmonic trap kicked along x, y and z on the GPU, its
  absorption spectrum against the oracle's run and spectrum;
* the field gradient with a field direction other than z against central
  differences of the GPU forward map.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_context, gpu_initial_state, oracle_mesh, rel
from oracle import scf, spectra as sp
from oracle.magnus import State, System, magnus_step

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

D = np.array([0.48, -0.6, 0.64])


def _cfg2_small(n_orb=3, nc=4, p=4):
    return W.scaled(W.CONFIGS[2], ncell=(nc, nc, nc), p=p, n_orb=n_orb)


def test_kick_matches_oracle():
    cfg = _cfg2_small()
    ctx = gpu_context(cfg, n_orb=3, k_max=8)
    m, _ = oracle_mesh(cfg)
    x = W.random_block(m.n_dof, 3, 4)
    g = torch.from_numpy(x).cuda()
    ctx.set_field_direction(D)
    ctx.kick(g, 0.37)
    assert rel(g.cpu().numpy(), sp.kick(x, m.dof_xyz, 0.37, D)) < 1e-14


@pytest.mark.parametrize("d", [(1.0, 0.0, 0.0), tuple(D)])
def test_magnus_with_field_direction_matches_oracle(d):
    cfg = W.CONFIGS[1]
    ctx = gpu_context(cfg, n_orb=1)
    ctx.set_field_direction(d)
    g = gpu_initial_state(ctx, cfg)
    m, vq = oracle_mesh(cfg)
    sysm = System(m, vq, tol=1e-12)
    st = State(sysm, W.initial_psibar(cfg, m.dof_xyz, m.M))
    for n in range(5):
        E = 0.02 * (n + 1)
        rep = ctx.magnus_step(g, cfg.dt, E, 1e-12)
        ref = magnus_step(sysm, st, cfg.dt, E, direction=d)
        assert np.abs(rep["mu"] - ref["dipole"]).max() < 1e-10 * np.abs(ref["dipole"]).max()
    assert rel(g.cpu().numpy(), st.psibar) < 1e-10


def test_scf_magnus_with_field_direction_matches_oracle():
    cfg = _cfg2_small(n_orb=2)
    ctx = gpu_context(cfg, n_orb=2)
    Z, R = W.atoms(cfg)
    ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=2)
    ctx.set_field_direction(D)
    g = gpu_initial_state(ctx, cfg)
    m, vq = oracle_mesh(cfg)
    sysm = System(m, vq, hartree=True, xc="x", Z=Z, R=R, tol=1e-12, pcg_tol=1e-14)
    st = State(sysm, W.initial_psibar(cfg, m.dof_xyz, m.M))
    for E in (0.01, -0.02, 0.005):
        rep = ctx.magnus_step(g, cfg.dt, E, 1e-12)
        ref = magnus_step(sysm, st, cfg.dt, E, direction=D)
        assert np.abs(rep["mu"] - ref["dipole"]).max() < 1e-10 * np.abs(ref["dipole"]).max()
    assert rel(g.cpu().numpy(), st.psibar) < 1e-10


def test_spectrum_kernels_match_oracle():
    from paper_1810_13130_amd import tdfe
    rng = np.random.default_rng(12)
    dt, n_t = 0.02, 3001
    t = dt * np.arange(n_t)
    mu = np.stack([1e-3 * np.sin(0.7 * t) * np.exp(-0.01 * t), 2e-3 * np.sin(1.3 * t),
                   1e-4 * rng.normal(size=n_t)]) + np.array([[0.5], [-0.1], [0.2]])
    field = np.stack([sp.field_gaussian(t, 2e-5, 3.0, 0.2)] * 2 + [sp.field_gaussian(t, -1e-5, 2.0, 0.3)])
    w = np.linspace(0.01, 4.0, 64)
    mu_d, w_d = torch.from_numpy(mu).cuda(), torch.from_numpy(w).cuda()
    S_kick = tdfe.absorption_spectrum(mu_d, dt, w_d, 0.005, kappa=1e-3).cpu().numpy()
    ref = sp.absorption_spectrum(mu, dt, w, 0.005, kappa=1e-3)
    assert rel(S_kick, ref) < 1e-12
    S_field = tdfe.absorption_spectrum(mu_d, dt, w_d, 0.005, field=torch.from_numpy(field).cuda()).cpu().numpy()
    ref = sp.absorption_spectrum(mu, dt, w, 0.005, field=field)
    assert rel(S_field, ref) < 1e-12
    P = tdfe.power_spectrum(mu_d[1].contiguous(), dt, w_d).cpu().numpy()
    assert rel(P, sp.power_spectrum(mu[1], dt, w)) < 1e-12
    # degenerate sizes: the smallest series each accepts
    P3 = tdfe.power_spectrum(mu_d[0, :3].contiguous(), dt, w_d).cpu().numpy()
    assert rel(P3, sp.power_spectrum(mu[0, :3], dt, w)) < 1e-12
    S2 = tdfe.absorption_spectrum(mu_d[:, :2].contiguous(), dt, w_d, 0.0, kappa=1e-3).cpu().numpy()
    assert rel(S2, sp.absorption_spectrum(mu[:, :2], dt, w, 0.0, kappa=1e-3)) < 1e-12


def test_kicked_trap_spectrum_end_to_end():
    """Harmonic trap, one orbital: kick along each axis, 63 steps of 0.1,
    absorption spectrum on the GPU; the oracle runs the same pipeline."""
    from paper_1810_13130_amd import tdfe
    cfg = W.CONFIGS[1]
    kappa, dt, nsteps = 1e-2, 0.1, 63
    ctx = gpu_context(cfg, n_orb=1)
    m, vq = oracle_mesh(cfg)
    psi0 = np.abs(W.initial_psibar(cfg, m.dof_xyz, m.M)).astype(np.complex128)
    psi0_gpu = np.abs(gpu_initial_state(ctx, cfg).cpu().numpy()).astype(np.complex128)
    mus_g, mus_r = [], []
    for a in range(3):
        e = np.eye(3)[a]
        ctx.set_field_direction(e)
        g = torch.from_numpy(np.ascontiguousarray(psi0_gpu)).cuda()
        mu0 = ctx.dipole(g)[0][a]
        ctx.kick(g, kappa)
        series = [ctx.dipole(g)[0][a] - mu0]
        for _ in range(nsteps):
            series.append(ctx.magnus_step(g, dt, 0.0, 1e-12)["mu"][a] - mu0)
        mus_g.append(series)
        sysm = System(m, vq, tol=1e-12)
        st = State(sysm, sp.kick(psi0, m.dof_xyz, kappa, e))
        r0 = scf.dipole(m, scf.density(m, psi0))[a]
        rs = [scf.dipole(m, scf.density(m, st.psibar))[a] - r0]
        for _ in range(nsteps):
            rs.append(magnus_step(sysm, st, dt)["dipole"][a] - r0)
        mus_r.append(rs)
    mus_g, mus_r = np.array(mus_g), np.array(mus_r)
    assert np.abs(mus_g - mus_r).max() < 1e-10 * kappa
    w = np.linspace(0.2, 2.0, 91)
    S = tdfe.absorption_spectrum(torch.from_numpy(mus_g).cuda(), dt, torch.from_numpy(w).cuda(), 0.0,
                                 kappa=kappa).cpu().numpy()
    S_ref = sp.absorption_spectrum(mus_r, dt, w, 0.0, kappa=kappa)
    assert rel(S, S_ref) < 1e-8
    assert abs(w[np.argmax(S)] - 1.0) < 0.05


def test_gradient_with_field_direction_against_finite_differences():
    cfg = W.scaled(W.CONFIGS[5], ncell=(3, 3, 3), p=3, n_orb=2)
    ctx = gpu_context(cfg)
    Z, R = W.atoms(cfg)
    ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=2)
    ctx.set_field_direction((0.6, 0.0, 0.8))
    psi = gpu_initial_state(ctx, cfg)
    E = W.field_amplitudes(4) * 50.0
    L, g = ctx.dipole_gradient(psi, E, cfg.dt, tol=1e-13, k_store=64)

    def forward(Ev):
        x = psi.clone()
        ctx.set_scf(hartree=True, xc=1, Z=Z, R=R, n_orb=2)  # reset the history
        for e in Ev:
            ctx.magnus_step(x, cfg.dt, float(e), 1e-13, report=False)
        return ctx.dipole(x)[0][2]

    assert abs(forward(E) - L) <= 1e-10 * max(abs(L), 1e-3)
    h = 1e-3
    for k in range(4):
        ep, em = E.copy(), E.copy()
        ep[k] += h
        em[k] -= h
        fd = (forward(ep) - forward(em)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-5 * np.abs(g).max()
    ctx.close()
