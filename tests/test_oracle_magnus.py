"""Pins of the oracle's Magnus step (CPU only).

* Harmonic trap (Ehrenfest): a ground state kicked by exp(+i 0.1 z) has
  mu_z(t) = 0.1 sin t exactly in the continuum; the discrete dipole must
  approach it under mesh refinement.
* Time-independent H: norm and energy are conserved by exp(-i dt Hbar).
* Predictor-corrector: second-order temporal convergence of the dipole
  (the paper reports q = 1.96 and 1.98); a planted first-order variant of the
  midpoint Hamiltonian must fail the same check.
"""
import numpy as np
import pytest

import workloads as W
from oracle import operators as op
from oracle.lanczos import lanczos_expm
from oracle.magnus import State, System, magnus_step
from oracle.mesh import Mesh


def _cfg1_system(nc):
    cfg = W.scaled(W.CONFIGS[1], ncell=(nc, nc, nc))
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    vq = W.external_potential(cfg, m.quad_xyz)
    return cfg, m, vq, System(m, vq, tol=1e-10)


def test_ehrenfest_dipole_converges_and_invariants():
    errs = []
    for nc in (4, 6):
        cfg, m, vq, s = _cfg1_system(nc)
        psi0 = W.initial_psibar(cfg, m.dof_xyz, m.M)
        st = State(s, psi0)
        e0 = np.vdot(psi0[:, 0], op.apply_Hbar(m, vq, psi0[:, 0])).real
        err = 0.0
        for _ in range(cfg.steps):
            rep = magnus_step(s, st, cfg.dt)
            err = max(err, abs(rep["dipole"][2] - 0.1 * np.sin(st.t)))
        e1 = np.vdot(st.psibar[:, 0], op.apply_Hbar(m, vq, st.psibar[:, 0])).real
        assert abs(np.linalg.norm(st.psibar) - 1.0) < cfg.steps * cfg.tol
        assert abs(e1 - e0) < cfg.steps * cfg.tol * 100
        errs.append(err)
    assert errs[0] < 1e-2 and errs[1] < errs[0] / 5


def _temporal_errors(step_fn):
    cfg = W.scaled(W.CONFIGS[2], ncell=(4, 4, 4), p=4, n_orb=2)
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    Z, R = W.atoms(cfg)
    vq = W.external_potential(cfg, m.quad_xyz)
    psi0 = W.initial_psibar(cfg, m.dof_xyz, m.M) * np.exp(-0.05j * m.dof_xyz[:, 2])[:, None]
    T = 0.2
    out = {}
    for dt in (0.1, 0.05, 0.025, 0.025 / 8):
        s = System(m, vq, hartree=True, xc="x", Z=Z, R=R, tol=1e-13)
        st = State(s, psi0)
        for _ in range(int(round(T / dt))):
            mu = step_fn(s, st, dt)
        out[dt] = mu[2]
    ref = out[0.025 / 8]
    e = [abs(out[d] - ref) for d in (0.1, 0.05, 0.025)]
    return np.log2(e[0] / e[1]), np.log2(e[1] / e[2])


@pytest.mark.slow
def test_predictor_corrector_is_second_order():
    q1, q2 = _temporal_errors(lambda s, st, dt: magnus_step(s, st, dt)["dipole"])
    assert 1.85 < q1 < 2.15 and 1.85 < q2 < 2.15


def _planted_midpoint_from_previous_step(s, st, dt):
    """Planted mistake: the midpoint Hamiltonian is taken at t_{n-1} (no predictor)."""
    from oracle import scf
    new, _, _ = s.expm(s.vext + st.W1, st.psibar, dt)
    st.W2, st.W1 = st.W1, s.W(new)[0]
    st.psibar = new
    return scf.dipole(s.mesh, scf.density(s.mesh, new))


@pytest.mark.slow
def test_planted_first_order_midpoint_fails_the_order_check():
    q1, q2 = _temporal_errors(_planted_midpoint_from_previous_step)
    assert q2 < 1.5
