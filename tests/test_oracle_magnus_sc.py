"""Pins of the oracle's fully self-consistent midpoint step (steps i-iv of
the section on the second-order Magnus propagator) and of the higher-order
extrapolation (CPU only).

* The extrapolation weights reproduce polynomials of their order exactly.
* Without density-dependent terms the step is one exponential, as in the
  predictor-corrector step.
* A converged step is a fixed point of the implicit midpoint rule:
  propagating psibar^{n-1} with (W_{n-1} + W[rho(psibar^n)])/2 returns psibar^n.
* The converged result does not depend on the initial extrapolation.
* Second-order temporal convergence of the dipole; a planted endpoint rule
  (midpoint W replaced by W_n) must fail the same check.
"""
import numpy as np
import pytest

import workloads as W
from oracle import scf
from oracle.magnus import State, System, extrapolation_weights, magnus_step, magnus_step_sc
from oracle.mesh import Mesh


def test_extrapolation_weights_are_exact_for_their_order():
    rng = np.random.default_rng(3)
    for order in (1, 2):
        for s in (0.25, 0.5, 1.0, -0.3):
            c = rng.normal(size=order + 1)
            poly = lambda x: sum(ck * x ** k for k, ck in enumerate(c))
            w = extrapolation_weights(s, order)
            assert abs(sum(wk * poly(-k) for k, wk in enumerate(w)) - poly(s)) < 1e-13
    assert extrapolation_weights(0.25, 1) == [1.25, -0.25]


def _small_scf(n_orb=2):
    cfg = W.scaled(W.CONFIGS[2], ncell=(3, 3, 3), p=3, n_orb=n_orb)
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    Z, R = W.atoms(cfg)
    vq = W.external_potential(cfg, m.quad_xyz)
    return cfg, m, Z, R, vq


def test_without_scf_terms_the_step_is_one_exponential():
    cfg = W.CONFIGS[1]
    m = Mesh(cfg.p, cfg.ncell, W.vertices(cfg), cfg.nq)
    vq = W.external_potential(cfg, m.quad_xyz)
    s = System(m, vq, tol=1e-12)
    a, b = State(s, W.initial_psibar(cfg, m.dof_xyz, m.M)), State(s, W.initial_psibar(cfg, m.dof_xyz, m.M))
    ra = magnus_step(s, a, 0.05, 0.01)
    rb = magnus_step_sc(s, b, 0.05, 0.01)
    assert np.array_equal(a.psibar, b.psibar) and rb["sc_iters"] == 1


def test_converged_step_is_a_fixed_point_of_the_midpoint_rule():
    cfg, m, Z, R, vq = _small_scf()
    s = System(m, vq, hartree=True, xc="x", Z=Z, R=R, tol=1e-13, pcg_tol=1e-14)
    st = State(s, W.initial_psibar(cfg, m.dof_xyz, m.M))
    for _ in range(2):
        magnus_step(s, st, cfg.dt)
    w_prev, psi_prev = st.W1.copy(), st.psibar.copy()
    rep = magnus_step_sc(s, st, cfg.dt, sc_tol=1e-12)
    assert rep["converged"] and rep["sc_iters"] > 1
    wn, _ = s.W(st.psibar)
    again, _, _ = s.expm(s.vext + 0.5 * (w_prev + wn), psi_prev, cfg.dt)
    assert np.abs(again - st.psibar).max() < 1e-10 * np.abs(st.psibar).max()


def test_converged_result_does_not_depend_on_the_extrapolation():
    cfg, m, Z, R, vq = _small_scf()
    out = []
    for order in (1, 2):
        s = System(m, vq, hartree=True, xc="x", Z=Z, R=R, tol=1e-13, pcg_tol=1e-14)
        st = State(s, W.initial_psibar(cfg, m.dof_xyz, m.M))
        its = []
        for _ in range(3):
            its.append(magnus_step_sc(s, st, cfg.dt, order=order, sc_tol=1e-12)["sc_iters"])
        out.append(st.psibar)
    assert np.abs(out[0] - out[1]).max() < 1e-10 * np.abs(out[0]).max()


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
def test_self_consistent_midpoint_is_second_order():
    q1, q2 = _temporal_errors(lambda s, st, dt: magnus_step_sc(s, st, dt, sc_tol=1e-11)["dipole"])
    assert 1.85 < q1 < 2.15 and 1.85 < q2 < 2.15


def _planted_endpoint_rule(s, st, dt):
    """Planted mistake: step (iii) takes W_n instead of the midpoint value."""
    wmid = st.W1
    for _ in range(50):
        new, _, _ = s.expm(s.vext + wmid, st.psibar, dt)
        wn, rho = s.W(new)
        change = np.max(np.abs(wn - wmid))
        wmid = wn
        if change <= 1e-11:
            break
    st.W3, st.W2, st.W1 = st.W2, st.W1, wn
    st.psibar = new
    return scf.dipole(s.mesh, rho)


@pytest.mark.slow
def test_planted_endpoint_rule_fails_the_order_check():
    q1, q2 = _temporal_errors(_planted_endpoint_rule)
    assert q2 < 1.5
