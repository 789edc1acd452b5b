"""Second-order Magnus step with the predictor-corrector midpoint (oracle).

Eqs. ApproxMagnus / PsiTimeDiscrete: psibar^n = exp(-i dt Hbar[rho(t_{n-1} +
dt/2)]) psibar^{n-1}.  The midpoint Hamiltonian follows the predictor-
corrector of Sec. "Approximating the second-order Magnus operator":
predict Hbar at t_{n-1} + dt/4 by extrapolation from earlier instants,
propagate psibar^{n-1} over dt/2, and evaluate Hbar at t_{n-1} + dt/2 from the
density of that half-step state.

Readings (the paper defers the details to another reference):
* only the density-dependent part W = V_H + V_xc is extrapolated, linearly
  from the integer instants: W(t_{n-1} + dt/4) ~ 1.25 W_{n-1} - 0.25 W_{n-2};
  the first step uses W_{-1} := W_0;
* the external and field potentials are evaluated exactly; a field of
  amplitude E_n along z is V_field = -E_n z (Eq. VField) held over step n
  (along a direction d: -E_n (d . r));
* the corrector restarts from psibar^{n-1} with the full dt;
* a density-independent H takes one exp(-i dt Hbar) per step;
* a nonlocal Kleinman-Bylander term (Eq. VPSP), when given, is part of Hbar
  in both exponentials;
* higher-order extrapolation (order 2) is the quadratic through the three
  latest integer instants, W(t_{n-1} + s dt) ~ sum_k l_k(s) W_{n-1-k}; the
  history before the first step repeats W_0.

The fully self-consistent alternative (same section, steps i-iv) is
``magnus_step_sc``: (i) extrapolate W to the midpoint t_{n-1} + dt/2 from
earlier instants; (ii) propagate psibar^{n-1} over dt with it and evaluate
W_n = W[rho(psibar^n)]; (iii) re-evaluate the midpoint W by interpolating
between W_{n-1} and W_n, i.e. (W_{n-1} + W_n)/2; (iv) repeat (ii)-(iii) until
the midpoint potential changes by at most ``sc_tol`` (largest change over the
Gauss points, a reading: the paper leaves the convergence test open).
"""
import numpy as np

from .lanczos import lanczos_expm
from .nonlocal_kb import apply_nonlocal_bar
from .operators import apply_Hbar
from . import scf


class System:
    """Everything that defines Hbar(t) for a run.

    vext: external potential at the Gauss points (n_cell, nq^3).
    hartree: solve the Poisson problem for V_H; nuclei (Z, R) give its
    boundary values.  xc: 'none', 'x' or 'xc'.  occ: occupations.
    """

    def __init__(self, mesh, vext, hartree=False, xc="none", Z=(), R=(), occ=None,
                 tol=1e-10, k_max=128, pcg_tol=1e-13, pcg_maxit=5000, nonlocal_kb=None):
        self.mesh = mesh
        # (C, E) of the Kleinman-Bylander term (oracle.nonlocal_kb.kb_matrix) or None
        self.nonlocal_kb = nonlocal_kb
        self.vext = np.asarray(vext, dtype=np.float64)
        self.hartree = scf.Hartree(mesh, Z, R, pcg_tol, pcg_maxit) if hartree else None
        self.xc = xc
        self.occ = occ
        self.tol, self.k_max = tol, k_max
        self.zq = mesh.quad_xyz[..., 2]
        self.scf = hartree or xc != "none"

    def W(self, psibar):
        """Density-dependent potential W = V_H + V_xc at the Gauss points."""
        rho = scf.density(self.mesh, psibar, self.occ)
        w = np.zeros_like(rho)
        if self.hartree is not None:
            w = w + self.hartree.solve(rho)[1]
        if self.xc != "none":
            w = w + scf.xc_potential(rho, self.xc)
        return w, rho

    def apply(self, v, x):
        y = apply_Hbar(self.mesh, v, x)
        if self.nonlocal_kb is not None:
            y = y + apply_nonlocal_bar(self.mesh, self.nonlocal_kb[0], self.nonlocal_kb[1], x)
        return y

    def expm(self, v, psibar, tau):
        return lanczos_expm(lambda x: self.apply(v, x), psibar, tau, self.tol, self.k_max)


class State:
    def __init__(self, system, psibar):
        self.psibar = np.array(psibar, dtype=np.complex128)
        if self.psibar.ndim == 1:
            self.psibar = self.psibar[:, None]
        self.n = 0
        self.t = 0.0
        if system.scf:
            w0, _ = system.W(self.psibar)
            self.W1 = w0
            self.W2 = w0
            self.W3 = w0
        self.ks = []


def extrapolation_weights(s, order):
    """Lagrange weights l_k(s), k = 0..order, for the instants 0, -1, .., -order
    (in steps from t_{n-1}) evaluated at s."""
    nodes = [-float(k) for k in range(order + 1)]
    w = []
    for k, xk in enumerate(nodes):
        lk = 1.0
        for j, xj in enumerate(nodes):
            if j != k:
                lk *= (s - xj) / (xk - xj)
        w.append(lk)
    return w


def _extrapolate(state, s, order):
    hist = [state.W1, state.W2, state.W3]
    return sum(wk * hk for wk, hk in zip(extrapolation_weights(s, order), hist))


def _field(system, E, direction):
    if direction is None:
        return -E * system.zq
    return -E * (system.mesh.quad_xyz @ np.asarray(direction, dtype=np.float64))


def magnus_step(system, state, dt, E=0.0, direction=None, order=1):
    """Advance ``state`` by one step; returns a report dict.  The field
    potential is -E z, or -E (d . r) for a field direction d; ``order`` is
    the predictor's extrapolation order (1 linear, 2 quadratic)."""
    vfield = _field(system, E, direction)
    psi0 = state.psibar
    rep = {}
    if system.scf:
        vP = system.vext + vfield + _extrapolate(state, 0.25, order)
        half, k1, e1 = system.expm(vP, psi0, 0.5 * dt)
        wh, _ = system.W(half)
        vC = system.vext + vfield + wh
        new, k2, e2 = system.expm(vC, psi0, dt)
        wn, rho = system.W(new)
        state.W3, state.W2, state.W1 = state.W2, state.W1, wn
        rep.update(k_pred=k1, k_corr=k2, err_pred=e1, err_corr=e2)
    else:
        new, k2, e2 = system.expm(system.vext + vfield, psi0, dt)
        rho = scf.density(system.mesh, new, system.occ)
        rep.update(k_corr=k2, err_corr=e2)
    state.psibar = new
    state.n += 1
    state.t += dt
    rep["dipole"] = scf.dipole(system.mesh, rho)
    rep["charge"] = scf.charge(system.mesh, rho)
    return rep


def magnus_step_sc(system, state, dt, E=0.0, direction=None, order=1, sc_tol=1e-10, max_iter=50):
    """Fully self-consistent midpoint step (steps i-iv above).  The report
    adds the iteration count and the last change of the midpoint potential;
    ``converged`` is False when max_iter iterations did not reach sc_tol (the
    last iterate is kept)."""
    vfield = _field(system, E, direction)
    psi0 = state.psibar
    rep = {"k_corr": [], "err_corr": []}
    if not system.scf:
        new, k, e = system.expm(system.vext + vfield, psi0, dt)
        rho = scf.density(system.mesh, new, system.occ)
        rep.update(k_corr=[k], err_corr=[e], sc_iters=1, sc_change=0.0, converged=True)
    else:
        wmid = _extrapolate(state, 0.5, order)                    # (i)
        it, change, converged = 0, np.inf, False
        while it < max_iter:
            new, k, e = system.expm(system.vext + vfield + wmid, psi0, dt)   # (ii)
            wn, rho = system.W(new)
            it += 1
            rep["k_corr"].append(k)
            rep["err_corr"].append(e)
            wmid_next = 0.5 * (state.W1 + wn)                     # (iii)
            change = float(np.max(np.abs(wmid_next - wmid)))
            wmid = wmid_next
            if change <= sc_tol:                                  # (iv)
                converged = True
                break
        state.W3, state.W2, state.W1 = state.W2, state.W1, wn
        rep.update(sc_iters=it, sc_change=change, converged=converged)
    state.psibar = new
    state.n += 1
    state.t += dt
    rep["dipole"] = scf.dipole(system.mesh, rho)
    rep["charge"] = scf.charge(system.mesh, rho)
    return rep
