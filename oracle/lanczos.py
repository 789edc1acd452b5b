"""Adaptive Lanczos approximation of exp(-i tau Hbar) psibar (oracle).

Sec. "Approximating the second-order Magnus operator":
* Eq. KrylovSubspace: K_k(A, psi) = span{psi, A psi, ..., A^(k-1) psi};
* Eq. zk: z_k = ||psi|| Q_k exp(T_k) e_1 with T_k = Q_k^H A Q_k tridiagonal;
* the small exponential by exact eigenvalue decomposition of T_k;
* Eq. AdaptiveLanczos: eps_k ~ |beta_{k+1,k}| ||psi|| |[exp(T_k)]_{k,1}|,
  the dimension k grown until eps_k is below the tolerance.

Readings (the paper is silent on these points):
* A = -i tau Hbar with Hbar real symmetric, so the recurrence is run on Hbar
  and T_k(A) = -i tau T_k(Hbar); |beta_{k+1,k}(A)| = |tau| beta_k(Hbar).
* e_1 is the first unit vector; Q^H replaces the printed Q^T (complex psi).
* each orbital has its own Krylov space (not a block Krylov method);
* eps_k is checked at every k from 1; no re-orthogonalisation;
* happy breakdown when beta_k <= 1e-14 max_j |alpha_j|;
* reaching k_max without eps_k <= tol is reported as non-convergence.
"""
import numpy as np
from scipy.linalg import eigh_tridiagonal


class NotConverged(RuntimeError):
    pass


def tridiag_expm_e1(alpha, beta, tau):
    """y = exp(-i tau T) e_1 for T = tridiag(beta, alpha, beta), by eigh."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    if len(alpha) == 1:
        return np.array([np.exp(-1j * tau * alpha[0])])
    theta, V = eigh_tridiagonal(alpha, beta)
    return V @ (np.exp(-1j * tau * theta) * V[0, :])


def lanczos_expm_vec(apply_hbar, psi, tau, tol, k_max=128, breakdown=1e-14):
    """exp(-i tau Hbar) psi for ONE complex vector psi (n_dof,).

    Returns (z, k, eps, info) where info holds alpha, beta and y.
    """
    psi = np.asarray(psi, dtype=np.complex128)
    nrm = np.linalg.norm(psi)
    if nrm == 0.0:
        return np.zeros_like(psi), 0, 0.0, {"alpha": [], "beta": [], "y": []}
    Q = [psi / nrm]
    alpha, beta = [], []
    q_prev = np.zeros_like(psi)
    b_prev = 0.0
    for k in range(1, k_max + 1):
        w = apply_hbar(Q[-1])
        a = float(np.real(np.vdot(Q[-1], w)))
        w = w - a * Q[-1] - b_prev * q_prev
        b = float(np.linalg.norm(w))
        alpha.append(a)
        y = tridiag_expm_e1(alpha, beta, tau)
        eps = abs(tau) * b * nrm * abs(y[-1])
        happy = b <= breakdown * max(abs(x) for x in alpha)
        if eps <= tol or happy:
            z = nrm * (np.stack(Q, axis=1) @ y)
            return z, k, eps, {"alpha": alpha, "beta": beta + [b], "y": y}
        beta.append(b)
        q_prev = Q[-1]
        b_prev = b
        Q.append(w / b)
    z = nrm * (np.stack(Q[:k_max], axis=1) @ y)
    raise NotConverged(f"Lanczos did not reach eps <= {tol} within k_max={k_max} (eps={eps:.3e})")


def lanczos_expm(apply_hbar, psibar, tau, tol, k_max=128):
    """exp(-i tau Hbar) applied to every column of psibar (n_dof, N).

    Returns (z, ks, errs).
    """
    psibar = np.asarray(psibar, dtype=np.complex128)
    if psibar.ndim == 1:
        psibar = psibar[:, None]
    out = np.empty_like(psibar)
    ks, errs = [], []
    for a in range(psibar.shape[1]):
        z, k, eps, _ = lanczos_expm_vec(apply_hbar, psibar[:, a], tau, tol, k_max)
        out[:, a] = z
        ks.append(k)
        errs.append(eps)
    return out, ks, errs
