"""Reverse-mode gradient of the final dipole w.r.t. per-step field amplitudes (oracle).

Not in the paper (the paper propagates forward only).  The forward map is the
predictor-corrector Magnus step of ``oracle.magnus`` with a field
V_field = -E_n z on step n (Eq. VField), written here with exact
exponentials of the dense H-bar (tiny meshes only), so the gradient is that
of the discrete scheme without Krylov truncation:

  V_P = V_ext - E_n z + 1.25 W_{n-1} - 0.25 W_{n-2}
  phi = exp(-i dt/2 Hbar(V_P)) psi^{n-1}
  V_C = V_ext - E_n z + W[rho(phi)]
  psi^n = exp(-i dt Hbar(V_C)) psi^{n-1},     W_n = W[rho(psi^n)]
  L = mu_z(psi^N) = sum_q varpi_q detJ_q z_q rho_q(psi^N)

Cotangents use the real inner product Re<a, b>.  The pieces:
* exponential: for z = exp(-i tau Hbar) x with cotangent zb,
  xb = exp(+i tau Hbar) zb (Hbar real symmetric), and the potential
  cotangent comes from the Frechet derivative of the exponential: with
  Hbar = U diag(lam) U^T, x~ = U^T x, z~ = U^T zb and P = I M^-1/2 U (the
  eigenvectors at the Gauss points),
    Vb_q = Re[ -i tau varpi_q detJ_q sum_alpha sum_ab conj(z~_a) P_qa G_ab P_qb x~_b ]
  where G_ab = int_0^1 exp(-i(1-s) tau lam_a) exp(-i s tau lam_b) ds is the
  divided difference of exp(-i tau .) (Daleckii-Krein);
* density: for rho_q = sum_alpha f_alpha |psi_alpha(x_q)|^2 with cotangent
  rhob, psib_alpha = 2 f_alpha M^-1/2 I^T (rhob * I M^-1/2 psibar_alpha);
* W = V_H + V_xc: rhob = f_xc(rho) Wb + 4 pi varpi detJ * I K00^-1 I^T Wb
  (K symmetric; the boundary lifting is constant);
* E enters V_P and V_C as -E_n z, so dL/dE_n = -sum_q (Vb_P + Vb_C)_q z_q.
"""
import numpy as np

from . import operators as op
from . import scf


def fxc(rho, mode):
    """d V_xc / d rho; exchange only (regularised to 0 at rho < 1e-30)."""
    if mode == "none":
        return np.zeros_like(rho)
    if mode != "x":
        raise NotImplementedError("f_xc is implemented for LDA exchange")
    rho = np.asarray(rho, dtype=np.float64)
    out = np.zeros_like(rho)
    m = rho > 1e-30
    out[m] = -(1.0 / 3.0) * np.cbrt(3.0 / np.pi) * rho[m] ** (-2.0 / 3.0)
    return out


class DenseAdjointSystem:
    """Forward scheme and its gradient with exact (dense) exponentials."""

    def __init__(self, mesh, vext, Z, R, xc="x", hartree=True, occ=None):
        self.mesh = mesh
        self.vext = np.asarray(vext, dtype=np.float64)
        self.xc = xc
        self.hartree = scf.Hartree(mesh, Z, R, tol=1e-14, maxit=20000) if hartree else None
        self.occ = occ
        self.zq = mesh.quad_xyz[..., 2]
        self.wdet = mesh.from_cell_quad(mesh.volume_weights)
        # interpolation from DoF coefficients (Loewdin scaled) to Gauss points
        self._interp = None

    # -- dense building blocks -----------------------------------------------------
    def interp_matrix(self):
        """I M^-1/2 as a dense (n_quad, n_dof) matrix, Gauss points in (n_cell, nq^3) order."""
        if self._interp is None:
            m = self.mesh
            eye = np.eye(m.n_dof)
            cols = []
            for j0 in range(0, m.n_dof, 256):
                blk = eye[:, j0:j0 + 256] * m.m_inv_sqrt[:, None]
                q = scf.quad_values(m, blk)  # (e, a, b, c, cols)
                cols.append(q.transpose(0, 3, 2, 1, 4).reshape(m.n_cell * m.nq ** 3, -1))
            self._interp = np.concatenate(cols, axis=1)
        return self._interp

    def eig(self, v):
        th, U = np.linalg.eigh(op.dense_Hbar(self.mesh, v))
        return th, U

    @staticmethod
    def expm(th, U, tau, x):
        return U @ (np.exp(-1j * tau * th)[:, None] * (U.T @ x))

    def W(self, psibar):
        rho = scf.density(self.mesh, psibar, self.occ)
        w = np.zeros_like(rho)
        if self.hartree is not None:
            w = w + self.hartree.solve(rho)[1]
        if self.xc != "none":
            w = w + scf.xc_potential(rho, self.xc)
        return w, rho

    # -- forward ---------------------------------------------------------------------
    def forward(self, psi0, E, dt):
        psi = np.array(psi0, dtype=np.complex128)
        W0, _ = self.W(psi)
        W1, W2 = W0, W0
        tape = []
        for n, e in enumerate(E):
            vP = self.vext - e * self.zq + 1.25 * W1 - 0.25 * W2
            thP, UP = self.eig(vP)
            phi = self.expm(thP, UP, 0.5 * dt, psi)
            Wh, rho_h = self.W(phi)
            vC = self.vext - e * self.zq + Wh
            thC, UC = self.eig(vC)
            new = self.expm(thC, UC, dt, psi)
            Wn, rho_n = self.W(new)
            tape.append(dict(psi=psi, phi=phi, rho_h=rho_h, rho_n=rho_n, new=new,
                             eP=(thP, UP), eC=(thC, UC)))
            W2, W1 = W1, Wn
            psi = new
        rho = scf.density(self.mesh, psi, self.occ)
        L = float(np.sum(self.wdet * self.zq * rho))
        return L, psi, tape

    # -- adjoint pieces ------------------------------------------------------------------
    def density_adjoint(self, psibar, rhob):
        """psib = 2 f M^-1/2 I^T (rhob * I M^-1/2 psibar)."""
        P = self.interp_matrix()
        occ = np.ones(psibar.shape[1]) if self.occ is None else np.asarray(self.occ)
        u = P @ psibar
        return 2.0 * (P.T @ (rhob.reshape(-1)[:, None] * u)) * occ[None, :]

    def W_adjoint(self, Wb, rho):
        """rhob from a cotangent Wb of W = V_H[rho] + V_xc(rho)."""
        rhob = fxc(rho, self.xc) * Wb
        if self.hartree is not None:
            m = self.mesh
            h = self.hartree
            interior = h.interior
            # I^T Wb (no quadrature weights) over the interior nodes
            B = m.ref.B
            ge = m.to_cell_quad(Wb)
            ce = np.einsum("ai,bj,ck,eabc->eijk", B, B, B, ge, optimize=True)
            c = np.zeros(m.n_nodes)
            np.add.at(c, m.cell_nodes.reshape(-1), ce.reshape(-1))
            x, _, _ = scf.pcg(h._A, 4.0 * np.pi * c[interior], np.zeros(int(interior.sum())), h.diag,
                              1e-14, 20000)
            phib = np.zeros(m.n_nodes)
            phib[interior] = x
            vh = m.from_cell_quad(scf.quad_values(m, phib, nodes=True))
            rhob = rhob + self.wdet * vh
        return rhob

    def exp_adjoint(self, eg, tau, x, zb):
        """(xb, Vb) for z = exp(-i tau Hbar(V)) x with cotangent zb."""
        th, U = eg
        xt = U.T @ x
        zt = U.T @ zb
        xb = U @ (np.exp(1j * tau * th)[:, None] * zt)
        d = th[:, None] - th[None, :]
        ea = np.exp(-1j * tau * th)
        with np.errstate(divide="ignore", invalid="ignore"):
            G = (ea[None, :] - ea[:, None]) / (-1j * tau * (th[None, :] - th[:, None]))
        same = np.abs(d) < 1e-12 * max(1.0, np.abs(th).max())
        G[same] = np.broadcast_to(ea[:, None], G.shape)[same]
        P = self.interp_matrix() @ U  # eigenvectors at the Gauss points
        acc = np.zeros(P.shape[0], dtype=np.complex128)
        for a in range(x.shape[1]):
            A = P * np.conj(zt[:, a])[None, :]
            Bm = P * xt[:, a][None, :]
            acc += np.einsum("qa,ab,qb->q", A, G, Bm, optimize=True)
        Vb = np.real(-1j * tau * acc) * self.wdet.reshape(-1)
        return xb, Vb.reshape(self.wdet.shape)

    def gradient(self, psi0, E, dt):
        """L and dL/dE for the per-step field amplitudes E."""
        N = len(E)
        L, psiN, tape = self.forward(psi0, E, dt)
        lam = self.density_adjoint(psiN, self.wdet * self.zq)
        Wb = {}
        dE = np.zeros(N)
        for n in range(N - 1, -1, -1):
            rec = tape[n]
            if n < N - 1 and (n + 1) in Wb:
                lam = lam + self.density_adjoint(rec["new"], self.W_adjoint(Wb.pop(n + 1), rec["rho_n"]))
            xC, VbC = self.exp_adjoint(rec["eC"], dt, rec["psi"], lam)
            dE[n] -= float(np.sum(VbC * self.zq))
            lam_h = self.density_adjoint(rec["phi"], self.W_adjoint(VbC, rec["rho_h"]))
            xP, VbP = self.exp_adjoint(rec["eP"], 0.5 * dt, rec["psi"], lam_h)
            dE[n] -= float(np.sum(VbP * self.zq))
            # W_{n} of the tape indexing is W of psi^{n} (state before step n+1):
            # step n (0-based) used W of psi^{n} (1.25) and of psi^{n-1} (-0.25)
            k1, k2 = n, max(n - 1, 0)
            Wb[k1] = Wb.get(k1, 0.0) + 1.25 * VbP
            Wb[k2] = Wb.get(k2, 0.0) - 0.25 * VbP
            lam = xC + xP
        return L, dE
