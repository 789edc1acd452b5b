"""CPU FP64 oracle for the spectral-finite-element real-time TDDFT step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library under
``paper_1810_13130_amd/``) imports, links or calls this package; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may.  It shares no code, tables or constants with the HIP path.

It is a plain, slow, obviously-correct numpy/scipy transcription of the
method of Kanungo & Gavini, "Real-time time-dependent density functional
theory using higher-order finite-element methods" (arXiv:1810.13130):

* ``fe``        reference element: GLL nodes/weights, Gauss rule, Lagrange
                basis (Sec. "Higher-order spectral finite-elements").
* ``mesh``      hexahedral mesh, node numbering, Dirichlet DoFs, diagonal
                GLL overlap M (Sec. "Semi-discrete solution", spectral FE).
* ``operators`` matrix-free and dense-assembled H and the Loewdin form
                Hbar = M^-1/2 H M^-1/2 (Eqs. DiscreteHamiltonian,
                TDKSMatVecStandard).
* ``lanczos``   adaptive Lanczos approximation of exp(-i tau Hbar) psi
                (Eqs. KrylovSubspace, zk, AdaptiveLanczos).
* ``scf``       density, dipole, Hartree Poisson solve, LDA exchange /
                Perdew-Zunger correlation (Eqs. VKS, Poisson,
                VHDiscretePoisson).
* ``magnus``    second-order Magnus step with the predictor-corrector
                midpoint Hamiltonian (Eqs. ApproxMagnus, PsiTimeDiscrete).
* ``adjoint``   reverse-mode gradient of the final dipole with respect to
                per-step field amplitudes (not in the paper; built from the
                Frechet derivative of the exponential).

Each function cites the passage it follows.  Where the paper is silent or
garbled the reading taken is stated in the function's docstring.
"""
