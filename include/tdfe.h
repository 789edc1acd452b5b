/*
 * tdfe.h -- C ABI of the MI355X spectral-finite-element real-time TDDFT step.
 *
 * Method: Kanungo & Gavini, "Real-time time-dependent density functional
 * theory using higher-order finite-element methods" (arXiv:1810.13130).
 * One call of tdfe_magnus_step advances a block of complex Kohn-Sham orbitals
 * psibar (Loewdin coordinates, Eq. TDKSMatVecStandard) by one second-order
 * Magnus step (Eqs. ApproxMagnus, PsiTimeDiscrete) whose exponential is
 * formed by adaptive Lanczos (Eqs. zk, AdaptiveLanczos) on
 * Hbar = M^-1/2 H M^-1/2 with M the diagonal GLL overlap (Sec. "Higher-order
 * spectral finite-elements") and H the FE Hamiltonian of
 * Eq. DiscreteHamiltonian.
 *
 * Conventions shared by every call
 *  - Mesh: a structured logical grid of ncell[0] x ncell[1] x ncell[2]
 *    hexahedra; cell (cx,cy,cz) is the trilinear image of [-1,1]^3 through
 *    its 8 corner vertices.  Cells are numbered cx + ncx (cy + ncy cz).
 *  - Global GLL nodes (I,J,K), 0 <= I <= ncx p, numbered I + Nx (J + Ny K)
 *    with Nx = ncx p + 1.  The unknowns (DoFs) are the interior nodes
 *    (homogeneous Dirichlet data, Eq. PsiExpansion), numbered
 *    lexicographically with x fastest; n_dof = (Nx-2)(Ny-2)(Nz-2).
 *  - Gauss points: nq = p + 1 per direction (tensor rule); point (a,b,c) of
 *    a cell has index a + nq (b + nq c).  Per-point arrays are
 *    [n_cell][nq^3] row-major FP64.
 *  - Orbitals at the boundary are ALWAYS psibar, complex128 interleaved
 *    (re, im), row-major [n_dof][n_orb]: element (j, alpha) at
 *    ((double*)ptr)[2 (j n_orb + alpha) + {0,1}].  Orbital psi = M^-1/2 psibar.
 *  - All device pointers are owned by the caller.  The library owns only its
 *    context and small host tables; all device scratch lives in the caller's
 *    workspace (tdfe_query / tdfe_bind_workspace).  No call frees caller
 *    memory.
 *  - All device work is enqueued on the hipStream_t given at setup.  Calls
 *    that return host values (scalars, reports) synchronise that stream.
 *  - Every call returns a tdfe_status; arguments are validated on the host
 *    before any device work.  Nothing aborts or throws across the ABI.  One
 *    context per stream; a context is not thread-safe.
 */
#ifndef TDFE_H
#define TDFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int tdfe_status;
#define TDFE_OK 0
#define TDFE_EINVAL (-1)     /* bad argument (sizes, nulls, order, tolerances) */
#define TDFE_ENOMEM (-2)     /* workspace missing or too small */
#define TDFE_EDEVICE (-3)    /* HIP runtime error; text in tdfe_last_error */
#define TDFE_ENOCONV (-4)    /* Lanczos reached k_max / PCG reached maxit */
#define TDFE_ESTATE (-5)     /* call out of order (e.g. apply before potential) */
#define TDFE_ENONFINITE (-6) /* NaN/Inf detected by an FP64 norm */

typedef struct tdfe_ctx tdfe_ctx;

/* working precision of the cell contractions and Krylov storage */
#define TDFE_FP64 0       /* everything FP64 (parity path) */
#define TDFE_MIXED_FP32 1 /* FP32 contractions and Krylov storage; FP64 scalars */
/* Matrix-core variants of the operator's 1D contractions (rectilinear box
 * meshes only; tdfe_fe_mesh_setup returns TDFE_EINVAL for any other mesh).
 * Storage, scalars and every other kernel are those of the base precision;
 * only the H-bar launches of the cell operator change engine:
 *   TDFE_FP32_MFMA: as TDFE_MIXED_FP32, contractions on FP32 matrix cores
 *                   (v_mfma_f32_16x16x4), p <= 7;
 *   TDFE_BF16_MFMA: as TDFE_MIXED_FP32, each contraction as three BF16
 *                   matrix-core products of split operands (head x head +
 *                   head x remainder + remainder x head, FP32 accumulation;
 *                   about 2^-16 relative per product), p <= 7;
 *   TDFE_FP64_MFMA: as TDFE_FP64, contractions on FP64 matrix cores
 *                   (v_mfma_f64_16x16x4), p <= 6. */
#define TDFE_FP32_MFMA 2
#define TDFE_BF16_MFMA 3
#define TDFE_FP64_MFMA 4

typedef struct {
  int p;                  /* element order, 1..8 (Sec. spectral FE) */
  int nq;                 /* Gauss points per direction; must be p + 1 */
  int ncell[3];           /* logical cells along x, y, z (each >= 1) */
  const double* vertices; /* HOST, (ncx+1)(ncy+1)(ncz+1) x 3, x fastest */
  int n_orb_max;          /* largest orbital block passed to any call */
  int k_max;              /* Krylov dimension cap, 1..1024 */
  int precision;          /* TDFE_FP64, TDFE_MIXED_FP32 or a matrix-core variant */
} tdfe_mesh_desc;

/* fe_mesh_setup: reference element (GLL nodes/weights, Gauss rule, 1D
 * interpolation/derivative tables) and mesh bookkeeping (Sec. "Higher-order
 * spectral finite-elements"; Eq. PsiExpansion for the Dirichlet DoFs).
 * No device memory is touched until tdfe_bind_workspace; the free memory of
 * the current device is queried once to size the Krylov basis: orbitals are
 * processed in chunks whose basis ((k_max + 2) vectors per orbital) fits in
 * 60% of it (128 GB if the query fails); the workspace also holds the
 * operator output of the widest soft-capped chunk (krylov_soft_chunk).
 * Environment read here: TDFE_MAX_CHUNK_ORB=n caps every Krylov chunk at n
 * orbitals; TDFE_BASIS_CHUNK_ORB=n caps only the basis memory at n orbitals
 * (soft-capped chunks may still be wider), as on a device with less memory;
 * TDFE_APPLY_VARIANT=line|pair|plane forces one operator kernel family
 * where it applies (the default picks per mesh, order and precision).
 * hip_stream: hipStream_t (may be 0).  *out receives a new context. */
tdfe_status tdfe_fe_mesh_setup(const tdfe_mesh_desc* d, void* hip_stream, tdfe_ctx** out);

/* sizes of the problem and of the device workspace the caller must provide */
tdfe_status tdfe_query(const tdfe_ctx* ctx, int64_t* n_dof, int64_t* n_cell, int64_t* n_quad,
                       size_t* workspace_bytes);

/* krylov_chunk: orbitals per Krylov chunk for a call on n_orb orbitals (the
 * operator launches of lanczos_expm and magnus_step cover one chunk, 2 *chunk
 * real columns, at a time); chunks are sized so that (k_max + 2) basis
 * vectors fit the memory limit stated at tdfe_fe_mesh_setup.  Host only. */
tdfe_status tdfe_krylov_chunk(const tdfe_ctx* ctx, int n_orb, int* chunk);

/* krylov_soft_chunk: the chunk and Krylov dimension limit that the next
 * exponential of lanczos_expm, magnus_step or propagate on n_orb orbitals
 * will use (the per-orbital adaptive dimension of Eq. AdaptiveLanczos does
 * not change).  Once an exponential has run, chunks may be wider than
 * krylov_chunk: w orbitals then share the basis memory of krylov_chunk
 * orbitals, which holds (k_max + 1) krylov_chunk / w - 1 vectors past the
 * first (*kcap); w is chosen so that *kcap is at least twice the largest
 * Krylov dimension of the last exponential and at least 32.  An orbital
 * that reaches *kcap unconverged sends its chunk back to k_max in chunks of
 * krylov_chunk before the chunk writes its output: the result is the same,
 * the exponential takes longer (and a soft-capped chunk waits for the device
 * once, before its combination).  *chunk = krylov_chunk and *kcap = k_max
 * when no wider chunk applies (no exponential yet, every orbital in one
 * chunk, or the field gradient's runs).  Host only; EINVAL for a null pointer
 * or n_orb outside 1..n_orb_max. */
tdfe_status tdfe_krylov_soft_chunk(const tdfe_ctx* ctx, int n_orb, int* chunk, int* kcap);

/* binds a caller-owned device buffer of >= workspace_bytes (256-byte aligned)
 * and computes the device-side geometry and the diagonal overlap
 * M_jj = sum_e w_i w_j w_k det J_e(node) (GLL quadrature, Sec. spectral FE). */
tdfe_status tdfe_bind_workspace(tdfe_ctx* ctx, void* dev, size_t bytes);

/* device outputs: DoF coordinates [n_dof][3], Gauss point coordinates
 * [n_cell][nq^3][3], overlap diagonal M [n_dof] */
tdfe_status tdfe_dof_coords(tdfe_ctx* ctx, double* dev_xyz);
tdfe_status tdfe_quad_coords(tdfe_ctx* ctx, double* dev_xyz);
tdfe_status tdfe_mass_diag(tdfe_ctx* ctx, double* dev_m);

/* set_potential: the static external potential V_ext at the Gauss points,
 * [n_cell][nq^3] FP64 device (Eq. VKS, local part).  Copied into the
 * workspace.  Also the total potential used by apply_H until SCF terms are
 * added by magnus_step. */
tdfe_status tdfe_set_potential(tdfe_ctx* ctx, const double* dev_v);

#define TDFE_XC_NONE 0
#define TDFE_XC_X 1   /* LDA exchange */
#define TDFE_XC_XC 2  /* LDA exchange + Perdew-Zunger 81 correlation */

typedef struct {
  int hartree;              /* solve K phi = 4 pi c for V_H (Eqs. Poisson, VHDiscretePoisson) */
  int xc;                   /* TDFE_XC_* (ALDA, Sec. TDKS equations) */
  int n_nuclei;             /* nuclei giving the Hartree boundary values f = sum Z/|r-R| */
  const double* Z;          /* HOST [n_nuclei] */
  const double* R;          /* HOST [n_nuclei][3] */
  const double* occupation; /* HOST [n_orb] occupations f_alpha, or NULL for all 1 */
  int n_orb;                /* orbitals the occupations refer to */
  double pcg_tol;           /* relative residual for curved meshes (box meshes solve exactly) */
  int pcg_maxit;
  int pcg_precond;          /* curved meshes: TDFE_PCG_FDM (0, default) or TDFE_PCG_JACOBI */
} tdfe_scf_desc;

/* Hartree solve on curved meshes: conjugate gradients on K phi = 4 pi c to
 * the relative residual pcg_tol, warm-started from the previous phi.  The
 * preconditioner is either the inverse diagonal of K (TDFE_PCG_JACOBI) or
 * TDFE_PCG_FDM: the exact inverse, by fast diagonalisation, of the stiffness
 * of a rectilinear stand-in mesh whose vertex coordinates along each axis are
 * the means of the true ones over the other two indices (on smoothly graded
 * meshes 20-30 iterations instead of the hundreds Jacobi needs).  Both stop at
 * the same residual test; box meshes always solve exactly.  Along axes of
 * more than 128 interior nodes the fast diagonalisation's 1D transforms are
 * rocBLAS DGEMMs; the first solve of a context times every rocBLAS solution
 * for each transform shape and keeps the fastest (a one-time cost of about
 * 0.1-0.5 s; two contexts may keep different solutions, which changes phi
 * at the level of the solve's tolerance). */
#define TDFE_PCG_FDM 0
#define TDFE_PCG_JACOBI 1

/* set_scf: density-dependent part of V_KS.  Resets the extrapolation history. */
tdfe_status tdfe_set_scf(tdfe_ctx* ctx, const tdfe_scf_desc* s);

/* Nonlocal pseudopotential term in the Kleinman-Bylander form (Eq. VPSP):
 * V_NL phi = sum_p (int u_p dV_p phi / D_p) u_p dV_p with D_p = int u_p dV_p u_p.
 * Its Galerkin matrix C^T diag(1/D) C, c_pj = int u_p dV_p N_j, is added (in
 * Loewdin form, M^-1/2 C^T diag(1/D) C M^-1/2) to every later application of
 * Hbar: apply_H*, lanczos_expm, magnus_step and the adjoint, in both
 * precisions (the mixed path keeps an FP32 copy of C M^-1/2 and accumulates
 * the projections in FP64).  All integrals use the Gauss rule of the mesh.
 *
 * Projectors are compact around their atoms: C M^-1/2 is stored on the
 * smallest box of the DoF grid that holds every entry above 2^-60 of the
 * projector's largest one (consecutive projectors with nearly the same box
 * share it), and the hot passes touch those boxes only.
 *
 * projector_query: *bytes = device store needed for n_proj projectors
 * (0 <= n_proj <= TDFE_MAX_PROJ): the bound n_proj n_dof 8 bytes (12 in
 * mixed contexts) for the boxes, plus scratch of about 8 (n_quad + n_dof)
 * bytes and 2 MB per 256 blocks of partial sums.
 *
 * set_projectors: dev_u, dev_dv are [n_proj][n_cell][nq^3] FP64 device
 * arrays of u_p and dV_p at the Gauss points; dev_store is a caller-owned
 * device buffer of >= the queried size (256-byte aligned) that the library
 * uses until the next set_projectors call or the context's destruction (the
 * caller keeps it alive and does not touch it).  n_proj = 0 removes the term
 * (pointers may then be NULL).  The inputs are read during the call only.
 * Synchronises the stream.  Errors: TDFE_ESTATE before bind_workspace,
 * TDFE_ENOMEM if store_bytes is too small, TDFE_EINVAL for null pointers,
 * misalignment, n_proj out of range or a D_p that is zero or not finite (the
 * term is then off). */
#define TDFE_MAX_PROJ 1024
tdfe_status tdfe_projector_query(const tdfe_ctx* ctx, int n_proj, size_t* bytes);
tdfe_status tdfe_set_projectors(tdfe_ctx* ctx, int n_proj, const double* dev_u, const double* dev_dv,
                                void* dev_store, size_t store_bytes);
/* projector_info: the compact layout chosen by the last set_projectors
 * (zeros when the term is off): number of groups sharing a box, stored
 * entries of C M^-1/2, DoFs in the boxes summed over groups (rows of x the
 * projection streams), and DoFs on the grid lines crossed by boxes (rows of
 * the output the add pass reads and writes, each once). */
tdfe_status tdfe_projector_info(const tdfe_ctx* ctx, int* n_groups, int64_t* stored, int64_t* box_dofs,
                                int64_t* line_dofs);

/* apply_H: dev_out = Hbar dev_psibar for n_orb orbitals (both [n_dof][n_orb]
 * complex128), Hbar = M^-1/2 (1/2 K + V-mass) M^-1/2 with the current total
 * potential (Eqs. DiscreteHamiltonian, TDKSMatVecStandard).  Gauss quadrature
 * for every term.  dev_out must not alias dev_psibar. */
tdfe_status tdfe_apply_H(tdfe_ctx* ctx, const void* dev_psibar, void* dev_out, int n_orb);

/* apply_H_add: dev_out += Hbar dev_psibar (same operator as apply_H, no
 * zeroing of dev_out): exactly one launch of the operator kernel (followed by
 * the nonlocal kernels when projectors are set), for composite operators and
 * for timing that kernel alone. */
tdfe_status tdfe_apply_H_add(tdfe_ctx* ctx, const void* dev_psibar, void* dev_out, int n_orb);

/* apply_H_add_f32: dev_out += Hbar dev_psibar in FP32 (the mixed-precision
 * operator kernel): both arrays complex64 interleaved [n_dof][n_orb]; the
 * potential is the FP32 copy of the current total potential.  Requires a
 * context created with TDFE_MIXED_FP32. */
tdfe_status tdfe_apply_H_add_f32(tdfe_ctx* ctx, const void* dev_psibar_c64, void* dev_out_c64, int n_orb);

/* lanczos_expm: psibar <- exp(-i tau Hbar) psibar in place, each orbital with
 * its own adaptive Krylov space (Eqs. KrylovSubspace, zk, AdaptiveLanczos):
 * stop at the first k with tau beta_k ||psibar|| |[exp(-i tau T_k)]_{k,1}| <= tol
 * or on happy breakdown (beta_k <= 1e-14 max|alpha|).  tau < 0 gives the
 * adjoint direction exp(+i|tau|Hbar).  In a TDFE_MIXED_FP32 context the
 * stop tolerance of orbital alpha is max(tol, 16 * 2^-24 * ||psibar_alpha||):
 * FP32 basis vectors cannot support a tighter estimate.  host_k [n_orb] and
 * host_err [n_orb] (may be NULL) receive the final dimension and error estimate.
 * Returns TDFE_ENOCONV (psibar holds the k_max iterate) if k_max is reached.
 * Returns TDFE_ENONFINITE if an orbital's FP64 norm ||psibar_alpha|| is NaN or
 * Inf (a non-finite entry), or if a recurrence coefficient (alpha_k, beta_k)
 * or the error estimate becomes non-finite: that orbital stops at once and
 * its output columns are not finite; the other orbitals are propagated as
 * usual.  ENONFINITE takes precedence over ENOCONV. */
tdfe_status tdfe_lanczos_expm(tdfe_ctx* ctx, void* dev_psibar, int n_orb, double tau, double tol,
                              int* host_k, double* host_err);

/* scf_fields: the density-dependent potential of the given orbitals, without
 * propagating them (Eq. VKS): rho of psibar (as tdfe_density), the Hartree
 * potential phi from K phi = 4 pi c, c_j = int rho N_j, with phi = f =
 * sum Z/|r - R| at the boundary nodes (Eqs. Poisson, VHDiscretePoisson;
 * exact fast diagonalisation on box meshes, Jacobi-PCG to pcg_tol on curved
 * ones, warm-started from and updating the context's last phi, as magnus_step
 * does), and W = V_H + V_xc at the Gauss points.
 *   dev_phi: [Nx Ny Nz] FP64 device, every node of the grid (boundary values
 *            included), node (I,J,K) at I + Nx (J + Ny K); or NULL.
 *   dev_w:   [n_cell][nq^3] FP64 device; or NULL (at least one is given).
 * The Magnus extrapolation history is not touched.  Synchronises the stream.
 * Errors: TDFE_ESTATE before set_scf (or with neither Hartree nor XC on),
 * TDFE_EINVAL for dev_phi without Hartree, TDFE_ENOCONV / TDFE_ENONFINITE
 * from the PCG solve. */
tdfe_status tdfe_scf_fields(tdfe_ctx* ctx, const void* dev_psibar, int n_orb, double* dev_phi, double* dev_w);

/* tridiag_expm: the small exponential of the Lanczos approximation (Eq. zk),
 * y = exp(-i tau T) e_1 for one real symmetric tridiagonal T of order k
 * (1 <= k <= 1024): diagonal dev_alpha[k], off-diagonal dev_beta[k-1]
 * (FP64 device; dev_beta may be NULL for k = 1); dev_y [k] complex128
 * interleaved (device).  The same evaluation the Lanczos stop test uses: a
 * Chebyshev series on the Gershgorin interval [c - r, c + r] of T with
 * Jacobi-Anger coefficients 2 (-i)^m J_m(|tau| r), about |tau| r terms, for
 * |tau| r up to about 6.5e4.  No context; dev_scratch (>= the queried bytes,
 * 256-byte aligned) holds the Bessel table.  Synchronises hip_stream;
 * *host_terms (may be NULL) receives the number of terms.  Errors: EINVAL for
 * bad arguments or |tau| r beyond the table, ENOMEM for a small or misaligned
 * scratch, ENONFINITE for an Inf or NaN spread of T. */
tdfe_status tdfe_tridiag_expm_query(int k, size_t* bytes);
tdfe_status tdfe_tridiag_expm(const double* dev_alpha, const double* dev_beta, int k, double tau, double* dev_y,
                              void* dev_scratch, size_t scratch_bytes, void* hip_stream, int* host_terms);

/* density at the Gauss points, rho_q = sum_alpha f_alpha |psi_alpha(x_q)|^2,
 * psi = M^-1/2 psibar interpolated with the GLL basis (Sec. TDKS equations).
 * dev_rho_q: [n_cell][nq^3] FP64 device. */
tdfe_status tdfe_density(tdfe_ctx* ctx, const void* dev_psibar, int n_orb, double* dev_rho_q);

/* dipole mu = sum_q varpi_q detJ_q x_q rho_q (electronic, +int r rho) and the
 * charge sum_q varpi_q detJ_q rho_q of the given orbitals.  host_mu[3]. */
tdfe_status tdfe_dipole(tdfe_ctx* ctx, const void* dev_psibar, int n_orb, double* host_mu,
                        double* host_charge);

typedef struct {
  int k_pred_max, k_corr_max; /* largest Krylov dimension of the two propagations */
  int k_pred_sum, k_corr_sum; /* sum over orbitals */
  double err_max;             /* largest Lanczos error estimate */
  int poisson_iters;          /* 0 for the exact box solver */
  double mu[3];               /* dipole of psibar^n */
  double charge;              /* charge of psibar^n */
  int sc_iters;               /* self-consistent midpoint: propagations over dt (0 in the predictor-corrector mode) */
  double sc_change;           /* self-consistent midpoint: last max change of the midpoint W */
} tdfe_step_report;

/* set_midpoint: how magnus_step evaluates Hbar at the step's midpoint (Sec.
 * "Approximating the second-order Magnus operator").
 *   TDFE_MIDPOINT_PC (default): the predictor-corrector below, its predictor
 *     W(t_{n-1} + dt/4) extrapolated from the order + 1 latest instants;
 *   TDFE_MIDPOINT_SC: the fully self-consistent iteration (steps i-iv):
 *     (i) W_mid = W(t_{n-1} + dt/2) extrapolated likewise; (ii) psibar^n =
 *     exp(-i dt Hbar(V_ext + V_field + W_mid)) psibar^{n-1}, W_n =
 *     W[rho(psibar^n)]; (iii) W_mid <- (W_{n-1} + W_n)/2; (iv) repeat (ii)-(iii)
 *     until max over the Gauss points of the change of W_mid <= sc_tol
 *     (Hartree), at most sc_maxit propagations; TDFE_ENOCONV beyond, with
 *     the last iterate written and kept as W_n.  One host synchronisation
 *     per iteration.
 * order: 1 (linear: weights 1.25, -0.25 at dt/4; 1.5, -0.5 at dt/2) or 2
 * (quadratic through W_{n-1}, W_{n-2}, W_{n-3}); the history before the
 * first step repeats W_0.  Applies to later magnus_step calls; the field
 * gradient supports the default only (TDFE_EINVAL otherwise). */
#define TDFE_MIDPOINT_PC 0
#define TDFE_MIDPOINT_SC 1
typedef struct {
  int mode;      /* TDFE_MIDPOINT_PC or TDFE_MIDPOINT_SC */
  int order;     /* extrapolation order, 1 or 2 */
  double sc_tol; /* SC: > 0 */
  int sc_maxit;  /* SC: >= 1 */
} tdfe_midpoint_desc;
tdfe_status tdfe_set_midpoint(tdfe_ctx* ctx, const tdfe_midpoint_desc* m);

/* magnus_step: one second-order Magnus step with the predictor-corrector
 * midpoint Hamiltonian (Eqs. ApproxMagnus, PsiTimeDiscrete; Sec.
 * "Approximating the second-order Magnus operator"; the self-consistent
 * alternative and the quadratic predictor are chosen by tdfe_set_midpoint):
 *   V_P = V_ext + V_field + 1.25 W_{n-1} - 0.25 W_{n-2}
 *   psibar^{n-1/2} = exp(-i dt/2 Hbar(V_P)) psibar^{n-1}
 *   V_C = V_ext + V_field + W[rho(psibar^{n-1/2})]
 *   psibar^n = exp(-i dt Hbar(V_C)) psibar^{n-1},   W_n = W[rho(psibar^n)]
 * with W = V_H + V_xc and V_field = -field_E (d . r) (Eq. VField), held over
 * the step; d is the field direction (tdfe_set_field_direction, z unless
 * set).  Without SCF terms the step is one exp(-i dt Hbar) psibar.  The first
 * call after set_scf computes W_0 from psibar (and W_{-1} := W_0).
 * psibar is updated in place; rep may be NULL.  The call synchronises its
 * stream once, at the end, to collect the Lanczos convergence status (and the
 * report); a device-side failure found there (TDFE_EINVAL for a Chebyshev
 * table overflow, TDFE_ENONFINITE for a non-finite orbital norm, Lanczos
 * coefficient or density, as in tdfe_lanczos_expm) is returned after psibar
 * has been written. */
tdfe_status tdfe_magnus_step(tdfe_ctx* ctx, void* dev_psibar, int n_orb, double dt, double field_E,
                             double tol, tdfe_step_report* rep);

/* propagate: n_steps magnus_step steps in one call, the field amplitude of
 * step n being host_E[n] (NULL: no field).  In the predictor-corrector mode
 * the steps are enqueued back to back with no synchronisation between them:
 * each step's Krylov results are folded on the device and its {charge,
 * mu_x, mu_y, mu_z} written to dev_mu + 4 n (dev_mu: [n_steps][4] FP64
 * device, or NULL); one readback and one synchronisation at the end.  The
 * self-consistent midpoint mode runs step by step.  rep (may be NULL)
 * receives the totals: largest Krylov dimension and the sum over all
 * propagations (in k_corr_max / k_corr_sum; per-step predictor and corrector
 * are not separated in the batched mode), largest error estimate, and the
 * last step's dipole and charge.  TDFE_ENOCONV if any Lanczos run reached
 * k_max (all steps are still taken); TDFE_ENONFINITE (checked at the end of
 * the batch, before ENOCONV) if any Lanczos run met a non-finite norm or
 * coefficient; other errors stop the run at the step that failed.  psibar is
 * updated in place. */
tdfe_status tdfe_propagate(tdfe_ctx* ctx, void* dev_psibar, int n_orb, int n_steps, double dt, const double* host_E,
                           double tol, double* dev_mu, tdfe_step_report* rep);

/* Excitations and observables (Sec. on the numerical studies and its table
 * of simulation parameters; Eq. VField).
 *
 * set_field_direction: d (HOST double[3], finite, not zero) of the field
 * potential V_field = -E_n (d . r) used by later magnus_step and
 * dipole_gradient calls and by tdfe_kick; used as given (a unit vector makes
 * E_n the field strength).  Default (0, 0, 1).
 *
 * kick: psibar <- exp(-i kappa d . r) psibar at the DoF nodes for n_orb
 * orbitals: the delta kick that excites a linear-response run.  It is the
 * impulse of the field E(t) = -kappa delta(t) in V_field.
 *
 * field_samples (host only, no context): out[i] = E(t[i]) for
 *   TDFE_FIELD_GAUSSIAN  params {kappa, t0, w}:  kappa exp(-(t - t0)^2 / w^2)
 *   TDFE_FIELD_SIN2      params {kappa, omega, T}: kappa sin^2(pi t / T) sin(omega t)
 *                        on [0, T], 0 outside.
 * A Magnus step from t_{n-1} holds the field at the step's midpoint,
 * E_n = E(t_{n-1} + dt / 2).  EINVAL for an unknown shape, non-finite
 * parameters, w <= 0 or T <= 0.
 *
 * absorption_spectrum: S(w_k) = (2 w_k / 3 pi) sum_a Im[mu~_a(w_k) / E~_a(w_k)]
 * for dev_omega[k], k < n_omega, written to dev_S[k].  dev_mu is [3][n_t]
 * FP64 device: row a holds the a-component of the dipole, sampled at
 * t_n = n dt (t_0 = 0 the excitation), of the run excited along axis a.
 *   mu~_a(w) = sum_n c_n e^{i w t_n} e^{-alpha t_n^2} (mu_a(t_n) - mu_a(0)) dt,
 *   E~_a(w)  = sum_n c_n e^{i w t_n} E_a(t_n) dt          (dev_field [3][n_t]),
 *            = -kappa                                      (dev_field NULL: kick),
 * c_n the trapezoid weights (1/2 at both ends).  alpha >= 0 is the Gaussian
 * window.  Enqueued on hip_stream; no context; EINVAL for n_t < 2, dt <= 0,
 * alpha < 0, a zero kick without field samples, null pointers.
 *
 * power_spectrum: P(w_k) = Im sum_{n=1}^{n_t-2} c_n e^{-i w_k t_n} mu''_n dt with
 * mu''_n = (mu_{n+1} - 2 mu_n + mu_{n-1}) / dt^2 and trapezoid weights over
 * n = 1 .. n_t - 2: the dipole power spectrum of a strong-field run from one
 * dipole component sampled at t_n = n dt (dev_mu [n_t]).  EINVAL for
 * n_t < 3, dt <= 0, null pointers. */
#define TDFE_FIELD_GAUSSIAN 1
#define TDFE_FIELD_SIN2 2
tdfe_status tdfe_set_field_direction(tdfe_ctx* ctx, const double* dir);
tdfe_status tdfe_kick(tdfe_ctx* ctx, void* dev_psibar, int n_orb, double kappa);
tdfe_status tdfe_field_samples(int shape, const double* params, int n, const double* t, double* out);
tdfe_status tdfe_absorption_spectrum(const double* dev_mu, const double* dev_field, int n_t, double dt, double kappa,
                                     double alpha, const double* dev_omega, int n_omega, double* dev_S,
                                     void* hip_stream);
tdfe_status tdfe_power_spectrum(const double* dev_mu, int n_t, double dt, const double* dev_omega, int n_omega,
                                double* dev_P, void* hip_stream);

/* A priori mesh (Sec. "Efficient spatio-temporal discretization", Eqs.
 * OptimalMeshMin, OptimalMeshSize): the element size h(r) = E g(r)^(-1/(p+3))
 * that minimises the dipole-error bound at a fixed element count, with
 *   g = sum over atoms of 2 Dbar^{p+1} phi + Dbar^{p+3} phi + Dbar^{p+1} V,
 *   Dbar^k f = sum over multi-indices |l| = k of |D^l f|,
 * phi = (pi s^2)^(-3/4) exp(-|r-R|^2/(2 s^2)) and V = -Z exp(-|r-R|^2/(2 a^2))
 * standing in for the atom's ground-state orbital and potential, and E from
 * int dr / h^3 = n_elem.  The mesh is rectilinear (no hanging nodes, so M
 * stays diagonal and the box kernels and the exact Hartree solver apply):
 * along each axis the spacing is the smallest h over the plane through the
 * point, h_a(s) = E (max over the plane of g)^(-1/(p+3)), sampled on a
 * uniform grid of samples^3 points of [lo, hi]^3; n_a = max(1, floor(c I_a
 * + 1/2)) cells with I_a = int ds / h_a (trapezoid rule) and
 * c^3 I_x I_y I_z = n_elem; the vertices equidistribute int ds / h_a
 * (linear inversion between samples).  The sampling runs on the GPU (one
 * thread per sample point; plane maxima and the count integral by fixed-order
 * block reductions), the 1D steps on the host.
 *
 * adaptive_axes_query: *bytes = device scratch for the call (about
 * 8 samples^3 bytes).
 * adaptive_axes: host_axes is [3][max_cells + 1]: row a receives the
 * n_a + 1 vertex coordinates of axis a (x, y, z), host_ncell[3] the counts,
 * *host_E (may be NULL) the constant E.  dev_scratch: caller-owned, 256-byte
 * aligned, >= the queried size.  Synchronises hip_stream.  EINVAL for a bad
 * description (p outside 1..8, hi <= lo, no atoms or more than
 * TDFE_MAX_ATOMS_MESH, non-positive widths, n_elem < 1, samples outside
 * 3..1024); ENOMEM if the scratch is too small or an axis needs more than
 * max_cells cells.  The vertices of fe_mesh_setup are then the tensor
 * product of the three axes (x fastest). */
#define TDFE_MAX_ATOMS_MESH 4096
typedef struct {
  int p;                /* element order the mesh is for */
  double lo, hi;        /* domain [lo, hi]^3 */
  int n_atoms;
  const double* R;      /* HOST [n_atoms][3] positions */
  const double* Z;      /* HOST [n_atoms] potential depths */
  const double* s_orb;  /* HOST [n_atoms] orbital widths */
  const double* a_pot;  /* HOST [n_atoms] potential widths */
  double n_elem;        /* target number of elements */
  int samples;          /* sample points per axis */
} tdfe_adapt_desc;
tdfe_status tdfe_adaptive_axes_query(const tdfe_adapt_desc* d, size_t* bytes);
tdfe_status tdfe_adaptive_axes(const tdfe_adapt_desc* d, void* dev_scratch, size_t scratch_bytes, void* hip_stream,
                               int max_cells, double* host_axes, int* host_ncell, double* host_E);

/* adaptive_axes_static: tdfe_adaptive_axes for callers that cannot allocate
 * device memory (serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results, with the scratch in a device array of
 * TDFE_AXES_STATIC_BYTES inside the library (one copy per GPU, held from the
 * library's load until the process ends).  No hipMalloc, hipFree or other
 * allocating call is made.  The array's address on the current device is
 * looked up on the first call with that device current; hip_stream must
 * belong to the current device.  Calls that overlap on one GPU (concurrent
 * streams or host threads) share the array and race; serialise them.
 * Synchronises hip_stream.  Errors: TDFE_EINVAL as tdfe_adaptive_axes;
 * TDFE_ENOMEM if the description needs more scratch than the array holds
 * (tdfe_adaptive_axes_query bytes > TDFE_AXES_STATIC_BYTES, i.e. samples
 * above 160) or an axis needs more than max_cells cells; TDFE_EDEVICE if the
 * array's address cannot be obtained. */
#define TDFE_AXES_STATIC_BYTES (32u * 1024u * 1024u)
tdfe_status tdfe_adaptive_axes_static(const tdfe_adapt_desc* d, void* hip_stream, int max_cells, double* host_axes,
                                      int* host_ncell, double* host_E);

/* Octree meshes with hanging nodes (Sec. "Efficient spatio-temporal
 * discretization": adaptive hexahedra that follow h(r) = E g(r)^(-1/(p+3))
 * of Eq. OptimalMeshSize).  Cell (level q, i, j, k) is the cube of edge
 * (hi - lo) / (n0 2^q) with lowest corner lo + (i, j, k) times that edge.
 *
 * octree_leaves: [lo, hi]^3 starts as n0^3 cubes; a cube of edge s is split
 * into its 8 octants while s > E (largest g over its 27 sample points:
 * corners, edge and face midpoints, centre)^(-1/(p+3)), at most max_level
 * times (E and g as for tdfe_adaptive_axes: E from the samples^3 grid); then
 * leaves that share a face, an edge or a corner are brought within one level
 * of each other by splitting the coarser.  g runs on the GPU, the decisions on
 * the host.  host_leaves receives n_leaf rows {q, i, j, k} in ascending
 * lexicographic order, host_E the constant E.  octree_leaves_query gives the
 * scratch bytes for max_leaves.  Synchronises hip_stream.  EINVAL for a bad
 * description (as tdfe_adaptive_axes, or n0 outside 1..64, max_level outside
 * 0..10); ENOMEM if the scratch is too small or the tree needs more than
 * max_leaves leaves. */
tdfe_status tdfe_octree_leaves_query(const tdfe_adapt_desc* d, int max_leaves, size_t* bytes);
tdfe_status tdfe_octree_leaves(const tdfe_adapt_desc* d, int n0, int max_level, void* dev_scratch,
                               size_t scratch_bytes, void* hip_stream, int max_leaves, int* host_leaves,
                               int* host_n_leaf, double* host_E);

/* fe_octree_setup: a context on the leaves of an octree (any leaf list that
 * tiles [lo, hi]^3 with neighbours -- across faces, edges and corners --
 * within one level; e.g. from tdfe_octree_leaves), in place of
 * tdfe_fe_mesh_setup.  Order-p GLL nodes of all leaves are merged by
 * position; a node on the closed boundary of a leaf that does not own it
 * (hanging) takes that leaf's polynomial value there (the tensor Lagrange
 * interpolant of its face or edge nodes), chains of such constraints are
 * substituted and masters on the domain boundary (Dirichlet) drop out.  The
 * DoFs are the remaining interior nodes, numbered by position (x slowest,
 * then y, then z); C maps DoF values to all nodes.  The overlap is lumped:
 * M_d = sum over nodes m of C_md N_m with N_m the GLL-rule mass of node m,
 * which keeps the GLL quadrature of every function of the constrained space
 * exact, and Hbar = M^-1/2 C^T H_nodes C M^-1/2.  Cells are numbered in the
 * order given; per-point arrays are [n_cell][nq^3] as for other meshes.
 * Supported afterwards: query, bind_workspace, dof_coords, quad_coords,
 * mass_diag, set_potential, apply_H, apply_H_add, lanczos_expm, density,
 * dipole, kick, set_field_direction, and magnus_step / propagate with a
 * fixed potential plus the field (set_scf may set occupations only).  EINVAL
 * from set_scf with Hartree or XC, set_projectors with projectors,
 * gradient_query and dipole_gradient; apply_H_add_f32 needs a mixed context,
 * which octree meshes do not have.  The device arrays (cell node lists, C and
 * C^T, two node work arrays of min(64, max(2 chunk, 2 n_orb_max)) columns)
 * live in the workspace.  EINVAL for p outside 1..8, n0 outside 1..64,
 * max_level outside 0..10, leaves that do not tile the domain or are not
 * balanced, precision other than TDFE_FP64, or a non-positive lumped
 * overlap. */
typedef struct {
  int p;             /* element order, 1..8 */
  double lo, hi;     /* domain [lo, hi]^3 */
  int n0;            /* root cubes per axis */
  int max_level;     /* finest level any leaf may have */
  int n_leaf;
  const int* leaves; /* HOST [n_leaf][4] = {q, i, j, k} */
  int n_orb_max;
  int k_max;
  int precision;     /* TDFE_FP64 */
} tdfe_octree_desc;
tdfe_status tdfe_fe_octree_setup(const tdfe_octree_desc* d, void* hip_stream, tdfe_ctx** out);
/* octree_info: counts of an octree context: all nodes, hanging nodes and
 * non-zeros of C (any pointer may be NULL); EINVAL on other contexts. */
tdfe_status tdfe_octree_info(const tdfe_ctx* ctx, int64_t* n_nodes, int64_t* n_hanging, int64_t* nnz);

/* gradient_query: device workspace bytes that tdfe_dipole_gradient needs for
 * n_orb orbitals, n_steps steps, a state checkpoint every checkpoint_every
 * steps and Krylov bases of up to k_store vectors (a multiple of 8, at most
 * k_max).  Memory grows as
 *   (n_steps/checkpoint_every + checkpoint_every + 8) states of n_dof x n_orb complex128
 *   + n_steps Gauss-point arrays + 3 k_store n_orb complex Gauss-point arrays. */
tdfe_status tdfe_gradient_query(tdfe_ctx* ctx, int n_orb, int n_steps, int checkpoint_every, int k_store,
                                size_t* bytes);

/* dipole_gradient: L = mu_z(psibar^N) after n_steps magnus_step steps from
 * dev_psibar0 with the field amplitudes host_E[n_steps] (V_field = -E_n (d . r)
 * on step n with d the field direction, z unless set; Eq. VField; Magnus step
 * as in tdfe_magnus_step, Eqs. ApproxMagnus,
 * PsiTimeDiscrete), and host_grad[n] = dL/dE_n of that discrete scheme
 * (reverse mode: exact adjoints of the density, Hartree, exchange and
 * extrapolation steps; the exponential's Frechet derivative is taken in the
 * Krylov spaces of the forward and adjoint Lanczos runs, exactly for their
 * tridiagonal matrices).  The paper propagates forward only; this is an
 * extension for optimal-control uses of the same step.
 *  - dev_psibar0 [n_dof][n_orb] complex128 is read, never written; the SCF
 *    history used by tdfe_magnus_step is left untouched (this call starts
 *    from W_{-1} = W_0 = W[rho(psibar0)]), and the operator potential is the
 *    external one again on return.
 *  - dev_work: >= tdfe_gradient_query bytes, 256-byte aligned, caller-owned.
 *  - n_orb must fit one Lanczos chunk (every n_orb <= n_orb_max does unless
 *    the Krylov basis of n_orb_max orbitals exceeds the chunk limit stated
 *    at tdfe_fe_mesh_setup); Hartree needs a box mesh;
 *    XC must be none or LDA exchange.
 *  - TDFE_EINVAL if a Lanczos run needs more than k_store vectors,
 *    TDFE_ENOCONV if one does not converge within k_max, TDFE_ENONFINITE
 *    if psibar0 has a non-finite entry (its norm is not finite) or a Lanczos
 *    coefficient or the gradient becomes non-finite.
 *  Synchronises the stream. */
tdfe_status tdfe_dipole_gradient(tdfe_ctx* ctx, const void* dev_psibar0, int n_orb, int n_steps,
                                 const double* host_E, double dt, double tol, int checkpoint_every,
                                 int k_store, void* dev_work, size_t work_bytes, double* host_L,
                                 double* host_grad);

/* text of the last error on this context (never NULL) */
const char* tdfe_last_error(const tdfe_ctx* ctx);

void tdfe_destroy(tdfe_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* TDFE_H */
