// Internal declarations of the tdfe HIP library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/tdfe.h"

#define TDFE_MAXN 9  // p <= 8

// one Krylov chunk holds at most this many real columns (2 per orbital)
#define TDFE_MAX_COLS 64
// a soft-capped chunk runs only with a cap of at least this many vectors and
// at least twice the largest Krylov dimension seen
#define TDFE_SOFT_CAP_MIN 32

struct tdfe_ctx {
  // ---- configuration -------------------------------------------------------
  int p = 0, n = 0, nq = 0;
  int ncx = 0, ncy = 0, ncz = 0;
  int64_t n_cell = 0, n_dof = 0, n_quad = 0, n_nodes = 0;
  int Nx = 0, Ny = 0, Nz = 0;
  int n_orb_max = 0, k_max = 0, precision = TDFE_FP64;
  bool box = false;  // rectilinear grid: axis-aligned cells
  // operator kernel choice (TDFE_APPLY_VARIANT at creation): 0 default policy
  // (see tdfe_launch_apply), 1 "line" everywhere, 2 "pair" for box cells of
  // even n in both precisions, 3 "plane" kernels wherever they exist
  int variant = 0;
  // the cell operator's contractions on the matrix cores (precision
  // TDFE_FP32_MFMA, TDFE_BF16_MFMA or TDFE_FP64_MFMA; box meshes)
  bool mfma = false;
  double* mfma_tab = nullptr;  // [6][16][16] stacked 1D tables
  hipStream_t stream = nullptr;
  std::string err;

  // ---- host tables ---------------------------------------------------------
  double xi[TDFE_MAXN], w[TDFE_MAXN];    // GLL nodes / weights
  double eta[TDFE_MAXN], wq[TDFE_MAXN];  // Gauss points / weights
  double B[TDFE_MAXN * TDFE_MAXN];       // B[a*n+i] = l_i(eta_a)
  double D[TDFE_MAXN * TDFE_MAXN];       // D[a*n+i] = l_i'(eta_a)
  double Dg[TDFE_MAXN * TDFE_MAXN];      // Dg[a*nq+b] = derivative at eta_a of the Gauss-point Lagrange basis b
  std::vector<double> vertices;          // (ncx+1)(ncy+1)(ncz+1)*3
  // box grids: the vertex coordinates along each axis; curved grids (after
  // set_scf with Hartree): their means over the other two indices, the
  // rectilinear stand-in mesh of the Hartree preconditioner
  std::vector<double> ax_x, ax_y, ax_z;

  // ---- workspace ------------------------------------------------------------
  char* ws = nullptr;
  size_t ws_bytes = 0, ws_need = 0;
  int chunk_orb = 0;  // orbitals per Krylov chunk
  // widest chunk the workspace holds with a soft cap on the Krylov dimension:
  // w orbitals fit (k_max + 1) chunk_orb / w - 1 basis vectors in the same
  // memory (operator output, partials and Bessel tables sized for w)
  int wide_orb = 0;
  int k_seen = 0;  // largest Krylov dimension of the last exponentials (0: none yet)

  // device pointers into the workspace
  double* tab = nullptr;      // device copy of the 1D tables (see tab_* offsets)
  double* minv = nullptr;     // [n_dof] M^-1/2
  float* minv32 = nullptr;    // [n_dof] FP32 copy (mixed contexts)
  double* mdiag = nullptr;    // [n_dof] M
  double* dofxyz = nullptr;   // [n_dof][3]
  double* nodexyz_ptr = nullptr;  // [n_nodes][3]
  double* m1x = nullptr;      // box: 1D M^-1/2 factors [Nx], [Ny], [Nz]
  double* m1y = nullptr;
  double* m1z = nullptr;
  double* cellgeo = nullptr;  // box: [n_cell][4] = {detJ*4/hx^2, .../hy^2, .../hz^2, detJ}
  double* corners = nullptr;  // [n_cell][8][3] (z-corner slowest, x fastest)
  double* xq = nullptr;       // [n_cell][nq^3][3]
  double* wdet = nullptr;     // [n_cell][nq^3] varpi_q detJ_q
  double* vext = nullptr;     // [n_cell][nq^3]
  double* vw = nullptr;       // [n_cell][nq^3] weighted total potential used by apply
  float* vw32 = nullptr;      // FP32 copy for the mixed path
  double* w1 = nullptr;       // W_{n-1}  (unweighted, [n_cell][nq^3])
  double* w2 = nullptr;       // W_{n-2}
  double* w3 = nullptr;       // W_{n-3}
  double* wn = nullptr;       // self-consistent midpoint: W_n of the current iterate
  double* scbuf = nullptr;    // [512] self-consistent midpoint: block maxima of the change
  double* wh = nullptr;       // W_{n-1/2}
  double* rho = nullptr;      // [n_cell][nq^3]
  double* phi = nullptr;      // [n_nodes] Hartree potential, boundary values included
  double* cload = nullptr;    // [n_nodes] load vector c_j
  double* fb = nullptr;       // [n_nodes] boundary values f (0 inside)
  double* lift = nullptr;     // [n_dof] (K f)_interior
  double* fdmS = nullptr;     // 1D eigenvector matrices Sx, Sy, Sz (row-major, n1 x n1), then their transposes
  double* fdmL = nullptr;     // 1D eigenvalues
  double* t0 = nullptr;       // [n_dof] scratch
  double* t1 = nullptr;       // [n_dof] scratch
  double* pcg = nullptr;      // 5 x [n_nodes] (r, z, p, Ap, x) for curved meshes
  double* dinvK = nullptr;    // [n_nodes] inverse stiffness diagonal (interior), 0 on boundary
  double* pcgs = nullptr;     // [16] CG scalars (rz, rr, bb, alpha, beta, pAp)
  void* krylov = nullptr;     // (k_max+1) x [n_dof][2 chunk_orb]
  void* hq = nullptr;         // [n_dof][2 max(chunk_orb, wide_orb)] apply output
  void* half = nullptr;       // [n_dof][2 n_orb_max] predictor state (complex128)
  double* partial = nullptr;  // reduction partials
  double* partial2 = nullptr; // [128][TDFE_MAX_COLS] first level of the two-level alpha reduction
  double* scal = nullptr;     // per-orbital Lanczos scalars
  double* jtab = nullptr;     // [max(chunk_orb, wide_orb)][TDFE_JTAB_STRIDE] Bessel tables of the small exponential
  unsigned* counters = nullptr;
  int64_t n_partial = 0;

  // host pinned poll buffer
  int* poll = nullptr;
  int flag_gen = 0;  // generation number of the Lanczos convergence flag (poll[32])
  void* blas = nullptr;        // rocBLAS handle on `stream` (fast diagonalisation along axes > 128 nodes)
  // rocBLAS solution of each fast-diagonalisation pass [axis][transposed],
  // chosen by timing at its first use (tuned: 0 not yet, 1 chosen)
  int fdm_tuned[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  int fdm_algo[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  int fdm_sol[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  hipEvent_t* evs = nullptr;  // [TDFE_N_EVENTS] look-ahead polling points
  int n_evs = 0;

  // ---- state -------------------------------------------------------------------
  bool bound = false, have_potential = false, have_scf = false, scf_init = false;
  int hartree = 0, xc = 0;
  std::vector<double> nucZ, nucR, occ, occ_host;
  int occ_ver = 0, occ_dev_ver = -1, occ_dev_n = -1;  // device copy of the occupations is current when equal
  double pcg_tol = 1e-13;
  int pcg_maxit = 5000;
  int pcg_precond = TDFE_PCG_FDM;  // curved meshes: CG preconditioner
  int last_poisson_iters = 0;
  double fdir[3] = {0.0, 0.0, 1.0};  // field direction d: V_field = -E_n (d . r)
  int mid_mode = TDFE_MIDPOINT_PC, mid_order = 1;  // midpoint Hamiltonian of the Magnus step
  double sc_tol = 1e-10;
  int sc_maxit = 50;
  // Kleinman-Bylander term: caller-owned store of the projector tables, off when n_proj == 0
  int n_proj = 0;
  void* nl_store = nullptr;
  int nl_groups = 0, nl_blocks = 0;  // projector groups (shared boxes) and blocks of the hot passes
  int nl_np_max = 0;                 // most projectors in one group
  int nl_lines = 0, nl_add_blocks = 0;  // grid lines crossed by boxes; segments (blocks) of the add pass
  int64_t nl_line_dofs = 0;                             // DoFs on those lines (x ranges)
  int64_t nl_packed = 0;             // stored entries of Cbar
  int64_t nl_box_dofs = 0;           // DoFs in the groups' boxes (summed over groups)

  // ---- octree meshes (tdfe_octree.hip) -------------------------------------------------------
  // host tables built at setup and copied into the workspace at bind; n_nodes
  // counts every merged GLL node (hanging and boundary ones included)
  bool octree = false;
  int oct_w = 0;  // real columns of the node work arrays
  int64_t oct_hanging = 0;
  std::vector<int> oct_cn_h;                 // [n_cell][n^3] node of every cell node (x fastest)
  std::vector<double> oct_s_h;               // [n_cell] cube edge
  std::vector<int> oct_eptr_h, oct_ecol_h;   // C: rows over nodes (DoF columns)
  std::vector<double> oct_eval_h;
  std::vector<double> oct_m_h, oct_dofxyz_h, oct_xq_h, oct_wdet_h;
  int* oct_cn = nullptr;
  double* oct_s = nullptr;
  int* oct_eptr = nullptr;
  int* oct_ecol = nullptr;
  double* oct_eval = nullptr;
  double* oct_xf = nullptr;  // [n_nodes][oct_w] expanded input (density; the operator's hanging values)
  double* oct_yf = nullptr;  // [n_nodes][oct_w] the operator's hanging-node output before C_h^T
  // the operator's view: per cell node slot its DoF index, -1 (boundary, or a
  // hanging node without interior masters: value 0) or -2 - h for hanging
  // node h; the hanging nodes' node indices; C^T restricted to the hanging
  // rows, by master DoF
  std::vector<int> oct_cd_h, oct_hv_h, oct_mptr_h, oct_md_h, oct_mh_h;
  std::vector<double> oct_mv_h;
  int* oct_cd = nullptr;
  int* oct_hv = nullptr;
  int* oct_mptr = nullptr;
  int* oct_md = nullptr;
  int* oct_mh = nullptr;
  double* oct_mv = nullptr;
};

// error helpers ----------------------------------------------------------------
tdfe_status tdfe_fail(tdfe_ctx* c, tdfe_status s, const char* fmt, ...);
#define TDFE_HIP(ctx, call)                                                          \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return tdfe_fail((ctx), TDFE_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)
#define TDFE_TRY(x)                      \
  do {                                   \
    tdfe_status s_ = (x);                \
    if (s_ != TDFE_OK) return s_;        \
  } while (0)

// layout of the device table block ----------------------------------------------
// tab[TAB_B + a*n + i], tab[TAB_D + ...], tab[TAB_DG + a*nq + b], tab[TAB_W3Q + q]
#define TAB_B 0
#define TAB_D (TDFE_MAXN * TDFE_MAXN)
#define TAB_DG (2 * TDFE_MAXN * TDFE_MAXN)
#define TAB_ETA (3 * TDFE_MAXN * TDFE_MAXN)
#define TAB_WQ (TAB_ETA + TDFE_MAXN)
#define TAB_W3Q (TAB_WQ + TDFE_MAXN)
#define TAB_SIZE (TAB_W3Q + TDFE_MAXN * TDFE_MAXN * TDFE_MAXN)

// operator launchers (tdfe_apply.hip) ------------------------------------------------
// y += kin-Laplacian-plus-potential applied to x on the DoF numbering, for
// `cols` real columns stored [n_dof][ld].  colscale[col/2] (may be NULL)
// scales the gathered input per orbital pair.  energy (may be NULL) receives
// per-block partial sums of x^T H x per column (layout [block][cols]).
struct ApplyArgs {
  const void* x;
  void* y;
  int ld;
  int cols;
  const double* colscale;
  double kin;           // 0.5 for H, 1.0 for K
  const double* vw;     // weighted potential or NULL
  const float* vw32;
  bool lowdin;          // scale by M^-1/2 on gather and scatter
  bool fullgrid;        // x / y are full node arrays (stiffness mode)
  double* energy;       // partials or NULL
  int64_t* n_blocks_out;
  const int* done_flag; // early-exit flag (device) or NULL
  bool fp32;            // x, y stored as float
  bool nonlocal;        // Hbar launches: add the Kleinman-Bylander term when projectors are set
};
tdfe_status tdfe_launch_apply(tdfe_ctx* c, const ApplyArgs& a);
// rectilinear-cell variant (tdfe_apply_box.hip), used by tdfe_launch_apply
bool tdfe_box_kernel_ok(const tdfe_ctx* c);
tdfe_status tdfe_launch_apply_box(tdfe_ctx* c, const ApplyArgs& a);
// lane-pair variant for box cells of even n (tdfe_apply_pair.hip)
bool tdfe_pair_kernel_ok(const tdfe_ctx* c);
tdfe_status tdfe_launch_apply_pair(tdfe_ctx* c, const ApplyArgs& a);
// trilinear-cell variant in the same layout (tdfe_apply_curved.hip)
bool tdfe_curved_kernel_ok(const tdfe_ctx* c, int cols, bool fp32);
#define TDFE_VARIANT_LINE 1
#define TDFE_VARIANT_PAIR 2
#define TDFE_VARIANT_PLANE 3
tdfe_status tdfe_launch_apply_curved(tdfe_ctx* c, const ApplyArgs& a);
// matrix-core variant for box cells (tdfe_apply_mfma.hip)
bool tdfe_mfma_kernel_ok(const tdfe_ctx* c, const ApplyArgs& a);
tdfe_status tdfe_launch_apply_mfma(tdfe_ctx* c, const ApplyArgs& a);
void tdfe_mfma_tables(int p, double* out);  // host: [6][16][16]
// FP32 Krylov storage and operator (mixed precision and its matrix-core variants)
inline bool tdfe_fp32(const tdfe_ctx* c) {
  return c->precision == TDFE_MIXED_FP32 || c->precision == TDFE_FP32_MFMA || c->precision == TDFE_BF16_MFMA;
}
// Krylov dimension that a chunk of w orbitals can reach in the basis memory
// of chunk_orb orbitals at k_max: (k_max + 1) chunk_orb / w - 1 vectors past
// the first, at most k_max
inline int tdfe_soft_cap(const tdfe_ctx* c, int w) {
  const long long v = (long long)(c->k_max + 1) * c->chunk_orb / (w > 0 ? w : 1) - 1;
  return (int)(v < c->k_max ? v : c->k_max);
}
// nonlocal term after the local kernel (tdfe_nonlocal.hip): Loewdin launches
// on the DoF numbering only; appends one row to the energy partials
tdfe_status tdfe_launch_nonlocal(tdfe_ctx* c, const ApplyArgs& a);

// mixed precision: floor of the Lanczos stop tolerance relative to ||psibar||
// (16 units of FP32 roundoff)
#define TDFE_MIXED_TOL_FLOOR (16.0 / 16777216.0)

// events for the host's look-ahead polling of device convergence flags (created once per context)
#define TDFE_N_EVENTS 16
tdfe_status tdfe_poll_events(tdfe_ctx* c);

// vector kernels (tdfe_lanczos.hip)
// zero fill of a word-aligned device range (a kernel, not hipMemsetAsync)
tdfe_status tdfe_zero(tdfe_ctx* c, void* p, size_t bytes);
// pinned readback area: ints [TDFE_READBACK_OFFSET_INTS, 4096) of c->poll
#define TDFE_READBACK_OFFSET_INTS 1024
#define TDFE_READBACK_BYTES (3072 * 4)
// enqueue a copy of `bytes` device bytes to readback offset `off`; *host is
// valid after the stream has been synchronised
tdfe_status tdfe_readback(tdfe_ctx* c, const void* dev_src, size_t bytes, size_t off, const void** host);
// called once per orbital chunk after the adaptive loop (before the combination):
// W = basis storage (k_max+1 vectors of vstride elements, float if fp32),
// scale[j*Nc+o] = 1/beta_{j}, kconv/alpha/beta/nrm as in the Lanczos scalar block
struct LanczosHook {
  virtual tdfe_status after_loop(tdfe_ctx* c, const void* W, int64_t vstride, int Nc, int o0, const double* scale,
                                 const int* kconv, const double* alpha, const double* beta, const double* nrm,
                                 int k_enqueued, bool fp32) = 0;
  virtual ~LanczosHook() {}
};
// defer = 0 or 1: leave the per-orbital results (k, status, error estimate)
// in device result slot `defer` and return without synchronising; the caller
// enqueues tdfe_lanczos_enqueue_results, synchronises the stream once and
// calls tdfe_lanczos_results (host outputs and hook must then be null)
tdfe_status tdfe_lanczos_run(tdfe_ctx* c, const double* vw, const void* in, void* out, int n_orb,
                             double tau, double tol, int* k_out, double* err_out, int* kmax_out,
                             int* ksum_out, double* errmax_out, LanczosHook* hook = nullptr, int defer = -1);
bool tdfe_lanczos_can_defer(const tdfe_ctx* c);
// device address of deferred result slot 0/1: k, status, error estimate per
// orbital ([n_orb_max] each, as doubles) and the table-overflow flag
double* tdfe_lanczos_result_slot(tdfe_ctx* c, int slot);
tdfe_status tdfe_lanczos_enqueue_results(tdfe_ctx* c, int slot, const void** host);
tdfe_status tdfe_lanczos_results(tdfe_ctx* c, const void* host, int n_orb, double tol, int* kmax_out,
                                 int* ksum_out, double* errmax_out);

// scf kernels (tdfe_scf.hip)
tdfe_status tdfe_density_dev(tdfe_ctx* c, const void* psibar, int n_orb, double* rho, double* partial3);
tdfe_status tdfe_dipole_dev(tdfe_ctx* c, const double* rho, double mu[3], double* charge);
tdfe_status tdfe_scf_potential(tdfe_ctx* c, const void* psibar, int n_orb, double* w_out,
                               double* mu, double* charge);
// the same, without synchronising: *host_red (if not null) receives the
// readback address of {charge, mu_x, mu_y, mu_z}, valid after a stream sync
tdfe_status tdfe_scf_potential_async(tdfe_ctx* c, const void* psibar, int n_orb, double* w_out,
                                     const void** host_red);
tdfe_status tdfe_fdm_setup(tdfe_ctx* c);
tdfe_status tdfe_compute_lift(tdfe_ctx* c);
// c->cload = sum_e I^T (w f), w = varpi detJ if weighted else 1 (full grid, zeroed first)
tdfe_status tdfe_load_vector(tdfe_ctx* c, const double* f, bool weighted);
// interior of phi_full <- K00^-1 (4 pi c_interior [- lift]); boundary entries untouched
tdfe_status tdfe_fdm_solve_into(tdfe_ctx* c, bool with_lift, double* phi_full);
void tdfe_blas_destroy(tdfe_ctx* c);
// out_q = phi(x_q) [+ V_xc(rho_q)] for a full-grid nodal field phi
tdfe_status tdfe_interp_field(tdfe_ctx* c, const double* phi_full, const double* rho, int xcmode, double* out);
// device array of the occupations f_alpha for n_orb orbitals
tdfe_status tdfe_occ_dev(tdfe_ctx* c, int n_orb, const double** dev);
// c->vw (and c->vw32 in mixed contexts) = wdet (vext - E z + ca A + cb B); A, B may be null
tdfe_status tdfe_assemble_vw(tdfe_ctx* c, const double* A, double ca, const double* B, double cb, double E);
// host symmetric eigen-decomposition A = U diag(lam) U^T (row-major n x n, U[i*n+k] = k-th vector)
void tdfe_sym_eigen(const std::vector<double>& A, int n, std::vector<double>& lam, std::vector<double>& U);

// octree meshes (tdfe_octree.hip): the operator as C^T (cell operators) C in
// the Loewdin scaling, the density at the Gauss points with the same 4
// partial sums per cell as the structured density kernel, and the upload of
// the host tables at bind
tdfe_status tdfe_launch_apply_octree(tdfe_ctx* c, const ApplyArgs& a);
tdfe_status tdfe_octree_density(tdfe_ctx* c, const double* psibar, int n_orb, const double* occ, double* rho,
                                double* partial4);
tdfe_status tdfe_octree_bind(tdfe_ctx* c);

// workspace carving (tdfe_setup.hip)
int64_t tdfe_blocks_apply(const tdfe_ctx* c, int cols);
