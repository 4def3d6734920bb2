/*
 * fsi.h - C ABI of the MI355X (gfx950) library for the Jacobian hot path of
 * the fully implicit, monolithic fictitious-domain / distributed-Lagrange-
 * multiplier (FD/DLM) immersed FSI method of arXiv 2601.08266.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array pointers are DEVICE pointers owned by the caller, unless an argument
 *   says "host".  The library never allocates, frees or retains caller memory.
 * - Work that needs scratch memory takes an explicit workspace (ws, ws_bytes)
 *   whose minimum size the matching *_workspace() query returns; a smaller
 *   workspace is rejected with FSI_ERR_WORKSPACE before anything is launched.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Calls enqueue work on it and return without synchronising, unless the
 *   comment says SYNCS.
 * - Arguments are validated before any launch; a bad argument returns
 *   FSI_ERR_ARG and launches nothing.  A failed HIP call returns FSI_ERR_HIP.
 *   fsi_last_error() returns a thread-local message for the last failure.
 *   No C++ exception crosses the ABI.
 * - Grids are uniform hexahedral: n[d] cells per axis, cell size h[d], origin
 *   x0[d]; Lagrange order p = `order` (1 or 2) for all four fields (the
 *   equal-order velocity/pressure pairs of section 2.1).  Nodes per axis
 *   N_d = p n[d] + 1, node id = i + N_0 (j + N_1 k).  Cells are numbered the
 *   same way with n[d].  Vectors are structure-of-arrays, field-major:
 *   x[f * N + node] with f = 0,1,2 the velocity components and f = 3 the
 *   pressure; velocity-only arrays are [3][N].
 * - Precision: `dtype` selects FP64 (double) or FP32 (float) for the floating
 *   point arrays named "T" below; the same call computes in that precision.
 */
#ifndef FSI_H
#define FSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FSI_OK = 0,
    FSI_ERR_ARG = -1,            /* invalid argument (nothing launched) */
    FSI_ERR_HIP = -2,            /* a HIP runtime call failed */
    FSI_ERR_WORKSPACE = -3,      /* workspace missing or too small */
    FSI_ERR_NOT_CONVERGED = -4,  /* iteration cap reached */
    FSI_ERR_BREAKDOWN = -5,      /* Krylov breakdown */
    FSI_ERR_NAN = -6,            /* NaN/Inf detected in a norm */
    FSI_ERR_UNSUPPORTED = -7     /* valid but not implemented combination */
} fsi_status;

typedef enum { FSI_F64 = 0, FSI_F32 = 1 } fsi_dtype;

typedef struct {
    int32_t n[3];      /* cells per axis, >= 1 */
    int32_t order;     /* 1 (Q1-Q1) or 2 (Q2-Q2) */
    double x0[3];      /* origin of the box */
    double h[3];       /* cell size per axis, > 0 */
} fsi_grid;

/*
 * Parameters of the Oseen-VMS operator (section 2.1, per unit density so the
 * paper's mu/rho is nu):
 *   nu   kinematic viscosity
 *   c_m  mass coefficient of the time discretisation (1/dt for backward Euler)
 *   dt   time step entering tau_m through C_T/dt^2
 *   C_T, C_I  constants of tau_m (4 and 36 in the paper)
 *   visc_strong  nonzero: the strong momentum residual keeps -nu(lap u + grad div u)
 */
typedef struct {
    double nu, c_m, dt, C_T, C_I;
    int32_t visc_strong;
} fsi_vms_params;

/* Static description of a status code (never NULL). */
const char *fsi_status_string(int status);
/* Thread-local message describing the last failure on this thread ("" if none). */
const char *fsi_last_error(void);
/* Library version string. */
const char *fsi_version(void);

/*
 * fsi_vms_apply - y = A(a, s) x, the VMS-stabilised Oseen operator.
 *
 * Section 2.1: the Galerkin weak form (eq. fluid_weak_form) linearised about
 * the advection field a, plus residual-based SUPG, PSPG and grad-div (LSIC)
 * terms with tau_m = (s (C_T/dt^2 + a.G a + C_I nu^2 G:G))^(-1/2),
 * tau_c = (tau_m tr G)^(-1), G_ij = sum_k dxi_k/dx_i dxi_k/dx_j (the
 * stabilisation-parameter equations; reference element [0,1]^3 so G = I/h^2).
 * These are the momentum/continuity blocks of the reduced system of section
 * 2.4.  Gauss quadrature with p+1 points per axis; a and s are interpolated
 * with the element basis, s clamped below by the cell's smallest nodal s.
 *
 *   grid, prm  host pointers
 *   a          T [3][N] advection field (device)
 *   s          T [N] interface scaling field, or NULL for s = 1 (device)
 *   dir_mask   uint32 bitmask over the 3N velocity DOFs (bit k of the stream
 *              = word k/32, bit k%32; k = f*N + node), or NULL.  Masked DOFs
 *              are Dirichlet: their columns are treated as zero and their rows
 *              as the identity (y_k = x_k).
 *   x          T [4][N] input (device);  y  T [4][N] output, overwritten.
 *              y must not overlap x, a or s.
 *   ws         workspace of at least fsi_vms_apply_workspace(grid, dtype) bytes.
 * Deterministic: identical inputs give bitwise identical outputs.
 */
size_t fsi_vms_apply_workspace(const fsi_grid *grid, fsi_dtype dtype);
int fsi_vms_apply(const fsi_grid *grid, const fsi_vms_params *prm, fsi_dtype dtype,
                  const void *a, const void *s, const uint32_t *dir_mask,
                  const void *x, void *y, void *ws, size_t ws_bytes, void *stream);

/*
 * fsi_dlm_locate - find the background cell and parametric position of each
 * solid point, sort the points by cell, and mark the interface band of s.
 *
 * Section 2.3 (eq. nodal_solid_velo evaluates fluid shape functions at the
 * current solid point positions) and appendix A (point search -> element
 * number and parametric position xi -> shape function evaluation).  Cell rule:
 * with breakpoints b_k = x0 + k h (FP64, as written, no fused multiply-add),
 * a coordinate X lies in cell i when b_i <= X <= b_{i+1}; the largest such i
 * is taken; X outside [b_0, b_n] on any axis marks the point outside
 * (cell = -1, not an error).  xi_d = (X_d - (x0_d + i_d h_d)) / h_d, computed
 * in FP64 and stored in `dtype`.
 *
 *   X          double [3][M] point positions (device)
 *   cell       int32 [M] out: cell id or -1
 *   xi         T [3][M] out: parametric position (0 for outside points)
 *   perm       int32 [M] out: point indices sorted by cell, stable (ties keep
 *              increasing point index), outside points last
 *   occ_cell   int32 [E] out: ascending ids of occupied cells (first n_occ used)
 *   occ_start  int32 [E+1] out: perm[occ_start[k] .. occ_start[k+1]) are the
 *              points of occ_cell[k]
 *   occ_index  int32 [E] out: k for the cell occ_cell[k], -1 for empty cells
 *   s_out      T [N] out or NULL: s = s_max on every node of an occupied cell,
 *              1 elsewhere (section 2.1's interface band, O(h) wide)
 *   n_occ_host, n_outside_host  HOST int64 out (may be NULL).  SYNCS the stream.
 *   ws         at least fsi_dlm_locate_workspace(grid, m) bytes.
 * M must be < 2^31 and the number of cells E < 2^31 - 1.
 */
size_t fsi_dlm_locate_workspace(const fsi_grid *grid, int64_t m);
int fsi_dlm_locate(const fsi_grid *grid, int64_t m, const double *X, fsi_dtype dtype,
                   int32_t *cell, void *xi, int32_t *perm, int32_t *occ_cell,
                   int32_t *occ_start, int32_t *occ_index, void *s_out, double s_max,
                   int64_t *n_occ_host, int64_t *n_outside_host,
                   void *ws, size_t ws_bytes, void *stream);

/*
 * fsi_dlm_B - interpolate the fluid velocity at the solid points:
 * (B u)_B = sum_A N_A(xi_B) u_A, per component (section 2.3, eq.
 * nodal_solid_velo; also the solid acceleration increment of section 2.4,
 * Delta U = (C^lambda)^T Delta V).
 *   cell, xi   from fsi_dlm_locate (device); points with cell = -1 give 0
 *   u          T [3][N] (device; the velocity part of a [4][N] vector works)
 *   Bu         T [3][M] out, overwritten
 */
int fsi_dlm_B(const fsi_grid *grid, fsi_dtype dtype, int64_t m, const int32_t *cell,
              const void *xi, const void *u, void *Bu, void *stream);

/*
 * Located order: position j of the cell-sorted point list of fsi_dlm_locate
 * (the points of occupied cell k at occ_start[k] .. occ_start[k+1] - 1, the
 * points outside the grid last), i.e. point perm[j].  Per-point vectors kept
 * in this order are read and written contiguously by fsi_dlm_B_located and by
 * fsi_dlm_BT with perm = NULL; in point order every point costs scattered
 * reads through perm.  A caller whose points move little between steps can
 * keep its per-point arrays in a previous step's located order.
 *
 * fsi_dlm_permute - nf fields of M points, T [nf][M]: to located order
 * (to_point = 0: dst[f][j] = src[f][perm[j]]) or back (to_point = 1:
 * dst[f][perm[j]] = src[f][j]); dst must not alias src.
 *
 * fsi_dlm_B_located - fsi_dlm_B with xi_loc (T [3][M]) and Bu_loc (T [3][M],
 * out) in located order; the points outside the grid get 0.  Bitwise equal
 * to fsi_dlm_B followed by fsi_dlm_permute.
 */
int fsi_dlm_permute(fsi_dtype dtype, int64_t m, int32_t nf, const int32_t *perm, int32_t to_point,
                    const void *src, void *dst, void *stream);
int fsi_dlm_B_located(const fsi_grid *grid, fsi_dtype dtype, int64_t m, const int32_t *occ_cell,
                      const int32_t *occ_start, int64_t n_occ, const void *xi_loc, const void *u,
                      void *Bu_loc, void *stream);

/*
 * fsi_dlm_BT - spread point forces to the fluid nodes:
 * y_A += sum_B N_A(xi_B) kappa_B lam_B, per component (section 2.3, eq.
 * fsi_constraint_matrix: C^lambda_AB = N_A(phi(X_B)) I, "force spreading").
 * Segmented: points are reduced per occupied cell in perm order, then each
 * node gathers the corner sums of its occupied neighbour cells in a fixed
 * order, so the result is deterministic without floating-point atomics.
 *   perm, occ_cell, occ_start, occ_index, n_occ  from fsi_dlm_locate
 *   lam        T [3][M];  kappa  T [M] or NULL (kappa = 1)
 *   y          T [3][N], ACCUMULATED (y += ...)
 *   ws         at least fsi_dlm_BT_workspace(grid, n_occ, dtype) bytes
 * perm = NULL: xi, lam and kappa are given in located order (see
 * fsi_dlm_permute), read without indirection; the result is bitwise that of
 * the point-order call on the same values.
 */
size_t fsi_dlm_BT_workspace(const fsi_grid *grid, int64_t n_occ, fsi_dtype dtype);
int fsi_dlm_BT(const fsi_grid *grid, fsi_dtype dtype, int64_t m, const int32_t *cell,
               const void *xi, const int32_t *perm, const int32_t *occ_cell,
               const int32_t *occ_start, const int32_t *occ_index, int64_t n_occ,
               const void *lam, const void *kappa, void *y, void *ws, size_t ws_bytes,
               void *stream);

/*
 * fsi_dlm_BT_noalloc - fsi_dlm_BT without a workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops that
 * forbid hipMalloc): the per-occupied-cell corner sums go to a scratch array
 * the library holds on each GPU it runs on until the process ends, of
 * fsi_dlm_BT_noalloc_max_bytes() bytes (32 MiB: up to 174,762 occupied Q1
 * cells in FP64, 349,525 in FP32).  Same arguments and result as fsi_dlm_BT
 * in point order (perm non-NULL; bitwise: the same kernels); n_occ whose
 * corner sums exceed the array ->
 * FSI_ERR_WORKSPACE before any device work.  It allocates nothing.  Calls that
 * overlap on one GPU (other streams or threads) share the array and race: keep
 * them in one stream order.
 */
size_t fsi_dlm_BT_noalloc_max_bytes(void);
int fsi_dlm_BT_noalloc(const fsi_grid *grid, fsi_dtype dtype, int64_t m, const int32_t *perm,
                       const void *xi, const int32_t *occ_cell, const int32_t *occ_start,
                       const int32_t *occ_index, int64_t n_occ, const void *lam, const void *kappa,
                       void *y, void *stream);

/*
 * fsi_dlm_gram - per occupied cell o, the block of B^T diag(kappa) B that
 * couples the cell's own (p+1)^3 nodes:
 *   gram[o][A][C] = sum_{B in cell o} kappa_B N_A(xi_B) N_C(xi_B)
 * (section 2.4: the C^lambda dR^s/dU (C^lambda)^T block with the per-point
 * stand-in kappa_B I; B from eq. nodal_solid_velo).  Because every point
 * couples only the nodes of its own cell, B^T diag(kappa) B u is the sum over
 * occupied cells of these blocks applied to the cell's nodal u.  Computed once
 * per point configuration and reused by every Jacobian apply.
 *   xi, perm, occ_start, n_occ  from fsi_dlm_locate; kappa T [M] or NULL (1)
 *   gram       T [n_occ][(p+1)^3][(p+1)^3] out (symmetric, row-major)
 * Deterministic (points summed in cell-sorted order).
 */
int fsi_dlm_gram(const fsi_grid *grid, fsi_dtype dtype, int64_t m, const void *xi,
                 const int32_t *perm, const int32_t *occ_start, int64_t n_occ,
                 const void *kappa, void *gram, void *stream);

/*
 * Mesh and material of the immersed solid for the hyperelastic solid block
 * (fsi_solid_setup / fsi_solid_apply below, which state the operator).
 */
typedef struct fsi_solid {
    int64_t n_nodes;            /* M: solid nodes (= the DLM points) */
    int64_t n_elem;             /* hexahedra */
    const double *X0;           /* [3][M] reference positions (device) */
    const int32_t *conn;        /* [n_elem][8] corner node indices (device); corner
                                   a + 2b + 4c sits at reference (a, b, c) in [0,1]^3 */
    const int32_t *node_start;  /* [M + 1] from fsi_solid_setup (device) */
    const int32_t *node_slot;   /* [8 n_elem] from fsi_solid_setup (device) */
    double C0, kappa_s;         /* eq. inc_neoHk */
    double rho_s0, rho_f, mu_f; /* solid reference density, fluid density and viscosity */
} fsi_solid;

/*
 * Everything the Jacobian of the reduced system needs (section 2.4):
 *   J = A_VMS(a, s) + [[B^T diag(kappa) B, 0], [0, 0]],
 * i.e. the paper's dR^{f,m}/dV + C^lambda dR^s/dU (C^lambda)^T block with the
 * solid tangent replaced by the per-point diagonal stand-in kappa_B I.
 * Dirichlet velocity DOFs (dir_mask) have identity rows and zero columns.
 * All arrays are device pointers in precision `dtype`, except the integer
 * point tables.  m = 0 (no solid) is allowed.  With `solid` set, the solid's own
 * tangent block replaces the per-point stand-in (see the field).
 */
typedef struct {
    fsi_grid grid;
    fsi_vms_params prm;
    fsi_dtype dtype;
    const void *a;             /* T [3][N] */
    const void *s;             /* T [N] or NULL */
    const uint32_t *dir_mask;  /* or NULL */
    int64_t m;                 /* number of solid points */
    const int32_t *cell;       /* [M] */
    const void *xi;            /* T [3][M] */
    const int32_t *perm;       /* [M] */
    const int32_t *occ_cell;   /* [n_occ] */
    const int32_t *occ_start;  /* [n_occ + 1] */
    const int32_t *occ_index;  /* [E] */
    int64_t n_occ;
    const void *kappa;         /* T [M] */
    const void *dlm_gram;      /* T [n_occ][nen][nen] from fsi_dlm_gram, or NULL: then the
                                  DLM block is applied point by point (B, kappa, B^T) */
    const fsi_solid *solid;    /* or NULL.  Set: every apply of this problem (fsi_jacobian_apply,
                                  fsi_fgmres_solve) uses the solid block B^T K_s B of
                                  fsi_jacobian_solid_apply (the points must be the solid's
                                  nodes) instead of B^T diag(kappa) B; kappa and dlm_gram then
                                  only describe the preconditioners' per-point approximation
                                  of that block.  fsi_vms_residual, fsi_tangent_apply and
                                  fsi_newton_solve reject it: the step with the solid's own
                                  residual is fsi_solid_step_residual / fsi_newton_solid_solve. */
    const double *solid_U;     /* double [3][M] solid displacement when solid != NULL */
    double solid_cM, solid_cK, solid_cV;  /* coefficients of K_s (fsi_solid_apply) */
} fsi_problem;

/*
 * fsi_jacobian_apply - y = J x for the problem above (x, y: T [4][N] device;
 * y overlaps neither x nor the problem's arrays).  ws: at least fsi_jacobian_workspace(problem) bytes.
 * Deterministic.
 */
size_t fsi_jacobian_workspace(const fsi_problem *problem);
int fsi_jacobian_apply(const fsi_problem *problem, const void *x, void *y, void *ws,
                       size_t ws_bytes, void *stream);

/*
 * fsi_jacobian_apply_block - the velocity rows of J on one block of the input, the
 * products with J's sub-matrices that the block preconditioners of section 2.4 take
 * (J = [[F, G], [D, C]], velocity rows first):
 *   block FSI_BLOCK_F: y_u = F x_u          = [J (x_u, 0)]_u   (x_p is not read)
 *   block FSI_BLOCK_G: y_u = G x_p          = [J (0, x_p)]_u   (x_u is not read; the DLM
 *                                             block, a function of the velocity, adds nothing)
 * x, y: T [4][N] device, as for fsi_jacobian_apply; only y's velocity part y[0..3N) is
 * written, its pressure part is left as it was.  Dirichlet velocity rows: x_u (block F),
 * 0 (block G).  Same workspace and aliasing rules as fsi_jacobian_apply.  Q1 grids only:
 * FSI_ERR_UNSUPPORTED for Q2.  Deterministic; equal to the corresponding rows of
 * fsi_jacobian_apply on the zero-padded input up to rounding order.
 */
#define FSI_BLOCK_F 1
#define FSI_BLOCK_G 2
int fsi_jacobian_apply_block(const fsi_problem *problem, int32_t block, const void *x, void *y,
                             void *ws, size_t ws_bytes, void *stream);

/*
 * Hyperelastic solid block (section 2.4's C^lambda dR^s/dU (C^lambda)^T with the
 * solid's own tangent in place of the per-point stand-in kappa_B I).  The solid
 * weak form is section 2.2's eq. solid_weak_form, the material the nearly-
 * incompressible neo-Hookean energy of eq. inc_neoHk,
 *   psi = C0/2 (tr Cbar - 3) + kappa_s/2 ((J^2 - 1)/2 - ln J),  Cbar = Fbar^T Fbar,
 *   Fbar = J^{-1/3} F (the isochoric part; the printed exponent +1/3 is read as -1/3),
 * discretised by trilinear hexahedra (2x2x2 Gauss points) whose nodes are the
 * multiplier points (section 2.3: delta functions at the solid nodes).  Applied to
 * solid-node velocities v:
 *   y = c_M M v + c_K K(U) v - c_V K_v(U) v,
 *   M   = int (rho_s0 - rho_f J) N_A N_B dOmega_0  (the inertia term with
 *         rho^s dOmega_t = rho_s0 dOmega_0 and rho^f dOmega_t = rho^f J dOmega_0),
 *   K   = int grad_0 N_A . dP/dF . grad_0 N_B dOmega_0  (P = dpsi/dF, F = I + grad_0 U),
 *   K_v = 2 mu_f int eps(N_A) : eps(N_B) dOmega_t  (the subtracted work of the
 *         artificial fluid, with the solid velocity interpolant, on the current
 *         configuration); the configuration is frozen within a linear solve for M
 *         and K_v.  c_M, c_K, c_V are the integrator's derivatives of the solid
 *         acceleration, displacement and velocity with respect to the new velocity
 *         (backward Euler: 1/dt, dt, 1).
 * Deterministic: element forces are summed per node in ascending element order.
 */


/*
 * fsi_solid_setup - per-mesh table of the element corners around every node
 * (node_start [M+1], node_slot [8 n_elem] = e*8 + c in ascending order), built on
 * the host from conn.  Rejects (FSI_ERR_ARG) any conn entry outside [0, M).
 * SYNCS the stream.
 */
int fsi_solid_setup(int64_t n_nodes, int64_t n_elem, const int32_t *conn, int32_t *node_start,
                    int32_t *node_slot, void *stream);

/*
 * fsi_solid_apply - y = (c_M M + c_K K(U) - c_V K_v(U)) v at the solid nodes.
 *   U        double [3][M] solid displacement (current = X0 + U; device)
 *   v, y     T [3][M] (device, not overlapping); y is overwritten
 *   ws       at least fsi_solid_workspace(n_elem, dtype) bytes
 */
size_t fsi_solid_workspace(int64_t n_elem, fsi_dtype dtype);
int fsi_solid_apply(const fsi_solid *solid, fsi_dtype dtype, const double *U, double cM, double cK,
                    double cV, const void *v, void *y, void *ws, size_t ws_bytes, void *stream);

/*
 * fsi_jacobian_solid_apply - y = J x for the reduced system with the solid block:
 *   J = A_VMS(a, s) + [[B^T K_s B, 0], [0, 0]],  K_s = c_M M + c_K K(U) - c_V K_v(U),
 * with B = (C^lambda)^T over the solid nodes (problem->m == solid->n_nodes; the
 * point tables come from fsi_dlm_locate on the current positions X0 + U;
 * problem->kappa and problem->dlm_gram are ignored).  Dirichlet velocity DOFs
 * (dir_mask) have identity rows and zero columns.  x, y: T [4][N] (device, not
 * overlapping).  ws: at least fsi_jacobian_solid_workspace(problem, solid) bytes.
 */
size_t fsi_jacobian_solid_workspace(const fsi_problem *problem, const fsi_solid *solid);
int fsi_jacobian_solid_apply(const fsi_problem *problem, const fsi_solid *solid, const double *U,
                             double cM, double cK, double cV, const void *x, void *y, void *ws,
                             size_t ws_bytes, void *stream);

/*
 * fsi_solid_residual - the solid's nonlinear residual at its nodes (eq.
 * solid_weak_form tested with each nodal shape function, no body force or
 * traction on the solid; same material, densities and viscous term as
 * fsi_solid_apply):  R^s = M_rho(U) A + f_int(U) - K_v(U) V,
 * f_int[A] = int P(F) : grad_0 N_A dOmega_0.  FP64.
 *   U, V, A  double [3][M] displacement, velocity, acceleration (device)
 *   R        double [3][M] out (not overlapping the inputs)
 *   ws       at least fsi_solid_workspace(n_elem, FSI_F64) bytes
 */
int fsi_solid_residual(const fsi_solid *solid, const double *U, const double *V, const double *A, double *R,
                       void *ws, size_t ws_bytes, void *stream);

/*
 * fsi_solid_step_residual - the step residual of section 2.4 with the solid in
 * place of the per-point stand-in: the solid velocity is the fluid's at the
 * solid nodes (eq. nodal_solid_velo), V = B u, the solid displacement and
 * acceleration are affine in it, U = U_base + cU V, A = cA V - A_base, and the
 * multiplier is eliminated by eq. nodal_lagrange (lambda = -R^s), so
 *   R = R_fluid(x; f) + [B^T R^s(U, V, A); 0],  Dirichlet rows u - gD,
 * with R_fluid as in fsi_vms_residual (problem->a, kappa, dlm_gram unused).
 * Backward Euler in velocity form: U_base = U_n, cU = dt, A_base = V_n / dt,
 * cA = 1 / dt.  Generalized-alpha in stage unknowns (the displacement advancing
 * through its rate V with the fluid's gamma): cU = gamma dt, U_base = U_n +
 * (alpha_f - gamma) dt V_n, cA = alpha_m / (gamma dt alpha_f), A_base = cA V_n -
 * (1 - alpha_m / gamma) Vdot_n.  A body force f per unit mass on the solid (the
 * (rho_s - rho_f)(A - f) of eq. solid_weak_form) enters as A_base + f.
 * problem: FP64, Q1 or Q2, problem->solid NULL, its points (located at the step's
 * configuration) the solid's nodes.
 *   U_base, A_base  double [3][M];  f, gD  double [3][N]
 *   x         double [4][N];  R  double [4][N] out
 *   U, V      double [3][M] out: the solid state of x
 *   ws        at least fsi_solid_step_workspace(problem, solid) bytes
 */
size_t fsi_solid_step_workspace(const fsi_problem *problem, const fsi_solid *solid);
int fsi_solid_step_residual(const fsi_problem *problem, const fsi_solid *solid, const double *U_base,
                            const double *A_base, double cU, double cA, const double *f, const double *gD,
                            const double *x, double *R, double *U, double *V, void *ws, size_t ws_bytes,
                            void *stream);

/*
 * fsi_vms_residual - nonlinear residual of one implicit step (Q1 and Q2), the
 * right-hand side of the Newton corrections of section 2.4:
 *   R = A(a = u, tau(u)) x - F(f) + [B^T diag(kappa) (B u - g); 0]
 * with A the operator of fsi_vms_apply evaluated with the velocity itself as
 * advection field (eq. fluid_weak_form's convective term and tau_m of the
 * stabilisation equations use v^f), F(f) = int (w + tau_m((u.grad)w + grad q)).f
 * the Galerkin/SUPG/PSPG weighting of the nodal source f = c_m u_old + body
 * force, and the DLM term from the per-cell blocks (problem->dlm_gram, needed
 * when n_occ > 0) minus lamg = B^T (kappa g) (g: prescribed solid-point
 * velocities, precomputed once per step with fsi_dlm_BT).  Dirichlet rows:
 * R = u - gD.  problem->a is ignored.
 *   f     T [3][N];  lamg  T [3][N] or NULL;  gD  T [3][N] (needed if dir_mask)
 *   x     T [4][N] current iterate (unmasked);  R  T [4][N] out
 *   ws    at least fsi_jacobian_workspace(problem) bytes
 */
int fsi_vms_residual(const fsi_problem *problem, const void *f, const void *lamg, const void *gD,
                     const void *x, void *R, void *ws, size_t ws_bytes, void *stream);

/*
 * Nodal 4x4 block-Jacobi preconditioner: for every node, the (u,v,w,p) x
 * (u,v,w,p) diagonal block of J (element contributions of the operator plus the
 * diagonal of the DLM block, Dirichlet rows/columns replaced by the identity),
 * inverted in FP64.  Section 2.4 preconditions the reduced 2x2 block system
 * with blocks taken from its sub-matrices; this is the node-local member of
 * that family.
 *   problem   FP64 problem (dtype FSI_F64; dlm_gram required when n_occ > 0)
 *   pinv64    double [16][N] out or NULL (entry (i,j) of node k at (4i+j)*N+k)
 *   pinv32    float  [16][N] out or NULL (the FP32 copy)
 *   blocks    double [16][N] out or NULL (the blocks before inversion)
 *   n_singular_host  HOST out or NULL: blocks that could not be inverted (set to
 *             the identity); SYNCS when non-NULL
 *   ws        at least fsi_bjacobi_workspace(grid) bytes
 * fsi_bjacobi_apply: z = P^{-1} v on [4][N] vectors in precision dtype.
 */
size_t fsi_bjacobi_workspace(const fsi_grid *grid);
int fsi_bjacobi_setup(const fsi_problem *problem, double *pinv64, float *pinv32, double *blocks,
                      int64_t *n_singular_host, void *ws, size_t ws_bytes, void *stream);
int fsi_bjacobi_apply(const fsi_grid *grid, fsi_dtype dtype, const void *pinv, const void *v,
                      void *z, void *stream);

/*
 * Schur-complement block preconditioner (section 2.4: the reduced 2x2 block
 * system J = [[F, G], [D, C]] is solved with block preconditioners built from
 * its sub-matrices).  This member uses
 *   F_hat = the nodal 3x3 velocity blocks of J (from fsi_bjacobi_setup's raw
 *           blocks), inverted per node;
 *   S_hat = a variable-coefficient pressure Laplacian -div(alpha grad p) on the
 *           node lattice (trilinear elements of side h/p), standing in for
 *           S = C - D F^{-1} G: the PSPG block C is tau_m times a Laplacian and
 *           G^T F^{-1} G acts like one scaled by 1/(c_m + DLM density), so
 *           alpha = tau_m + mean over the lattice cell's corners of
 *           1/(c_m + max(d_A, 0)/v_A), d_A = (B^T kappa)_A, v_A the node's
 *           lumped lattice volume; tau_m from the stabilisation-parameter
 *           equation with the corner means of a and s.  Dirichlet rows of the
 *           Laplacian: boundary nodes whose velocity is not fully prescribed
 *           (node 0 if there is none).  S_hat^{-1} is one multigrid V(2,2)
 *           cycle: Jacobi smoothing (weight 8/9), trilinear prolongation,
 *           restriction = its transpose, alpha averaged 2x2x2 per coarser
 *           level while all cell counts are even and the level has more than
 *           64 nodes, the coarsest level (at most 1000 nodes) solved with a
 *           dense inverse.
 *   FSI_PC_SCHUR_DIAG: z_p = S_hat^{-1} v_p, z_u = F_hat^{-1} v_u.
 *   FSI_PC_SCHUR_TRI:  z_p as above, z_u = F_hat^{-1} (v_u - [J (0, z_p)]_u)
 *                      (the upper factor [[F_hat, G], [0, S_hat]]; one extra
 *                      Jacobian apply per preconditioner apply).
 *   vel_steps = k > 0: F_hat^{-1} t becomes k minimal-residual steps on F (the
 *                      velocity rows of J [u; 0]) preconditioned by the nodal
 *                      blocks: r = t, z = 0; p = blocks^{-1} r, q = F p,
 *                      alpha = (q.r)/(q.q), z += alpha p, r -= alpha q (one
 *                      Jacobian apply per step; the step lengths stay on the
 *                      device).  0 <= k <= 16.
 * fsi_schur_size: bytes of the preconditioner object for a grid (0 if the
 *   lattice cannot be coarsened to at most 1000 nodes).  The object holds the
 *   coefficients, the inverses and the V-cycle's vectors: an apply writes into
 *   it, so applies that share one object must not overlap.
 * fsi_schur_setup: builds the object from the FP64 problem (a, s, dir_mask,
 *   dlm_gram needed when n_occ > 0) and blocks = double [16][N], the raw nodal
 *   blocks of fsi_bjacobi_setup for the same problem.  SYNCS (the coarsest
 *   operator is factorised on the host).
 * fsi_schur_apply: z = P^{-1} v ([4][N] device, precision J->dtype, not
 *   overlapping); J is only applied in FSI_PC_SCHUR_TRI or with vel_steps > 0,
 *   with ws of at least fsi_jacobian_workspace(J) bytes (ws may be NULL
 *   otherwise).
 * fsi_schur_info: levels of the hierarchy, their lattice-cell counts
 *   (ncell[3 l + d], up to 16 levels) and the byte offsets of each level's
 *   FP64 alpha array inside the object (for inspection).
 */
typedef enum { FSI_PC_BJACOBI = 0, FSI_PC_SCHUR_DIAG = 1, FSI_PC_SCHUR_TRI = 2 } fsi_precond;
size_t fsi_schur_size(const fsi_grid *grid);
int fsi_schur_info(const fsi_grid *grid, int32_t *n_levels, int32_t *ncell, int64_t *alpha_offset);
int fsi_schur_setup(const fsi_problem *P64, const double *blocks, void *pc, size_t pc_bytes,
                    void *stream);
int fsi_schur_apply(const fsi_problem *J, int32_t mode, int32_t vel_steps, void *pc, const void *v,
                    void *z, void *ws, size_t ws_bytes, void *stream);

/*
 * fsi_fgmres_solve - solve J x = b with restarted flexible GMRES, right
 * preconditioned by the nodal block-Jacobi blocks or the Schur-complement block
 * preconditioner (section 2.4: the reduced system is solved iteratively with
 * block preconditioners).
 * FP64: Krylov basis, classical Gram-Schmidt with re-orthogonalisation, Givens
 * rotations, x, and the residual b - J x recomputed at every restart.  With
 * opts->basis = FSI_F32 (only with inner = FSI_F32 and restart <= 52) the basis
 * vectors are stored rounded to FP32 while every product and sum of the
 * Gram-Schmidt passes, and the Gram matrix of the stored vectors, stay FP64
 * (half the bytes per pass; a cycle stops at the FP32 level anyway).
 * Inner precision (opts->inner): the preconditioner and Jacobian applies of
 * each cycle and the stored preconditioned vectors; with FSI_F32 the restarts
 * are iterative-refinement steps (a cycle stops once its residual estimate
 * fell by opts->inner_reduction or reached the target).
 *   J64   FP64 problem (true residuals; also the inner applies if inner = F64)
 *   J32   FP32 problem (same data rounded to FP32) when inner = F32, else NULL
 *   pinv  opts->precond = FSI_PC_BJACOBI: [16][N] inverse blocks in the inner
 *         precision, or NULL (no preconditioner); FSI_PC_SCHUR_*: the object of
 *         fsi_schur_setup (its scratch vectors are written during the solve)
 *   b     double [4][N];  x  double [4][N] in: initial guess, out: solution
 *   stats HOST out (may be NULL).  SYNCS: with opts->host_ring (pinned host
 *         memory of the caller, e.g. from hipHostMalloc, at least
 *         restart * (restart + 2) doubles) the Arnoldi steps are enqueued back
 *         to back and the host reads each step's coefficients from the ring
 *         one step behind the device (so a cycle may compute one step past its
 *         stopping point; that step is not used); without it (NULL) each step
 *         waits for its coefficients.  It waits for the stream at every
 *         restart.  The call creates its per-step events and destroys them
 *         before it returns; it keeps nothing.
 * Returns FSI_OK when ||b - J x||_2 <= rtol ||b||_2 (FP64 residual),
 * FSI_ERR_NOT_CONVERGED (x = last iterate) on the iteration cap or on
 * stagnation (three restart cycles in a row without a 0.1 % residual
 * reduction), FSI_ERR_NAN (NaN/Inf in b, in a residual or in an Arnoldi
 * vector), FSI_ERR_BREAKDOWN.
 */
typedef struct {
    int32_t restart;          /* Krylov vectors per cycle (e.g. 50) */
    int32_t max_iters;        /* total Arnoldi steps */
    double rtol;              /* relative FP64 residual target */
    fsi_dtype inner;          /* FSI_F32 (mixed precision) or FSI_F64 */
    double inner_reduction;   /* FP32 cycles stop at this relative reduction (e.g. 1e-5) */
    int32_t precond;          /* fsi_precond (0: block-Jacobi) */
    int32_t vel_steps;        /* Schur forms: minimal-residual steps on the velocity block */
    double *host_ring;        /* pinned host ring of the caller, or NULL (see below) */
    int64_t host_ring_len;    /* doubles in host_ring */
    fsi_dtype basis;          /* storage of the Krylov basis: FSI_F64 (0) or FSI_F32 (see above) */
} fsi_solve_opts;

typedef struct {
    int32_t iters, cycles, status;
    double bnorm, res0, res_final;   /* ||b||, initial and final FP64 residual norms */
    double t_total_ms;
} fsi_solve_stats;

size_t fsi_fgmres_workspace(const fsi_problem *J64, const fsi_problem *J32,
                            const fsi_solve_opts *opts);
int fsi_fgmres_solve(const fsi_problem *J64, const fsi_problem *J32, const void *pinv,
                     const double *b, double *x, const fsi_solve_opts *opts,
                     fsi_solve_stats *stats, void *ws, size_t ws_bytes, void *stream);

/*
 * fsi_newton_solve - one implicit time step: Newton's method on
 * R(x) = 0 (fsi_vms_residual), each correction from J(u_k) dx = -R(x_k)
 * solved by fsi_fgmres_solve with the preconditioner opts->precond of J(u_k)
 * (of J(u_0) at every iterate with opts->pc_reuse), from dx = 0
 * (section 2.4: Newton iterations on the monolithic system, each solving the
 * reduced block system).  J(u_k) is the Picard/Oseen linearisation: the
 * operator of fsi_vms_apply with advection field u_k plus the DLM block.
 *   P64   FP64 problem: s, dir_mask, point tables, kappa, dlm_gram (a ignored)
 *   P32   FP32 copy of the same data when opts->inner = FSI_F32, else NULL
 *   f, lamg, gD  as in fsi_vms_residual (FP64)
 *   x     double [4][N] in: guess (Dirichlet values imposed), out: solution
 * Stops when ||R||_2 <= opts->tol_abs; each linear solve uses the relative
 * tolerance max(eta', 0.5 tol_abs / ||R||) with eta' = eta for the Picard
 * operator; for the full tangent eta' = min(eta, sqrt(0.5 tol_abs / ||R||)) in
 * the first iteration and 0.5 tol_abs / ||R|| after it (with quadratic
 * convergence two iterations then reach the target).
 * stats: HOST out.  SYNCS.
 */
typedef struct {
    int32_t max_newton;       /* Newton iterations cap (e.g. 20) */
    double tol_abs;           /* absolute residual target */
    double eta;               /* linear forcing term (e.g. 1e-3) */
    int32_t restart, max_krylov;
    fsi_dtype inner;          /* inner precision of the Krylov cycles */
    double inner_reduction;
    int32_t precond;          /* fsi_precond: block-Jacobi (0) or a Schur form (see pc_reuse) */
    int32_t vel_steps;        /* Schur forms: minimal-residual steps on the velocity block */
    int32_t tangent;          /* 0: Picard/Oseen J(u_k); 1: full Newton tangent (fsi_tangent_apply) */
    double *host_ring;        /* passed to every FGMRES solve (fsi_solve_opts), or NULL */
    int64_t host_ring_len;
    int32_t pc_reuse;         /* 0: the preconditioner is rebuilt at every Newton iterate; 1: it is
                                 built at the first iterate of the call and reused (a lagged
                                 preconditioner: FGMRES accepts any preconditioner, the operator
                                 stays J(u_k), so only the Krylov counts can change) */
    fsi_dtype basis;          /* Krylov basis storage of every FGMRES solve (fsi_solve_opts) */
} fsi_newton_opts;

typedef struct {
    int32_t newton_iters, krylov_iters, status;
    double res_hist[32];      /* ||R|| before each Newton iteration, then the final one */
    double t_total_ms, t_residual_ms, t_setup_ms, t_krylov_ms;
} fsi_newton_stats;

size_t fsi_newton_workspace(const fsi_problem *P64, const fsi_problem *P32,
                            const fsi_newton_opts *opts);

/*
 * fsi_tangent_apply - the full Newton tangent of the step residual (section 2.4:
 * Newton's method on the monolithic system; section 2.1 for the terms), i.e.
 * the derivative of fsi_vms_residual with respect to x, applied to v:
 *   y = J_full(x) v = A(a = u, tau(u)) v~ + [B^T kappa B v~_u; 0]
 *       + (reactive convection (dv.grad)u in the Galerkin, SUPG and PSPG terms)
 *       + (SUPG test-function derivative ((dv.grad)w) . rho)
 *       + (derivatives of tau_m and tau_c along dv: d tau_m = -tau_m^3 s (u.G dv),
 *          d tau_c = -(tau_c / tau_m) d tau_m),
 * where rho = r_m(u, p) - f is the state's strong momentum residual and
 * v~ = v with its velocity Dirichlet entries zeroed; velocity Dirichlet rows
 * y = v.  The DLM block is linear, so its derivative is the Picard one.
 *   P  the problem in the precision of the call (P->dtype): s, dir_mask, point
 *      tables, kappa, dlm_gram or the pointwise path; P->a is ignored (the
 *      advection field is the state's velocity); no solid block
 *   x  state (u, p), T [4][N];  f  source c_m u_old + body force, T [3][N]
 *      (lamg and gD of the residual are constant and drop out)
 *   v, y  T [4][N], y must not alias x, f or v
 * Q1 only.  ws: at least fsi_tangent_workspace(P) bytes.  Deterministic.
 * fsi_newton_solve uses it as the Krylov operator when opts->tangent = 1 (in
 * the inner precision; the preconditioner keeps the Picard operator).
 */
size_t fsi_tangent_workspace(const fsi_problem *P);
int fsi_tangent_apply(const fsi_problem *P, const void *x, const void *f, const void *v, void *y,
                      void *ws, size_t ws_bytes, void *stream);
int fsi_newton_solve(const fsi_problem *P64, const fsi_problem *P32, const double *f,
                     const double *lamg, const double *gD, double *x,
                     const fsi_newton_opts *opts, fsi_newton_stats *stats, void *ws,
                     size_t ws_bytes, void *stream);

/*
 * fsi_newton_solid_solve - one time step with the hyperelastic solid: Newton on
 * fsi_solid_step_residual from x, each iteration solving with the matrix
 * A(a = u_k) + B^T (c_M M + c_K K(U_k) - c_V K_v(U_k)) B, (c_M, c_K, c_V)
 * = (cA, cU, 1) (the configuration frozen for M and K_v, as the Picard
 * linearisation of the fluid), by FGMRES with the options' preconditioner built
 * from the problems' per-point kappa and per-cell blocks (an approximation of
 * the solid block that the caller chooses; dlm_gram is required).  After the
 * step, U and V hold the solid state of the converged x (backward Euler:
 * U_{n+1} = U_n + dt V_{n+1}, the solid update Delta U = (C^lambda)^T Delta V of
 * section 2.4 integrated).
 * opts->tangent must be 0.  Other arguments as fsi_newton_solve and
 * fsi_solid_step_residual; ws: fsi_newton_solid_workspace(P64, P32, solid, opts).
 */
size_t fsi_newton_solid_workspace(const fsi_problem *P64, const fsi_problem *P32, const fsi_solid *solid,
                                  const fsi_newton_opts *opts);
int fsi_newton_solid_solve(const fsi_problem *P64, const fsi_problem *P32, const fsi_solid *solid,
                           const double *U_base, const double *A_base, double cU, double cA,
                           const double *f, const double *gD, double *x, double *U, double *V,
                           const fsi_newton_opts *opts, fsi_newton_stats *stats, void *ws, size_t ws_bytes,
                           void *stream);

/*
 * Learned warm start (an addition to the method: a better Newton initial
 * guess for the predictor of section 2.4; it never changes the converged
 * answer, which the residual tolerance decides).  A stack of 3x3x3
 * convolutions on the fluid node lattice, BF16 operands with FP32
 * accumulation on the matrix cores, trained with MSE and Adam.
 *
 * Layouts: activations channels-last [V][C] (uint16 = bfloat16 bits, or
 * float), V = dims[0] dims[1] dims[2], voxel v = i + dims[0] (j + dims[1] k);
 * C (cin, cout) a multiple of 32.  Weights [27][cout][cin] with tap =
 * dx + 3 (dy + 3 dz) reading the neighbour at offset (dx-1, dy-1, dz-1); zero
 * padding outside the lattice.
 *
 * fsi_conv3d_fwd     Y[v][o] = bias[o] + sum_tap sum_i X[v+off][i] W[tap][o][i];
 *                    then, if gate != NULL, Y = 0 where gate[v][o] <= 0 (ReLU
 *                    backward mask); then ReLU if relu != 0.  Y_bf16 and/or
 *                    Y_f32 receive the result (either may be NULL).
 *                    With W from fsi_conv3d_flip_transpose (Wd[tap][i][o] =
 *                    W[26-tap][o][i]) the same call is the data gradient.
 *                    X, W, Y_f32 16-byte aligned, Y_bf16 and gate 8-byte
 *                    aligned, V cin 2 < 2^31 bytes (else FSI_ERR_ARG).
 * fsi_conv3d_wgrad   dW[tap][o][i] = sum_v dY[v][o] X[v+off][i] (float),
 *                    db[o] = sum_v dY[v][o] (float, or db = NULL).  Split over
 *                    voxel ranges summed in a fixed order: deterministic.
 * fsi_mse_loss       over channels < used: loss = mean (pred - target)^2 (HOST
 *                    out, SYNCS if non-NULL), dpred = 2 (pred - target) / count
 *                    as bfloat16 (0 in unused channels).
 * fsi_adam_step      w, m, v float [n]; t >= 1; w_bf16 (optional) gets the
 *                    rounded copy of the updated w.
 * fsi_nn_pack        out[v][c] = (ca_c a_c[v] + cb_c b_c[v] + cc_c c_c[v] + cst_c
 *                    - shift_c) * scale_c for c < nch (a NULL pointer
 *                    contributes 0), 0 for nch <= c < C; a_c, b_c, c_c are
 *                    double [V] device arrays.
 * fsi_nn_moments     per channel, sum and sum of squares over V (HOST out
 *                    [C][2] doubles, SYNCS).
 * fsi_nn_unpack      x[f][v] = base[f][v] + out[v][f] / scale_f + shift_f for
 *                    f < 4; Dirichlet velocity DOFs (dir_mask) take gD (or 0).
 */
typedef struct {
    const double *a[32];
    const double *b[32];
    const double *c[32];
    double ca[32], cb[32], cc[32];
    double cst[32];
    double shift[32];
    double scale[32];
    int32_t nch;
} fsi_nn_pack_spec;

typedef struct {
    double shift[4];
    double scale[4];
} fsi_nn_unpack_spec;

int fsi_conv3d_fwd(const int32_t *dims, int32_t cin, int32_t cout, const uint16_t *X,
                   const uint16_t *W, const float *bias, int32_t relu, const uint16_t *gate,
                   uint16_t *Y_bf16, float *Y_f32, void *stream);
size_t fsi_conv3d_wgrad_workspace(const int32_t *dims, int32_t cin, int32_t cout);
int fsi_conv3d_wgrad(const int32_t *dims, int32_t cin, int32_t cout, const uint16_t *dY,
                     const uint16_t *X, float *dW, float *db, void *ws, size_t ws_bytes,
                     void *stream);
int fsi_conv3d_flip_transpose(int32_t cin, int32_t cout, const uint16_t *W, uint16_t *Wd,
                              void *stream);
size_t fsi_mse_workspace(void);
int fsi_mse_loss(int64_t nvox, int32_t c, int32_t used, const float *pred, const float *target,
                 uint16_t *dpred, double *loss_host, void *ws, size_t ws_bytes, void *stream);
int fsi_adam_step(int64_t n, float *w, const float *g, float *m, float *v, uint16_t *w_bf16,
                  int32_t t, float lr, float b1, float b2, float eps, void *stream);
int fsi_to_bf16(int64_t n, const float *in, uint16_t *out, void *stream);
int fsi_nn_pack(int64_t nvox, int32_t c, const fsi_nn_pack_spec *p, float *out, void *stream);
size_t fsi_nn_moments_workspace(int32_t c);
int fsi_nn_moments(int64_t nvox, int32_t c, const float *data, double *sums_host, void *ws,
                   size_t ws_bytes, void *stream);
int fsi_nn_unpack(int64_t nvox, int32_t c, const float *out, const double *base,
                  const fsi_nn_unpack_spec *u, const uint32_t *dir_mask, const double *gD, double *x,
                  void *stream);

/*
 * BLAS-1 helpers used by the drivers (FP64 device vectors):
 *   fsi_axpby  y = alpha x + beta y (beta = 0: y = alpha x, y's old contents ignored)
 *   fsi_dot    HOST out = x . y, deterministic fixed-order reduction.  SYNCS.
 */
int fsi_axpby(int64_t n, double alpha, const double *x, double beta, double *y, void *stream);
int fsi_dot(int64_t n, const double *x, const double *y, double *out_host, void *ws,
            size_t ws_bytes, void *stream);
size_t fsi_dot_workspace(void);

/*
 * Kernel timing (tracing aid, not part of the method).  fsi_profile_enable(1)
 * creates a pool of hipEvents, resets the totals and brackets each later launch
 * of an instrumented kernel with two events recorded on that launch's stream;
 * fsi_profile_enable(0) stops recording and destroys the events and the totals
 * (read them before).  This timing registry is the only state the library keeps
 * between calls besides the per-thread error text, and it exists only while
 * profiling is on; do not switch it while another thread is inside a call.  fsi_profile_read(name, ...) waits for the recorded events
 * (SYNCS) and returns the summed elapsed milliseconds and the number of
 * launches of the kernel `name` ("vms_q1_cells", "vms_q2_cells",
 * "vms_gather", "dlm_cell_reduce", "dlm_locate", ...; unknown names read 0).
 */
int fsi_profile_enable(int on);
int fsi_profile_read(const char *kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* FSI_H */
