/*
 * pd.h -- C ABI of libpd, the MI355X (gfx950) pressure solver for the staggered spectral
 * semi-implicit discontinuous Galerkin scheme of Fambri & Dumbser, "Spectral semi-implicit and
 * space-time discontinuous Galerkin methods for the incompressible Navier-Stokes equations on
 * staggered Cartesian grids", arXiv:1602.05806 (Section 2, "Spectral semi-implicit DG schemes on
 * staggered Cartesian grids").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Grid. Uniform Cartesian grid with nx*ny(*nz) main cells of size h_d = len[d]/ncell[d],
 *    periodic in every direction (periodic_mask must have one bit per dimension set). Main cell
 *    i covers [i h, (i+1) h]; the dual cell i of a velocity component staggered along d covers
 *    [(i+1/2) h, (i+3/2) h], i.e. it overlaps the right half of main cell i and the left half of
 *    main cell i+1 (the edge-based staggering of Section 2.1 with the periodic wrap of eq. pSyst1d).
 *  * DoF layout (element-blocked). A field is (N+1)^d nodal values per cell at the Gauss-Legendre
 *    nodes of that cell. Flat index = cell * (N+1)^d + node, with cell = (k*ny + j)*nx + i and
 *    node = (l3*(N+1) + l2)*(N+1) + l1 (x fastest in both). Pressure-like fields live on the main
 *    grid; velocity component d lives on its own dual grid with the same index formula.
 *  * Pointers. Every array argument is a DEVICE pointer owned by the caller, of PD_FP64 (double)
 *    or PD_FP32 (float) elements as the call states; the library never frees caller memory.
 *    Arrays may not alias unless a call says so.
 *  * Streams. All work is enqueued on `hip_stream` (a hipStream_t; NULL = the null stream) and
 *    returns without waiting, except where a call says it synchronises (solves read their
 *    convergence information back).
 *  * Errors. Negative PD_E* codes are returned, never thrown; pd_last_error() gives the message.
 *    A context is not thread safe; use one context per stream.
 */
#ifndef PD_H
#define PD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pd_ctx pd_ctx;

/* Status codes. */
enum {
  PD_OK = 0,
  PD_EINVAL = -1,      /* invalid argument or unsupported configuration                    */
  PD_ENOMEM = -2,      /* device allocation failed                                           */
  PD_EDEVICE = -3,     /* a HIP call failed (message holds the HIP error string)             */
  PD_ENOCONV = -4,     /* maxit reached before the tolerance                                 */
  PD_EBREAKDOWN = -5   /* CG breakdown: <p, A p> <= 0 or not finite (e.g. NaN in the RHS)   */
};

/* Precision of a call. PD_FP64: FP64 arrays and arithmetic. PD_FP32: FP32 arrays and arithmetic
 * with FP64 dot-product accumulation (pd_apply only). PD_FP32_REFINE64: FP64 arrays at the
 * boundary; the solve runs one conjugate-gradient iteration on FP32 vectors (operator applies
 * and vector updates in FP32, dot products accumulated in FP64) and periodically flushes the
 * FP32 correction into the FP64 solution and replaces the FP32 residual by the FP64 residual
 * b - A x (iterative refinement by residual replacement, keeping the search direction); it
 * stops on the FP64 residual. */
enum { PD_FP64 = 0, PD_FP32 = 1, PD_FP32_REFINE64 = 2 };

/* Operators. PD_OP_PRESSURE: A_p = dt * K with K = sum_d h_d^-2 (M on the other directions)
 * (x) H_d and H_d = D_d^T M^-1 D_d the block-tridiagonal 1D operator with blocks L, C, R of
 * eq. (pSyst) / (PerPrSyst); it acts on q = P^{n+theta} (eq. LOpressure). PD_OP_VISCOUS:
 * A_v = M^{xyz} + nu dt K, the implicit-viscosity operator of eq. (implicitviscosity) with the
 * dt and h factors of eqs. (uSDG12), (Ux) made explicit. Both are symmetric; A_v is positive
 * definite, A_p positive semi-definite with null space Z = null of the weak gradient. */
enum { PD_OP_PRESSURE = 0, PD_OP_VISCOUS = 1 };

/* Per-solve report. iters: CG iterations (FP32 plus FP64 ones for PD_FP32_REFINE64);
 * outer_iters: FP64 residual recomputations (refinement: one per replacement; PD_FP64: the
 * CG runs, 1 plus the replacements made when the recurrence met rtol but the recomputed residual
 * b - A x did not); restarts:
 * refinement replacements that also restarted the search direction; fallback_iter: for
 * PD_FP32_REFINE64, the iteration at which the solve continued in FP64 because the FP64
 * residual had stopped decreasing under FP32 iterations (FP32 rounding of A p dominates the
 * smallest eigenvalues once eps_32 * cond(A) approaches 1), -1 if it never did; status: PD_OK /
 * PD_ENOCONV / PD_EBREAKDOWN; rel_res_recur: last recurrence (FP64: CG recurrence; refinement:
 * last FP64) residual / ||b||; rel_res_true: true FP64 residual ||b - A x||/||b|| recomputed at
 * exit; ms: wall time of the solve on the stream. ||b|| is taken after the null-space projection
 * for PD_OP_PRESSURE. */
typedef struct {
  int iters, outer_iters, status, restarts, fallback_iter, reserved;
  double rel_res_recur, rel_res_true, ms;
} pd_solve_info;

/* Create a context: computes the 1D tables of eq. (matrices), eq. (pSyst) and eq. (l2forward) in
 * FP64 on the host for degree N (0 <= N <= 8), uploads FP64 and FP32 copies, and allocates the
 * solver workspace. dim is 2 or 3; ncell[d] >= 1 and len[d] > 0 for d < dim; dt > 0;
 * 0.5 <= theta <= 1 (theta of eq. uSDG1); nu >= 0. periodic_mask: bit d set = periodic along d
 * (bits at or above dim: PD_EINVAL). A clear bit puts homogeneous Dirichlet pressure walls at
 * both ends of direction d (p = 0 on the wall, the boundary case of eq. (pSyst)): the ghost
 * cell beyond a wall holds the adjacent cell's pressure reflected about the wall with its sign
 * flipped, so the wall rows of the 1D operator are (C - L J) P_0 + R P_1 and
 * L P_{m-2} + (C - R J) P_{m-1}, J reversing the node order. Along such a direction the null
 * space of A_p shrinks to the part of the cell-periodic kernel that is odd about the cell centre
 * (none for even N, so A_p is then definite). Walls cover pd_apply, pd_cg_solve,
 * pd_project_null and pd_project_null_noalloc; every velocity, step, adjoint and loss entry
 * point requires a fully periodic context (PD_EINVAL otherwise). On error
 * *out is NULL and the message is available from pd_last_error(NULL). */
int pd_setup(pd_ctx** out, int dim, const int ncell[3], const double len[3], int N,
             double dt, double theta, double nu, unsigned periodic_mask, void* hip_stream);

/* Release the context's device memory (waits for its stream). NULL is ignored. */
void pd_destroy(pd_ctx* ctx);

/* Last error message of ctx (or of the last failed pd_setup if ctx is NULL). Never NULL. */
const char* pd_last_error(const pd_ctx* ctx);

/* Sizes: number of main cells, DoFs per field (cells * (N+1)^dim) and dim. Host call. */
int pd_sizes(const pd_ctx* ctx, long long* ncells, long long* ndof, int* dim);

/* Copy the N+1 Gauss-Legendre nodes and weights on [0,1] used by ctx to host arrays. */
int pd_nodes(const pd_ctx* ctx, double* xi, double* w);

/* Host-only query of the FP64 1D tables the library builds for degree N (0..8), no device use:
 * which = PD_TAB_NODES (N+1 Gauss-Legendre nodes on [0,1]), PD_TAB_WEIGHTS (N+1 weights),
 * PD_TAB_L / PD_TAB_C / PD_TAB_R ((N+1)^2 entries, row-major: the blocks L, C, R of the 1D
 * pressure operator of eq. (pSyst) / (PerPrSyst)), PD_TAB_PNULL ((N+1)^2: orthogonal projector
 * onto the cell-periodic kernel of the weak gradient, null(R~ - L~)), PD_TAB_PNULL_ODD
 * ((N+1)^2: orthogonal projector onto the part of that kernel odd about the cell centre, the
 * 1D null space along a Dirichlet direction; all zeros for even N), PD_TAB_PV ((N+1)^2,
 * row-major V[m][l]: the generalised eigenvectors of the diagonal block, C V = M V diag(lambda),
 * V^T M V = I, which the cell-block Jacobi preconditioner uses), PD_TAB_PLAM (N+1: lambda).
 * out must hold that many doubles. Returns the number of values written, or PD_EINVAL. */
enum { PD_TAB_NODES = 0, PD_TAB_WEIGHTS = 1, PD_TAB_L = 2, PD_TAB_C = 3, PD_TAB_R = 4,
       PD_TAB_PNULL = 5, PD_TAB_PNULL_ODD = 6, PD_TAB_PV = 7, PD_TAB_PLAM = 8 };
int pd_table_1d(int N, int which, double* out);

/* y = A x for op PD_OP_PRESSURE or PD_OP_VISCOUS; x, y: ndof elements of precision prec
 * (PD_FP64 or PD_FP32). Matrix-free: tensor-product application of the 1D blocks along each
 * direction (eq. tensorP1) with the diagonal Gauss-Legendre masses. */
int pd_apply(pd_ctx* ctx, int op, int prec, const void* x, void* y, void* hip_stream);

/* Solve A x = b with unpreconditioned conjugate gradients (the paper's matrix-free CG,
 * Section 2.1). b, x: ndof FP64 arrays. x holds the initial guess on entry (set it to zero for
 * the paper's choice) and the solution on exit. For PD_OP_PRESSURE, b is first projected onto
 * range(A_p) (orthogonal complement of the null space of the weak gradient) and x is projected
 * at exit, so the result is the minimum-norm solution. PD_FP64 stops when the CG recurrence
 * residual <= rtol ||b||_2 and the recomputed FP64 residual ||b - A x||_2 is too: when the latter
 * is above but within 16x, it replaces the recurrence residual and the iterations continue (up
 * to 8 times, while each replacement at least halves it; a larger gap is the FP64 rounding
 * floor of b - A x and ends the solve with PD_OK, rel_res_true reporting it).
 * PD_FP32_REFINE64 stops on the recomputed FP64 residual. b and x must not alias (PD_EINVAL).
 * Synchronises with the stream at exit; info may be NULL.
 * Returns PD_OK, PD_ENOCONV (maxit reached) or PD_EBREAKDOWN. */
int pd_cg_solve(pd_ctx* ctx, int op, int prec, const void* b, void* x, double rtol, int maxit,
                pd_solve_info* info, void* hip_stream);

/* b = sum_d B_d u_d with B_d = h_d^-1 (M on the other directions) (x) D_d^T: the right-hand
 * side of eq. (LOpressure) from the dual velocity components u[0..dim-1] (FP64, dual layout).
 * The discrete divergence of eq. (pSDG1) is -b. */
int pd_rhs_div(pd_ctx* ctx, void* const u[3], void* b, void* hip_stream);

/* Velocity update of eqs. (LOvelocityU)-(LOvelocityW): u_d -= dt h_d^-1 M_d^-1 D_d q for every
 * direction d, with q = P^{n+theta} (FP64, main grid) and u[d] the FP64 dual components,
 * updated in place. */
int pd_project_velocity(pd_ctx* ctx, const void* q, void* const u[3], void* hip_stream);

/* Null-space projection v <- v - Z Z^T v of an FP64 (prec = PD_FP64) or FP32 main-grid field,
 * Z = orthonormal basis of null(A_p) (tensor products of the cell-periodic null vectors of the
 * 1D weak gradient: 1 per direction for even N, 2 for odd N; along a Dirichlet direction only the
 * odd one, so no projection at all when N is even and a wall exists). In place. */
int pd_project_null(pd_ctx* ctx, int prec, void* v, void* hip_stream);

/* Allocation-free variant of pd_project_null, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments, kernels and result (bit-identical to pd_project_null), but the projection's scratch
 * (per-block node sums and the correction) lives in a fixed device array of the library,
 * 256 x 729 + 729 doubles (1.5 MB, the maximum for N <= 8 in 3D), one copy per device held
 * until the process ends; the call allocates nothing and calls no allocating routine. Every call
 * on a device shares that device's array: calls that overlap on one device (several streams or
 * host threads) race and must be serialised by the caller. PD_EINVAL for (N+1)^dim beyond the
 * array (not reachable for N <= 8). */
int pd_project_null_noalloc(pd_ctx* ctx, int prec, void* v, void* hip_stream);

/* L2 projections between a dual grid and the main grid along direction d (eq. l2forward and
 * eq. l2backward): dir = 0: main = pi_{*->#}(dual); dir = 1: dual = pi_{#->*}(main). FP64. */
int pd_l2_project(pd_ctx* ctx, int d, int dir, const void* in, void* out, void* hip_stream);

/* One explicit convection step of eqs. (Fu)-(Fw) on the main grid with the third-order TVD
 * Runge-Kutta scheme: um[d] (FP64 main-grid velocity components) are replaced by the
 * predicted Fu, Fv, Fw. Rusanov flux with s = 2 max(|v_e^-|, |v_e^+|) on faces normal to e.
 * With PD_CFG_EXPLICIT_VISC set, the explicit viscous flux is included (see pd_configure);
 * with PD_CFG_CONVECTION = 0 as well, only the viscous flux. */
int pd_convect(pd_ctx* ctx, void* const um[3], void* hip_stream);

/* One semi-implicit fractional step (eqs. LOdiffusionU-LOvelocityW): u[d] = dual velocity
 * components U^n (in) / U^{n+1} (out), p = P^n (in) / P^{n+1} (out), all FP64. info[0..dim-1]
 * report the viscous solves, info[3] the pressure solve (info may be NULL). Synchronises.
 * Solver settings come from pd_configure. */
int pd_step(pd_ctx* ctx, void* const u[3], void* p, pd_solve_info info[4], void* hip_stream);

/* ---- Space-time step (Section 3) -------------------------------------------------------------
 * One step of the space-time scheme of degree M in time on the slab [t^n, t^n + dt] with the
 * Picard pressure correction of Section 3.3 (eqs. LOdiffusionU_HO-LOvelocityW_HO), M + 1
 * iterations. The velocity is a polynomial of degree M in time on the nodal Gauss-Legendre basis
 * psi_0..psi_M of [0, 1]; the time matrices are those of eqs. (tmatrix1)-(tmatrix3)
 * (M^t = diag(omega), At = M1 - MV). Iteration k forms, at every time node p, the right-hand
 * side of the momentum equations (eq. uSDG1_ST) on the dual grids,
 *   R_p = pi_{#->*}(psi_p(0) F) - omega_p G P_p      (k = 0: F = F^n, the semi-implicit
 *         predictor of pd_step at t^n, i.e. TVD-RK3 advection and, for M = 0, the implicit
 *         viscous solve; P = 0)
 *   R_p = pi_{#->*}(psi_p(0) pi_{*->#} U^n + dt omega_p L(pi_{*->#} U_p)) - omega_p G P_p
 *         (k >= 1: the space-time advective term of eq. Fu_ST at the current iterate; L is the
 *         explicit DG rate, with the viscous flux when PD_CFG_EXPLICIT_VISC is set),
 * solves the M + 1 decoupled pressure systems omega_s A_p dP_s = sum_d B_d R_{s,d} (eq. pSyst_ST2;
 * each a pd_cg_solve with the step's precision and PD_CFG_P_RTOL), and sets
 * U_s = sum_p Ainv[s][p] (R_p - omega_p G dP_p), P_s += dP_s: every iterate is discretely
 * divergence free at every time node (eq. pSDG1_ST). M = 0 is the semi-implicit step of pd_step
 * with theta = 1.
 * u[0..dim-1]: FP64 dual components, U^n on entry (the previous slab's end value), the end value
 * u(t^{n+1}) = sum_s psi_s(1) U_s on return. p_nodes: FP64 array of (M+1) * ndof, overwritten
 * with the pressure at the M + 1 time nodes (node s at offset s * ndof). 0 <= M <= 4; M >= 1
 * requires nu = 0 or PD_CFG_EXPLICIT_VISC (the non-symmetric space-time implicit viscous solve
 * of eq. implicitviscosity_ST is not provided: PD_EINVAL). info: NULL or 3 + (M+1)^2 entries:
 * [0..dim-1] the viscous solves (M = 0 with implicit viscosity, else zero), [3 + k (M+1) + s]
 * the pressure solve of iteration k at node s. Allocates its workspace on first use of each M
 * (about 3 dim (M+1) + M + 2 dim + 2 vectors of ndof doubles). Synchronises. */
int pd_step_st(pd_ctx* ctx, int M, void* const u[3], void* p_nodes, pd_solve_info* info,
               void* hip_stream);

/* Host-only query of the time tables the library builds for degree M (0..4), no device use:
 * which = PD_TTAB_NODES / PD_TTAB_WEIGHTS / PD_TTAB_PSI0 / PD_TTAB_PSI1 (M+1 values: Gauss-
 * Legendre nodes tau and weights omega on [0, 1], psi_p(0), psi_p(1)), PD_TTAB_MV / PD_TTAB_AINV
 * ((M+1)^2 values, row-major: MV of eq. tmatrix3 and the inverse of At = M1 - MV). Returns the
 * number of values written, or PD_EINVAL. */
enum { PD_TTAB_NODES = 0, PD_TTAB_WEIGHTS = 1, PD_TTAB_PSI0 = 2, PD_TTAB_PSI1 = 3,
       PD_TTAB_MV = 4, PD_TTAB_AINV = 5 };
int pd_time_table(int M, int which, double* out);

/* ---- Adjoint (transposed linearisation) of the fractional step --------------------------------
 * The step maps the dual velocity U^n to U^{n+1} (P^n does not enter U^{n+1}). Its adjoint maps
 * a cotangent Ubar of U^{n+1} to the cotangent of U^n, in reverse order of the step: the velocity
 * update and pressure solve (q = A_p^+ b is symmetric, so the adjoint pressure solve is a second
 * CG solve on A_p from zero with the same settings), B_d^T, pi_{#->*}^T, the viscous solve
 * (A_v symmetric: a CG solve with A_v, then the mass matrix), the transposed linearisation of the
 * explicit TVD-RK3 convection at the forward stages (Rusanov speed differentiated on the branch of
 * the forward state), and pi_{*->#}^T. All arrays FP64; solver settings come from pd_configure.
 * Transposes of the single operators are exposed for testing and custom adjoints. */

/* out = pi^T in along direction d: dir 0 transposes pi_{*->#} (in: main layout, out: dual),
 * dir 1 transposes pi_{#->*} (in: dual, out: main). in and out must not alias. */
int pd_l2_project_adjoint(pd_ctx* ctx, int d, int dir, const void* in, void* out,
                          void* hip_stream);

/* ubar[d] = B_d^T bbar for every direction d (bbar: main layout; ubar[d]: dual layout of
 * component d), B_d the divergence map of pd_rhs_div. Overwrites ubar. */
int pd_rhs_div_adjoint(pd_ctx* ctx, const void* bbar, void* const ubar[3], void* hip_stream);

/* qbar = -sum_d G_d^T ubar[d]: transpose of the velocity update of pd_project_velocity with
 * respect to q (G_d = dt h_d^-1 M_d^-1 D_d). Overwrites qbar (main layout). */
int pd_project_velocity_adjoint(pd_ctx* ctx, void* const ubar[3], void* qbar, void* hip_stream);

/* Adjoint of pd_convect (one TVD-RK3 step of the explicit convection on the main grid) at the
 * state um (the input of that pd_convect call, unchanged): ubar holds the cotangent of the output
 * on entry and the cotangent of the input on return. um and ubar must not alias. */
int pd_convect_adjoint(pd_ctx* ctx, void* const um[3], void* const ubar[3], void* hip_stream);

/* Adjoint of pd_step at U^n: u holds U^n (dual components, unchanged), ubar holds the cotangent of
 * U^{n+1} on entry and that of U^n on return. info[0..dim-1] report the adjoint viscous solves,
 * info[3] the adjoint pressure solve (info may be NULL). Synchronises. */
int pd_step_adjoint(pd_ctx* ctx, void* const u[3], void* const ubar[3], pd_solve_info info[4],
                    void* hip_stream);

/* Mean kinetic energy of a dual velocity field, the K = (1/|Omega|) int |v|^2 / 2 of the 3D
 * Taylor-Green subsection of Section 2.4 (the loss of the adjoint rollout): every component is
 * integrated by Gauss-Legendre quadrature on its own dual grid, so on the uniform grid
 * K = (1 / (2 ncells)) sum_d sum_i W_i u_d,i^2 with W_i the product of the GL weights of node i.
 * u[0..dim-1]: FP64 dual components (read only). *energy (host) receives K. grad may be NULL;
 * otherwise grad[d] (FP64, dual layout of component d, must not alias any u[e]) is overwritten
 * with gscale * dK/du_d = gscale W u_d / ncells, the cotangent of the velocity for an incoming
 * loss cotangent gscale (finite). Synchronises. */
int pd_kinetic_energy(pd_ctx* ctx, void* const u[3], double gscale, void* const grad[3],
                      double* energy, void* hip_stream);

/* Settings used by pd_step and the timing hooks (key, value):
 *   PD_CFG_STEP_PREC     PD_FP64 (default) or PD_FP32_REFINE64 for the step's solves
 *   PD_CFG_P_RTOL        pressure tolerance in pd_step (default 1e-10)
 *   PD_CFG_V_RTOL        viscous tolerance in pd_step (default 1e-12)
 *   PD_CFG_MAXIT         iteration cap for the step's solves (default 100000, at most 2^30)
 *   PD_CFG_CONVECTION    1 (default) = explicit convection on, 0 = off (unsteady Stokes step)
 *   PD_CFG_RU_FACTOR     PD_FP32_REFINE64: the FP32 residual is replaced by the FP64 residual
 *                        b - A x each time it has dropped by this factor (default 0.1)
 *   PD_CFG_TIMING        s >= 1: the dispatch of every s-th launch of the operator kernel
 *                        inside solves carries start/stop HIP events (see pd_timing; 1 = every
 *                        launch; events add a few microseconds per timed launch), 0 (default) =
 *                        off
 *   PD_CFG_CHECK_EVERY   convergence poll interval of the solve loop in iterations (default 32,
 *                        at most 2^20)
 *   PD_CFG_KZ            3D operator kernel: planes per column segment (0 = automatic, at most
 *                        2^30)
 *   PD_CFG_TILES_PER_WG  2D operator kernel: tiles per persistent workgroup (0 = automatic, at
 *                        most 2^30)
 *   PD_CFG_PREFETCH      1 (default) = the operator kernel prefetches the next tile (2D) or the
 *                        next plane's halo (3D) into registers during compute, 0 = no prefetch
 *   PD_CFG_TILE_VARIANT  2D operator kernel tile shape: 0 (default) = the largest tile of cells
 *                        whose LDS box fits, 1 / 2 = one / two sizes smaller (more workgroups);
 *                        a grid with walls always runs 0 with prefetch (both settings ignored)
 *   PD_CFG_DEFER_X       where CG iteration k's x += alpha_k p_k is made: 1 (default) = in the
 *                        operator kernel of iteration k + 1 (it reads p_k anyway; 9 instead of
 *                        10 vector words per DoF and iteration), 0 = in the update kernel
 *   PD_CFG_PRECOND       1 = preconditioned CG in pd_cg_solve, pd_step and pd_step_st (both
 *                        precisions, both operators; the paper names preconditioning as future
 *                        work for its matrix-free CG, end of Section 2.1): z = P r with P the
 *                        cell-block Jacobi preconditioner, the inverse of each cell's diagonal
 *                        (N+1)^d x (N+1)^d block of the operator, applied in the generalised
 *                        eigenbasis of the 1D blocks (C, M) (tensor products of (N+1) x (N+1)
 *                        transforms); beta = <r', z'> / <r, z>; the stopping test stays on
 *                        ||r||_2. Allocates z in both precisions on first use. The one-kernel form
 *                        is not used with it. Every cell uses the interior block C along each
 *                        direction: next to a Dirichlet wall, and across a periodic direction of a
 *                        single cell, the true diagonal block also holds the wall or wrap
 *                        couplings; P stays symmetric positive definite there, only less exact.
 *                        0 (default) = the paper's unpreconditioned CG.
 *   PD_CFG_EXPLICIT_VISC 1 = the explicit-viscosity variant of Section 2.2: the viscous flux
 *                        -nu grad q is part of the explicit TVD-RK3 step of pd_step and pd_convect
 *                        (broken gradient at the nodes, averaged normal derivatives on faces,
 *                        Rusanov speed plus 2 nu (2N+1) / (h_e sqrt(pi/2)), eqs. Fu-Fw) and the
 *                        implicit viscous solves are skipped; pd_step then requires the viscous
 *                        part of the CFL condition eq. (CFL), dt (2N+1)^2 sum_d 2 nu / h_d^2 <= 1
 *                        (PD_EINVAL otherwise); pd_step_adjoint and pd_convect_adjoint reject it.
 *                        0 (default) = implicit viscosity (eq. implicitviscosity).
 *   PD_CFG_ONE_KERNEL    2D only: 1 = one kernel per CG iteration: the operator kernel of
 *                        iteration k also makes the residual update of iteration k - 1,
 *                        r_k = r_{k-1} - alpha_{k-1} q_{k-1}, and its x update (8 vector words
 *                        per DoF and iteration instead of 9, one launch instead of two), with
 *                        rho_k = |r_k|^2 expanded from <r_{k-1}, q_{k-1}> and <q_{k-1}, q_{k-1}>;
 *                        0 (default) = operator kernel + update kernel (measured as fast or
 *                        faster on gfx950). 3D solves always use two kernels.
 * The last six only change the launch shape; results are identical up to the block order of
 * the dot-product partial sums (for PD_CFG_DEFER_X also the rounding of x, for
 * PD_CFG_ONE_KERNEL the rounding of rho_k). */
enum {
  PD_CFG_STEP_PREC = 0, PD_CFG_P_RTOL = 1, PD_CFG_V_RTOL = 2, PD_CFG_MAXIT = 3,
  PD_CFG_CONVECTION = 4, PD_CFG_RU_FACTOR = 5, PD_CFG_TIMING = 6, PD_CFG_CHECK_EVERY = 7,
  PD_CFG_KZ = 8, PD_CFG_TILES_PER_WG = 9, PD_CFG_PREFETCH = 10, PD_CFG_TILE_VARIANT = 11,
  PD_CFG_DEFER_X = 12, PD_CFG_ONE_KERNEL = 13, PD_CFG_EXPLICIT_VISC = 14, PD_CFG_PRECOND = 15
};
int pd_configure(pd_ctx* ctx, int key, double value);

/* Timing hook: total milliseconds and launch count of the fused CG operator-apply kernel of
 * precision prec (PD_FP64: FP64 solves; PD_FP32: inner solves of PD_FP32_REFINE64) launched inside
 * pressure solves since the last reset (reset != 0 clears after reading). The sampled launches
 * (every PD_CFG_TIMING-th; requires PD_CFG_TIMING >= 1) carry start/stop HIP events in their
 * dispatch on the solve's stream; launches after convergence (early exits) are not counted.
 * bytes_per_launch: algorithmic bytes of one launch of the last timed solve (reads r and p_old,
 * writes p and A p, and with the deferred x update also reads and writes x: 6 words per DoF,
 * else 4; the one-kernel 2D form also reads A p_{k-1} and writes r: 8 words). Synchronises with
 * the last stream. */
int pd_timing(pd_ctx* ctx, int prec, double* total_ms, long long* launches,
              double* bytes_per_launch, int reset);

/* ---- Batched 2D pressure solves -------------------------------------------------------------
 * A batch holds `count` independent periodic 2D pressure systems A_p x = b (the PD_OP_PRESSURE
 * operator above, applied problem by problem): problem j has ncell[2j] x ncell[2j+1] cells on a
 * len[2j] x len[2j+1] domain and degree N[j] (0..8); all share dt. Batch vectors are packed: one
 * FP64 array in which problem j occupies elements [off[j], off[j+1]) in the element-blocked
 * layout of a single 2D problem (pd_batch_layout gives off). A solve advances all problems
 * together, each with its own CG scalars, stopping test and iteration count: a fixed chunk of
 * iterations (plus, for PD_FP32_REFINE64, the FP64 residual replacement of every unfinished
 * problem) is captured once into a HIP graph and replayed until every problem has stopped. */
typedef struct pd_batch pd_batch;

/* pd_batch_setup flags. PD_BATCH_AUTOTUNE: pick the operator tile shape (the three variants of
 * PD_CFG_TILE_VARIANT) per (degree, size bucket, precision) by timing the shapes on the batch's
 * own problems; size bucket = the largest power of two <= max(ncell). Choices are read from and
 * added to the text file named by the environment variable PD_AUTOTUNE_CACHE when it is set
 * (one "key variant" pair per line). PD_BATCH_RETUNE: time every bucket again, ignoring cached
 * choices. Without flags, cached choices are used where present, else variant 0. */
enum { PD_BATCH_AUTOTUNE = 1, PD_BATCH_RETUNE = 2 };

/* Create a batch (tables, descriptors, packed workspace; tuning if asked). ncell, len: 2*count
 * host values; N: count host values; dt > 0; each problem has at most 2^26 cells. The batched
 * operator runs one tile of cells per workgroup and every workgroup of a problem re-sums that
 * problem's per-tile partial sums at each iteration (O(tiles^2) reads per launch): the batch is
 * meant for many problems of up to about 512^2 cells; a single larger problem is better solved
 * with pd_cg_solve. On error *out is NULL and the message is available from
 * pd_batch_last_error(NULL). Synchronises. */
int pd_batch_setup(pd_batch** out, int count, const int* ncell, const double* len, const int* N,
                   double dt, unsigned flags, void* hip_stream);

/* Release the batch's device memory and graphs (waits for the device). NULL is ignored. */
void pd_batch_destroy(pd_batch* batch);

/* Last error message of batch (or of the last failed pd_batch_setup if NULL). Never NULL. */
const char* pd_batch_last_error(const pd_batch* batch);

/* offsets: count + 1 host values; offsets[j] = first packed element of problem j,
 * offsets[count] = total packed length. */
int pd_batch_layout(const pd_batch* batch, long long* offsets);

/* variants: count host values; tile variant (0..2) problem j uses in precision prec (PD_FP64, or
 * PD_FP32 for the inner iterations of PD_FP32_REFINE64). */
int pd_batch_variants(const pd_batch* batch, int prec, int* variants);

/* Settings (key, value):
 *   PD_BCFG_CHUNK  iterations per graph replay: even, 2..4096 (default 64). With
 *                  PD_FP32_REFINE64 the FP64 residual is replaced once per chunk.
 *   PD_BCFG_GRAPH  1 (default) = replay the captured graph, 0 = enqueue the same kernels one by
 *                  one each chunk (identical arithmetic; for comparison and debugging).
 *   PD_BCFG_RU_FACTOR  PD_FP32_REFINE64: a problem's FP32 iterations pause (until the chunk's
 *                  residual replacement) once their residual has dropped by this factor below the
 *                  last replaced one, in (0, 1) (default 1e-2). This keeps fast-converging
 *                  problems from iterating on FP32 rounding noise.
 *   PD_BCFG_PRECOND  1 = preconditioned CG with the cell-block Jacobi preconditioner of
 *                  PD_CFG_PRECOND (each problem's own degree and cell sizes), in both precisions;
 *                  the stopping tests stay on ||r||_2; 0 (default) = plain CG. */
enum { PD_BCFG_CHUNK = 0, PD_BCFG_GRAPH = 1, PD_BCFG_RU_FACTOR = 2, PD_BCFG_PRECOND = 3 };
int pd_batch_configure(pd_batch* batch, int key, double value);

/* Solve every problem of the batch: b = packed FP64 right-hand sides (read only; each problem's
 * part is first projected onto range(A_p) as in pd_cg_solve), x = packed FP64 solutions (out;
 * the initial guess is zero; each problem's result is projected onto range(A_p), the minimum
 * norm solution). prec: PD_FP64 (when the recurrence residual meets rtol ||b_j|| at an even
 * iteration, the FP64 residual b_j - A x_j recomputed at the chunk end decides: above the goal
 * but within 16x of it, the iterations resume from it with the same direction, at most 8 times,
 * each halving it; a larger gap is the FP64 rounding floor and ends the problem, as in
 * pd_cg_solve) or PD_FP32_REFINE64 (stop when the FP64 residual recomputed at a chunk end is
 * <= rtol ||b_j||). maxit caps each problem's iterations. info: count entries or NULL; iters
 * counts the iterations a problem ran (a problem stopped inside a chunk waits for the chunk end
 * without iterating); ms is the whole batch's time; rel_res_true is recomputed in FP64 for every
 * problem after the solve; outer_iters counts the chunk-end FP64 residual evaluations (at least
 * 1); fallback_iter: FP32 iterations run before a refinement problem continued in FP64 (-1 =
 * none). Synchronises. Returns PD_OK when every problem converged, else PD_EBREAKDOWN if any
 * problem broke down, else PD_ENOCONV. */
int pd_batch_cg_solve(pd_batch* batch, int prec, const void* b, void* x, double rtol, int maxit,
                      pd_solve_info* info, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* PD_H */
