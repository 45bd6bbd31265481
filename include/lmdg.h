/*
 * lmdg.h - C ABI of the MI355X (gfx950) low-memory S_N-DG transport solver.
 *
 * The library solves the scaled steady linear transport equation
 *     Omega . grad Psi + (sigma_s/eps + eps sigma_a) Psi = (sigma_s/eps) Psibar + eps q
 * (Sun & Hauck, "Low-memory, discrete ordinates, discontinuous Galerkin methods for
 * radiative transport", Sec. 1, eq-main) on a uniform Cartesian mesh of
 * [0, length_0] x [0, length_1] (x [0, length_2] in 3D) with multilinear (Q^1) upwind
 * DG in space and a discrete ordinates set in angle (Sec. 2.1), for three spaces:
 *   LMDG_SCHEME_STD    standard S_N-DG                       (Sec. 2.1, eq-sndg-scheme)
 *   LMDG_SCHEME_LMDG   low-memory space V_{h,0} + D_{h,1}    (Sec. 3.2, eq-gene-scheme)
 *   LMDG_SCHEME_RLMDG  low-memory space with upwind slope reconstruction
 *                                                            (Sec. 3.3, eq-rlmdg-vari)
 * Each is solved through the paper's dimension-reduced system with a Krylov method
 * (GMRES here); the operator of that system is applied with transport sweeps.
 * Slab geometry (Sec. 4.1, eq-1d) is a 2D handle with one row of cells and directions
 * (mu, 0), created with dim 1 (see lmdg_create).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int status (LMDG_OK on success).  No C++ exception and
 *   no abort crosses this boundary.  lmdg_status_string() names a status; the handle
 *   keeps a longer message for the last failure (lmdg_last_error()).
 * - Cells are numbered x fastest: p = i + n_0 * j (2D), p = i + n_0 * (j + n_1 * k) (3D).
 * - A "moment vector" holds Legendre moments of a Q^1 field on every cell, moment
 *   major: v[r * n_cells + p], r = 0..n_P-1.  2D: n_P = 4, basis 1, xi, eta, xi*eta
 *   (xi = 2(x - x_c)/h_0, eta = 2(y - y_c)/h_1).  3D: n_P = 8, basis index
 *   r = bx + 2 by + 4 bz for xi^bx eta^by zeta^bz (1, xi, eta, xi eta, zeta, xi zeta,
 *   eta zeta, xi eta zeta).  Krylov vectors, right-hand sides and scalar fluxes all
 *   use this layout (n_P * n_cells doubles).  For LMDG/RLMDG moment 0 is X_0
 *   (per-cell scalar-flux average) and moments 1..n_P-1 are X_1 of Sec. 3.2 Step 3.
 * - Right-hand sides: a handle carries n_rhs sources (1 after lmdg_set_materials,
 *   n after lmdg_set_sources).  Every vector argument of lmdg_sweep, lmdg_apply,
 *   lmdg_rhs, lmdg_recover and lmdg_solve then holds the n_rhs fields stacked:
 *   v[(k * n_P + r) * n_cells + p] for right-hand side k (sweep outputs and angular
 *   fluxes likewise, with their own per-right-hand-side sizes).  All right-hand sides
 *   share each sweep launch; the solver runs one GMRES instance per right-hand side.
 * - Pointers documented as "device" must point to memory of the handle's GPU
 *   (e.g. torch CUDA tensors); "host" pointers are ordinary CPU memory.  The caller
 *   owns every array it passes; the handle owns its internal workspaces.
 * - `stream` is a hipStream_t (NULL = the default stream).  All device work of a
 *   call is enqueued on it; calls that report iteration counts or residuals
 *   synchronise it before returning.
 * - lmdg_sweep, lmdg_apply, lmdg_rhs and lmdg_recover only enqueue work and return at
 *   once.  The sweeps hand data between workgroups through progress words, and every
 *   wait for one is bounded: a wait that gives up (a fault of the device or of the
 *   library, never of the caller's data) sets a sticky flag in the handle and the
 *   kernel still finishes, with wrong numbers.  The flag is read and cleared by the
 *   next synchronising call on the handle (lmdg_synchronize, lmdg_solve,
 *   lmdg_adjoint_solve), which then returns LMDG_HIP_ERROR; callers of the
 *   asynchronous functions check their results with lmdg_synchronize.
 * - A handle is not re-entrant: calls on one handle must not overlap.
 * - Supported: dim = 2 (STD, LMDG, RLMDG) with prescribed inflow and sources given by
 *   their cell moments (isotropic or per direction); dim 3 (LMDG, RLMDG) with vacuum
 *   inflow and per-cell constant sources; per-cell constant cross sections and eps.
 *   Anything else returns LMDG_UNSUPPORTED.
 */
#ifndef LMDG_H
#define LMDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LMDG_OK 0
#define LMDG_INVALID_ARG 1
#define LMDG_NOT_CONVERGED 2
#define LMDG_NONFINITE 3
#define LMDG_HIP_ERROR 4
#define LMDG_UNSUPPORTED 5

#define LMDG_SCHEME_STD 0
#define LMDG_SCHEME_LMDG 1
#define LMDG_SCHEME_RLMDG 2

/* arithmetic of the sweeps (local solves and quadrature sums); reductions into
 * moment vectors, B_11, GMRES and residuals are always FP64 */
#define LMDG_PREC_FP64 0
#define LMDG_PREC_FP32 1

/* solve modes */
#define LMDG_MODE_FP64 0   /* FP64 sweeps inside FP64 GMRES */
#define LMDG_MODE_MIXED 1  /* FP32 sweeps inside FP64 GMRES, FP64 iterative refinement */

/* preconditioners of the reduced system (lmdg_set_preconditioner) */
#define LMDG_PRECOND_NONE 0
#define LMDG_PRECOND_CELL 1       /* cell blocks of K only */
#define LMDG_PRECOND_TWO_LEVEL 2  /* cell blocks + the diffusion-limit correction */

typedef struct lmdg_handle lmdg_t;

typedef struct lmdg_info {
  int iterations;           /* total inner GMRES iterations (operator applications) */
  int restarts;             /* GMRES restart cycles */
  int ir_passes;            /* outer refinement passes (MIXED), 1 for FP64 */
  int converged;            /* 1 when the true relative residual met tol */
  double rel_residual;      /* ||b - K x||_2 / ||b||_2 with the FP64 operator */
  double time_total_ms;     /* wall time of the call */
  double time_apply_ms;     /* time in operator applications (event timed) */
} lmdg_info;

/* Message for a status code (static storage). */
const char* lmdg_status_string(int status);

/* Message of the last failure on this handle (static storage if h is NULL). */
const char* lmdg_last_error(const lmdg_t* h);

/*
 * Level-symmetric LQ_N quadrature (host).  Sec. 2.1, eq-polyquad: positive weights,
 * exact for polynomials of degree <= 2 in Omega.  Levels mu_i^2 = mu_1^2 +
 * (i-1) 2(1-3 mu_1^2)/(N-2); octant points (mu_i, mu_j, mu_k), i+j+k = N/2+2;
 * permutation classes share a weight solving the even-moment equations (minimum
 * norm for N = 16); mu_1 makes the next even moment exact.  dim 2 keeps the
 * Omega_z > 0 hemisphere projected to (Omega_x, Omega_y), weights renormalised.
 *   order    N in {4, 6, 8, 12, 16}
 *   capacity size of the caller's arrays in directions (>= N(N+2)/2 for dim 2,
 *            N(N+2) for dim 3)
 *   n_dir    out: number of directions
 *   omega    out, host, n_dir x dim row-major
 *   w        out, host, n_dir, sum 1
 * Errors: INVALID_ARG for other orders/dims or too small capacity.
 */
int lmdg_quadrature_level_symmetric(int dim, int order, int capacity, int* n_dir,
                                    double* omega, double* w);

/*
 * Create a handle on the current HIP device for a uniform mesh of n[0] x ... x
 * n[dim-1] cells of [0, length[0]] x ... (host arrays of dim entries) and the
 * quadrature (omega: n_dir x dim, w) (host arrays, copied).  The quadrature must
 * satisfy eq-polyquad (i)-(iii) to 1e-12, have positive weights and no zero
 * component (the upwind direction along every axis must be defined), and at most 36
 * directions per quadrant / octant (2D S16 has 36, 3D S8 has 10).
 * dim 1 (slab geometry, eq-1d): n[0] cells of [0, length[0]], omega = the n_dir values
 * mu (nonzero, sum w = 1, sum w mu = 0, sum w mu^2 = 1/3, e.g. a Gauss rule with weights
 * halved, at most 36 per sign of mu).  The handle is the 2D problem on n[0] x 1 cells of
 * [0, length[0]] x [0, 1] with directions (mu, 0): no y face carries flux, so its 1 and
 * xi moments are the slab scheme's.  Vectors use the 2D layout (4 moments per cell);
 * rows 0 and 1 are the slab moments, rows 2 and 3 (eta, xi eta) carry no slab
 * quantity and stay zero (RLMDG reconstructs along x only on slab handles).  lmdg_adjoint_solve returns UNSUPPORTED on slab handles.
 * Errors: INVALID_ARG (NULL pointers, sizes < 1, quadrature violations),
 *         UNSUPPORTED (dim not 1, 2 or 3), HIP_ERROR (allocation).
 */
int lmdg_create(int dim, const int64_t* n, const double* length, int n_dir,
                const double* omega, const double* w, lmdg_t** out);

void lmdg_destroy(lmdg_t* h);

/*
 * Cross sections, source and inflow data (device arrays, copied into the handle):
 * sigma_s >= 0, sigma_a >= 0, eps > 0 per cell (eq-main; a per-cell eps describes a
 * multiscale medium), q = per-cell constant source (n_cells each).  sigma_a = 0 is
 * accepted; the paper's analysis assumes sigma_a >= delta_a > 0, and without
 * absorption the reduced systems can be arbitrarily ill-conditioned.
 * alpha: the inflow boundary values Psi = alpha on Gamma^- of eq-main, NULL for vacuum.
 *   2D (device, n_dir x (n_1 + n_0) x 3 doubles): for direction l (the caller's index)
 *   entries f = 0..n_1-1 describe the x-inflow face of mesh row f (x = 0 if
 *   Omega_x > 0, x = length_0 otherwise), entries f = n_1 + i the y-inflow face of
 *   column i (y = 0 if Omega_y > 0, y = length_1 otherwise).  Each entry holds
 *   (a0, a1, m): a0 = (1/|F|) int_F alpha, a1 = (3/|F|) int_F alpha t with t in
 *   [-1, 1] the cell coordinate along the face (eta on x faces, xi on y faces), so that
 *   a0 + a1 t is the L2 projection onto the face's linear functions, which is all the
 *   Q^1 test functions see of alpha (the boundary term of Q in eq-Ljk), and m = alpha
 *   at the face midpoint, the upwind value the reconstruction of Sec. 3.3.1 uses in the
 *   inflow cell (RLMDG).  Slab handles (dim 1): n_dir doubles, alpha of direction l at
 *   its inflow end (x = 0 for mu > 0, x = length_0 otherwise).  3D: must be NULL.
 *   Faces on the outflow side of a direction are never read.
 * The call replaces any sources set before (one right-hand side, q).
 * Errors: INVALID_ARG (NULL, negative values, eps <= 0), NONFINITE,
 *         UNSUPPORTED (alpha on a 3D handle).
 */
int lmdg_set_materials(lmdg_t* h, const double* sigma_s, const double* sigma_a,
                       const double* eps, const double* q, const double* alpha,
                       void* stream);

/*
 * Replace the handle's source by one given through its cell moments (2D and slab
 * handles; eq-Ljk: Q_{l,K}(v) = eps int_K q_l v):
 *   per_direction 0: qm[r * n_cells + p] = (1/|K_p|) int_{K_p} q b_r dx, r = 0..3, an
 *                    isotropic source (the four Legendre moments of each cell);
 *   per_direction 1: qm[(l * 4 + r) * n_cells + p], the same for the source q_l of
 *                    direction l (the caller's index), e.g. a manufactured source.
 * Device array.  The inflow data of lmdg_set_materials stay; the handle has one
 * right-hand side afterwards.  Slope moments of the source enter the low-memory
 * schemes through the isotropic slope rows of the reduced right-hand side (Step 1 of
 * Sec. 3.2), direction-dependent constant moments through the source sweep.
 * Errors: INVALID_ARG (materials not set, NULL, per_direction not 0 or 1), NONFINITE,
 *         UNSUPPORTED (3D handle).
 */
int lmdg_set_source_moments(lmdg_t* h, int per_direction, const double* qm, void* stream);

/*
 * n_rhs per-cell constant sources q (device, n_rhs * n_cells doubles, right-hand
 * side k at q[k * n_cells + p]) replacing the single source of lmdg_set_materials;
 * the cross sections and eps stay.  The source term of right-hand side k is
 * eps q_k (eq-main).  All right-hand sides are swept together (one schedule, one
 * set of per-cell coefficients per launch); solves run one GMRES instance each.
 * Errors: INVALID_ARG (materials not set, NULL, n_rhs < 1 or > 64), NONFINITE.
 */
int lmdg_set_sources(lmdg_t* h, int n_rhs, const double* q, void* stream);

/*
 * One sweep of all directions followed by the angular reductions (Sec. 2.1.1 for
 * STD, eq-nonrec-block for LMDG, Sec. 3.3.2 for RLMDG), without the identity/B_11
 * part of the reduced operator.  Solves, per direction, L_l Psi_l = S_l with
 *   S = M x + Q            (STD; x, Q optional)
 *   S = M_0 x_0 + L_01 Sigma^T x_1 + Q~_0     (LMDG, RLMDG; L~_00 for RLMDG)
 * and returns the per-cell sums over directions (device, out_moments x n_cells):
 *   STD:   n_P moments of P Psi
 *   LMDG:  [P_0 Psi ; Sigma L_10 Psi (xi, eta, xi*eta rows)]
 *   RLMDG: [P_0 Psi ; G Psi (3 rows) ; P_1 R Psi (xi, eta)] with the second block row
 *          G = Sigma (L_10 + L_11 R) - Sigma M_1 P_1 R of Sec. 3.3.2 (the scattering
 *          part is taken per direction, where it cancels most of L_11 R)
 *   3D (rows of Sigma L_10 and G indexed by slope moment 1..7):
 *   STD:   the 8 moments of P Psi (8 x 8 local solves of eq-Ljk)            8 rows
 *   LMDG:  [P_0 Psi ; Sigma L_10 Psi (7 rows)]                              8 rows
 *   RLMDG: [P_0 Psi ; G Psi (7 rows) ; P_1 R Psi (xi, eta, zeta)]           11 rows
 *   x        device moment vector or NULL (= 0)
 *   use_q    1 adds the source Q, 0 omits it
 *   out      device, n_out * n_cells doubles (n_out = 4, 4, 6 for STD, LMDG, RLMDG in
 *            2D; 8, 8, 11 in 3D)
 *   psi      optional device output of the angular flux (cell averages for
 *            LMDG/RLMDG, all n_P moments for STD), layout psi[(l*m + r)*n_cells + p]
 *            with l the caller's direction index, m = 1 (LMDG/RLMDG) or n_P (STD);
 *            FP64, NULL to skip.
 */
int lmdg_sweep(lmdg_t* h, int scheme, int prec, const double* x, int use_q,
               double* out, double* psi, void* stream);

/* K x of the reduced system (device moment vectors).  Unit of the
 * cell-direction-updates/s metric: one call = n_cells * n_dir updates.  The standard
 * scheme on 3D handles applies the operator as printed, K Phi = Phi - P L^{-1} M Phi
 * (eq-sndg-phi); the 2D standard and all low-memory operators use the defect form,
 * the same operator with the sigma_s/eps parts cancelled before the sweep. */
int lmdg_apply(lmdg_t* h, int scheme, int prec, const double* x, double* y, void* stream);

/*
 * lmdg_apply for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same K x, with
 * the sweep workspace (quadrant partials, edge traces, 3D per-cell coefficients, progress words,
 * ticket counter, wait flag) taken from a fixed array of 64 MiB that the library holds
 * on each GPU it runs on until the process ends, instead of the handle's buffers.  The
 * call allocates nothing (no hipMalloc, no event creation); the caller passes x and y
 * as for lmdg_apply, and the handle's device must be the current device.  Every call on
 * a GPU shares that GPU's array and starts by clearing its counters: calls that
 * overlap on one GPU (several streams, threads or handles at once) race and must be
 * serialised by the caller.  A failed bounded wait is carried over to the handle's own
 * flag and reported by its next synchronising call, as for lmdg_apply.
 * Errors: INVALID_ARG (as lmdg_apply; the handle's device not current; a workspace
 * larger than the fixed array, e.g. the 2D S16 or several-source workloads on large
 * meshes - lmdg_workspace_bytes does not apply, the message gives the size),
 * HIP_ERROR.
 */
int lmdg_apply_noalloc(lmdg_t* h, int scheme, int prec, const double* x, double* y, void* stream);

/* Right-hand side b of the reduced system (device moment vector). */
int lmdg_rhs(lmdg_t* h, int scheme, int prec, double* b, void* stream);

/* Step 4 / eq-sndg-final-sweep: scalar-flux moments phi (device moment vector)
 * from a solution x of the reduced system; psi as in lmdg_sweep (nullable). */
int lmdg_recover(lmdg_t* h, int scheme, int prec, const double* x, double* phi,
                 double* psi, void* stream);

/*
 * Solve K x = b with restarted GMRES(restart) from x0 (device, NULL = 0) until the
 * true FP64 relative residual ||b - K x|| / ||b|| <= tol, then recover the scalar
 * flux.  mode FP64: FP64 sweeps.  mode MIXED: an FP64 refinement loop around inner
 * GMRES solves that use FP32 sweeps and keep their Krylov basis in FP32 (products and
 * sums in FP64, lmdg_set_refinement sets their target); the FP64 operator defines the
 * residual.  The
 * restarts are augmented with earlier corrections when lmdg_set_augment set k > 0.
 *   x_out    device moment vector (solution of the reduced system)
 *   phi_out  device moment vector (scalar flux), NULL to skip
 *   info     host, filled also when NOT_CONVERGED is returned; with several
 *            right-hand sides rel_residual is the largest over them, converged
 *            means all converged, and iterations counts shared operator applications
 * Errors: INVALID_ARG (tol <= 0, restart < 1, max_iter < 1), NOT_CONVERGED.
 */
int lmdg_solve(lmdg_t* h, int scheme, int mode, double tol, int restart, int max_iter,
               const double* x0, double* x_out, double* phi_out, lmdg_info* info,
               void* stream);

/*
 * Reconstruction of the RLMDG scheme (Sec. 3.3.1) used by every later RLMDG call on
 * this handle (2D and slab handles).  The paper names two variants without formulas;
 * the library takes these readings:
 *   stencil 2   the two-cell upwind difference of Sec. 3.3.1 (the default);
 *   stencil 3   RLMDG* (discussion of fig-efficiency): in cells with two upwind
 *               neighbours along an axis the slope is the derivative at the cell centre
 *               of the quadratic through the three upwind-inclusive cell averages,
 *               Legendre coefficient s (3 u - 4 u_up + u_upup) / 4; two-cell difference
 *               with one upwind neighbour, boundary difference in the inflow cell;
 *   suppress 1  (examp-disccross1) no slope along an axis where the upwind neighbour
 *               has other cross sections (sigma_s/eps or eps sigma_a); a three-cell
 *               stencil falls back to two cells when its far cell differs.
 * With a variant the RLMDG operator is applied in the plain form of eq-nonrec-block
 * (the defect form that keeps FP32 sweeps accurate at small eps covers the default
 * reconstruction only), and the sweeps hand four trace values downwind.
 * Errors: INVALID_ARG (stencil not 2 or 3, suppress not 0 or 1), UNSUPPORTED (a variant
 * on a 3D handle).
 */
int lmdg_set_reconstruction(lmdg_t* h, int stencil, int suppress);

/*
 * Restart augmentation of the handle's GMRES solves (lmdg_solve, lmdg_adjoint_solve
 * and the inner solves of mode MIXED).  With k > 0 each restart cycle also searches
 * the corrections of the last k cycles (LGMRES of Baker, Jessup and Manteuffel,
 * SIAM J. Matrix Anal. Appl. 26, 2005): after the restart Krylov steps the basis is
 * extended with the stored images K z of those corrections, which costs no operator
 * application, so the cycle minimises the residual over the Krylov space plus the
 * span of the old corrections.  This counters the stagnation of restarted GMRES on
 * the reduced systems of small eps, whose spectra reach close to zero.
 *   k  0 (plain GMRES, the default) .. 250 - restart; a larger k is clamped in each
 *      solve to 250 - restart.  Memory: 3 k + 2 further vectors of the solve's length.
 * Errors: INVALID_ARG (k < 0 or k > 249).
 */
int lmdg_set_augment(lmdg_t* h, int k);

/*
 * Iterative refinement of mode MIXED (lmdg_solve, lmdg_adjoint_solve): each pass
 * computes the FP64 residual r and solves K d = r with FP32 sweeps until the inner
 * relative residual is inner_tol (or the FP32 operator stops making progress); fewer
 * digits per pass mean more passes, each of which restarts the Krylov space, more
 * digits mean longer inner solves.  Which is faster depends on the system: 1e-3
 * (the default) suits the preconditioned 2D solves, 1e-4 the 3D ones.
 *   inner_tol  1e-6 .. 0.5 (FP32 sweeps carry about 1e-6 relative error)
 * Errors: INVALID_ARG (inner_tol outside that range).
 */
int lmdg_set_refinement(lmdg_t* h, double inner_tol);

/*
 * Preconditioner of the handle's GMRES solves of the reduced LMDG and RLMDG systems
 * (lmdg_solve, the LMDG adjoint solve and the inner solves of mode MIXED), applied on
 * the right: GMRES works on K M^{-1} u = b and the iterate is X = M^{-1} u, so the
 * solution and the stopping test on ||b - K X|| are those of the unpreconditioned
 * solve.  The paper leaves preconditioning of the dimension-reduced system to future
 * work (Sec. 5, item (ii)); this one is built on its eps -> 0 limit of the low-memory
 * scheme (Sec. 3.1, eq-difflimPF):
 *     M^{-1} r = K_loc^{-1} r + Z B^{-1} W r.
 * K_loc is, per cell, the 4 x 4 diagonal block of K (rows and columns X_0, X_1 of the
 * cell).  W turns the residual into the source it stands for in the full scheme (cell
 * moments (sigma_s/eps) r_0 and -r_m / (|K| n_m), n = 1/3, 1/3, 1/9) loaded onto nodal
 * Q^1 functions.  B is the eq-difflimPF form with coefficient 1/(3 sigma_t) and
 * absorption eps sigma_a plus 1/2 of the boundary mass (vacuum), absorption and boundary
 * terms lumped, keeping the couplings of nodes of equal parity of i + j (all of them on
 * square cells).  Z maps nodal values to [cell average ; minus the slope moments], for
 * RLMDG plus the angular average of the reconstructed slopes of the cell averages.  B^{-1}
 * is applied by `cycles` multigrid V-cycles (one per parity class; Galerkin coarse
 * operators, Gauss-Seidel smoothing, dense coarsest solve), a fixed linear map.
 *   kind    LMDG_PRECOND_NONE (default), LMDG_PRECOND_CELL (K_loc^{-1} only) or
 *           LMDG_PRECOND_TWO_LEVEL.
 *   cycles  1 .. 50 V-cycles per application (kind TWO_LEVEL; one is usually enough).
 * The setup (cell blocks for the scheme of the solve, multigrid hierarchy) runs at the
 * first use after lmdg_set_materials; its memory (16 doubles per cell, about 5 per node
 * of the multigrid) is counted by lmdg_workspace_bytes, and a preconditioned solve holds
 * two further vectors of the solve's length.  Solves of STD, of an RLMDG reconstruction
 * variant and of the RLMDG adjoint system run without it.
 * Errors: INVALID_ARG (kind or cycles out of range), UNSUPPORTED (a 3D or slab handle
 * with kind != NONE).
 */
int lmdg_set_preconditioner(lmdg_t* h, int kind, int cycles);

/*
 * z = M^{-1} r for every right-hand side of the handle (device moment vectors of the
 * reduced system; see lmdg_set_preconditioner) with the handle's kind and cycles; kind
 * NONE copies r.  Enqueues on `stream`; builds the preconditioner first if needed.
 * Errors: INVALID_ARG (NULL vectors, materials not set), UNSUPPORTED (a scheme or handle
 * the preconditioner does not cover), HIP_ERROR.
 */
int lmdg_precond_apply(lmdg_t* h, int scheme, const double* r, double* z, void* stream);

/*
 * Detector response and its gradients (2D, all three schemes).
 * J = int_D phi_h d dx for detector moments det (device moment vector,
 * det[r*n_cells + p] = int_{K_p} d b_r dx; for the indicator of a box, the exact
 * integral of each basis function over the part of the cell inside the box).
 * The scheme's discrete system A y = b (eq-sndg-scheme; eq-lmdg-block with the
 * trial map of eq-gene-scheme; eq-rlmdg-vari) is solved forward, then A^T lambda =
 * dJ/dy, and the derivatives of the bilinear form of eq-Ljk with respect to the
 * per-cell data give
 *   g_sigma_a = -eps sum_l w_l int_K psi_l lambda_l,
 *   g_sigma_s = -(1/eps) (sum_l w_l int_K psi_l lambda_l - int_K phi Lambda),
 *   g_q       =  eps int_K Lambda           (Lambda = sum_l w_l lambda_l),
 * i.e. dJ/d(sigma_s, sigma_a, q) of cell K for the discrete J, with psi the forward
 * field of the trial space (for RLMDG including its reconstructed slopes) and lambda
 * the adjoint field of the test space.  Both solves use mode, tol, restart and
 * max_iter as lmdg_solve does.  The quadrature must be centrally symmetric (-Omega with
 * the same weight for every Omega): the adjoint sweep of direction Omega is then a
 * forward-type sweep of -Omega.  STD and LMDG are Galerkin, so their adjoint is the
 * forward system with the detector as source.  RLMDG is Petrov-Galerkin: its adjoint is
 * the scheme with trial space V^lm and test functions reconstructed from the downwind
 * side, which the library solves by its own reduced system (sweeps with the local
 * operator L_00 + R'^T L_10, R' the downwind reconstruction, and the same GMRES).
 *   det                device, 4 * n_cells doubles (moment-major)
 *   g_sigma_s, g_sigma_a, g_q   device outputs, n_cells doubles each
 *   J_out              host output
 *   info               host; iterations, restarts and passes summed over both solves
 * The angular fluxes are never stored for all directions: the gradient sum is built
 * one quadrant at a time, recomputing that quadrant's forward fluxes and the opposite
 * quadrant's adjoint-type fluxes with two restricted sweeps (the handle keeps
 * 2 x slots x n_cells doubles for LMDG and RLMDG, 8 x slots x n_cells for STD, slots =
 * the padded directions per quadrant; RLMDG also n_dir x n_cells for the adjoint source).
 * Errors: UNSUPPORTED (3D meshes, slab handles, RLMDG with a reconstruction variant),
 * INVALID_ARG (NULL pointers, bad solver arguments, quadrature without central symmetry,
 * more than one right-hand side on the handle), NOT_CONVERGED (either solve, or the
 * conjugate gradients of B_11 that give the slope part of the LMDG adjoint source),
 * HIP_ERROR.
 */
int lmdg_adjoint_solve(lmdg_t* h, int scheme, int mode, const double* det, double tol,
                       int restart, int max_iter, double* g_sigma_s, double* g_sigma_a,
                       double* g_q, double* J_out, lmdg_info* info, void* stream);

/*
 * Device memory of the handle (host outputs, bytes): *held = what it owns now (mesh
 * and direction tables, materials and source data, sweep workspaces for its current
 * number of right-hand sides, Krylov and adjoint buffers of earlier solves);
 * *solve = what an lmdg_solve with this restart (and the augmentation set by
 * lmdg_set_augment) would allocate on top of that (0 once a solve of that size ran).
 * Errors: INVALID_ARG (NULL, restart < 1 or > 250).
 */
int lmdg_workspace_bytes(const lmdg_t* h, int restart, int64_t* held, int64_t* solve);

/*
 * Wait for all work of the handle on `stream` and report whether any sweep launched
 * since the last synchronising call had a wait that gave up (LMDG_HIP_ERROR; the flag
 * is cleared).  LMDG_OK means every result enqueued so far is complete and valid.
 */
int lmdg_synchronize(lmdg_t* h, void* stream);

/*
 * Bounded waits of the sweeps, for tests of the failure path: every wait for a
 * progress word polls it at most `spins` times (default 2^25, about a second) before
 * it gives up; unreachable = 1 makes every wait target a value no producer writes, so
 * every wait that is reached gives up after `spins` polls while all kernels still run
 * to completion (the numbers are then wrong and the next synchronising call reports
 * LMDG_HIP_ERROR).  unreachable = 0 restores normal waits.
 * Errors: INVALID_ARG (spins < 1, unreachable not 0 or 1).
 */
int lmdg_set_wait_limit(lmdg_t* h, long long spins, int unreachable);

/*
 * Kernel timing for measurement: while enabled, every sweep-kernel launch of this
 * handle is bracketed by HIP events recorded on its launch stream.
 * lmdg_sweep_kernel_time() waits for the recorded events and returns the summed
 * kernel time in milliseconds and the number of launches since the last query
 * (or since enabling), then clears the record.  Host pointers.
 */
int lmdg_profile(lmdg_t* h, int enable);
int lmdg_sweep_kernel_time(lmdg_t* h, double* total_ms, int* launches);

#ifdef __cplusplus
}
#endif

#endif /* LMDG_H */
