/*
 * bddc.h -- C ABI of libbddc.so: BDDC-preconditioned conjugate gradients for
 * Q1 finite-element diffusion problems on box partitions, on one MI355X.
 *
 * Method: the BDDC preconditioner of Goebel, Cojean and Anzt, "BDDC
 * preconditioning on GPUs for Cardiac Simulations" (arXiv 2410.14786), Sec. 2:
 *   A = sum_i R_i^T A_i R_i,
 *   coarse basis Phi_i from the saddle-point systems of eq. (1),
 *   A_c = sum_i R_ci^T Phi_i^T A_i Phi_i R_ci,
 *   constraints: full values at corners, averages over edges and faces,
 *   weights w = 1/kappa (kappa = number of subdomains sharing a dof),
 *   M^{-1} r = v1 + v2 + v3 with v1 the coarse correction (eq. (2)), v2 the
 *   weighted constrained local solves (eqs. (3), (4)) and v3 the
 *   static-condensation correction on subdomain interiors applied to
 *   r1 = r - A (v1 + v2) (eq. (5)),
 * inside CG preconditioned by M (Sec. 2 and Sec. 3).
 *
 * Problem statement fixed by this ABI (the paper's unit-square Poisson
 * setting, Sec. 3, extended to 3D and per-element conductivity):
 *   -div(theta grad u) = f on the unit square (dim 2) or cube (dim 3),
 *   u = 0 on the whole boundary, Q1 elements on a uniform grid of nel[a]
 *   elements per axis, theta > 0 constant per element.  The unknowns are the
 *   interior nodes; free dof index (ix-1) + (nx-1)*((iy-1) + (ny-1)*(iz-1)),
 *   x fastest.  The right-hand side b is the assembled load vector itself.
 *
 * Conventions for every entry point:
 *   - Return value 0 (BDDC_OK) or a negative bddc_status; nothing throws.
 *   - Vector arguments (r, z, b, x, u, lam, g) are DEVICE pointers to float64
 *     arrays owned by the caller, which must stay valid until the ctx's stream
 *     has passed the call.  They must not alias each other.
 *   - All work is enqueued on the stream given at setup (a hipStream_t, e.g.
 *     torch.cuda.current_stream().cuda_stream; NULL = the default stream).
 *   - One ctx per stream; a ctx has no internal locking.
 */
#ifndef BDDC_H
#define BDDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BDDC_OK = 0,
  BDDC_EINVAL = -1,      /* bad dimension, sizes, cuts, pointers or options      */
  BDDC_ENOTSPD = -2,     /* theta <= 0, a non-positive pivot in a local or the
                            coarse Cholesky factor, or a box that touches no
                            Dirichlet boundary while corner constraints are off
                            (its A_RR is singular; found by the planner)          */
  BDDC_ENOMEM = -3,      /* device or host allocation failed                      */
  BDDC_EHIP = -4,        /* a HIP runtime call failed                             */
  BDDC_ENOCONV = -5,     /* maxit reached; x and info are still filled            */
  BDDC_EBREAKDOWN = -6,  /* CG breakdown: (p, A p) <= 0 or (r, z) <= 0 or NaN     */
  BDDC_ENOTIMPL = -7     /* a valid request the library does not support          */
} bddc_status;

/* Constraint selection (paper Sec. 2: corner values, edge and face averages).
 * BDDC_ALL_PRIMAL makes every interface node a primal (point) constraint; it
 * exists for tests (the preconditioner is then an exact inverse on interface
 * residuals) and needs at most 64 constraints per subdomain. */
enum { BDDC_CORNERS = 1, BDDC_EDGES = 2, BDDC_FACES = 4, BDDC_ALL_PRIMAL = 8 };

/* Setup option flag for tests: when setup fails after the device stage
 * started (e.g. ENOTSPD), still return the context in *out so that its data
 * can be inspected with bddc_debug_read; it must then be destroyed. */
enum { BDDC_SETUP_KEEP_ON_ERROR = 1 };

/* Setup option flag: iterate CG on the whole space with the three-part
 * preconditioner exactly as written in the paper (Sec. 2: M^{-1} r = v1 + v2 + v3
 * applied every iteration, r1 and v3 included).  Without it, bddc_pcg_solve runs
 * the same preconditioned CG restricted to interface dofs: from x0 = P_I b every
 * residual vanishes on subdomain interiors and every search direction is
 * discrete-harmonic, so CG with A on those vectors is CG with the assembled
 * Schur complement S = sum_i R_i^T (A_BB - A_BI A_II^{-1} A_IB)_i R_i, and the
 * preconditioned residual restricted to the interface is v1 + v2 (v3 only
 * changes interior values).  Both give the same iterates in exact arithmetic;
 * the interior values of x are recovered once at the end by the interior
 * solves of eq. (5).  bddc_apply always applies the full three-part operator.
 * The interface operator and the interior solves come from the local factors
 * and must be exact, so the interface form keeps FP64 factors also with
 * local_bits = 32 and runs the preconditioner's local solves (there explicit
 * interface matrices) in FP32; see bddc_options.local_bits. */
enum { BDDC_SETUP_FULL_SPACE = 2 };

/* Setup option flag, beyond the paper (which fixes w = 1/kappa, Sec. 2):
 * coefficient-aware weights (rho-scaling).  rho_i(x) is the largest
 * conductivity among subdomain i's elements that contain node x and
 * w_i(x) = rho_i(x) / sum_j rho_j(x) over the subdomains sharing x: a partition
 * of unity that equals 1/kappa for a constant conductivity.  Only the weights
 * W_i change; every step of the method is otherwise the same. */
enum { BDDC_SETUP_RHO_SCALING = 4 };

/* Setup option flag: solve the coarse problem of eq. (2) by CG, as the paper
 * does (Sec. 2), instead of the explicit inverse of its dense FP64 Cholesky
 * factor: CG on the assembled A_c with its diagonal as preconditioner (the
 * paper's CG is unpreconditioned), from zero to a relative residual of 1e-13
 * (at most 2000 iterations) at every application of the preconditioner, in one
 * workgroup when A_c and the CG vectors fit its LDS, else with the rows of A_c
 * split over 64 workgroups that meet at grid barriers (their waits are bounded
 * by the "wait_polls" limit of bddc_set_limit).  No dense coarse factor or
 * inverse is formed; A_c is checked for a positive diagonal only, and a coarse
 * matrix that is not positive definite ends that inner CG early instead of
 * failing setup.  The explicit inverse is faster on one GPU. */
enum { BDDC_SETUP_COARSE_CG = 8 };

/* Solve flags. */
enum { BDDC_X0_GIVEN = 1 /* use x on entry as the initial guess */ };

typedef struct bddc_ctx bddc_ctx;  /* opaque; owns all device state */

/* Q1 mesh on the unit square (dim 2, nel[2] ignored) or cube (dim 3). */
typedef struct {
  int32_t dim;
  int64_t nel[3];
} bddc_mesh;

/* Tensor-product box partition, HOST arrays: per axis a,
 * cuts[a][0] = 0 < cuts[a][1] < ... < cuts[a][nsub[a]] = nel[a].
 * Box (bx, by, bz) has index bx + nsub[0]*(by + nsub[1]*bz).  Every box must
 * be at least 2 elements long along each axis. */
typedef struct {
  int32_t nsub[3];
  const int64_t* cuts[3];
} bddc_partition;

/* Per-element conductivity, prod(nel) values, element (ex,ey,ez) at
 * ex + nx*(ey + ny*ez).  on_device = 0: host pointer; 1: device pointer. */
typedef struct {
  const double* theta;
  int32_t on_device;
} bddc_coefficients;

typedef struct {
  int32_t local_bits;   /* 64: local factors and solves in FP64.  32: the
                           preconditioner's local solves in FP32, with FP32
                           accumulation; the outer CG, r1, the coarse factor and
                           solve stay FP64.  With BDDC_SETUP_FULL_SPACE the local
                           Cholesky factors and every triangular solve are FP32.
                           In the interface form the factors are FP64 and the
                           local solves of the preconditioner (the matrices X^T X
                           and W_G^T X of eqs. (2)-(4) on the interface) are
                           stored and applied in FP32; bddc_apply then applies
                           the FP64 three-part operator. */
  int32_t use_graph;    /* 1: replay PCG iterations from a captured HIP graph   */
  int32_t nb_override;  /* 0 = default tile size (64); other values: ENOTIMPL   */
  void* stream;         /* hipStream_t for all work of this ctx                 */
  int32_t flags;        /* BDDC_SETUP_FULL_SPACE, BDDC_SETUP_RHO_SCALING,
                           BDDC_SETUP_COARSE_CG and/or BDDC_SETUP_KEEP_ON_ERROR */
} bddc_options;

typedef struct {
  int32_t iters;        /* CG iterations taken                                  */
  double relres_true;   /* ||b - A x||_2 / ||b||_2 at exit                       */
  double relres_rec;    /* recursively updated ||r||_2 / ||b||_2 at exit         */
  double cond_est;      /* Lanczos estimate of cond(M^{-1} A) from the CG
                           coefficients (1 when no iteration was taken)          */
  double t_setup_ms;    /* wall time of bddc_setup                               */
  double t_solve_ms;    /* wall time of this solve                               */
} bddc_pcg_info;

/* Build the preconditioner (paper Sec. 2): assemble A and every A_i from theta,
 * classify interface dofs into corner / edge / face classes, factor the local
 * problems, form Phi_i implicitly and A_ci = Phi_i^T A_i Phi_i, assemble and
 * factor A_c.  Synchronous.  On success *out owns all device state.
 * Errors: EINVAL (shapes, cuts, options), ENOTSPD (theta <= 0 or a failed
 * pivot), ENOMEM, EHIP, ENOTIMPL (more than 64 constraints on a subdomain). */
int bddc_setup(const bddc_mesh* mesh, const bddc_partition* part,
               const bddc_coefficients* coef, uint32_t constraints,
               const bddc_options* opts, bddc_ctx** out);

/* z = M^{-1} r = v1 + v2 + v3 (paper Sec. 2, eqs. (2)-(5)).  r and z are device
 * arrays of n_free float64.  Asynchronous on the ctx stream. */
int bddc_apply(bddc_ctx* ctx, const double* r, double* z);

/* Solve A x = b by CG preconditioned with M (paper Sec. 2, Sec. 3) from
 * x0 = P_I b (the static-condensation guess: interior solves of eq. (5)
 * applied to b) unless flags has BDDC_X0_GIVEN.  Stops when
 * ||r_k||_2 <= rtol ||b||_2 and the true residual confirms it.  Synchronous.
 * Returns OK, ENOCONV (x holds the last iterate), EBREAKDOWN, EINVAL. */
int bddc_pcg_solve(bddc_ctx* ctx, const double* b, double* x, double rtol,
                   int32_t maxit, int32_t flags, bddc_pcg_info* info);

/* The same z = M^{-1} r as bddc_apply (the same kernels in the same order, so
 * the same bits), for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * It calls no hipMalloc, hipFree or other allocating routine and records no
 * timing event.  The buffers that one application starts afresh (published
 * triangular-solve values and ticket counters) live in a
 * fixed device workspace of 64 MiB that the library holds on every GPU it runs
 * on until the process ends, instead of in the ctx.  Every call on one GPU
 * uses that GPU's workspace, whatever the ctx: calls that overlap on one GPU
 * (different streams, or different host threads) race and must be ordered by
 * the caller.  Each call re-initialises the part it uses before reading it.
 * Errors: EINVAL (NULL or aliased vectors, or a problem whose apply workspace
 * 4 * n_vec * (4 or 8 bytes) + the ticket counters exceeds 64 MiB; the
 * message gives both sizes), EHIP (no workspace address on this device).
 * Asynchronous on the ctx stream. */
int bddc_apply_noalloc(bddc_ctx* ctx, const double* r, double* z);

/* y = A x with the assembled global matrix (paper Sec. 2).  Asynchronous. */
int bddc_spmv(bddc_ctx* ctx, const double* x, double* y);

/* Per-element derivative of lam^T A(theta) u with the sign of an adjoint
 * gradient: g_e = -lam_e^T K_ref u_e, where K_ref = dK_e/dtheta_e is the
 * unit-conductivity Q1 element matrix; g has prod(nel) entries.
 * Asynchronous. */
int bddc_elem_grad(bddc_ctx* ctx, const double* lam, const double* u, double* g);

/* Setup statistics (for the factorisation's compute roofline): the floating-
 * point operations of the batched local tile Cholesky inside the factors'
 * envelope (diagonal factor 64^3/3, panel solve 64^3, off-diagonal update 2*64^3,
 * diagonal update 64^3 per tile operation) and its GPU time at setup in ms
 * (measured with stream events around the factorisation launches).  Either
 * pointer may be NULL.  Errors: EINVAL (NULL ctx). */
int bddc_setup_stats(bddc_ctx* c, double* factor_flops, double* factor_ms);

/* Sizes: free dofs, subdomains, global coarse dofs, device bytes held.
 * Any output pointer may be NULL. */
int bddc_query(bddc_ctx* ctx, int64_t* n_free, int32_t* n_sub, int32_t* n_coarse,
               int64_t* dev_bytes);

/* Host-only planning check (no GPU needed): validates the arguments and runs
 * the host stage of bddc_setup (dof numbering, multiplicities, interface
 * classes, local orderings), returning its sizes.  stats[0..7] =
 * {n_free, n_sub, n_coarse, n_corner_classes, n_edge_classes,
 *  n_face_classes, sum_i n_i, max_i n_ci}. */
int bddc_plan_stats(const bddc_mesh* mesh, const bddc_partition* part,
                    uint32_t constraints, int64_t stats[8]);

/* Kernel timing: when enabled, every launch of the named kernel family is
 * bracketed by HIP events on the ctx stream; bddc_kernel_time returns the
 * number of timed launches and their summed duration in ms (synchronising
 * the stream).  Families: "trsv_fwd_rr", "trsv_bwd_rr", "trsv_fwd_ii",
 * "trsv_bwd_ii" (full-space solves), "op" (the symmetric mat-vec with the
 * local Schur complements of the interface operator), "pc" (the symmetric
 * mat-vec of the interface preconditioner), "schur" (the whole operator),
 * "spmv", "apply".  While timing is enabled, PCG iterations are
 * launched eagerly even when use_graph is set.  Launches that returned at once
 * because the solve had already converged (shorter than a fifth of the
 * family's longest) are not counted.  Each query resets the family.
 * Unknown names give EINVAL. */
int bddc_set_timing(bddc_ctx* ctx, int32_t enabled);
int bddc_kernel_time(bddc_ctx* ctx, const char* family, int64_t* launches,
                     double* total_ms);

/* Test access to one subdomain's setup data, copied to host memory (synchronous).
 * what: "sizes" -> {n_R, n_I, n_A, n_P, T, n_i} (6 values);
 *       "factor" -> the local factor L of the equilibrated A_RR as a dense
 *                   (T*64) x (T*64) row-major lower triangle (padding rows included);
 *       "border" -> the bordering rows W^T = (L^{-1} D B)^T, 64 x (T*64) row-major;
 *       "schur"  -> the bordering diagonal tile (-W^T W), 64 x 64;
 *       "aci"    -> A_ci = Phi_i^T A_i Phi_i, 64 x 64 (constraint order: averages
 *                   then corners);
 *       "envelope" -> 2T values: for each tile row k of the factor, the first tile
 *                   column holding a nonzero (tiles left of it are zero and are
 *                   never stored into or read), then the same over the interior
 *                   rows only (meaningful for k < ceil(n_I / 64));
 *       "gmap"   -> global free dof of each local dof (n_i values);
 *       "dscale" -> equilibration factor of each local dof (n_i values).
 * Returns the number of values written (<= cap) or a negative status. */
int64_t bddc_debug_read(bddc_ctx* ctx, const char* what, int32_t sub, double* host_out, int64_t cap);

/* Device-side limits, mainly for tests of the failure paths:
 *   "wait_polls"      polls of a published value before a triangular-solve task
 *                     gives up, and polls of a grid barrier of the coarse CG
 *                     over 64 workgroups (default 4194304, about a second); the
 *                     task then uses 0 (the coarse CG stops), finishes normally
 *                     and marks the ctx's device status word; a negative value
 *                     makes every wait give up at once;
 *   "coarse_cg_maxit" iteration limit of the coarse CG (BDDC_SETUP_COARSE_CG,
 *                     default 2000); a coarse CG that stops at it (or breaks
 *                     down) marks the device status word;
 *   "sym_lds_cols"    interface form: the tile columns (0..64, default 64)
 *                     whose partial products a mat-vec workgroup sums over its
 *                     rows before storing them; the others store one per tile
 *                     (results agree to rounding);
 *   "sym_row_pieces"  interface form: row pieces (0..28, default 28) a mat-vec
 *                     workgroup keeps until its range is done; the others are
 *                     stored at once (results are bitwise the same).
 * The last two select code paths for tests; they are not tuning knobs.
 * A marked status word is reported, and cleared, by the next bddc_pcg_solve
 * (EHIP for a wait that gave up, ENOCONV for the coarse CG; x and info are
 * still filled) or bddc_sync.  Captured graphs are dropped.
 * Errors: EINVAL (unknown name, negative coarse_cg_maxit, sym_* out of range). */
int bddc_set_limit(bddc_ctx* ctx, const char* what, int32_t value);

/* Waits for all work queued on the ctx stream and reports the device status
 * word since it was last reported: OK, EHIP (a triangular-solve wait or a
 * coarse-CG grid barrier gave up, e.g. in an asynchronous bddc_apply) or
 * ENOCONV (the coarse CG did not converge); the word is cleared. */
int bddc_sync(bddc_ctx* ctx);

/* Launch shape of the persistent kernels (triangular solves and tile
 * mat-vecs): wg_per_cu resident workgroups per compute unit, 1..16 (default
 * 4).  Captured graphs are dropped and recaptured with the new shape. */
int bddc_set_tuning(bddc_ctx* ctx, int32_t wg_per_cu);

/* Autotuner: for each of the ncand candidate wg_per_cu values, runs `iters`
 * PCG iterations on a fixed right-hand side (after one untimed warm-up run)
 * and times them with HIP events; keeps the fastest setting.  *best receives
 * it and ms_out[i] (may be NULL) the time of candidate i.  Synchronous. */
int bddc_autotune(bddc_ctx* ctx, const int32_t* candidates, int32_t ncand, int32_t iters, int32_t* best,
                  double* ms_out);

/* Frees every device and host resource of ctx (NULL is allowed). */
void bddc_destroy(bddc_ctx* ctx);

/* Static message for a status code. */
const char* bddc_strerror(int code);

/* Detail of the last error on the calling thread (static buffer). */
const char* bddc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BDDC_H */
