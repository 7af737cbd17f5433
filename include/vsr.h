/*
 * vsr.h -- C ABI of the MI355X (gfx950) vertex-star FDM/sparse relaxation solver.
 *
 * Method: Brubeck & Farrell, "A scalable and robust vertex-star relaxation for
 * high-order FEM" (SIAM J. Sci. Comput., 2022), Sec. 2.  The library solves the
 * Poisson problem -div(kappa grad u) = f with homogeneous Dirichlet conditions
 * (weak form of Sec. 2.1), discretized with continuous Q_p on a structured mesh
 * of trilinear hexahedra, by PCG (Sec. 2.8) preconditioned with the hybrid
 * two-level V(1,1) cycle of Sec. 2.5: vertex-star additive Schwarz relaxation
 * in the FDM basis (Sec. 2.4) with exact sparse-Cholesky patch solves (Sec. 2.6)
 * of the separable surrogate form (Sec. 2.7), and a Q1 coarse correction.
 *
 * Conventions shared by every call
 *  - Every call returns a vsr_status and never throws.  On error the outputs are
 *    unspecified and vsr_last_error() describes the failure (thread-local text,
 *    valid until the next failing call on that thread).  A problem stays usable
 *    after any error except VSR_EDEVICE.
 *  - Host arrays passed to vsr_setup are copied; the caller may free them on
 *    return.  Vector arguments are caller-owned FP64 device buffers (HIP device
 *    memory on the current device) of length vsr_num_dofs(); inputs and outputs
 *    must not alias.  The library owns, and vsr_destroy frees, everything else.
 *  - Vector layout: the free DOFs are the interior nodes of the global GLL
 *    lattice of (p*nx+1) x (p*ny+1) x (p*nz+1) nodes, in lexicographic order
 *    with x fastest: index (i-1) + (j-1)*Lx + (k-1)*Lx*Ly, Lx = p*nx-1, ...
 *  - Work runs on options.stream (NULL = the default stream).  Apply calls are
 *    asynchronous; vsr_pcg_solve returns after the solve has completed.
 */
#ifndef VSR_H
#define VSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vsr_problem vsr_problem;

typedef enum {
    VSR_OK = 0,
    VSR_EINVAL = 1,   /* bad argument: p outside [2,15], a mesh axis with < 2 cells,
                         a non-finite input, a NULL pointer, an unknown mode */
    VSR_EMESH = 2,    /* a cell with det(DF) <= 0 at a quadrature point */
    VSR_ENOTSPD = 3,  /* a non-positive pivot in a patch or coarse Cholesky factor
                         (e.g. a coefficient kappa <= 0) */
    VSR_ENOCONV = 4,  /* PCG stopped at max_iterations before reaching rtol, or broke down */
    VSR_EDEVICE = 5,  /* a HIP runtime error */
    VSR_ENOMEM = 6    /* device or host allocation failed */
} vsr_status;

/* Structured hexahedral mesh (Sec. 2.1): nx*ny*nz cells, vertex (i,j,k) at
 * vertices[3*(i + (nx+1)*(j + (ny+1)*k)) + c], c = 0,1,2 the coordinates.
 * Cell (ex,ey,ez) is the trilinear image of [-1,1]^3 whose reference corner
 * (a,b,c) in {0,1}^3 maps to vertex (ex+a, ey+b, ez+c).  Host memory, copied. */
typedef struct {
    int32_t nx, ny, nz;
    const double *vertices;
} vsr_mesh;

/* Coefficients.  kappa: host, one positive value per cell (cell index
 * ex + nx*(ey + ny*ez)), NULL means kappa = 1.  mu_override: host, 3 values per
 * cell replacing the averaged surrogate scalings mu_j of Sec. 2.7 (used by a
 * learned surrogate); NULL means the cell averages of the paper. */
typedef struct {
    const double *kappa;
    const double *mu_override;
} vsr_coefficients;

typedef struct {
    int32_t relax_fp32;      /* 1: relaxation, coarse correction and the cycle's inner
                                operator applies in FP32 (outer PCG stays FP64); 0: all FP64 */
    int32_t cycle;           /* 0: hybrid multiplicative V(1,1) (Sec. 2.5, default);
                                1: additive z = S r + P A0^{-1} P^T r */
    int32_t quad_points;     /* GLL points per direction; 0 => ceil(3(p+1)/2) (Sec. 2.8) */
    int32_t lanczos_steps;   /* CG-Lanczos steps for the damping estimate; 0 => 20 */
    int32_t max_iterations;  /* PCG iteration cap; 0 => 1000 */
    int32_t interior_patches_only; /* 1: patches only around interior vertices; 0: every vertex */
    uint64_t seed;           /* seed of the splitmix64 Lanczos start vector */
    double omega;            /* > 0: use this damping instead of the Lanczos estimate */
    void *stream;            /* hipStream_t; NULL => default stream */
    int32_t autotune;        /* 1: pick launch shapes (cells or workgroups per cell of the
                                operator, patch-panel unroll and workgroup size) by timing the
                                candidates on this problem at setup, once per (GPU
                                architecture, p, precision, operator kind) per process and
                                per cache file; 0: fixed defaults.  Shapes never change the
                                arithmetic of any output value. */
    int32_t batch_streams;   /* batched solves: HIP streams the members are spread over; 0 => 4 */
    int32_t batch_eager;     /* batched solves: 1 launches every iteration from the host;
                                0 (default) records one lockstep iteration of all members into
                                a hipGraph once and replays it */
    const char *tune_cache;  /* autotune: text file of tuned shapes to read and append to;
                                NULL => in-process cache only */
    int32_t share_factors;   /* 1: stars of the same class whose cell scalings agree to 11
                                significant digits (e.g. every interior star of a uniform
                                Cartesian mesh with constant kappa) are factored once and share
                                the first one's stored factor (the others' patch matrices differ
                                from it by ~1e-11 relative).  0: one factor per star (default). */
    int32_t deterministic;   /* 1: every patch-panel partial sum is taken by one thread in a fixed
                                order instead of being combined with LDS atomics, so relaxations,
                                preconditioner applies and PCG iterates repeat bit for bit from run
                                to run (the operator, load vector, transfers, assembly and dot
                                products are always in a fixed order); slower panels.
                                0: atomics where they are faster (default). */
    int32_t coarse_solver;   /* solver of the Q1 coarse problem (Sec. 2.5, 2.8): 1: dense inverse
                                of its Galerkin matrix (exact); 2: one V(1,1) cycle of geometric
                                multigrid (damped point-Jacobi with weight 2/3 on every level, 2x2x2
                                cell coarsening while every axis has an even number >= 4 of cells,
                                Galerkin levels, dense inverse on the coarsest level); 0 (default):
                                dense up to 8,000 coarse unknowns (21^3 cells), multigrid above */
    int32_t stagnation_window; /* relax_fp32 only: a solve whose ||r||_2 has not fallen below
                                stagnation_factor times its reference value (||b||_2 at the start,
                                then each value that did fall below it) for this many consecutive
                                iterations stops as stagnated and continues from its x with the
                                FP64 relaxation: PCG on A e = b - A x to the remaining tolerance,
                                x += e.  The FP64 setup of the same problem this needs is made at
                                the first stagnation and kept with the problem (twice its device
                                memory from then on).  0 => 10; < 0: never.  Solves in profiling
                                mode do not test for stagnation. */
    double stagnation_factor; /* see stagnation_window; 0 => 1 (any decrease counts) */
} vsr_options;

typedef struct {
    int32_t iterations;        /* number of x updates */
    int32_t converged;         /* 1 if ||r||_2 <= rtol ||b||_2 was reached */
    double rel_residual;       /* recursive residual norm / ||b||_2 at exit */
    double true_rel_residual;  /* ||b - A x||_2 / ||b||_2 recomputed in FP64 at exit */
    double omega, lambda_min, lambda_max;  /* damping and its Lanczos estimates */
    double setup_seconds, solve_seconds;
    /* CG-Lanczos on the solve itself (Sec. 4, Table tab:poisson-cond): extreme eigenvalues of the
     * tridiagonal built from this run's step lengths alpha_j and direction updates beta_j
     * (diagonal 1/alpha_j + beta_{j-1}/alpha_{j-1}, off-diagonal sqrt(beta_j)/alpha_j), which
     * approach the extreme eigenvalues of P^{-1} A from inside, and their ratio, the estimate
     * of kappa(P^{-1} A).  All three are 0 when no step was taken (b = 0) or a step length
     * was not positive. */
    double ritz_min, ritz_max, kappa_estimate;
    int32_t fp64_iterations;   /* iterations taken on the FP64 relaxation after a stagnation
                                  (included in iterations; the Ritz values are those of the
                                  FP32-relaxation run); 0 if none */
} vsr_solve_info;

/* ---- Primal linear elasticity with the SDC relaxation (Sec. 3.1) -------------------------
 * a(v, u) = int 2 mu eps(v) : eps(u) + lambda div v div u, Q_p in each displacement
 * component, homogeneous Dirichlet conditions on the whole boundary, on a tensor grid of
 * axis-aligned boxes.  A displacement vector (device, FP64) holds 3 n values, component
 * after component, each in the scalar layout above (n = vsr_num_dofs of the same mesh).  The
 * preconditioner is the hybrid V(1,1) of Sec. 2.5 with the SDC relaxation (block-Jacobi over
 * the components; component j's block solved by the vertex-star FDM patches with the exact
 * separable scalings of A_jj on boxes) and Q1 in every component as the coarse space (exact
 * dense solve, at most 12,000 coarse unknowns). */
typedef struct vsr_elasticity vsr_elasticity;

/* opt: relax_fp32 (the component relaxations in FP32), lanczos_steps, seed, omega,
 * max_iterations, stream and deterministic are used; NULL = defaults.  Returns VSR_EINVAL for a
 * mesh that is not a tensor grid of boxes, mu <= 0 or lambda < 0. */
vsr_status vsr_elasticity_setup(const vsr_mesh *mesh, int32_t p, double mu, double lambda, const vsr_options *opt,
                                vsr_elasticity **out);
int64_t vsr_elasticity_num_dofs(const vsr_elasticity *el);
/* b = [b_1; b_2; b_3] from the body force f_dev: 3 blocks of ncell q^3 values (the samples of
 * vsr_load_vector), one per component. */
vsr_status vsr_elasticity_load_vector(vsr_elasticity *el, const double *f_dev, double *b_dev);
vsr_status vsr_elasticity_apply_operator(vsr_elasticity *el, const double *x_dev, double *y_dev);
/* mode 0: the hybrid V(1,1) preconditioner; 1: the SDC relaxation alone (undamped); 2: the
 * coarse correction. */
vsr_status vsr_elasticity_apply_relaxation(vsr_elasticity *el, const double *r_dev, double *z_dev, int32_t mode);
vsr_status vsr_elasticity_damping(const vsr_elasticity *el, double *omega, double *lambda_min, double *lambda_max);
/* PCG (Sec. 2.8) from x = 0 until ||r||_2 <= rtol ||b||_2, driven from the device (scalars
 * and the stopping test on the GPU; the host polls one iteration behind).  info as for
 * vsr_pcg_solve, without stagnation handling.  Returns VSR_ENOCONV at max_iterations and
 * VSR_EINVAL for a non-finite b.  The iterations run on the library's own stream, forked from
 * and joined back to the options' stream, as replays of one recorded iteration (kept for the
 * next solve into the same x_dev); calls on one object must not overlap. */
vsr_status vsr_elasticity_pcg_solve(vsr_elasticity *el, const double *b_dev, double *x_dev, double rtol,
                                    vsr_solve_info *info);
void vsr_elasticity_destroy(vsr_elasticity *el);

/* Fill *opt with the defaults listed above (all zero except the library's defaults). */
void vsr_default_options(vsr_options *opt);

/* Build everything the solve needs (Sec. 2.2-2.7): 1D GLL/FDM data, geometry and
 * surrogate scalings, the Cholesky factor of every vertex-star patch, the Q1
 * coarse matrix and its inverse, the damping omega (CG-Lanczos unless given).
 * p in [2, 15]; mesh axes >= 2 cells.  *out receives a new problem. */
vsr_status vsr_setup(const vsr_mesh *mesh, int32_t p, const vsr_coefficients *coef,
                     const vsr_options *opt, vsr_problem **out);

/* Number of free DOFs (length of every vector argument), or -1 for NULL. */
int64_t vsr_num_dofs(const vsr_problem *prob);

/* Load vector b_i = sum_K sum_q w_q |det DF(x_q)| phi_i(x_q) f_{K,q} (Sec. 2.1).
 * f_dev: device FP64, one sample per cell and quadrature point, cell-major, points
 * in x-fastest tensor order (ncell * quad_points^3 values).  b_dev: device FP64 (n). */
vsr_status vsr_load_vector(vsr_problem *prob, const double *f_dev, double *b_dev);

/* y = A x, the matrix-free sum-factorized Galerkin operator (Sec. 2.1, 2.7), FP64. */
vsr_status vsr_apply_operator(vsr_problem *prob, const double *x_dev, double *y_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): y = A x exactly as vsr_apply_operator
 * computes it (same kernels, same summation order, bitwise the same y), with the operator's
 * element vector (2 * ncell * (p+1)^3 FP64 values at most) placed in a static device
 * workspace of 64 MiB that the library holds on each GPU it runs on until the process ends,
 * instead of the problem's own buffer.  The call allocates nothing: no hipMalloc, hipFree or
 * allocating library routine.  Call it with the problem's device current.  Every call on a
 * GPU shares that GPU's workspace, so calls that overlap on one GPU (from several threads or
 * streams) race; the workspace keeps the last call's contents, which no call reads before
 * writing.  VSR_EINVAL if 2 * ncell * (p+1)^3 * 8 bytes exceeds 64 MiB (e.g. more than 1,024
 * cells at p = 15). */
vsr_status vsr_apply_operator_noalloc(vsr_problem *prob, const double *x_dev, double *y_dev);

/* z = M r with mode 0: the full preconditioner (cycle chosen at setup);
 * mode 1: the patch relaxation alone, z = T (sum_j Rbar_j^T A_j^{-1} Rbar_j) T^T r
 * (Sec. 2.4-2.6, undamped); mode 2: the coarse correction z = P A0^{-1} P^T r. */
vsr_status vsr_apply_relaxation(vsr_problem *prob, const double *r_dev, double *z_dev, int32_t mode);

/* PCG (Sec. 2.8) from x = 0 until ||r||_2 <= rtol ||b||_2; x_dev receives the
 * solution.  info may be NULL.  Returns VSR_ENOCONV if max_iterations is reached. */
vsr_status vsr_pcg_solve(vsr_problem *prob, const double *b_dev, double *x_dev, double rtol,
                         vsr_solve_info *info);

/* Damping and Lanczos estimates chosen at setup. */
vsr_status vsr_get_damping(const vsr_problem *prob, double *omega, double *lambda_min,
                           double *lambda_max);

/* Timing of the patch-solve kernel (the dominant kernel; one launch per relaxation
 * solves the stars of all vertices, interior ones first).  enable != 0 makes every later
 * relaxation record HIP events around that launch on the problem's stream;
 * vsr_kernel_stats returns the launch count, total milliseconds and the algorithmic
 * bytes one launch moves (factor entries read twice plus the patch vectors read and
 * written), and resets the counters. */
vsr_status vsr_set_profiling(vsr_problem *prob, int32_t enable);
vsr_status vsr_kernel_stats(vsr_problem *prob, int64_t *launches, double *total_ms,
                            double *bytes_per_launch);

/* Sizes of the patch factorization: number of patches and stored factor entries. */
vsr_status vsr_factor_info(const vsr_problem *prob, int64_t *num_patches, int64_t *factor_entries);

/* ---------------------------------------------------------------------------
 * Learned separable surrogate (an extension of the averaged surrogate of Sec. 2.7;
 * the paper has no learned part).  Cells are passed by their 8 corners: host
 * array corners[24*cell + 3*((c*2+b)*2+a) + coord], corner (a,b,c) in {0,1}^3
 * of the reference cube [-1,1]^3, x fastest.  kappa (host, per cell) may be NULL.
 * All host arrays are read or written synchronously; device arrays are HIP
 * device memory.  Errors as for the solver calls.
 * ------------------------------------------------------------------------- */

/* Number of MLP parameters (74 -> 64 -> 64 -> 3, GELU): W1 (64x74 row-major), b1 (64),
 * W2 (64x64), b2, W3 (3x64), b3, packed in that order as float32. */
int32_t vsr_mlp_num_params(void);

/* Features per cell (device float32, ncell x 74): 8 (DF / |det DF(0)|^(1/3) - I) at the
 * 2x2x2 Gauss points (x fastest, DF row-major), then log kappa and 0.  mu_avg (host, ncell x 3, may be NULL):
 * the cell averages of diag(G_hat) of Sec. 2.7 with kappa = 1 and the degree-p
 * quadrature rule.  features_dev may be NULL. */
vsr_status vsr_surrogate_features(int64_t ncell, const double *corners, const double *kappa, int32_t p,
                                  float *features_dev, double *mu_avg);

/* Theorem 1 (Sec. 2.7) spectral ratio C_K / c_K of mu^{-1/2} G_hat mu^{-1/2} over the
 * 27 points xi in {-1,0,1}^3, for host scalings mu (ncell x 3, positive); ratio: host (ncell). */
vsr_status vsr_surrogate_ratio(int64_t ncell, const double *corners, const double *mu, double *ratio);

/* Minimax labels: delta (host, ncell x 3) with mu = mu_avg exp(delta) minimising the
 * Theorem-1 ratio on a fixed coarse-to-fine grid over delta = (a, b, 0), shifted so the
 * spectrum is centred at 1; ratio (host, ncell, may be NULL) is the ratio attained. */
vsr_status vsr_surrogate_labels(int64_t ncell, const double *corners, int32_t p, double *delta, double *ratio);

/* Y = MLP(X) for n samples (device float32, X: n x 74, Y: n x 3).  bf16 != 0 rounds the
 * weights to bfloat16 for the arithmetic (FP32 accumulation). */
vsr_status vsr_mlp_forward(const float *params_dev, int32_t bf16, const float *X_dev, int64_t n, float *Y_dev);

/* Gradient (device, vsr_mlp_num_params() floats) of the mean squared error between MLP(X)
 * and T (device, n x 3) with respect to the parameters; loss_dev (1 float) may be NULL. */
vsr_status vsr_mlp_gradient(const float *params_dev, int32_t bf16, const float *X_dev, const float *T_dev, int64_t n,
                            float *grad_dev, float *loss_dev);

/* `steps` Adam steps (beta 0.9 / 0.999, eps 1e-8, learning rate lr) on the FP32 master
 * parameters; minibatch s uses the rows order_dev[s*batch .. (s+1)*batch) of X and T
 * (device int32, steps*batch entries).  step0 counts earlier steps (bias correction).
 * adam_m_dev, adam_v_dev: device state (num_params floats each, zero initially).
 * loss_dev (device, steps floats, may be NULL) receives each minibatch loss. */
vsr_status vsr_mlp_train(float *params_dev, float *adam_m_dev, float *adam_v_dev, int32_t bf16, const float *X_dev,
                         const float *T_dev, int64_t n, const int32_t *order_dev, int32_t batch, int32_t steps,
                         int32_t step0, float lr, float *loss_dev);

/* Surrogate scalings for the solver (pass as vsr_coefficients.mu_override): per cell
 * mu = kappa mu_avg exp(MLP(features)), kept only where its Theorem-1 ratio is below that
 * of the averaged scalings (else kappa mu_avg).  mu_out: host ncell x 3; learned (host,
 * ncell, may be NULL): 1 where the network's scalings were kept. */
vsr_status vsr_surrogate_scalings(int64_t ncell, const double *corners, const double *kappa, int32_t p,
                                  const float *params_dev, int32_t bf16, double *mu_out, int32_t *learned);

/* Launch shapes in use: shapes[0..5] = Cartesian-operator cells per workgroup (FP64,
 * FP32), patch-panel unroll, general-operator workgroups per cell (FP64, FP32; 0 = chosen
 * by size: 2 where one workgroup's FP64 column state would not fit in registers, else 1),
 * threads per patch workgroup. */
vsr_status vsr_get_tuning(const vsr_problem *prob, int32_t shapes[6]);

/* Set the launch shapes (same order; cells per workgroup in {1, 2, 4}, used only for
 * Cartesian meshes with p <= 7; unroll in {4, 8, 16}; workgroups per cell in {0, 1, 2};
 * patch threads 256, 512 or 1024, the last with an unroll of 4 or 8).  VSR_EINVAL for any
 * other value. */
vsr_status vsr_set_tuning(vsr_problem *prob, const int32_t shapes[6]);

void vsr_destroy(vsr_problem *prob);

/* ---------------------------------------------------------------------------
 * Batched solves: many independent problems (any mix of sizes, degrees, meshes
 * and coefficients) solved together.  Every member runs its own PCG (Sec. 2.8
 * settings) with its own scalars; the members iterate in lockstep, the stopping
 * test of each is taken on the device and a member that has stopped skips all
 * further work (its kernels return at once).  Members are spread over
 * options.batch_streams streams (largest first onto the least loaded stream) so
 * small members run concurrently; one lockstep iteration of all members is
 * recorded into a hipGraph and replayed until none is active (the stop flags sit
 * in mapped host memory and are read one replay behind, so the next replay is
 * always queued).  Each member gives the same iterates as vsr_pcg_solve on it up
 * to the order of the floating-point additions that the patch panels make with
 * LDS atomics.
 * ------------------------------------------------------------------------- */
typedef struct vsr_batch vsr_batch;

/* Set up `count` members: meshes[i], p[i], coefs[i] (coefs may be NULL: kappa = 1
 * everywhere), all with *opt.  Setup is as vsr_setup for each member. */
vsr_status vsr_setup_batch(int32_t count, const vsr_mesh *meshes, const int32_t *p,
                           const vsr_coefficients *coefs, const vsr_options *opt,
                           vsr_batch **out);

/* Form a batch from `count` problems already set up with vsr_setup.  On success the batch
 * takes ownership of them (vsr_destroy_batch frees them; do not vsr_destroy them); on
 * error they stay with the caller.  Only opt->batch_streams and opt->batch_eager are read
 * (opt may be NULL: defaults).  A problem may belong to one batch only. */
vsr_status vsr_batch_create(int32_t count, vsr_problem *const *members, const vsr_options *opt, vsr_batch **out);

int32_t vsr_batch_size(const vsr_batch *batch);

/* Member i, owned by the batch (valid until vsr_destroy_batch): use it for
 * vsr_num_dofs, vsr_load_vector, the applies and single solves. */
vsr_problem *vsr_batch_member(vsr_batch *batch, int32_t i);

/* Solve A_i x_i = b_i for every member from x_i = 0 to ||r_i||_2 <= rtol ||b_i||_2.
 * b_dev, x_dev: host arrays of count device pointers (FP64, length vsr_num_dofs of
 * the member).  infos (host, count entries, may be NULL) receives per-member
 * results; solve_seconds is the wall time of the whole batch.  Returns after
 * completion; VSR_ENOCONV if any member stopped without converging (its info says
 * which). */
vsr_status vsr_pcg_solve_batch(vsr_batch *batch, const double *const *b_dev, double *const *x_dev, double rtol,
                               vsr_solve_info *infos);

void vsr_destroy_batch(vsr_batch *batch);

/* Description of the last failure on the calling thread ("" if none). */
const char *vsr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VSR_H */
