/*
 * lrpost — low-rank posterior covariance for a space-time Bayesian inverse
 * problem governed by the 2D heat equation, on AMD Instinct MI355X (gfx950).
 *
 * Method: Benner, Qiu, Stoll, "Low-rank computation of posterior covariance
 * matrices in Bayesian inverse problems".  The posterior covariance
 * Gamma_post = (A^T Gamma_noise^{-1} A + Gamma_prior^{-1})^{-1} (Sec. 2 eq.
 * postcov1) is approximated from the dominant eigenpairs of the
 * prior-preconditioned misfit Hessian (Sec. 2 eq. prior_pre) through the
 * Sherman-Morrison-Woodbury update of Sec. 2, the eigenpairs coming from a
 * Krylov process whose space-time vectors are kept as low-rank factors
 * (Sec. 4 eq. lr_vec, Algorithm 1).  Each Hessian apply needs one forward and
 * one adjoint space-time solve of (I_nt kron L + C kron M) vec(X) = vec(F)
 * (Sec. 6.1 eq. st_pde), done here in low-rank matrix-equation form.
 *
 * Problem (all entry points):
 *   y_t = Laplace(y) + u on [0,1]^2, y = 0 on the boundary, y(0) = 0;
 *   Q1 elements on a uniform N x N mesh, n = N-1 interior nodes per side,
 *   nx = n^2, nodes numbered (j-1) n + (i-1) for node (i h, j h), x1 fastest;
 *   implicit Euler with tau = T/nt; the parameter is the space-time source u;
 *   observations are nodal values inside a closed box at t_1..t_nt with noise
 *   covariance sigma^2 I; Gamma_prior^{-1} = P = alpha tau (I_nt kron (K+M)).
 *
 * Space-time vectors: X in R^{nx x nt} (column k is time t_{k+1}) held as
 * X = W1 W2^T.  In every lrpost_lowrank the spatial factor W1 is DEVICE memory
 * (nx rows, leading dimension nx, column-major, float64) and the temporal
 * factor W2 is HOST memory (nt rows, leading dimension nt, column-major,
 * float64).  `cap` is the number of columns allocated in both; `rank` the
 * number in use.  The caller allocates and owns both buffers.
 *
 * Errors: every call returns 0 on success or a negative code below; no C++
 * exception crosses this interface.  lrpost_last_error() returns a
 * thread-local message describing the last failure on the calling thread.
 *
 * Concurrency: one problem handle must not be used by two threads at once.
 * Work is ordered on the HIP stream given in the description; without one,
 * on a blocking stream the problem creates (ordered after earlier work of
 * the null stream, like every blocking stream).  Every entry point except
 * lrpost_gram_noalloc returns after its results are complete.
 */
#ifndef LRPOST_H
#define LRPOST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LRPOST_OK 0
#define LRPOST_EINVAL -1      /* invalid argument: shape, rank above cap, sigma/alpha <= 0, empty box */
#define LRPOST_ENOMEM -2      /* device allocation failed or request exceeds the HBM budget */
#define LRPOST_ENOCONV -3     /* an iteration did not reach its tolerance within its limit */
#define LRPOST_EBREAKDOWN -4  /* numerical breakdown that survived the fallback */
#define LRPOST_EHIP -5        /* a HIP runtime call failed */

#define LRPOST_FP64 0         /* every step in float64 */
#define LRPOST_MIXED 1        /* float32 stencil/multigrid, float64 small factorizations */

#define LRPOST_MISFIT 0       /* y = H_mis x = sigma^-2 F^T F x */
#define LRPOST_PRECOND 1      /* y = G x = P^{-1} H_mis x (prior-preconditioned Hessian) */

#define LRPOST_BLOCK_LANCZOS 0
#define LRPOST_RANDOMIZED 1

typedef struct lrpost_problem lrpost_problem;
typedef struct lrpost_eigs lrpost_eigs;

/* Problem description (the configuration of one inverse problem). */
typedef struct {
  int32_t N;          /* mesh cells per side; a power of two, 4 <= N <= 4096 */
  int32_t nt;         /* implicit-Euler steps, >= 1 */
  double T;           /* final time (> 0) */
  double alpha;       /* prior precision scale (> 0) */
  double sigma;       /* noise standard deviation (> 0) */
  double box[4];      /* closed observation box x1lo, x1hi, x2lo, x2hi (must hold >= 1 node) */
  double trunc_tol;   /* relative Frobenius truncation tolerance of factors, in (0, 1) */
  int32_t rank_cap;   /* maximal factor rank kept after truncation, >= 1 */
  int32_t precision;  /* LRPOST_FP64 or LRPOST_MIXED */
  int32_t mg_levels;  /* must be 0: the V-cycle always coarsens to levels of at most 31
                         nodes per side, solved inside one workgroup (any other value
                         is rejected with LRPOST_EINVAL) */
  uint64_t seed;      /* seed of the Lanczos start block */
  void* hip_stream;   /* hipStream_t to order work on, or NULL for a blocking stream of the problem's own */
} lrpost_problem_desc;

/* A low-rank space-time vector X = W1 W2^T (see the header comment for memory). */
typedef struct {
  int32_t nx, nt, rank, cap;
  double* W1; /* device, nx x cap */
  double* W2; /* host,   nt x cap */
} lrpost_lowrank;

/* Statistics of the last operation on a problem (for logs and tests). */
typedef struct {
  int64_t applies;        /* Hessian applies since creation */
  int32_t last_rank_y;    /* rank of the last forward state */
  int32_t last_rank_p;    /* rank of the last adjoint state */
  int32_t last_rank_out;  /* rank of the last apply's output */
  int32_t last_basis;     /* spatial basis size of the last space-time solve */
  int32_t lanczos_steps;  /* block steps of the last eigensolve */
  int32_t st_enrichments; /* space-time solve batches that needed the enriched pole set */
  int32_t st_unresolved;  /* of those, batches still above the threshold after enrichment */
  int32_t st_direct_grams; /* pole blocks (per source) whose swept block needed its own Gram
                             in the second orthogonalization sweep (see the space-time solve) */
  double last_tail;       /* relative tail dropped by the last truncation */
  double last_st_resid;   /* largest relative residual ||tau K Y + M Y C^T - F||_F / ||F||_F
                             (C for the adjoint) of the solutions of the last space-time
                             solve batch, for the truncated factors returned (Sec. 6.1,
                             eq. st_pde); -1 while the check is off or no solve ran */
  double last_st_presid;  /* the same residual preconditioned by two multigrid V-cycles of
                             M + tau K per time step, relative to the same preconditioned
                             source (the block-diagonal preconditioner of Sec. 6.1,
                             eq. pre_1): it tracks the relative error of the solution and is
                             what the check of lrpost_set_st_check compares */
  double ritz_resid;      /* largest relative Ritz residual ESTIMATE of the last
                             eigensolve: block Lanczos takes it from the coupling block of
                             the recurrence, the randomized solver from the Grams of its
                             two passes.  Neither includes the truncation of the Ritz
                             vectors after the loop; lrpost_eig_residuals measures that */
  int64_t pool_mallocs;   /* device allocations the problem's caching pool made since creation */
  int64_t pool_trims;     /* times the pool released its cached blocks to satisfy one */
  double pool_malloc_s;   /* host seconds spent in those allocations and releases */
} lrpost_stats;

/* Create a problem: validates the description, builds the multigrid
 * hierarchy, the observation mask and the prior variance diag(P^{-1}).
 * Allocates device memory owned by the handle.  Sec. 2 (problem), Sec. 6
 * (Q1 heat equation, implicit Euler). */
int lrpost_create(const lrpost_problem_desc* desc, lrpost_problem** out);
int lrpost_destroy(lrpost_problem* p);
/* Re-target a problem to another prior precision scale alpha, noise level
 * sigma, observation box and start-block seed, keeping its mesh, time steps,
 * tolerance, rank cap, precision, stream, multigrid hierarchy, device memory
 * pool and captured graphs: every later result equals that of a problem
 * created with the new description (a resident problem for requests of one
 * size class).  Eigenpair handles made before belong to the old target and
 * are rejected afterwards (LRPOST_EINVAL).  alpha, sigma <= 0 or an empty
 * box: LRPOST_EINVAL, with the problem unchanged. */
int lrpost_retarget(lrpost_problem* p, double alpha, double sigma, const double* box, uint64_t seed);

/* Hessian apply on one low-rank vector (Sec. 6.1 eq. misfit, Sec. 4
 * Algorithm 1 matrix-vector step): forward space-time solve of the source
 * tau M X, observation and noise weighting, adjoint space-time solve,
 * tau M, and for LRPOST_PRECOND the prior solve alpha^{-1} (K+M)^{-1}.
 * x->rank may be 0 (y->rank is then 0).  y->cap must hold the truncated
 * output (at most desc.rank_cap columns).  Returns LRPOST_EINVAL on shape
 * mismatch. */
int lrpost_hess_apply(lrpost_problem* p, const lrpost_lowrank* x, lrpost_lowrank* y, int which);
/* nvec independent applies (x[i] -> y[i]) sharing spatial passes. */
int lrpost_hess_apply_batch(lrpost_problem* p, int nvec, const lrpost_lowrank* x, lrpost_lowrank* y, int which);

/* Low-rank space-time solve (Sec. 6.1 eq. st_pde with L = tau K):
 * forward (adjoint = 0):  tau K Y + M Y C^T = F1 F2^T  (time runs forward),
 * adjoint (adjoint = 1):  tau K Y + M Y C   = F1 F2^T  (time runs backward).
 * Output truncated at desc.trunc_tol in the M-weighted Frobenius norm.
 * Every space-time solve (also inside the Hessian applies) measures the
 * relative residual of its truncated output (lrpost_stats.last_st_resid) and
 * the residual preconditioned by M + tau K (last_st_presid); above the check
 * threshold the spatial basis is enriched once by a refined and extended pole
 * set (the residual monitor and basis enrichment of the AMEn solver of
 * Sec. 6.1).  A solve still above it is counted in st_unresolved, and in the
 * strict check mode returns LRPOST_ENOCONV. */
int lrpost_spacetime_solve(lrpost_problem* p, const lrpost_lowrank* f, lrpost_lowrank* y, int adjoint);
/* Residual check of the space-time solves: mode 0 off (last_st_resid =
 * last_st_presid = -1), 1 measure only, 2 (default) measure and enrich, 3
 * (strict) measure, enrich and return LRPOST_ENOCONV when a solve stays
 * above the threshold; rtol is the threshold on the preconditioned relative
 * residual (0: 50 trunc_tol, and at least 1e-4 with LRPOST_MIXED, whose
 * float32 multigrid bounds the attainable value).  Enrichment: the pole set refined by the
 * geometric midpoints of neighbouring poles and extended at the original
 * spacing up to min(24 tau / h^2, 1e4).  mode outside 0..3 or rtol < 0: LRPOST_EINVAL. */
int lrpost_set_st_check(lrpost_problem* p, int mode, double rtol);

/* Eigensolve for the k largest eigenpairs of G (Sec. 4 Algorithm 1, as block
 * Lanczos with full re-orthogonalization in the P inner product; or a
 * randomized two-pass range finder with k + oversample probes).  The result
 * handle owns device-resident eigenvector factors.
 * Convergence: every wanted pair must reach a relative Ritz residual
 * estimate (lrpost_stats.ritz_resid) of at most rtol, by default
 * max(1e-9, 0.1 trunc_tol) in FP64 and max(1e-7, 0.1 trunc_tol) mixed, block
 * Lanczos within at most min(max(8k, 64), 800) vectors (lrpost_set_eig_limits
 * overrides both).  Otherwise the call returns LRPOST_ENOCONV and *out STILL
 * holds the pairs reached, which the caller reads and frees as usual. */
int lrpost_eigensolve(lrpost_problem* p, int k, int method, int oversample, lrpost_eigs** out);
/* Limits of lrpost_eigensolve / lrpost_eigensolve_probes on this problem:
 * max_vectors caps the block-Lanczos basis (0: default), rtol the relative
 * Ritz residual target (0: default).  Negative values: LRPOST_EINVAL. */
int lrpost_set_eig_limits(lrpost_problem* p, int max_vectors, double rtol);
/* Measured relative residuals ||G v_i - lambda_i v_i||_P / |lambda_i| of the
 * k stored pairs of e (one extra Hessian apply per pair, batched four at a
 * time; the residual's P-norm from a weighted Gram product of the low-rank
 * concatenation [G v_i, v_i]).  e must come from p (else LRPOST_EINVAL);
 * resid: caller-owned host array of k doubles.  The bound |lambda - theta|
 * <= ||G v - theta v||_P of a P-normalized v certifies each eigenvalue up to
 * the accuracy of the library's (truncated) apply. */
int lrpost_eig_residuals(lrpost_problem* p, const lrpost_eigs* e, double* resid);
/* The two-pass randomized eigensolver (method LRPOST_RANDOMIZED) on caller
 * probes: Y_j = G Omega_j, a P-orthonormal basis Q of range(Y) through the
 * Gram [<Y_i, Y_j>_P], T = Q^T P G Q from a second pass of applies, Ritz
 * pairs of T (Halko, Martinsson, Tropp 2011, range finder and Rayleigh-Ritz;
 * the pencil is the one of Sec. 2, eq. prior_pre).  probes: nprobe low-rank
 * space-time vectors (W1 device, W2 host), read only.  Returns
 * min(k, rank of the probes' images) pairs; their largest relative Ritz
 * residual is in lrpost_stats.ritz_resid.  With method LRPOST_RANDOMIZED,
 * lrpost_eigensolve draws k + oversample probes G1 G2^T / sqrt(r),
 * r = min(32, rank_cap), from the library's counter-based normal generator. */
int lrpost_eigensolve_probes(lrpost_problem* p, int k, int nprobe, const lrpost_lowrank* probes,
                             lrpost_eigs** out);
int lrpost_eig_count(const lrpost_eigs* e);
/* Eigenvalues, descending, into caller-owned host array of length k. */
int lrpost_eig_values(const lrpost_eigs* e, double* lambda);
/* Copy eigenvector i (P-orthonormal) into v (v->cap must suffice; sets v->rank). */
int lrpost_eig_vector(const lrpost_eigs* e, int i, lrpost_lowrank* v);
int lrpost_eig_vector_rank(const lrpost_eigs* e, int i);
int lrpost_eigs_free(lrpost_eigs* e);
/* Build an eigs handle from caller eigenpairs (lambda host, vectors as
 * low-rank factors), e.g. to evaluate the posterior of a known basis. */
int lrpost_eigs_from_pairs(lrpost_problem* p, int k, const double* lambda, const lrpost_lowrank* v,
                           lrpost_eigs** out);

/* Number of observed nodes (the interior nodes inside the closed box), or -1
 * for a null handle. */
int lrpost_obs_count(const lrpost_problem* p);
/* Posterior mean, which for this linear-Gaussian problem is the MAP point of
 * Sec. 2 (eq. map1 and the minimization after it, with zero prior and noise
 * means): the solution of (H_mis + P) u = sigma^{-2} F^T y.  Solved as
 * (G + I) u = P^{-1} sigma^{-2} F^T y in the P inner product by block
 * Lanczos with full re-orthogonalization started from the right-hand side
 * (the Lanczos form of conjugate gradients; block size 4, three seeded
 * start vectors beside the right-hand side), every Krylov vector a low-rank
 * space-time vector.  y_obs: host, nobs x nt column-major (nobs =
 * lrpost_obs_count, observed nodes in increasing node order, column k the
 * observations at t_{k+1}), caller-owned, read only.  max_vectors caps the
 * Krylov vectors (0: 800); rtol is the target of the relative residual
 * estimate ||(G + I) u - rhs||_P / ||rhs||_P (0: max(1e-7, 1e3 trunc_tol)).
 * The apply's truncation error bounds the attainable accuracy (it enters as
 * about trunc_tol times the largest eigenvalue of G relative to the shift
 * 1), so meaningful means need tight tolerances.  mean: output (cap columns,
 * rank set); rel_resid (may be NULL): the final estimate.  Returns
 * LRPOST_ENOCONV, with mean and rel_resid still written, when the target is
 * not met within max_vectors. */
int lrpost_posterior_mean(lrpost_problem* p, const double* y_obs, int max_vectors, double rtol, lrpost_lowrank* mean,
                          double* rel_resid);

/* diag(Gamma_post,k) = diag(P^{-1}) - sum_i d_i v_i^2, d_i = lambda_i/(1+lambda_i)
 * (Sec. 2, Sherman-Morrison-Woodbury step), as an nx x nt array
 * (column-major, caller-owned; `on_device` says whether diag is device memory). */
int lrpost_post_variance(lrpost_problem* p, const lrpost_eigs* e, double* diag, int on_device);
/* diag(P^{-1}) over one time step (nx values, host). */
int lrpost_prior_variance(lrpost_problem* p, double* dprior);

/* ns zero-mean posterior samples s = (I - V diag(p_i) V^T P) L xi with
 * p_i = 1 - (1+lambda_i)^{-1/2} and L = (alpha tau)^{-1/2} (I kron (K+M)^{-1/2})
 * (the symmetric root, applied through the sine basis that diagonalizes K and
 * M).  The covariance of s is Gamma_post,k: the low-rank update of Sec. 2
 * (eq. prior_pre) written as a factor L_post L_post^T.  xi: caller-supplied
 * standard normal draws; xi and out: ns * nx * nt float64 each (sample-major,
 * each sample nx x nt column-major), caller-owned, device memory when
 * on_device != 0, else host.  ns * nt <= 65535. */
int lrpost_sample(lrpost_problem* p, const lrpost_eigs* e, int ns, const double* xi, double* out, int on_device);

int lrpost_get_stats(const lrpost_problem* p, lrpost_stats* s);

/* Progress logging: level > 0 prints one JSON line per eigensolver step to
 * stderr (step, vectors, applies, time in applies and in re-orthogonalization,
 * worst relative Ritz residual of the wanted pairs). */
int lrpost_set_log(lrpost_problem* p, int level);

/* Kernel timing for measurement: while enabled, every launch of the
 * multigrid kernels below is bracketed by HIP events on the problem's stream
 * and credited with its algorithmic traffic in bytes (elements of the
 * precision it runs in, float32 for the V-cycles of LRPOST_MIXED):
 *   LRPOST_KERNEL_SMOOTHER_STEP  one Chebyshev step: read x_cur, x_prev and b
 *                                once, write x_new once (absent operands are
 *                                not counted);
 *   LRPOST_KERNEL_MG_DOWN        level-fused pre-smoothing, residual and
 *                                restriction: read b, write x and the coarse
 *                                right-hand side;
 *   LRPOST_KERNEL_MG_UP          level-fused prolongation and post-smoothing:
 *                                read the pre-smoothed x, the coarse
 *                                correction and b, write x;
 *   LRPOST_KERNEL_GRAM           the matrix-core stage of the float64 Gram
 *                                products A^T B (nx x m and nx x q operands):
 *                                read A and B once, 2 m q nx flops;
 *   LRPOST_KERNEL_PROJ           the float64 matrix-core projection
 *                                C = beta C + A Q (A nx x m, C nx x p): read A
 *                                once, read C once when beta != 0, write C
 *                                once, 2 m p nx flops;
 *   LRPOST_KERNEL_STENCIL        the Q1 stencil Y = a K X + b M X (+ c Z) on
 *                                the finest mesh (the operator applies and
 *                                the residuals of the multigrid correction
 *                                cycles): read X (and Z) once, write Y once.
 *   LRPOST_KERNEL_GRAM32,        the same Gram products and projections on
 *   LRPOST_KERNEL_PROJ32         the float32 matrix cores (the first
 *                                Gram-Schmidt sweep of the mixed-precision
 *                                basis building): the basis operand A is read
 *                                as float32 (4 bytes per element), the others
 *                                as for the float64 kinds.
 *   LRPOST_KERNEL_SINE           the sine transform along x1 of the
 *                                convection-diffusion solves (a dense product
 *                                with the n x n sine matrix on the float64
 *                                matrix cores): read X once, write Y once,
 *                                2 n flops per node;
 *   LRPOST_KERNEL_TRIDIAG        the tridiagonal systems along x2 of those
 *                                solves: the right-hand side read once, the
 *                                eliminated values and multipliers written
 *                                and read back once, the solution written:
 *                                six float64 streams per node.
 * lrpost_profile_read synchronizes, returns for one kind the launch count, the
 * summed kernel time in ms, the counted bytes and (if flops is not NULL) the
 * counted floating-point operations since the last read, and resets that
 * kind's counters. */
enum {
  LRPOST_KERNEL_SMOOTHER_STEP = 0,
  LRPOST_KERNEL_MG_DOWN = 1,
  LRPOST_KERNEL_MG_UP = 2,
  LRPOST_KERNEL_GRAM = 3,
  LRPOST_KERNEL_PROJ = 4,
  LRPOST_KERNEL_STENCIL = 5,
  LRPOST_KERNEL_GRAM32 = 6,
  LRPOST_KERNEL_PROJ32 = 7,
  LRPOST_KERNEL_SINE = 8,
  LRPOST_KERNEL_TRIDIAG = 9
};
int lrpost_profile(lrpost_problem* p, int enable);
int lrpost_profile_read(lrpost_problem* p, int kernel, int64_t* launches, double* total_ms, double* bytes,
                        double* flops);

/* Multigrid kernel choice: on (the default) runs each V-cycle level on meshes
 * of up to 1023 nodes per side as two level-fused kernels (pre-smoothing with
 * residual and restriction; prolongation with post-smoothing), off as one
 * kernel per smoother step, residual-restriction and prolongation.  Both
 * compute the same iterates; finer meshes always take the per-step kernels. */
int lrpost_set_mg_fused(lrpost_problem* p, int on);

/* Autotuned tile shape of the Q1 stencil kernel: the strip height (8, 16 or
 * 32 mesh rows per workgroup) of every shape class -- precision, mesh side,
 * column count rounded up to a power of two, with or without the added term
 * -- is chosen by timing the three heights on the class's first launch (the
 * fastest is kept for the process).  Every height computes every node with
 * the same operations, so results do not depend on the choice.
 * lrpost_set_autotune(0) uses a fixed rule (tall strips when there are
 * enough columns for a few thousand workgroups) for classes not yet timed.
 * lrpost_autotune_report writes the table (one text line per class: its
 * choice and the three times) into buf (len bytes, NUL-terminated,
 * truncated to fit) and returns the full length. */
int lrpost_set_autotune(int on);
int lrpost_autotune_report(char* buf, size_t len);

/* Batch size of the randomized eigensolver's probe applies: n > 0 applies
 * at most n probes per batched pass (one multigrid solve for all their pole
 * solves); 0 (the default) takes as many as fit in half of the device memory
 * that was free when the problem was created, by an estimate of 56 bytes per
 * node, pole and probe column in mixed precision (about 38 rank-32 probes per
 * pass on the 512 x 512, nt = 500 workload).  Results do not depend on the
 * batch size.  n < 0: LRPOST_EINVAL. */
int lrpost_set_apply_batch(lrpost_problem* p, int n);

/* HIP graphs of the multigrid V-cycles: with on (the default) every V-cycle
 * launch sequence (the level kernels down, the LDS coarse solve, the level
 * kernels up) is captured once per precision, column count and buffers into
 * a HIP graph on the problem's stream and replayed from then on, one graph
 * launch in place of 2L + 1 kernel launches; off launches the kernels one by
 * one (and frees the captured graphs).  Both give the same bits.  Runs with
 * kernel timing enabled (lrpost_profile) launch directly.
 * lrpost_graph_info returns the number of graphs captured and of graph
 * launches since the problem was created. */
int lrpost_set_graphs(lrpost_problem* p, int on);
int lrpost_graph_info(const lrpost_problem* p, int64_t* captured, int64_t* launches);

/* ---- the initial-condition problem of the paper's experiments ----------
 * Sec. 6 (eqs. pde, obj, dis_obj, postvar, misfit) and Sec. 6.2: the unknown
 * is the initial state u = y(0), one value per interior node (node index
 * j n + i, x1 fastest); the state follows the source-free heat equation
 * from it on the problem's mesh and time steps, (M + tau K) y_1 = M u,
 * (M + tau K) y_k = M y_{k-1}, i.e. the space-time system of eq. st_pde with
 * right-hand side (M u) e_1^T; the observations are the problem's observed
 * nodes at t_1..t_nt with noise sigma^2 I (sigma from the description), and
 * the prior covariance is prior_var * I (the paper's experiments: 10 I with
 * sigma^-2 = 1e4 / prior_var).  The prior-preconditioned misfit Hessian of
 * eq. misfit is then G = prior_var sigma^-2 C^T K^-T B^T B K^-1 C with
 * C = e_1 kron M, a symmetric operator on nodal vectors.  The space-time
 * solves inside are the low-rank solver of lrpost_spacetime_solve, so the
 * accuracy follows the description's trunc_tol.  Each call is independent:
 * nothing of it is stored in the problem. */

/* Observed nodes from a mask: mask[i] != 0 for each observed interior node
 * (host, nx bytes, caller-owned).  Replaces the observation box of the
 * description for every later call (the space-time source problem uses it
 * too); eigenpair handles made before are rejected afterwards.  An all-zero
 * mask: LRPOST_EINVAL. */
int lrpost_set_obs_mask(lrpost_problem* p, const uint8_t* mask);

/* Y = G U for nvec initial states: U and Y are nx x nvec column-major device
 * buffers (caller-owned, distinct).  prior_var <= 0 or a null buffer with
 * nvec > 0: LRPOST_EINVAL. */
int lrpost_ic_apply(lrpost_problem* p, double prior_var, int nvec, const double* U, double* Y);

/* The k leading eigenpairs of G (Sec. 4, Algorithm 1 for the self-adjoint G:
 * block Krylov steps of 4 applies (8 when k >= 32) with full re-orthogonalization by
 * classical Gram-Schmidt twice, and Rayleigh-Ritz on the whole basis).
 * values: host, k doubles, descending.  vectors: device, nx x k
 * column-major, Euclidean-orthonormal (caller-owned).  Stops when every
 * wanted pair has ||G x - theta x|| <= rtol theta_1 (theta_1 the largest
 * Ritz value, the norm of G: every apply carries the truncation error of its
 * space-time solves relative to the whole operator; rtol <= 0: max(1e-8,
 * 0.1 trunc_tol), in mixed precision max(1e-6, 0.1 trunc_tol)), or when
 * another block would pass max_vectors basis vectors (<= 0: max(8k, 40));
 * then LRPOST_ENOCONV, with the Ritz pairs reached written all the same.
 * used_vectors (may be NULL) receives the basis size. */
int lrpost_ic_eigensolve(lrpost_problem* p, double prior_var, int k, int max_vectors, double rtol, double* values,
                         double* vectors, int* used_vectors);

/* Posterior variance diag(prior_var (I + G)^-1) from k eigenpairs of G
 * (eq. postvar with the Sherman-Morrison-Woodbury update):
 * out[i] = prior_var - prior_var sum_j values[j] / (1 + values[j]) vectors[i, j]^2.
 * values host (k), vectors device (nx x k), out nx doubles on the device
 * (on_device != 0) or on the host. */
int lrpost_ic_post_variance(lrpost_problem* p, double prior_var, int k, const double* values, const double* vectors,
                            double* out, int on_device);

/* ---- the convection-diffusion operator (Sec. 6.3) ------------------------
 * L = -nu Laplace + w . grad with the wind w = (0, wind) along x2,
 * discretized by SUPG bilinear elements on the problem's mesh (homogeneous
 * Dirichlet conditions).  For bilinear elements the stabilized operator is
 * nu K + wind N + delta wind^2 S: N the convection matrix (w . grad phi_j,
 * phi_i)/wind, S the streamline matrix (d phi_j/dx2, d phi_i/dx2); the time
 * derivative keeps the mass matrix M (eq. st_pde with L in place of K).
 *
 * lrpost_set_convection switches the spatial operator of
 * lrpost_spacetime_solve and of the initial-condition problem (lrpost_ic_*)
 * to L: forward solves use L, adjoint solves L^T (eq. postvar's K^-T), so G
 * stays symmetric.  nu > 0 sets it; delta < 0 takes the element Peclet rule
 * (delta = h / (2|wind|) (1 - 1/Pe) for Pe = |wind| h / (2 nu) > 1, else 0),
 * delta >= 0 is used as given (below the rule the shifted solves lose their
 * stability guarantee); nu <= 0 returns to the heat operator K.  While L is
 * set, the calls of the space-time source problem (hess_apply*,
 * eigensolve*, eig_residuals, posterior_mean) return LRPOST_EINVAL.
 * Non-finite parameters: LRPOST_EINVAL.  The shifted solves (tau L + p M) of
 * the rational Krylov basis are exact: a sine transform along x1 (where the
 * operator is symmetric), one tridiagonal system along x2 per sine mode, and
 * the inverse transform. */
int lrpost_set_convection(lrpost_problem* p, double nu, double wind, double delta);
/* Host settings of the convection-diffusion operator for a mesh of N cells
 * per side and nt steps over [0, T] (no problem, no device work): out[0]
 * delta (the Peclet rule when delta < 0), out[1], out[2] the rectangle
 * [1, out[1]] x i[-out[2], out[2]] that holds the field of values of every
 * projected I + tau Q^T L Q with Q^T M Q = I, out[3] the Newton-Schulz start
 * alpha (X_0 = alpha I), out[4] the bound r < 1 of the numerical radius of
 * I - alpha (I + tau Q^T L Q), out[5] the step count (2 r^(2^k) <= 1e-18),
 * out[6] the lower spectral bound of the symmetric part of M^{-1} L.
 * out: host, 7 doubles.  N < 2, nt < 1, T <= 0, nu <= 0 or non-finite
 * values: LRPOST_EINVAL. */
int lrpost_convdiff_params(int N, int nt, double T, double nu, double wind, double delta, double* out);
/* Building blocks for kernel-level parity tests (DEVICE float64 buffers, nx x
 * ncols column-major, leading dimension nx; coef: host, 2 ncols doubles
 * (a_j, b_j)):
 *   apply: Y[:,j] = (a_j L + b_j M) X[:,j]  (transpose != 0: L^T);
 *   solve: X[:,j] = (a_j L + b_j M)^{-1} B[:,j] (transpose != 0: L^T), with
 *          a_j, b_j >= 0 and a_j + b_j > 0 (LRPOST_EINVAL otherwise); B may
 *          equal X.
 * LRPOST_EINVAL without a convection operator set. */
int lrpost_convdiff_apply(lrpost_problem* p, int ncols, const double* X, double* Y, const double* coef,
                          int transpose);
int lrpost_convdiff_solve(lrpost_problem* p, int ncols, const double* B, double* X, const double* coef,
                          int transpose);

/* Device memory kept for reuse: a problem's allocator caches the blocks its
 * calls free (results stay valid; the cache only speeds up the next call).
 * lrpost_release_cache waits for the problem's stream, returns every cached
 * block to the device and stores the bytes released in *released_bytes (if
 * not NULL).  Call it before allocating large buffers elsewhere on the same
 * device (the binding does so when a device allocation of its own fails).
 * Buffers held by live eigenpair handles are not cached and stay valid. */
int lrpost_release_cache(lrpost_problem* p, uint64_t* released_bytes);

/* ---- building blocks, exported for kernel-level parity tests ----------
 * All pointers are DEVICE memory, float64, column-major with leading
 * dimension nx (the problem's nx). */

/* Y[:,j] = (a_j K + b_j M) X[:,j] + c_j Z[:,j] for j < ncols on the finest mesh
 * (Z may be NULL); coef: host array of 3*ncols doubles (a_j, b_j, c_j). */
int lrpost_stencil_apply(lrpost_problem* p, int ncols, const double* X, double* Y, const double* Z,
                         const double* coef);
/* X[:,j] approx (a_j K + b_j M)^{-1} B[:,j] by `cycles` multigrid V-cycles from
 * X = 0 (coef: host, 2*ncols doubles a_j >= 0, b_j >= 0, a_j + b_j > 0). */
int lrpost_mg_solve(lrpost_problem* p, int ncols, const double* B, double* X, const double* coef, int cycles);
/* C = A^T B  (A: nx x m, B: nx x q, C: host m x q column-major). */
int lrpost_gram(lrpost_problem* p, int m, const double* A, int q, const double* B, double* C_host);
/* C = A^T B like lrpost_gram, with A (nx x m) in float32 DEVICE memory and
 * B (nx x q) float64: the float32 matrix-core kernel of the first
 * Gram-Schmidt sweep of mixed precision (B rounded to float32 as it is
 * staged, float32 accumulation within a row chunk, float64 across chunks);
 * C host, m x q column-major. */
int lrpost_gram_f32(lrpost_problem* p, int m, const float* A, int q, const double* B, double* C_host);
/* Mixed precision only: the first of the two Gram-Schmidt sweeps that build
 * the rational Krylov basis of every space-time solve runs on the float32
 * matrix cores against a float32 copy of the basis (fp32_first != 0, the
 * default), or in float64 like the second.  The second sweep is float64
 * either way; it removes what the first leaves (Sec. 4's re-orthogonalization
 * done twice). */
int lrpost_set_sweep_precision(lrpost_problem* p, int fp32_first);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the Gram
 * product of lrpost_gram, C = A^T B, with C in DEVICE memory (m x q,
 * column-major, leading dimension m, caller-owned) instead of host memory.
 * Its partial products go to a static scratch array of 64 MiB per device
 * (resolved when the first problem is created on that device and held until
 * the process ends); the call allocates and frees nothing and does not
 * synchronize: the work is enqueued on p's stream and C is complete when the
 * stream reaches it.  Every call on one device shares that array, so calls
 * whose work overlaps on one device (two streams, two threads) race; calls
 * ordered on one stream do not.  Returns LRPOST_EINVAL when the product needs
 * more than the array holds (e.g. m = q = 4096 on a 32 x 32 mesh); the same
 * kernels and chunking as lrpost_gram give the same bits. */
int lrpost_gram_noalloc(lrpost_problem* p, int m, const double* A, int q, const double* B, double* C_dev);
/* Truncate X = W1 W2^T in place to tolerance tol (<= 0: desc.trunc_tol) and
 * rank <= cap; weighted = 1 measures in the M-norm in space. */
int lrpost_truncate(lrpost_problem* p, lrpost_lowrank* x, double tol, int weighted);

/* ---- serving loop ------------------------------------------------------
 * Posterior requests (the k leading eigenpairs by block Lanczos and, when
 * want_diag != 0, diag(Gamma_post,k) over nx * nt points; Sec. 2, Sec. 6
 * eq. postvar) of any mesh and time size, served concurrently.  `workers`
 * threads (1..16) each own a HIP stream; a worker takes a pending request
 * whose device-memory estimate fits in what is left of hbm_budget_bytes (one
 * of its resident size class among the first eight pending if there is one,
 * else the oldest; a request always runs when nothing else does), so that
 * requests arriving while others run are admitted as workers and memory free
 * up and overlap with them on the device.  Each worker keeps the problem of
 * the last size class (mesh, nt, T, tolerance, rank cap, precision) it served
 * resident on the device and prefers pending requests of that class, which
 * it serves on that problem re-targeted to their prior, noise and box (a
 * parked problem's memory estimate stays counted against the budget); a
 * request's result is the one it would have alone.
 * submit copies the description and returns a ticket at once; wait blocks
 * until that request is done, writes k eigenvalues (host) and, if diag is
 * not NULL and the request asked for it, nx * nt variances (host,
 * column-major nx x nt), and the latency from submit to completion in
 * seconds, then forgets the ticket.  A request's error code and message are
 * returned by its wait.  destroy finishes running requests, fails pending
 * ones, and must not run concurrently with a wait on the same server. */
typedef struct lrpost_server lrpost_server;
int lrpost_server_create(size_t hbm_budget_bytes, int workers, lrpost_server** out);
int lrpost_server_submit(lrpost_server* s, const lrpost_problem_desc* desc, int k, int want_diag, uint64_t* ticket);
int lrpost_server_wait(lrpost_server* s, uint64_t ticket, double* lambda, int k, double* diag, double* latency_s);
/* largest number of requests that ran at once and largest admitted memory estimate */
int lrpost_server_info(lrpost_server* s, int* peak_running, size_t* peak_admitted_bytes);
/* requests served so far, and how many of them ran on a worker's resident
 * problem of their size class (re-targeted, lrpost_retarget) */
int lrpost_server_class_stats(lrpost_server* s, int64_t* served, int64_t* resident_hits);
int lrpost_server_destroy(lrpost_server* s);

/* Attainable float64 rates of the current device (instrumentation; no
 * passage of the paper): times v_mfma_f64_16x16x4f64 (the instruction of the
 * float64 Gram, projection and sine-transform kernels) and the vector FMA
 * with operands in registers only, each over 2048 workgroups of 256 threads
 * and `iters` (1..100000) unrolled rounds, best of three launches after one
 * untimed.  out[0] = matrix-core TFLOP/s, out[1] = vector-FMA TFLOP/s (host
 * memory, two doubles).  Allocates and frees 4 MiB of device memory and a
 * stream of its own; synchronizes.  EINVAL for iters out of range or a NULL
 * out, EHIP for a failed HIP call. */
int lrpost_measure_fp64_rates(int iters, double* out);

const char* lrpost_last_error(void);
const char* lrpost_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LRPOST_H */
