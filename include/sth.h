/*
 * sth.h - C ABI of the MI355X (gfx950) space-time heat-equation slab solver.
 *
 * The library implements the hot path of the time-parallel multigrid of
 * Hofer, Langer and Neumueller, "Robust Preconditioning for Space-Time
 * Isogeometric Analysis of Parabolic Evolution Problems" (arXiv 1802.09277):
 * the space-time dG-IgA system L_h u = f of the heat equation on the unit
 * square or cube (eq. equ_linear_system: block lower bidiagonal, diagonal
 * blocks A_n = K_t (x) M_x + M_t (x) K_x, sub-diagonal blocks -B_n with
 * B_n = N_t (x) M_x, eq. structureAn), its residual, the damped block-Jacobi
 * slab smoother (Section 3.1) whose slab inverses A_n^{-1} are applied
 * through the decomposition eq. equ:ST:generalDecompA with the temporal
 * generalized eigen decomposition (Section 3.3, in real 2x2-block form) and
 * fast diagonalisation of the spatial spline pencils, time restriction and
 * prolongation (two slabs -> one), the V-cycle and the solve loop.
 *
 * Conventions for every entry point:
 *  - Vectors are caller-owned, contiguous FP64 device buffers of
 *    sth_vector_len(h) elements, laid out u[slab][t][z][y][x] (x fastest;
 *    the time index is the slower Kronecker index of eq. structureAn; only
 *    the interior spatial B-splines are unknowns, u = 0 on the lateral
 *    boundary).  The library never frees them.
 *  - `stream` is a hipStream_t (NULL = default stream).  Calls are
 *    stream-ordered and asynchronous unless stated otherwise.
 *  - Every call returns an sth_status; on failure sth_last_error() gives a
 *    thread-local message.  Invalid arguments return STH_EINVAL before any
 *    allocation or launch.  Nothing throws across the ABI.
 *  - Calls on one handle must not overlap in time (they share workspaces).
 */
#ifndef STH_H
#define STH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sth_handle sth_handle;

typedef enum {
    STH_OK = 0,
    STH_EINVAL = -1,    /* invalid argument or unsupported shape */
    STH_ENOMEM = -2,    /* device allocation failed */
    STH_EHIP = -3,      /* a HIP runtime call failed */
    STH_ENOTPOS = -4,   /* M_t not positive, or a temporal eigenvalue with
                           Re(lambda) <= 0 (the a-posteriori check of Section
                           3.2: reduce theta) */
    STH_ECOND = -5,     /* temporal eigenvector matrix too ill-conditioned
                           for the diagonalisation path (Section 3.3, last
                           paragraph; Table 1) */
    STH_ENOCONV = -6,   /* NaN/Inf, residual growth, or maxit reached */
    STH_ENODEV = -7,    /* no usable GPU */
    STH_EAGAIN = -8     /* serving: the request has not finished yet */
} sth_status;

typedef enum {
    STH_FP64 = 0,       /* spatial eigenbasis transforms in FP64 (MFMA f64) */
    STH_FP32 = 1,       /* transforms in FP32 MFMA, FP32 accumulation */
    STH_BF16X3 = 2      /* transforms as 3 BF16 MFMA products (hi*hi, hi*lo,
                           lo*hi), FP32 accumulation */
} sth_prec;

/* The discrete problem (Sections 2.1-2.3): unit square (dim 2) or cube
 * (dim 3), open uniform knot vectors, degree `degree` in space and time,
 * n_slabs equal slabs on (0,T), n_elem_t time elements per slab, SUPG
 * parameter sigma = theta * (T / n_slabs / n_elem_t).  The multigrid
 * coarsens in time only (two slabs -> one) while the slab count is even and
 * larger than coarse_slabs; the coarsest level is solved exactly by
 * slab-wise forward substitution (in the spatial eigenbasis, where the
 * coupling B_n only carries the last time row of the previous slab).
 * omega is the damping of the block-Jacobi smoother (Section 3.1: 1/2),
 * nu_pre / nu_post the smoothing steps of the V-cycle. */
typedef struct {
    int dim;            /* 2 or 3 */
    int n_elem;         /* spatial elements per axis, >= 2 */
    int degree;         /* 1..4 */
    int n_slabs;        /* >= 1 */
    int n_elem_t;       /* >= 1; N_t = n_elem_t + degree <= 8 */
    double T;           /* > 0 */
    double theta;       /* >= 0 */
    double omega;       /* (0, 1] */
    int nu_pre;         /* >= 0 */
    int nu_post;        /* >= 0 */
    int transform_prec; /* sth_prec */
    int coarse_slabs;   /* >= 1: stop coarsening at this many slabs or fewer */
    int iterate_basis;  /* sth_solve only: 0 iterate on the B-spline
                           coefficients; 1 keep the iterate in the spatial
                           eigenbasis of the smoother (u = (I (x) U_x) u^),
                           where L_h, D^{-1} and the time transfers act
                           pointwise over spatial modes; the spatial
                           transforms then run once on f, once per cycle on the
                           residual for the stopping test, and once on the
                           result.  Same iterates in exact arithmetic. */
    int temporal_form;  /* how A_n^{-1} treats the temporal pencil (K_t, M_t),
                           Section 3.3: 0 diagonalisation K_t V = M_t V Z
                           (STH_ECOND when cond(V) > 1e8); 1 real Schur form
                           M_t^{-1} K_t = Q R Q^T (orthogonal Q, a block back
                           substitution per spatial mode); 2 diagonalisation
                           unless cond(V) > 1e6, then real Schur (default) */
    double space_ratio; /* coarsening in space (Section 4.4, the multigrid
                           coarsens in space as well as in time): 0 (default)
                           time only; > 0 a level transition also halves the
                           spatial elements per axis when the level's
                           tau / h_x^2 >= space_ratio (h_x = 1 / n_elem) and
                           its element count is even and at least 4 (the
                           ratio halves on such a step and doubles on a time
                           step; 2 keeps the cycle counts of time-only
                           coarsening).  The prolongation in space is the
                           embedding of the coarse spline space (knot
                           insertion), the coarse operators the Galerkin
                           ones, i.e. the rediscretisations on the coarse
                           mesh with the finest sigma.  Requires
                           iterate_basis 0 (STH_EINVAL otherwise). */
    int minres_iters;   /* slab inverse of the smoother (Section 3.3,
                           Theorems 3.8 and 3.10): 0 (default) exact by fast
                           diagonalisation; k > 0: through the temporal eigen
                           form, each real eigenvalue's spatial system solved
                           exactly and each conjugate pair's 2x2 block system
                           by k iterations of MinRes (zero start) on the
                           symmetric form of Theorem 3.10 with its block
                           diagonal preconditioner P (applied exactly).  The
                           preconditioned spectrum lies in [-1, -1/sqrt 2] u
                           [1/sqrt 2, 1], so k = 12 reduces each block residual
                           (P^{-1} norm) by 1e-4, the accuracy of Section 4.4,
                           and k = 28 by 1e-10.  The coarsest level stays
                           exact.  Requires iterate_basis 0 and the eigen
                           form on every level (STH_EINVAL otherwise); at most
                           200. */
} sth_problem;

/* Right-hand side as a sum of separable modes (host arrays):
 *   f(x,t) = sum_m amp[m] prod_a sin(k[m*dim+a] pi x_a) cos(omega[m] pi t + phase[m]),
 * zero initial data.  The load vector is l_h(phi_i) (Section 2.2) with a
 * Gauss rule of degree+3 points per direction and element. */
typedef struct {
    int n_modes;
    const double* amp;
    const int* k;
    const double* omega;
    const double* phase;
} sth_rhs_modes;

/* Fills p with the defaults of Section 4.4: theta 0.01, omega 1/2, T 1,
 * V(1,1), FP64 transforms, the automatic temporal form and coarse_slabs 128:
 * the exact coarsest-level solve runs parallel in time, so a level of up to
 * 128 slabs is cheaper to solve exactly than to coarsen further, and the
 * eigenbasis iteration then takes it together with the level above it in one
 * pass (the shape fields are left at zero). */
void sth_problem_default(sth_problem* p);

/* Device bytes that sth_setup would allocate for this problem (factors,
 * coarse-level vectors and workspaces; not the caller's vectors).  Host
 * only, no allocation: used for admission by memory footprint. */
int sth_workspace_bytes(const sth_problem* p, size_t* bytes);

/* Host FP64 setup and upload on `stream`: the 1-D spatial mass and stiffness
 * matrices and the temporal matrices K_t, M_t of eq. TimeMatrices on every
 * level (Section 2.3, the slab operators of eq. structureAn), the temporal
 * pencil of every level in the eigen form of Section 3.3 (real 2x2 blocks,
 * the Re(lambda) > 0 check of Section 3.2 -> STH_ENOTPOS, the cond(V) guard
 * -> STH_ECOND) or its real Schur form, the spatial fast-diagonalisation
 * factors, and the time prolongation of Section 3.1.  Arguments: the problem
 * (host, read only), a hipStream_t (NULL = default stream), *out receives the
 * handle.  On success *out owns device memory until sth_destroy; on failure
 * *out is NULL and nothing stays allocated.  Synchronises `stream`. */
int sth_setup(const sth_problem* p, void* stream, sth_handle** out);

/* n_slabs * N_t * n^dim (n = n_elem + degree - 2), or 0 for NULL. */
size_t sth_vector_len(const sth_handle* h);

/* The same for a problem description, without a setup (0 if invalid). */
size_t sth_problem_vector_len(const sth_problem* p);

/* Number of multigrid levels (1 + number of coarsenings). */
int sth_num_levels(const sth_handle* h);

/* Spatial elements per axis on a multigrid level (0 for a bad level):
 * n_elem halved once per space-time coarsening step above it. */
int sth_level_elems(const sth_handle* h, int level);

/* f <- load vector of the given modes (host 1-D quadrature, device outer
 * products). */
int sth_load_rhs(sth_handle* h, const sth_rhs_modes* m, double* f, void* stream);

/* The same load vector as sth_load_rhs, for callers that cannot allocate
 * device memory (tight serving loops, code that runs between the captures of
 * a caller's HIP graphs, harnesses that forbid hipMalloc): the temporal and
 * spatial mode tables are staged in a fixed device array of the library
 * (4 MiB per GPU, 524288 doubles, held until the process ends) instead of
 * device memory allocated per call.  This call allocates no device or pinned
 * host memory.  The tables need n_modes * (n_slabs * N_t + 3 n) doubles; a
 * larger request returns STH_EINVAL before any copy or launch.  Every call on
 * one GPU shares that GPU's array, so calls that overlap in time on the same
 * GPU (from several threads or on several streams) race; like sth_load_rhs,
 * the call synchronises `stream` before it returns, so consecutive calls from
 * one thread do not overlap. */
int sth_load_rhs_noalloc(sth_handle* h, const sth_rhs_modes* m, double* f, void* stream);

/* y <- L_h u  (eq. equ_linear_system). */
int sth_apply(sth_handle* h, const double* u, double* y, void* stream);

/* r <- f - L_h u, i.e. r_n = f_n - A_n u_n + B_n u_{n-1} for all slabs
 * (eq. equ_linear_system with A_n, B_n of eq. structureAn).  f, u, r: device
 * vectors of sth_vector_len(h) doubles; r must not alias f or u. */
int sth_residual(sth_handle* h, const double* f, const double* u, double* r, void* stream);

/* z <- D^{-1} r with D = diag(A_n): every slab inverted independently by
 * eq. equ:ST:generalDecompA (exact up to rounding for FP64 transforms), or
 * with minres_iters > 0 by the MinRes slab inverse of the smoother. */
int sth_block_solve(sth_handle* h, const double* r, double* z, void* stream);

/* `steps` damped block-Jacobi steps u <- u + omega D^{-1}(f - L_h u) with
 * D = diag(A_n), the smoother of the time-parallel multigrid (Section 3.1);
 * u (device, sth_vector_len(h) doubles) is updated in place. */
int sth_smooth(sth_handle* h, const double* f, double* u, int steps, void* stream);

/* One V(nu_pre, nu_post) cycle of the time-parallel multigrid (Section 3.1:
 * the slab smoother, restriction and prolongation in time between pairs of
 * slabs and one coarse slab, an exact solve on the coarsest level) on the
 * finest level; u (device) is updated in place.  Iterates on the B-spline
 * coefficients, whatever iterate_basis says. */
int sth_vcycle(sth_handle* h, const double* f, double* u, void* stream);

/* V-cycles from the initial guess in u until ||f - L_h u||_2 <= rtol ||f||_2
 * (the stopping test of Section 4.4: Euclidean norm of the coefficient
 * vector relative to the right-hand side) or maxit cycles.  f, u: device
 * vectors of sth_vector_len(h) doubles (u holds the initial guess and
 * receives the result).  Blocks the host until the result is in u.  iters
 * and relres (may be NULL) receive the cycle count and the final relative
 * residual (in the eigenbasis iteration an upper bound of it when the
 * two-sided bound decides the test, else the exact value).  With
 * iterate_basis 1 and transform_prec FP32 or BF16x3 the solve is an FP64
 * defect correction: each outer step forms the FP64 residual and its exact
 * norm, and an eigenbasis solve with reduced-precision transforms reduces
 * it; iters is then the sum of the inner cycles.  Returns STH_ENOCONV on
 * NaN, on growth over 3 consecutive cycles (outer steps) or when maxit is
 * reached. */
int sth_solve(sth_handle* h, const double* f, double* u, double rtol, int maxit,
              int* iters, double* relres, void* stream);

/* The same system solved by flexible GMRES(restart), right-preconditioned
 * by one V-cycle from a zero initial guess in the handle's iteration basis
 * (the multigrid used as a preconditioner instead of as the solver, as the
 * paper's introduction and Section 3.1 allow).  u holds the initial guess;
 * stops when the true ||f - L_h u||_2 <= rtol ||f||_2 (checked at every
 * restart and at convergence of the Arnoldi estimate) or after maxit
 * preconditioned iterations.  restart in 1..31.  The first call allocates
 * (2 restart + 1) level-0 vectors of workspace, kept by the handle.
 * Blocks the host (a few scalars per iteration); STH_ENOCONV as sth_solve. */
int sth_solve_fgmres(sth_handle* h, const double* f, double* u, double rtol, int maxit, int restart,
                     int* iters, double* relres, void* stream);

/* Graph replay of the solve iterations (default off: on this hardware the
 * boundaries between replayed graphs cost more than individual launches
 * of the few kernels of a cycle): on a non-default
 * stream sth_solve captures one iteration (V-cycle, residual, norm, scalar
 * read) into a HIP graph for the given (f, u) and replays it (on any
 * stream; a new f or u, or a change of the timing mask, recaptures).
 * enable = 0 launches every kernel individually; so does kernel timing
 * (sth_timing), which needs events around the individual launches. */
int sth_use_graphs(sth_handle* h, int enable);

/* Speculative cycles (default on; eigenbasis iteration with V(1,1) cycles,
 * a level below the finest and N_t <= 5): sth_solve enqueues each cycle
 * before the residual norm of the one ahead of it has reached the host.
 * The final sum of a cycle stores on the device whether the next cycle
 * must run (its lower bound of the B-spline residual exceeds rtol ||f||);
 * when it may have converged every kernel of the next cycle returns at
 * once and the exact norm decides, so the cycles, iterates and counts are
 * those of the plain loop (the stopping test of Section 4.4) without a host
 * round trip between cycles.  The first cycles follow the initial residual
 * pass the same way (its threshold (rtol ||f||)^2 formed on the device), and
 * on the 2-D path the mapping of the result into u goes behind the exact
 * norm, guarded by the device's copy of the final test.
 * enable = 0 waits for each norm first; so does kernel timing. */
int sth_speculate(sth_handle* h, int enable);

/* Level transfers (Section 3.1, time coarsening by combining two slabs):
 * rc <- (P_t^T (x) I) r on slab pairs of `level` (rc has the slab count of
 * level+1), and u <- u + (P_t (x) I) ec; where the transition below `level`
 * coarsens in space too, I is replaced by P_x (x) .. (x) P_x (P_x^T in the
 * restriction; see space_ratio), and neither vector may be one of the
 * handle's own workspaces.  Vectors of a level have sth_level_len(h, level)
 * elements. */
int sth_restrict(sth_handle* h, int level, const double* r, double* rc, void* stream);
int sth_prolong_add(sth_handle* h, int level, const double* ec, double* u, void* stream);
size_t sth_level_len(const sth_handle* h, int level);

/* ||v||_2 of a level-0 vector with a reduction order fixed by the vector
 * length only; the result is written to *out (host) after a stream sync. */
int sth_norm(sth_handle* h, const double* v, double* out, void* stream);

int sth_destroy(sth_handle* h);

/* Thread-local message of the last failure in this thread. */
const char* sth_last_error(void);

/* ---- host-side introspection (no GPU needed) ------------------------- */

/* Setup quantities of one level, copied into caller-provided host arrays
 * (any pointer may be NULL).  n = interior functions per axis, N_t time
 * functions per slab.
 *   M1, K1  : n*n   1-D spatial mass / stiffness (row-major)
 *   U, mu   : n*n, n  K1 U = M1 U diag(mu), U^T M1 U = I
 *   Kt, Mt  : N_t*N_t temporal matrices of eq. TimeMatrices on this level
 *   Pt      : 2N_t*N_t prolongation level -> level+1 (if level < levels-1)
 *   V, W    : N_t*N_t real eigenvector block form, W = (M_t V)^{-1}, so
 *             that W K_t V = Z (block diagonal) and W M_t V = I
 *   eig_re, eig_im : N_t; a complex pair occupies two consecutive entries
 *             with eig_im = +beta, -beta and Z block [[a, b], [-b, a]].
 * Also returns cond(V) (2-norm) and the number of levels. */
typedef struct {
    int n, N_t, n_levels;
    double cond_V;
    double *M1, *K1, *U, *mu, *Kt, *Mt, *Pt, *V, *W, *eig_re, *eig_im;
    int schur;          /* 1: real Schur form, V = Q, W = Q^T M_t^{-1} and
                           W K_t V = R (quasi upper triangular, copied to R) */
    double* R;          /* N_t*N_t, may be NULL */
    double* mode_weights; /* 2n, may be NULL: per 1-D spatial mode j, G_jj and
                           sum_k |G_jk| of G = C^T C, C = M1 U (interleaved);
                           the eigenbasis solve bounds the B-spline residual
                           norm below by sum_m (2 prod G_jj - prod sum_k |G_jk|)
                           |r^_m|^2 over the modes m = (j_x, j_y[, j_z]) */
} sth_factors;
int sth_host_factors(const sth_problem* p, int level, sth_factors* out);

/* 1-D load vectors used by sth_load_rhs for one mode: time part per slab
 * (n_slabs*N_t, test functions psi + sigma psi') and spatial part per axis
 * (n, interior functions). */
int sth_host_load_1d(const sth_problem* p, double omega, double phase, int k,
                     double* time_part, double* space_part);

/* The prolongation of the interior spatial functions from a mesh of
 * n_elem_c elements on (0,1) to the mesh of 2 n_elem_c elements (degree p,
 * Boehm knot insertion of every element midpoint): out is row-major
 * (n_f x n_c), n_f = 2 n_elem_c + p - 2, n_c = n_elem_c + p - 2. */
int sth_host_space_prolongation(int n_elem_c, int degree, double* out);

/* ---- kernel timing (measurement support) ----------------------------- */

/* Kernel classes timed with HIP events when timing is enabled. */
typedef enum {
    STH_K_RESIDUAL = 0, STH_K_XFORM_X = 1, STH_K_XFORM_S = 2, STH_K_TIMEMIX = 3,
    STH_K_RESTRICT = 4, STH_K_PROLONG = 5, STH_K_NORM = 6, STH_K_OTHER = 7,
    STH_K_XFORM_2D = 8,     /* both axes of 2-D images in one kernel */
    STH_K_EIG_SMOOTH = 9,   /* eigenbasis iteration: residual + slab inverse + update */
    STH_K_EIG_RESID = 10,   /* eigenbasis iteration: residual (and restriction) */
    STH_K_RESNORM = 11,     /* eigenbasis iteration: residual mapped to B-splines, sum of squares */
    STH_K_EIG_CYCLE_END = 12, /* eigenbasis iteration: residual norm, next smoothing step and
                               restriction in one pass on the finest level */
    STH_K_EIG_CYCLE_CLOSE = 13, /* the same pass preceded by the prolongation and the
                                 post-smoothing step of the finest level */
    STH_K_EIG_COARSE = 14,  /* eigenbasis iteration: the two coarsest levels in one pass */
    STH_K_MINRES = 15,      /* MinRes slab inverse: the 2x2 block operator (tensor stencils) */
    STH_K_COUNT = 16
} sth_kernel_class;

/* Record an event pair around every launch of the kernel classes whose bit
 * (1 << sth_kernel_class) is set in class_mask; 0 stops recording.  A
 * nonzero mask clears the previous records. */
int sth_timing(sth_handle* h, unsigned class_mask);

/* Restrict the recording to launches on one multigrid level (0 = finest;
 * -1, the default, records every level). */
int sth_timing_level(sth_handle* h, int level);

/* Totals over the recorded launches of one class: launches, summed kernel
 * time in ms, summed algorithmic FLOPs and HBM bytes (the minimum traffic
 * of the operation: every input read once, every output written once).
 * Synchronises on the recorded events. */
int sth_timing_report(sth_handle* h, int kclass, int* launches, double* ms,
                      double* flops, double* bytes);

/* ---- serving: continuous batching of independent solves ------------- */

/* A server owns a scheduler thread and a setup thread, `max_active` HIP
 * streams (one per request in flight) and a cache of setups keyed by the
 * problem description.  Requests (a problem, a right-hand side given by
 * modes, a tolerance) are admitted in arrival order as soon as a stream is
 * free and their device footprint (sth_workspace_bytes plus the setup's own
 * f and u) fits into hbm_budget_bytes together with every cached setup;
 * idle cached setups are evicted, least recently used first, to make room.
 * Admitted requests run concurrently: each solve is driven one V-cycle at a
 * time (individual launches on its own stream, each cycle enqueued behind
 * the device flag of the cycle before it), so a request that arrives while
 * others run starts as soon as it is admitted.  The result is copied into
 * the caller's device buffer u_out (sth_problem_vector_len elements, valid
 * until the request finishes); the kernels are deterministic, so a result
 * does not depend on which other requests ran beside it.  The solve starts
 * from u = 0 and stops at ||f - L_h u|| <= rtol ||f|| or after maxit cycles
 * (Section 4.4).  All calls are thread-safe. */
typedef struct sth_server sth_server;

typedef struct {
    int status;             /* sth_status of the solve (STH_EAGAIN while pending) */
    int iters;              /* V-cycles */
    double relres;          /* final ||f - L_h u|| / ||f|| */
    double queue_ms;        /* submit -> admitted */
    double setup_ms;        /* admitted -> right-hand side loaded (includes a new setup) */
    double solve_ms;        /* right-hand side loaded -> result in u_out */
    double latency_ms;      /* submit -> result in u_out */
    size_t footprint_bytes; /* device bytes of the setup the request used */
    int setup_reused;       /* 1 if the setup came from the cache */
    char message[160];      /* failure message, empty on success */
} sth_request_stats;

/* max_active >= 1 streams; fails with STH_EINVAL on a zero budget. */
int sth_server_create(size_t hbm_budget_bytes, int max_active, sth_server** out);

/* Queues a request; the mode arrays are copied.  STH_ENOMEM if its footprint
 * alone exceeds the budget, STH_EINVAL for an invalid problem.  *ticket
 * identifies the request in the calls below. */
int sth_server_submit(sth_server* s, const sth_problem* p, const sth_rhs_modes* rhs, double rtol,
                      int maxit, double* u_out, long long* ticket);

/* STH_EAGAIN while the request is pending or running; otherwise STH_OK and
 * *stats (if not NULL) filled, after which the ticket is released. */
int sth_server_poll(sth_server* s, long long ticket, sth_request_stats* stats);

/* Blocks until the request has finished, then as sth_server_poll. */
int sth_server_wait(sth_server* s, long long ticket, sth_request_stats* stats);

/* Setups made from now on replay each solve iteration from a captured HIP
 * graph (sth_use_graphs) on their request's stream, instead of launching
 * its kernels one by one: one graph launch per cycle for the scheduler
 * thread.  A cached setup keeps the mode it was made with.  Results are
 * bitwise those of eager launches. */
int sth_server_use_graphs(sth_server* s, int enable);

/* Device bytes held by cached setups (busy or idle) and their count. */
int sth_server_resident(sth_server* s, size_t* bytes, int* setups);

/* Waits for the requests in flight, then frees every setup and stream. */
int sth_server_destroy(sth_server* s);

#ifdef __cplusplus
}
#endif
#endif /* STH_H */
