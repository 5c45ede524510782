/* saamg.h -- C ABI of the MI355X (gfx950) smoothed-aggregation AMG library.
 *
 * The method is smoothed aggregation AMG (SA-AMG) with the four prolongator adaptations of
 * Hu, Siefert and Tuminaro, "Smooth Aggregation for Difficult Stretched Mesh and Coefficient
 * Variation Problems" (arXiv 2103.10476): 1Norm (Sec. 2.1-2.2), OffLmp (Sec. 2.3,
 * Algorithm 2), Cnstrnt (Sec. 2.4, Algorithm 3) and Sprsfy (Sec. 2.5).  Setup builds the
 * hierarchy of Sec. 1.1 (strength criterion, aggregates, tentative prolongator, prolongator
 * smoothing, Galerkin coarse operators); solve runs CG preconditioned by the V-cycle of
 * Algorithm 1 with the degree-2 Chebyshev smoother of Sec. 3.1.
 *
 * Conventions
 *  - Matrices are CSR: int32 row pointers (n+1) and column indices (nnz < 2^31), columns
 *    strictly ascending within each row, diagonal stored, float64 values.
 *  - Device pointers are HIP device addresses on the current device; host pointers are
 *    ordinary host memory.  Every pointer argument is borrowed for the duration of the call
 *    only; the library copies what it keeps.
 *  - All work is queued on the stream given at setup (NULL = the null stream); every call
 *    returns after its results are complete.  A hierarchy may be used by one thread at a
 *    time; distinct hierarchies are independent.
 *  - No C++ exception crosses this boundary.  A negative status is a failure: outputs are
 *    left untouched (sa_solve leaves x unspecified on SA_ERR_BREAKDOWN).  sa_last_error()
 *    returns a thread-local description of the last failure.
 *  - Setup is deterministic: with fixed options the hierarchy is bit-identical run to run.
 */
#ifndef SAAMG_H
#define SAAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SA_OK = 0,
  SA_NOT_CONVERGED = 1,      /* iteration cap reached; last iterate written              */
  SA_PENDING = 2,            /* serving: request not finished yet                         */
  SA_ERR_INVALID_ARG = -1,   /* bad argument, bad options, non-finite input               */
  SA_ERR_BAD_CSR = -2,       /* unsorted/duplicate/out-of-range column, missing diagonal  */
  SA_ERR_NONPOSITIVE_DIAG = -3, /* zero filtered diagonal (plain SA) or A_ii <= 0         */
  SA_ERR_NEGATIVE_EIGENVALUE = -4, /* eigenvalue estimate <= 0 or not finite (Sec. 3.1)   */
  SA_ERR_COARSEN_STALLED = -5,     /* an aggregation did not reduce the size              */
  SA_ERR_COARSE_FACTOR = -6,       /* coarsest pivot <= 0 (Cholesky) or 0 (LU), coarsest
                                      too large, or nonsymmetric under Cholesky            */
  SA_ERR_OOM = -7,                 /* device allocation failed / over the memory budget   */
  SA_ERR_HIP = -8,                 /* a HIP runtime call failed                           */
  SA_ERR_BREAKDOWN = -9            /* CG breakdown: p'Ap <= 0 or r'z <= 0                 */
} sa_status;

typedef enum { SA_HOST = 0, SA_DEVICE = 1 } sa_location;

/* Variant bits (the paper's four adaptations). */
#define SA_SPRSFY 1u  /* Sec. 2.5: aggregate-aware second dropping stage            */
#define SA_OFFLMP 2u  /* Sec. 2.3: sign-aware lumping of dropped entries (Alg. 2)   */
#define SA_1NORM 4u   /* Sec. 2.1-2.2: 1-norm diagonal with the sigma safeguard     */
#define SA_CNSTRNT 8u /* Sec. 2.4: bound-constrained prolongator rows (Alg. 3)      */

enum { SA_AGG_NATURAL = 0, SA_AGG_HASHED = 1 };
enum { SA_CHEBYSHEV = 0, SA_JACOBI = 1 };
enum { SA_FP64 = 0, SA_FP32_VCYCLE = 1 };
enum { SA_BETA_FR = 0, SA_BETA_PR = 1 };
enum { SA_COARSE_CHOLESKY = 0, SA_COARSE_LU = 1 };
enum { SA_ISOLATED_LEFT_OUT = 0, SA_ISOLATED_SINGLETON = 1 };

/* Options.  struct_size must be sizeof(sa_options); sa_default_options fills the defaults
 * given in brackets (the paper's settings where it states them). */
typedef struct {
  uint32_t struct_size;
  uint32_t variants;      /* OR of SA_SPRSFY | SA_OFFLMP | SA_1NORM | SA_CNSTRNT [0]        */
  double theta;           /* strength threshold, Sec. 1.1 [0.02]                            */
  double tau;             /* OffLmp ddom growth bound, Sec. 2.3 (value: Sec. 3.1) [1.1]    */
  double sigma;           /* 1Norm root-value safeguard, Sec. 2.2 [1/3]                     */
  int32_t one_norm_power; /* 0: lambda = 1 for 1Norm (Sec. 2.1); 1: power method [0]        */
  int32_t power_iters;    /* power-method steps for every eigenvalue estimate [10]          */
  uint64_t seed;          /* counter-based generator seed (start vectors, hashed order)     */
  int32_t agg_order;      /* SA_AGG_NATURAL | SA_AGG_HASHED [natural]                       */
  int32_t max_levels;     /* [10]                                                           */
  int32_t max_coarse;     /* coarsen until n <= max_coarse, Sec. 3.1 [1000]                 */
  int32_t smoother;       /* SA_CHEBYSHEV | SA_JACOBI [Chebyshev]                           */
  int32_t degree;         /* smoother degree / sweeps, Sec. 3.1 [2]                         */
  int32_t precision;      /* SA_FP64 | SA_FP32_VCYCLE [FP64]                                */
  double cheb_ratio;      /* Chebyshev interval [lambda/ratio, lambda], Sec. 3.1 [10]       */
  double cheb_boost;      /* multiplier on the smoother eigenvalue estimate [1]             */
  double rtol;            /* CG stops when ||r|| <= rtol ||b|| (recurrence residual) [1e-8] */
  int32_t max_iter;       /* CG iteration cap [500]                                         */
  int32_t pcg_beta;       /* SA_BETA_FR | SA_BETA_PR (flexible) [FR; PR in FP32 mode]       */
  int32_t dist_power;     /* sa_setup_coords weight 1/distance^p, p = 1 or 2, Sec. 3.1 [1]  */
  int32_t coarse_solver;  /* SA_COARSE_CHOLESKY (symmetric coarsest operator; a nonsymmetric
                             one is SA_ERR_COARSE_FACTOR) | SA_COARSE_LU (no pivoting; for
                             nonsymmetric matrices solved with GMRES, Sec. 3.4) [Cholesky]     */
  int32_t isolated;       /* a vertex without strong connections: SA_ISOLATED_LEFT_OUT (in no
                             aggregate, a zero row of the tentative prolongator; smoothed
                             only) | SA_ISOLATED_SINGLETON (an aggregate of its own, so the
                             aggregates cover every vertex as in Sec. 1.1) [left out].  Systems
                             SA always leaves such nodes out                                   */
} sa_options;

typedef struct {
  int32_t n;               /* rows = columns                                              */
  int64_t nnz;             /* stored entries (< 2^31)                                     */
  const int32_t *row_ptr;  /* n+1                                                          */
  const int32_t *col;      /* nnz                                                          */
  const double *val;       /* nnz                                                          */
  sa_location loc;         /* where the three arrays live                                  */
} sa_csr;

typedef struct {
  void *stream;            /* hipStream_t for all work; NULL = the null stream             */
} sa_context;

typedef struct sa_hierarchy sa_hierarchy;

typedef struct {
  int32_t levels;
  int32_t n[16];            /* rows per level                                              */
  int64_t nnz[16];          /* stored entries of A_l per level                             */
  int64_t nnz_p[16];        /* stored entries of P_l (0 on the coarsest)                   */
  double lambda[16];        /* prolongator-smoothing eigenvalue estimate per level         */
  double omega[16];         /* damping 4/(3 lambda), Sec. 1.1                              */
  double smoother_lambda[16];
  int32_t mis_rounds[16];   /* rounds of the parallel root selection per level             */
  double operator_complexity; /* sum_l nnz(A_l) / nnz(A_1), Sec. 3.1                       */
  int64_t device_bytes;     /* device memory held by the hierarchy                         */
  double setup_seconds;
} sa_info;

/* What sa_export_level can copy out (parity tests and diagnostics). */
typedef enum {
  SA_PART_A_RP = 0, SA_PART_A_COL = 1, SA_PART_A_VAL = 2, SA_PART_MASK = 3,
  SA_PART_AGG = 4, SA_PART_ROOT = 5, SA_PART_ABAR_RP = 6, SA_PART_ABAR_COL = 7,
  SA_PART_ABAR_VAL = 8, SA_PART_INVD = 9, SA_PART_P_RP = 10, SA_PART_P_COL = 11,
  SA_PART_P_VAL = 12, SA_PART_R_RP = 13, SA_PART_R_COL = 14, SA_PART_R_VAL = 15,
  SA_PART_SM_INVD = 16, SA_PART_COARSE_INV = 17,
  SA_PART_COORDS = 18,      /* node coordinates, points x dim (distance strength only)     */
  /* systems hierarchies (sa_setup_system) only: */
  SA_PART_PT_RP = 19, SA_PART_PT_COL = 20, SA_PART_PT_VAL = 21, /* QR tentative prolongator */
  SA_PART_NULLSPACE = 22,   /* the level's nullspace, n x k row-major                        */
  SA_PART_NODE_MASK = 23, SA_PART_NODE_RP = 24, SA_PART_NODE_COL = 25  /* node graph, labels */
} sa_part;

/* Fills *o with the defaults listed above (struct_size included). */
void sa_default_options(sa_options *o);

/* Builds the hierarchy of Sec. 1.1 with the selected adaptations of Sec. 2.
 *  A          the fine matrix, host or device (A->loc); validated (SA_ERR_BAD_CSR).
 *  nullspace  NULL for the constant vector (the paper's case); otherwise n nonzero finite
 *             values in A->loc memory, handled by the exact scaling D_B A D_B.
 *  o          options (NULL = defaults).
 *  out        receives the new hierarchy; owned by the caller until sa_destroy.
 * Errors: SA_ERR_INVALID_ARG, SA_ERR_BAD_CSR, SA_ERR_NONPOSITIVE_DIAG,
 * SA_ERR_NEGATIVE_EIGENVALUE, SA_ERR_COARSEN_STALLED, SA_ERR_COARSE_FACTOR, SA_ERR_OOM,
 * SA_ERR_HIP.  On failure *out is NULL and nothing is leaked.
 * The root selection's rounds are launched back to back while the calling thread polls a
 * pinned status word written by the kernels (it spins on one host core meanwhile); if a word
 * does not arrive within SAAMG_STATUS_SPIN_NS nanoseconds (environment, default 20000000),
 * the thread synchronises the stream and reads the device flags instead.  The small readbacks
 * of sizes and scalars (here and in the solves) are polled the same way, from a tag word the
 * copy writes after its data, with the same limit before the stream is synchronised.  Levels
 * of at most SAAMG_MIS_WG_MAX_N vertices (default 4096) run their rounds after the first
 * inside one workgroup, and levels from SAAMG_MIS_V_MIN_N vertices on (default 524288) give
 * each thread of a round's passes four vertices.  The result is the same in every case. */
sa_status sa_setup(const sa_context *ctx, const sa_csr *A, const double *nullspace,
                   const sa_options *o, sa_hierarchy **out);

/* sa_setup with the strength test of Sec. 3.1 taken on a distance Laplacian instead of on
 * the level operator.  L^(d) has the operator's pattern; an off-diagonal entry is -1/d_ij^p
 * with d_ij the Euclidean distance between the two nodes (o->dist_power p = 1, the paper's
 * definition, the default; p = 2 takes the reciprocal of the squared distance and needs no
 * square root) and the diagonal makes every row sum zero; entry (i,j) is strong iff
 * |L_ij| >= theta sqrt(L_ii L_jj).  Coarse levels take as coordinates the
 * centroids of their aggregates (members summed in ascending order, divided by the count).
 * Everything else is sa_setup's.
 *  coords  n x dim float64 node coordinates, row-major (node i at coords[i*dim .. i*dim+dim-1]),
 *          in A->loc memory, finite; NULL makes this sa_setup.
 *  dim     1, 2 or 3.
 * Errors: those of sa_setup; SA_ERR_INVALID_ARG also for a bad dim, a non-finite coordinate
 * or two nodes connected by a stored entry of some level's operator at zero distance. */
sa_status sa_setup_coords(const sa_context *ctx, const sa_csr *A, const double *nullspace,
                          const double *coords, int32_t dim, const sa_options *o,
                          sa_hierarchy **out);

/* Smoothed aggregation for systems with a multi-vector nullspace (the paper's algorithms are
 * scalar; it names systems as future work).  The unknowns are numbered node-major, block_size
 * per node (1..16, dividing A->n); nullspace is A->n x k row-major (1 <= k <= 16), in A->loc
 * memory, e.g. the six rigid-body modes of 3-D elasticity.
 *  - Strength is taken between nodes: with F_IJ the sum of squares of the block A_IJ, (I,J)
 *    is strong iff F_IJ^2 >= theta^4 F_II F_JJ (the scalar test for block_size 1); with
 *    coords (one point per node, A->n / block_size x dim) the distance Laplacian of the node
 *    graph decides instead.  Couplings between two nodes take their pair's label; couplings
 *    inside a node are kept.  Lumping (plain or OffLmp), the smoothing diagonal (plain or
 *    1Norm) and lambda are the scalar definitions applied to rows.
 *  - Aggregates are sets of nodes.  Aggregate J's rows of the nullspace (members ascending,
 *    components ascending) are factored B_J = Q_J R_J by Householder reflections with R's
 *    diagonal non-negative; the tentative prolongator holds Q_J in columns kJ..kJ+k-1 and
 *    the next level's nullspace holds R_J (so the coarse level has k unknowns per node).
 *  - P = P_t - omega D^-1 Abar P_t; R = P^T; Galerkin products as for sa_setup.
 *  - Sprsfy and Cnstrnt (defined for a scalar constant nullspace) are refused.
 * Errors: those of sa_setup; SA_ERR_INVALID_ARG also for a bad block size or k, a
 * non-finite nullspace entry, or an aggregate with fewer unknowns than k. */
sa_status sa_setup_system(const sa_context *ctx, const sa_csr *A, int32_t block_size,
                          const double *nullspace, int32_t k, const double *coords, int32_t dim,
                          const sa_options *o, sa_hierarchy **out);

/* Numeric re-setup: new values for the matrix given to sa_setup, on the same pattern (val
 * holds nnz values in that matrix's CSR order; nullspace as in sa_setup, NULL = ones; both in
 * `loc` memory).  Every symbolic decision of the setup is kept: strength labels and Sprsfy
 * drops, aggregates, and the sparsity patterns of the filtered matrices, P, R and every level
 * operator.  The numbers are recomputed in the setup's own order: filtered values (plain or
 * OffLmp lumping), smoothing diagonal, eigenvalue estimate and damping, P (and Cnstrnt), R,
 * the Galerkin products, the smoothers and the coarsest inverse.  The result is bit-identical
 * to what sa_setup gives on the new values whenever that setup would take the same symbolic
 * decisions.  For a sequence of systems with one pattern (time steps, repeated requests) this
 * skips the strength test and root selection.  The first re-setup also builds, per level, the
 * lists of products that form every entry of A P and R (A P) (in Gustavson order) and keeps
 * A P; later re-setups then take R, A P and the coarse operators through those lists, without
 * the products' symbolic passes (bitwise the same values).  This costs device memory of about
 * 8 bytes per Galerkin product plus A P (held until sa_destroy); the environment variable
 * SAAMG_RESETUP_PLAN=0 keeps the full products instead.  Errors as for sa_setup (values
 * only); after a failure the hierarchy can only be destroyed or re-set up again (solves return
 * SA_ERR_INVALID_ARG).  A systems hierarchy keeps its nullspace (nullspace must be NULL). */
sa_status sa_resetup(sa_hierarchy *h, const double *val, const double *nullspace,
                     sa_location loc);

/* Solves A x = b with CG preconditioned by one V-cycle (Algorithm 1) per iteration, from
 * x0 = 0, until dot(r,r) <= rtol^2 dot(b,b) or max_iter.  b and x are n-vectors in `loc`
 * memory (x is written).  iterations and rel_residual = sqrt(dot(r,r)/dot(b,b)) may be
 * NULL.  Returns SA_OK, SA_NOT_CONVERGED (last iterate written) or an error. */
sa_status sa_solve(sa_hierarchy *h, const double *b, double *x, sa_location loc,
                   int32_t *iterations, double *rel_residual);

/* Solves A x = b with restarted flexible GMRES(restart) preconditioned on the right by one
 * V-cycle per iteration: the paper's solver for its nonsymmetric wind-turbine systems
 * (Sec. 3.4).  For a nonsymmetric A, set up with coarse_solver = SA_COARSE_LU.
 *  - x0 = 0; Arnoldi by classical Gram-Schmidt applied twice; Givens rotations; the flexible
 *    form keeps the preconditioned vectors, so an FP32 V-cycle is a valid preconditioner.
 *  - Stops when the least-squares residual norm is <= rtol ||b||; at each restart the true
 *    residual b - A x is formed and tested; max_iter bounds the Arnoldi steps.
 *  - restart: 1..1024.  Device scratch of (2 restart + 1) n doubles is taken from the
 *    library's cache for the call.
 *  - iterations (Arnoldi steps) and rel_residual (the last residual norm over ||b||) may be
 *    NULL.
 * Returns SA_OK, SA_NOT_CONVERGED (last iterate written), SA_ERR_BREAKDOWN (non-finite
 * residual or a singular least-squares system; x unspecified) or another error. */
sa_status sa_solve_gmres(sa_hierarchy *h, const double *b, double *x, sa_location loc,
                         int32_t restart, int32_t *iterations, double *rel_residual);

/* sa_solve_gmres for callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same iteration and results, but
 * the workspace lives in a fixed 128 MiB array compiled into the library (held by each GPU
 * the library runs on until the process ends) instead of memory taken for the call.  No
 * device memory is allocated and the fine-level SpMV timing of sa_profile_enable is off for
 * the call.  The hierarchy's device must be current.
 *  - The workspace takes 8 ((2 restart + 1) n + about (restart + 1) n / 4096 + restart^2)
 *    bytes plus alignment; a call needing more than 128 MiB (e.g. restart 30 with n above
 *    about 270,000) returns SA_ERR_INVALID_ARG without running (sa_last_error names the
 *    size).
 *  - Every call on one GPU uses that GPU's one array: calls that overlap on a GPU (other
 *    threads, other streams) race and must be serialised by the caller.  Each call writes the
 *    workspace it uses before reading it.
 * Returns as sa_solve_gmres. */
sa_status sa_solve_gmres_noalloc(sa_hierarchy *h, const double *b, double *x, sa_location loc,
                                 int32_t restart, int32_t *iterations, double *rel_residual);

/* Solves count systems A_k x_k = b_k, each on its own hierarchy hs[k], in lockstep: each CG
 * iteration of every still-running system is advanced by grouped launches (one launch per
 * step for all systems: V-cycle levels, inner products, updates) on hs[0]'s stream.  Each
 * system's arithmetic is exactly that of sa_solve on it alone, so x[k], iterations[k] and
 * rel_residual[k] equal what sa_solve returns for it.  b[k], x[k]: n_k-vectors in `loc`
 * memory.  status[k] receives each system's status (SA_OK, SA_NOT_CONVERGED or an error,
 * with x[k] unspecified on SA_ERR_BREAKDOWN); iterations and rel_residual may be NULL.
 * The hierarchies must be distinct and not in use by another call.  Returns SA_OK when
 * every system was run (whatever their statuses), otherwise SA_ERR_INVALID_ARG, SA_ERR_OOM or
 * SA_ERR_HIP. */
sa_status sa_solve_many(sa_hierarchy *const *hs, int32_t count, const double *const *b,
                        double *const *x, sa_location loc, int32_t *iterations,
                        double *rel_residual, sa_status *status);

/* Applies one V-cycle z = M^{-1} f (f, z device vectors of the fine size). */
sa_status sa_vcycle(sa_hierarchy *h, const double *f, double *z);

/* Level sizes, eigenvalue estimates, complexity and memory of a hierarchy. */
sa_status sa_hierarchy_info(const sa_hierarchy *h, sa_info *info);

/* Number of elements of `what` on `level` (0 if the level does not hold it). */
sa_status sa_export_size(const sa_hierarchy *h, int32_t level, sa_part what, int64_t *count);

/* Copies `what` of `level` into host_buf (bytes must be at least count * element size:
 * 4 for row pointers, columns and aggregates, 1 for MASK/ROOT, 8 for values). */
sa_status sa_export_level(const sa_hierarchy *h, int32_t level, sa_part what, void *host_buf,
                          size_t bytes);

/* Kernel timing for roofline reports: while enabled, every launch of the SpMV kernel on the
 * fine-level operator during sa_solve is bracketed with HIP events on the hierarchy's
 * stream.  sa_profile_read returns the number of such launches, their summed device time
 * (ms) and their summed algorithmic HBM bytes (entries x 12 B + row pointers + every vector
 * the fused epilogue reads or writes, each once), accumulated since enabling. */
sa_status sa_profile_enable(sa_hierarchy *h, int32_t on);
sa_status sa_profile_read(const sa_hierarchy *h, int64_t *launches, double *ms, double *bytes);

/* Releases the hierarchy and all its device memory (NULL is ignored).  Device blocks go back
 * to the library's per-stream cache for reuse by later work on the same stream. */
void sa_destroy(sa_hierarchy *h);

/* ---- serving: many independent setup + solve requests on one GPU ------------------------
 * A server owns max_slots setup workers, each a host thread with its own HIP stream (default
 * priority), and one solve batcher with its own stream.  Requests are admitted in submission
 * order (FIFO) while the sum of the admitted requests' device-byte estimates
 * (sa_estimate_bytes) stays within hbm_budget.  An admitted request runs sa_setup on a free
 * slot's stream (up to max_slots setups overlap on the GPU), then joins the solve group: each
 * tick of the batcher advances every request in the group by one CG iteration with grouped
 * launches, as sa_solve_many does, and a request leaves the group, with its result copied to
 * host memory and all its device memory released, as soon as it converges, fails or reaches
 * its iteration cap.  A slot takes its next request as soon as its setup is done (continuous
 * batching: requests arriving while others are on the GPU are admitted as slots and memory
 * free up, and their work overlaps on the device).  Requests share nothing but the GPU and
 * the grouped kernels run each request's standalone arithmetic, so a request's x, iteration
 * count and residual are bitwise the same alone (sa_setup + sa_solve) or in any mix.  The
 * server serves the use of many SA-AMG solves (Sec. 3) on one device; it adds no numerical
 * method of its own. */
typedef struct sa_server sa_server;

typedef struct {
  int32_t status;          /* the request's own status: SA_OK, SA_NOT_CONVERGED or an error */
  int32_t n;               /* rows                                                           */
  int32_t iterations;      /* CG iterations                                                  */
  int32_t levels;          /* hierarchy levels                                               */
  double rel_residual;     /* sqrt(r.r / b.b) at exit                                        */
  double queue_seconds;    /* submission -> admission                                        */
  double setup_seconds;    /* sa_setup                                                       */
  double solve_seconds;    /* sa_solve                                                       */
  double latency_seconds;  /* submission -> result ready                                     */
  int64_t reserved_bytes;  /* estimate charged against the budget at admission               */
  int64_t peak_bytes;      /* device bytes the request actually held at its peak             */
} sa_result;

typedef struct {
  int64_t submitted, completed, failed, queued, running;
  int64_t budget_bytes;
  int64_t reserved_bytes;       /* estimates of the running requests                         */
  int64_t peak_reserved_bytes;  /* maximum of reserved_bytes so far                          */
  int64_t peak_measured_bytes;  /* maximum over time of the summed measured live bytes       */
  int64_t solve_ticks;          /* grouped CG iterations run                                 */
  double mean_group;            /* requests advanced per tick, on average                    */
  int64_t max_group;            /* most requests advanced by one tick                        */
} sa_server_stats;

/* Device bytes a request on an n x n matrix with nnz entries is charged at admission: an
 * upper bound on its peak device memory (hierarchy + setup temporaries + solve workspace)
 * for operator complexities up to about 3. */
int64_t sa_estimate_bytes(int32_t n, int64_t nnz);

/* Creates a server.  ctx may be NULL (current device).  hbm_budget: bytes (> 0);
 * max_slots: concurrent requests, 1..32.  Errors: SA_ERR_INVALID_ARG, SA_ERR_HIP. */
sa_status sa_server_create(const sa_context *ctx, size_t hbm_budget, int32_t max_slots,
                           sa_server **out);

/* Queues a request: A (validated by sa_setup when the request runs), b (n values) and the
 * options (NULL = defaults) are copied to host memory before the call returns (A->loc gives
 * where A and b live).  *ticket receives the request's id.  Errors: SA_ERR_INVALID_ARG
 * (bad arguments, or the server shutting down), SA_ERR_OOM (a request whose estimate alone
 * exceeds the budget: it could never be admitted), SA_ERR_HIP. */
sa_status sa_server_submit(sa_server *s, const sa_csr *A, const double *b, const sa_options *o,
                           uint64_t *ticket);

/* As sa_server_submit, but nothing is copied at submission: the request keeps A's arrays and
 * b (host or device memory, A->loc) and reads them when its setup starts and during its solve.
 * The caller must keep them valid and unchanged until sa_server_poll or sa_server_wait has
 * returned the request's result, or sa_server_destroy has returned.  For clients whose inputs
 * already sit in memory they own: submission then costs no copy of the matrix (a host copy of
 * a large request runs at memcpy speed, about 0.1 s per GB).  Errors as sa_server_submit. */
sa_status sa_server_submit_borrowed(sa_server *s, const sa_csr *A, const double *b,
                                    const sa_options *o, uint64_t *ticket);

/* Non-blocking: SA_PENDING while the request is queued or running.  Once it has finished,
 * writes x (n values in `loc` memory; may be NULL) and *r (may be NULL), forgets the ticket
 * and returns the request's status (SA_OK, SA_NOT_CONVERGED or its error; sa_last_error then
 * gives the request's message).  Unknown ticket: SA_ERR_INVALID_ARG. */
sa_status sa_server_poll(sa_server *s, uint64_t ticket, double *x, sa_location loc,
                         sa_result *r);

/* As sa_server_poll, but blocks until the request has finished. */
sa_status sa_server_wait(sa_server *s, uint64_t ticket, double *x, sa_location loc,
                         sa_result *r);

/* Blocks until no request is queued or running (results stay available to poll). */
sa_status sa_server_drain(sa_server *s);

sa_status sa_server_get_stats(const sa_server *s, sa_server_stats *st);

/* Finishes the running requests, drops the queued ones, joins the workers and releases the
 * server (NULL is ignored). */
void sa_server_destroy(sa_server *s);

const char *sa_status_string(sa_status s);
const char *sa_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SAAMG_H */
