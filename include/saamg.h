/* saamg.h -- C ABI of the MI355X (gfx950) smoothed-aggregation AMG library.
 *
 * The method is smoothed aggregation AMG (SA-AMG) with the four prolongator adaptations of
 * Hu, Siefert and Tuminaro, "Smooth Aggregation for Difficult Stretched Mesh and Coefficient
 * Variation Problems" (arXiv 2103.10476): 1Norm (Sec. 2.1-2.2), OffLmp (Sec. 2.3,
 * Algorithm 2), Cnstrnt (Sec. 2.4, Algorithm 3) and Sprsfy (Sec. 2.5).  Setup builds the
 * hierarchy of Sec. 1.1 (strength criterion, aggregates, tentative prolongator, prolongator
 * smoothing, Galerkin coarse operators); solve runs CG preconditioned by the V-cycle of
 * Algorithm 1 with the degree-2 Chebyshev smoother of Sec. 4.1.
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
  SA_ERR_NEGATIVE_EIGENVALUE = -4, /* eigenvalue estimate <= 0 or not finite (Sec. 4.1)   */
  SA_ERR_COARSEN_STALLED = -5,     /* an aggregation did not reduce the size              */
  SA_ERR_COARSE_FACTOR = -6,       /* coarsest Cholesky pivot <= 0 or coarsest too large  */
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

/* Options.  struct_size must be sizeof(sa_options); sa_default_options fills the defaults
 * given in brackets (the paper's settings where it states them). */
typedef struct {
  uint32_t struct_size;
  uint32_t variants;      /* OR of SA_SPRSFY | SA_OFFLMP | SA_1NORM | SA_CNSTRNT [0]        */
  double theta;           /* strength threshold, Sec. 1.1 [0.02]                            */
  double tau;             /* OffLmp ddom growth bound, Sec. 2.3/4.1 [1.1]                   */
  double sigma;           /* 1Norm root-value safeguard, Sec. 2.2 [1/3]                     */
  int32_t one_norm_power; /* 0: lambda = 1 for 1Norm (Sec. 2.1); 1: power method [0]        */
  int32_t power_iters;    /* power-method steps for every eigenvalue estimate [10]          */
  uint64_t seed;          /* counter-based generator seed (start vectors, hashed order)     */
  int32_t agg_order;      /* SA_AGG_NATURAL | SA_AGG_HASHED [natural]                       */
  int32_t max_levels;     /* [10]                                                           */
  int32_t max_coarse;     /* coarsen until n <= max_coarse, Sec. 4.1 [1000]                 */
  int32_t smoother;       /* SA_CHEBYSHEV | SA_JACOBI [Chebyshev]                           */
  int32_t degree;         /* smoother degree / sweeps, Sec. 4.1 [2]                         */
  int32_t precision;      /* SA_FP64 | SA_FP32_VCYCLE [FP64]                                */
  double cheb_ratio;      /* Chebyshev interval [lambda/ratio, lambda], Sec. 4.1 [10]       */
  double cheb_boost;      /* multiplier on the smoother eigenvalue estimate [1]             */
  double rtol;            /* CG stops when ||r|| <= rtol ||b|| (recurrence residual) [1e-8] */
  int32_t max_iter;       /* CG iteration cap [500]                                         */
  int32_t pcg_beta;       /* SA_BETA_FR | SA_BETA_PR (flexible) [FR; PR in FP32 mode]       */
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
  double operator_complexity; /* sum_l nnz(A_l) / nnz(A_1), Sec. 4.1                       */
  int64_t device_bytes;     /* device memory held by the hierarchy                         */
  double setup_seconds;
} sa_info;

/* What sa_export_level can copy out (parity tests and diagnostics). */
typedef enum {
  SA_PART_A_RP = 0, SA_PART_A_COL = 1, SA_PART_A_VAL = 2, SA_PART_MASK = 3,
  SA_PART_AGG = 4, SA_PART_ROOT = 5, SA_PART_ABAR_RP = 6, SA_PART_ABAR_COL = 7,
  SA_PART_ABAR_VAL = 8, SA_PART_INVD = 9, SA_PART_P_RP = 10, SA_PART_P_COL = 11,
  SA_PART_P_VAL = 12, SA_PART_R_RP = 13, SA_PART_R_COL = 14, SA_PART_R_VAL = 15,
  SA_PART_SM_INVD = 16, SA_PART_COARSE_INV = 17
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
 * SA_ERR_HIP.  On failure *out is NULL and nothing is leaked. */
sa_status sa_setup(const sa_context *ctx, const sa_csr *A, const double *nullspace,
                   const sa_options *o, sa_hierarchy **out);

/* Solves A x = b with CG preconditioned by one V-cycle (Algorithm 1) per iteration, from
 * x0 = 0, until dot(r,r) <= rtol^2 dot(b,b) or max_iter.  b and x are n-vectors in `loc`
 * memory (x is written).  iterations and rel_residual = sqrt(dot(r,r)/dot(b,b)) may be
 * NULL.  Returns SA_OK, SA_NOT_CONVERGED (last iterate written) or an error. */
sa_status sa_solve(sa_hierarchy *h, const double *b, double *x, sa_location loc,
                   int32_t *iterations, double *rel_residual);

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

/* Releases the hierarchy and all its device memory (NULL is ignored). */
void sa_destroy(sa_hierarchy *h);

const char *sa_status_string(sa_status s);
const char *sa_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SAAMG_H */
