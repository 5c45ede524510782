/* CPU oracle for the SA-AMG setup and PCG solve -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded reference of what the GPU library computes, written from
 * Hu, Siefert and Tuminaro, "Smooth Aggregation for Difficult Stretched Mesh and Coefficient
 * Variation Problems" (arXiv 2103.10476).  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.  It shares no code,
 * header or constant table with the GPU library.
 *
 * Conventions: CSR with int32 row pointers/columns (columns strictly ascending per row,
 * diagonal stored), float64 values.  All pointers are host pointers owned by the caller.
 * Every function returns 0 on success or a negative status (same numbering as the GPU
 * library's status codes):  -1 invalid argument, -2 malformed CSR, -3 non-positive/zero
 * diagonal, -4 non-positive or non-finite eigenvalue estimate, -5 coarsening stalled,
 * -6 coarse factorisation failed, -9 CG breakdown; +1 = not converged (result written).
 */
#ifndef SA_ORACLE_H
#define SA_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double theta;           /* strength threshold (Sec. 1.1, strength criterion)          */
  int32_t variants;       /* bit0 Sprsfy, bit1 OffLmp, bit2 1Norm, bit3 Cnstrnt           */
  int32_t one_norm_power; /* 0: use 1 for the 1Norm eigenvalue (Sec. 2.1); 1: power method */
  double tau;             /* OffLmp ddom growth bound (Sec. 2.3), 1.1 in Sec. 3.1          */
  double sigma;           /* 1Norm safeguard root value (Sec. 2.2), 1/3                    */
  int32_t power_iters;    /* power-method steps for eigenvalue estimates, 10               */
  int32_t agg_order;      /* 0 natural vertex order, 1 hashed order                        */
  uint64_t seed;          /* seed of the counter-based generator                           */
  int32_t max_levels;     /* 10                                                            */
  int32_t max_coarse;     /* stop coarsening at <= this many unknowns (Sec. 3.1), 1000      */
  int32_t smoother;       /* 0 Chebyshev, 1 Jacobi                                         */
  int32_t degree;         /* smoother degree / sweeps, 2                                   */
  double cheb_ratio;      /* Chebyshev interval [lambda/ratio, lambda], 10                 */
  double cheb_boost;      /* multiplier on the smoother eigenvalue estimate, 1            */
  double rtol;            /* PCG relative residual reduction                               */
  int32_t max_iter;       /* PCG iteration cap                                             */
  int32_t pcg_beta;       /* 0 Fletcher-Reeves, 1 Polak-Ribiere (flexible)                 */
  int32_t dist_power;     /* distance-Laplacian weight 1/d^p: 1 (the text of Sec. 3.1) or 2 */
  int32_t coarse_solver;  /* 0 Cholesky (symmetric coarsest operator), 1 LU without pivoting */
  int32_t singletons;     /* vertices without strong connections: 0 left out of every
                             aggregate, 1 a singleton aggregate each (Sec. 1.1 covering)    */
} orc_options;

void orc_default_options(orc_options *o);
const char *orc_last_error(void);

/* ---- whole method ---- */
int orc_setup(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
              const double *nullspace /* NULL = ones */, const orc_options *o, void **h);
/* the same with the distance-Laplacian strength (Sec. 3.1): coords[n*dim] node coordinates
 * (row-major, dim 1..3); coarse levels take their aggregates' centroids; coords == NULL is
 * orc_setup */
int orc_setup_coords(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                     const double *nullspace, const double *coords, int32_t dim,
                     const orc_options *o, void **h);
/* systems SA: bs dofs per node (node-major), nullspace B (n x k, row-major, k <= 16), QR
 * tentative prolongator per aggregate; coords per node (n/bs x dim) or NULL */
int orc_setup_system(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                     int32_t bs, const double *B, int32_t k, const double *coords, int32_t dim,
                     const orc_options *o, void **h);
/* s[0..5] = block size, k, nnz(P_t), nodes, nnz(node graph), size of the level's nullspace */
int orc_level_block(const void *h, int lvl, int64_t *s);
/* numeric re-setup: new values (nnz of the setup's matrix, its CSR order), same symbolic
 * decisions (strength labels, Sprsfy drops, aggregates, patterns) */
int orc_resetup(void *h, const double *val, const double *nullspace /* NULL = ones */);
int orc_num_levels(const void *h);
/* sizes[0..7] = n, nnz(A), nc, nnz(Abar), nnz(P), nnz(R), nnz(S graph), is_coarsest */
int orc_level_sizes(const void *h, int lvl, int64_t *sizes);
/* scal[0..3] = lambda (prolongator), omega, smoother lambda, unused */
int orc_level_scalars(const void *h, int lvl, double *scal);
/* what: 0 A.rp 1 A.col 2 A.val 3 mask(u8) 4 agg(i32) 5 is_root(u8) 6 Abar.rp 7 Abar.col
 *       8 Abar.val 9 invD(f64) 10 P.rp 11 P.col 12 P.val 13 R.rp 14 R.col 15 R.val
 *       16 smoother invD(f64) 17 setup matrix (scaled) .val 18 coordinates (n*dim f64,
 *       distance strength only)  systems: 19 P_t.rp 20 P_t.col 21 P_t.val 22 nullspace
 *       (n x k) 23 node labels (u8) 24 node graph rp 25 node graph col                   */
int orc_export(const void *h, int lvl, int what, void *buf);
int orc_vcycle(const void *h, const double *f, double *u);
int orc_solve(const void *h, const double *b, double *x, int32_t *iters, double *relres,
              double *rr_history /* NULL or max_iter+1 entries */);
/* restarted flexible GMRES(restart), V-cycle as right preconditioner (Sec. 3.4's solver);
 * rr_history: NULL or max_iter+1 entries of the residual norm (index 0 = ||b||) */
int orc_solve_gmres(const void *h, const double *b, double *x, int32_t restart, int32_t *iters,
                    double *relres, double *rr_history);
void orc_destroy(void *h);

/* ---- single steps (inputs given explicitly) ---- */
int orc_strength(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                 double theta, uint8_t *mask);
int orc_distance_strength(int32_t n, const int32_t *rp, const int32_t *col,
                          const double *coords, int32_t dim, double theta, int32_t dist_power,
                          uint8_t *mask);
int orc_aggregate(int32_t n, const int32_t *rp, const int32_t *col, const uint8_t *mask,
                  int32_t order, uint64_t seed, int32_t level, int32_t singletons,
                  int32_t *agg, uint8_t *is_root, int32_t *nc);
int orc_sprsfy(int32_t n, const int32_t *rp, const int32_t *col, uint8_t *mask,
               const int32_t *agg, const uint8_t *is_root, int32_t nc);
/* filtered matrix; out_rp [n+1], out_col/out_val capacity nnz(A) */
int orc_lump(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
             const uint8_t *mask, int32_t offlmp, double tau, int32_t *out_rp,
             int32_t *out_col, double *out_val);
int orc_diag(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
             int32_t one_norm, double sigma, double *invD);
// y = A x for an nr x nc CSR matrix, in the row-sum order of the oracle's spmv.
int orc_spmv(int32_t nr, int32_t nc, const int32_t *rp, const int32_t *col, const double *val,
             const double *x, double *y);
int orc_power(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
              const double *invD, int32_t iters, uint64_t seed, int32_t level,
              int32_t stream, double *lambda);
int orc_prolongator(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                    const double *invD, const int32_t *agg, double omega, int32_t *out_rp,
                    int32_t *out_col, double *out_val);
int orc_cnstrnt(int32_t n, const int32_t *rp, const int32_t *col, double *val,
                const int32_t *agg);
/* one row of X*Y; returns the count written (cols ascending) or a negative status */
int orc_spgemm_row(const int32_t *xrp, const int32_t *xcol, const double *xval,
                   const int32_t *yrp, const int32_t *ycol, const double *yval,
                   int32_t ncols_y, int32_t row, int32_t *out_col, double *out_val);
double orc_dot(int64_t n, const double *x, const double *y);
uint64_t orc_splitmix64(uint64_t seed, uint64_t k);

#ifdef __cplusplus
}
#endif
#endif
