// Host-side launchers of the library's kernels (internal).
#pragma once
#include "common.hpp"

namespace sa {

// ---------------- solve-phase kernels (solve_kernels.hip) ------------------------------
// y = A x with every row of at most 64 entries summed sequentially in ascending column order
// from 0 (products staged through LDS).  A longer row is summed the same way when `plain` is
// set -- the setup's eigenvalue estimates, whose results decide the hierarchy bit for bit --
// and otherwise, in the solve, as 64 interleaved in-order partial sums added in order, which
// cuts the row's dependent chain of adds from L to about L/64 + 64 (a rounding-level
// difference from the sequential sum).  Variants fuse the row-local epilogue used by the
// smoother, residual and transfer steps.
template <class T>
struct SpmvArgs {
  int32_t n;
  const int32_t *rp;
  const int32_t *col;
  const T *val;
  const T *x;
  const int32_t *bstart;  // row partition from spmv_plan: (first row, first entry) pairs
  int32_t nblk;
  // sliced-ELL copy (see Sell); when sval is set the SpMV runs on it instead of the CSR
  const int32_t *sptr = nullptr;
  const int32_t *scol = nullptr;
  const T *sval = nullptr;
  int32_t nslice = 0;
  bool plain = false;  // long rows in sequential order too (see above)
};
// Row partition for the SpMV kernels: block b owns the rows whose cost rp[r] + 8 r lies in
// [2048 b, 2048 (b+1)), i.e. at most 256 rows and (long rows aside) at most 2048 entries;
// stored as nblk+1 (first row, first entry) pairs, 8-byte aligned.
void spmv_plan(Csr &A, Arena &ar, hipStream_t s);
template <class T>
inline SpmvArgs<T> spmv_args(const Csr &A, const T *val, const T *x) {
  return SpmvArgs<T>{A.n, A.rp, A.col, val, x, A.bstart, A.nblk};
}
// Switches an SpMV to the sliced-ELL copy S with values val (no change when S is not built).
template <class T>
inline SpmvArgs<T> with_sell(SpmvArgs<T> a, const Sell &S, const T *val) {
  if (S.ptr && val) {
    a.sptr = S.ptr;
    a.scol = S.col;
    a.sval = val;
    a.nslice = S.nslice;
  }
  return a;
}
// Builds the sliced-ELL copy of A (FP32 values too when f32) if it pays: rows averaging at
// most 12 entries (longer rows keep the CSR kernel, whose products are formed by the whole
// block), none longer than 64 (the longer ones are summed in the split order by a
// wavefront) and padding at most a quarter of the entries.  Returns whether it did.
bool sell_build(const Csr &A, Sell &S, bool f32, Arena &ar, hipStream_t s);
// Copies A's current values into a built copy (after a numeric re-setup).
void sell_values(const Csr &A, const Sell &S, hipStream_t s);
// Sorts the entries of every row by column (values follow when val != nullptr); keys within a
// row must be distinct.  Short rows per thread, long rows per block (bitonic in LDS).
void sort_rows(int32_t n, const int32_t *rp, int32_t *col, double *val, hipStream_t s);

template <class T> void spmv_store(const SpmvArgs<T> &a, T *y, hipStream_t s);
template <class T> void spmv_scale(const SpmvArgs<T> &a, const T *d, T *y, hipStream_t s);
// y = d (A x), plus max |y_i| (bit patterns of non-negative doubles) maximised atomically
// into slots[0..kMaxSlots), one atomic per row block of the CSR kernels (the sliced-ELL copy,
// if set, is not used)
constexpr int kMaxSlots = 256;
template <class T>
void spmv_scale_max(const SpmvArgs<T> &a, const T *d, T *y, unsigned long long *slots,
                    hipStream_t s);
template <class T> void spmv_resid(const SpmvArgs<T> &a, const T *f, T *r, hipStream_t s);
template <class T> void spmv_add(const SpmvArgs<T> &a, T *u, hipStream_t s);
// r = f - A u; d = (invD .* r) / theta
template <class T>
void spmv_cheb_start(const SpmvArgs<T> &a, const T *f, const T *invD, T theta, T *r, T *d,
                     hipStream_t s);
// x = d: rout = rin - A d; dn = c1 d + c2 (invD .* rout); u = (uzero ? 0 : u) + d, and when
// `last` also u += dn.  dout must differ from d (= a.x).
template <class T>
void spmv_cheb_step(const SpmvArgs<T> &a, const T *rin, T *rout, const T *invD, T c1, T c2,
                    T *u, bool uzero, T *dout, bool last, hipStream_t s);
// x = u: u2 = u + w (invD .* (f - A u))
template <class T>
void spmv_jacobi(const SpmvArgs<T> &a, const T *f, const T *invD, T w, T *u2, hipStream_t s);

// d = (invD .* f) / theta; if write_u: u = 0 + d
template <class T>
void cheb_first(int32_t n, const T *f, const T *invD, T theta, T *d, T *u, bool write_u,
                hipStream_t s);
// u = u + d
template <class T> void vec_add(int32_t n, T *u, const T *d, hipStream_t s);
// u = 0 + w (invD .* f)
template <class T>
void jacobi_first(int32_t n, const T *f, const T *invD, T w, T *u, hipStream_t s);

void cast_f64_to_f32(const double *a, float *b, int64_t n, hipStream_t s);
void cast_f32_to_f64(const float *a, double *b, int64_t n, hipStream_t s);

// Dense y = M x for the coarsest level (M row-major n x n, float64).
void gemv_f64(int32_t n, const double *M, const double *x, double *y, hipStream_t s);

// ---- GMRES (solve_kernels.hip) ----------------------------------------------------------
// Device state of one GMRES cycle with restart length m: the Hessenberg matrix (row-major,
// (m+1) x m), the rotations, the right-hand side g of the least-squares problem, its
// solution y, Gram-Schmidt coefficients c and the scalars the host reads after each step.
struct GmresScalars {
  double res;  // |g[j+1]| after the step's rotation
  double hn;   // norm of the new Arnoldi vector
  double hn2;  // its square (canonical dot)
  double nrm2; // dot(r, r) of a residual
  double beta; // its norm
  int32_t err, pad;
};
// c[i] = dot(V_i, w) for i < nv, V_i = V + i * ldv (the canonical dot, each independently);
// ws holds nv * dot_ws_size(n) doubles.
void multi_dot_f64(const double *V, int64_t ldv, int32_t nv, const double *w, int64_t n,
                   double *c, double *ws, hipStream_t s);
// w[k] = w[k] - c[0] V_0[k] - c[1] V_1[k] - ... (nv terms in ascending order); with add,
// w[k] = w[k] + c[0] V_0[k] + ... instead.
void multi_axpy_f64(const double *V, int64_t ldv, int32_t nv, const double *c, double *w,
                    int64_t n, bool add, hipStream_t s);
// H[i][j] = c[i] (pass 0) or H[i][j] + c[i] (pass 1), i <= j.
void gmres_accum(double *H, int32_t m, int32_t j, const double *c, int32_t pass, hipStream_t s);
// hn = sqrt(hn2), H[j+1][j] = hn; v = w / hn when hn > 0 (elementwise, in place allowed).
void gmres_normalize(GmresScalars *S, double *H, int32_t m, int32_t j, const double *w,
                     double *v, int64_t n, hipStream_t s);
// Rotations of column j and the new one; g updated, S->res = |g[j+1]|.
void gmres_givens(double *H, int32_t m, int32_t j, double *cs, double *sn, double *g,
                  GmresScalars *S, hipStream_t s);
// y = H[0:k,0:k]^{-1} g (back substitution); err 1 on a zero diagonal entry.
void gmres_backsolve(const double *H, int32_t m, int32_t k, const double *g, double *y,
                     GmresScalars *S, hipStream_t s);
// beta = sqrt(nrm2); v = r / beta; g[0] = beta.
void gmres_start(GmresScalars *S, const double *r, double *v, int64_t n, double *g,
                 hipStream_t s);

// PCG device scalars.
struct PcgScalars {
  double rho, pq, alpha, rr, rho1, beta, rw, spare;
  int32_t err, pad;
};
// x = x + alpha p; r = r - alpha q  (alpha = S->alpha)
void pcg_update_xr(int32_t n, double *x, double *r, const double *p, const double *q,
                   const PcgScalars *S, hipStream_t s);
// p = z + beta p
void pcg_update_p(int32_t n, double *p, const double *z, const PcgScalars *S, hipStream_t s);
// w = z - zold
void vec_sub(int32_t n, const double *z, const double *zold, double *w, hipStream_t s);
// alpha = rho / pq (err on pq <= 0)
void pcg_alpha(PcgScalars *S, hipStream_t s);
// beta (FR: rho1/rho; PR: rw/rho), err on rho1 <= 0, then rho = rho1
void pcg_beta(PcgScalars *S, bool pr, hipStream_t s);
// rho = rho1 (initial), err on <= 0
void pcg_init_rho(PcgScalars *S, hipStream_t s);

// ---------------- setup kernels (setup_kernels.hip) ------------------------------------
// Validates a CSR (ascending in-range columns, diagonal present, finite values); flags
// bits in *err: 1 bad structure, 2 missing diagonal, 4 non-finite value, 2048 row pointers
// not spanning [0, nnz] (nnz: the length of col and val).
void validate_csr(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col,
                  const double *val, int32_t *err, hipStream_t s);
// dval[i] = A_ii.
void find_diag(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
               double *dval, hipStream_t s);
// mask per entry (0 weak, 1 strong, 3 diagonal) and scount[i] = strong entries in row i.
// `wave`: one wavefront per row (levels whose rows are long); same results.
void strength(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
              const double *dval, double th2, uint8_t *mask, int32_t *scount, bool wave,
              hipStream_t s);
int32_t max_row_length(int32_t n, const int32_t *rp, hipStream_t s);
// Distance-Laplacian weights (Sec. 3.1): w[k] = 1/|x_i - x_j|^power off the diagonal (0 on
// it; power 1 or 2), Ld[i] = sum of row i's weights; xyz is n x dim (dim 1..3).  Sets
// *err |= ebit when two connected nodes coincide.  strength() on (w, Ld) gives the labels.
void distance_weights(int32_t n, const int32_t *rp, const int32_t *col, const double *xyz,
                      int32_t dim, int32_t power, double *w, double *Ld, int32_t *err,
                      int32_t ebit, hipStream_t s);
// Member lists of the nc aggregates: mrp[nc+1] offsets into mem (unaggregated vertices left
// out); members in scatter order, or ascending when `sorted`.  Arrays from ar.
void member_lists(int32_t n, const int32_t *agg, int32_t nc, bool sorted, Arena &ar,
                  int32_t **mrp_out, int32_t **mem_out, hipStream_t s);

// ---- systems SA (systems.hip) ----------------------------------------------------------
// Node graph of a node-major block matrix (bs dofs per node): G.rp/G.col over A.n / bs nodes.
void node_graph(const Csr &A, int32_t bs, Arena &ar, Csr &G, hipStream_t s);
// Node labels on G from block Frobenius norms (0 weak, 1 strong, 3 diagonal) and the strong
// count per node.
void block_strength(const Csr &A, int32_t bs, const Csr &G, double theta, uint8_t *nmask,
                    int32_t *scount, hipStream_t s);
// Dof labels of A from node labels (entries inside a node kept).
void dof_mask(const Csr &A, int32_t bs, const Csr &G, const uint8_t *nmask, uint8_t *mask,
              hipStream_t s);
// QR tentative prolongator of n dofs (node aggregates agg, nc of them) for the nullspace B
// (n x k): Pt (n x nc k) from ar, Bc (nc k x k) the coarse nullspace; *err |= ebit when an
// aggregate has fewer dofs than k.
void tentative_qr(int32_t n, int32_t bs, int32_t k, const int32_t *agg, int32_t nc,
                  const double *B, Arena &ar, Csr &Pt, double *Bc, int32_t *err, int32_t ebit,
                  hipStream_t s);
// P = P_t - (omega invD_i) (Abar P_t)_i on the pattern of Abar P_t.
void smooth_tentative(const Csr &abar, const Csr &Pt, const double *invD, const double *omega,
                      Arena &ar, Csr &P, hipStream_t s);

// *err |= ebit when some x[0..m) is not finite.
void check_finite(const double *x, int64_t m, int32_t *err, int32_t ebit, hipStream_t s);
// cxyz[J] = centroid of aggregate J's members (nc x dim), summed in ascending vertex order.
void aggregate_centroids(int32_t n, const int32_t *agg, int32_t nc, const double *xyz,
                         int32_t dim, double *cxyz, hipStream_t s);
// Symmetrised strength graph G = S u S^T as CSR (grp[n+1], gcol[nnzG]); returns nnzG.
int64_t strength_graph(int32_t n, const int32_t *rp, const int32_t *col, const uint8_t *mask,
                       const int32_t *scount, bool wave, Arena &ar, int32_t **grp,
                       int32_t **gcol, hipStream_t s);
// Aggregation (roots = lexicographically-first distance-2 MIS in priority order; phase-2
// join).  A vertex without strong connections joins no aggregate (agg -1), or is the root of
// a singleton aggregate when `singletons` is set (the covering reading).  Returns nc;
// agg[n], is_root[n], root_vertex[nc].
int32_t aggregate(int32_t n, int64_t nnzG, const int32_t *grp, const int32_t *gcol, int32_t order,
                  uint64_t seed, int32_t level, bool singletons, int32_t *agg,
                  uint8_t *is_root, Arena &ar, int32_t **root_vertex, int32_t *rounds,
                  hipStream_t s);
// Sprsfy: marks dropped strong entries (mask 1 -> 2).
void sprsfy(int32_t n, const int32_t *rp, const int32_t *col, uint8_t *mask,
            const int32_t *agg, const int32_t *root_vertex, int32_t nc, hipStream_t s);
// Filtered matrix (plain or OffLmp) and the smoothing diagonal inverse of the n-row CSR with
// nnz_a entries; returns nnz(Abar).  err bit 8: zero filtered diagonal with the plain diagonal.
int64_t lump(int32_t n, int64_t nnz_a, const int32_t *rp, const int32_t *col, const double *val,
             const uint8_t *mask, bool offlmp, double tau, bool one_norm, double mult,
             bool wave, Arena &ar, Csr &abar, double *invD, int32_t *err, hipStream_t s);
// Power method; writes the estimate to *lam (device).  ws: 3n doubles + dot workspace.
void power_method(const Csr &M, const double *invD, int32_t iters, uint64_t seed,
                  int32_t level, int32_t stream_id, double *lam, hipStream_t s);
// omega = 4/(3 lambda) (or lambda = 1 first when `unit`), err bit 16 if lambda <= 0.
void damping(double *lam, double *omega, bool unit, int32_t *err, hipStream_t s);
// P = (I - omega invD Abar) Ptent; returns nnz(P).  long_rows: the per-aggregate sums come
// from a SpGEMM with the 0/1 aggregate matrix (the same sums in the same order).
int64_t prolongator(const Csr &abar, const double *invD, const int32_t *agg, int32_t nc,
                    const double *omega, Arena &ar, Csr &P, hipStream_t s,
                    bool long_rows = false);
void cnstrnt(const Csr &P, const int32_t *agg, hipStream_t s);
void scale_rows(const Csr &P, const double *B, hipStream_t s);
// R = P^T with ascending columns per row.
void transpose(const Csr &P, Arena &ar, Csr &R, hipStream_t s);
// 1/A_ii with err bit 32 when A_ii <= 0.
void inv_diag(int32_t n, const double *dval, double *invD, int32_t *err, hipStream_t s);
// Ahat = D_B A D_B
void scale_sym(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
               const double *B, double *out, hipStream_t s);

// ---------------- SpGEMM (spgemm.hip) --------------------------------------------------
// C = X * Y with Gustavson-order accumulation per output entry (ascending inner index);
// output rows sorted; cancellations stored.  C's arrays are allocated from `ar`.
void spgemm(const Csr &X, const Csr &Y, Arena &ar, Csr &C, hipStream_t s);
// Numeric plan of C = X Y on a fixed pattern (re-setup): for each entry p of C, the products
// that form it in ascending position of X's row (ascending inner index), as pairs of an X
// entry le[t] and a Y entry lq[t] for t in [lrp[p], lrp[p+1]).
struct SpgemmPlan {
  int64_t *lrp = nullptr;
  int32_t *le = nullptr, *lq = nullptr;
  int64_t nprod = 0;
};
// Builds the plan from X, Y and the pattern of C (C = X Y as spgemm formed it); err bit
// `bit` if a product's column is missing from C's row (never, for that C).
void spgemm_plan(const Csr &X, const Csr &Y, const Csr &C, Arena &ar, SpgemmPlan &pl,
                 int32_t *err, int32_t bit, hipStream_t s);
// C.val from X.val and Y.val through the plan: every entry summed over its list in order,
// from 0 (Gustavson order, as spgemm: bitwise the same values).
void spgemm_numeric(const Csr &X, const Csr &Y, const SpgemmPlan &pl, Csr &C, hipStream_t s);
// Position of every P entry in R = P^T (R's rows sorted), and R.val from P.val through it.
void transpose_perm(const Csr &P, const Csr &R, Arena &ar, int32_t **perm, hipStream_t s);
void transpose_values(const Csr &P, const int32_t *perm, Csr &R, hipStream_t s);

// ---------------- coarsest level (coarse.hip) ------------------------------------------
// Dense inverse of the coarsest operator via Cholesky (err bit 64 on a pivot <= 0).
// lu: LU without pivoting (any operator); otherwise Cholesky, with err bit 256 when the
// operator is not symmetric to 1e-10 relative.  err bit 64: a pivot <= 0 (Cholesky) or zero.
void coarse_inverse(const Csr &A, double *Ainv, int32_t *err, bool lu, hipStream_t s);

}  // namespace sa
