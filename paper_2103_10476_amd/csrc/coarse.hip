// Coarsest level (Sec. 3.1: a direct solve once the hierarchy reaches <= 1000 unknowns, or
// a level left without strong connections): blocked dense Cholesky A_L = L L^T with the
// trailing updates on the FP64 matrix cores, L^{-1} by blocks (the off-diagonal blocks on
// the matrix cores), and A_L^{-1} = L^{-T} L^{-1} on the matrix cores (v_mfma_f64_16x16x4f64).
// Nonsymmetric operators (GMRES, Sec. 3.4) take a blocked LU without pivoting instead,
// A_L = L U, and A_L^{-1} = U^{-1} L^{-1} = W^T L^{-1} with W = (U^T)^{-1}.
// The V-cycle then applies A_L^{-1} as a dense GEMV.  The factor's rounding order differs
// from a sequential factorization, so this is the one setup result that matches a CPU
// reference to rounding (~1e-16 relative) rather than bit for bit.
#include "kernels.hpp"

namespace sa {

typedef double v4d __attribute__((ext_vector_type(4)));

__global__ void k_dense_scatter(int32_t n, int32_t ld, const int32_t *rp, const int32_t *col,
                                const double *val, double *D) {
  const int64_t i64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i64 >= n) return;
  const int32_t i = (int32_t)i64;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) D[(int64_t)i * ld + col[k]] = val[k];
}

// ---- blocked right-looking Cholesky, 64 x 64 blocks ---------------------------------------
// D is ld x ld row-major (ld a multiple of 64) and holds the matrix in its lower triangle;
// rows and columns n..ld-1 are an identity pad, so every block is full.  Step kb factors the
// diagonal block, solves the panel below it, and updates the trailing lower triangle on the
// FP64 matrix cores.  The factor's rounding order differs from the sequential textbook
// Cholesky; the result is checked against a dense inverse to ~1e-16 relative.
constexpr int kNB = 64;

__global__ void k_pad_identity(int32_t n, int32_t ld, double *D) {
  const int32_t i = n + blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ld) D[(int64_t)i * ld + i] = 1.0;
}

// Diagonal block at (k0, k0): unblocked right-looking Cholesky in LDS (err bit 64 on a
// pivot <= 0).
__global__ __launch_bounds__(256) void k_potrf_diag(int32_t ld, int32_t k0, double *D,
                                                    int32_t *err) {
  __shared__ double a[kNB][kNB + 1];
  const int tid = threadIdx.x;
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int i = q / kNB, j = q % kNB;
    a[i][j] = (j <= i) ? D[(int64_t)(k0 + i) * ld + k0 + j] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < kNB; ++j) {
    if (tid == 0) {
      const double d = a[j][j];
      if (!(d > 0.0)) atomicOr(err, 64);
      a[j][j] = sqrt(d);
    }
    __syncthreads();
    const double ljj = a[j][j];
    for (int i = j + 1 + tid; i < kNB; i += 256) a[i][j] /= ljj;
    __syncthreads();
    // trailing update over the (63-j)^2 square below and right of (j, j) only
    const int m = kNB - 1 - j;
    for (int q = tid; q < m * m; q += 256) {
      const int i = j + 1 + q / m, k = j + 1 + q % m;
      if (k <= i) a[i][k] -= a[i][j] * a[k][j];
    }
    __syncthreads();
  }
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int i = q / kNB, j = q % kNB;
    if (j <= i) D[(int64_t)(k0 + i) * ld + k0 + j] = a[i][j];
  }
}

// Panel below the diagonal block: row i of L in columns k0..k0+63 solves x L_kk^T = d by
// forward substitution (one thread per row, the 64 unknowns in registers).
__global__ __launch_bounds__(256) void k_trsm_panel(int32_t ld, int32_t k0, double *D) {
  __shared__ double lk[kNB][kNB + 1];
  const int tid = threadIdx.x;
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int i = q / kNB, j = q % kNB;
    lk[i][j] = (j <= i) ? D[(int64_t)(k0 + i) * ld + k0 + j] : 0.0;
  }
  __syncthreads();
  const int64_t i = (int64_t)k0 + kNB + (int64_t)blockIdx.x * 256 + tid;
  if (i >= ld) return;
  double *row = D + i * ld + k0;
  double x[kNB];
#pragma unroll
  for (int j = 0; j < kNB; ++j) x[j] = row[j];
#pragma unroll
  for (int j = 0; j < kNB; ++j) {
    double t = x[j];
#pragma unroll
    for (int m = 0; m < j; ++m) t -= x[m] * lk[j][m];
    x[j] = t / lk[j][j];
  }
#pragma unroll
  for (int j = 0; j < kNB; ++j) row[j] = x[j];
}

// Trailing update after step kb: D[ib][jb] -= L[ib][kb] L[jb][kb]^T for every block pair
// kb < jb <= ib < nbk (workgroup t = the t-th pair, row-major over the lower triangle).  The
// two 64 x 64 panels are staged in LDS; each of the 4 wavefronts computes a 16 x 64 strip
// as four 16 x 16 tiles with v_mfma_f64_16x16x4f64 (lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and receives D[4v + l/16][l%16] in result register v).  Diagonal blocks are
// updated whole; their upper parts are never read.
__global__ __launch_bounds__(256) void k_syrk_mfma(int32_t ld, int32_t kb, int32_t nbk,
                                                   double *D) {
  __shared__ double As[kNB][kNB + 1];
  __shared__ double Bs[kNB][kNB + 1];
  const int64_t t = blockIdx.x;
  int32_t a = (int32_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)a * (a + 1) / 2 > t) --a;
  while ((int64_t)(a + 1) * (a + 2) / 2 <= t) ++a;
  const int32_t b = (int32_t)(t - (int64_t)a * (a + 1) / 2);
  const int32_t ib = kb + 1 + a, jb = kb + 1 + b;
  if (ib >= nbk || jb > ib) return;  // block-uniform; the grid holds exactly the pairs
  const int64_t r0 = (int64_t)ib * kNB, c0 = (int64_t)jb * kNB, k0 = (int64_t)kb * kNB;
  const int tid = threadIdx.x;
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int r = q / kNB, k = q % kNB;
    As[r][k] = D[(r0 + r) * ld + k0 + k];
    Bs[r][k] = D[(c0 + r) * ld + k0 + k];
  }
  __syncthreads();
  const int w = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < kNB; kk += 4) {
      const double av = As[16 * w + lr][kk + lk];
      const double bv = Bs[16 * ct + lr][kk + lk];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 16 * w + 4 * v + lk;
      const int64_t col = c0 + 16 * ct + lr;
      D[row * ld + col] -= acc[v];
    }
  }
}

// ---- blocked inverse of the triangular factor, Li = L^{-1} ------------------------------------
// Step 0 inverts every 64 x 64 diagonal block.  Then L X = I is solved by right-looking block
// forward substitution with the whole identity as right-hand side, in place in Li (zero
// below the diagonal blocks to start with): for block row ib = 0, 1, ..., its tiles are
// finalised, X[ib][kb] = Li[ib][ib] B[ib][kb] (kb < ib), and every later block row is
// updated, B[i][kb] -= L[i][ib] X[ib][kb] (i > ib, kb <= ib).  Each launch is one tile
// product deep, so the dependent chain is two launches per block row.

// 64 x 64 product on the matrix cores: wavefront w accumulates rows 16w..16w+15 of As * Bs
// (As[r][k] = A[r][k], Bs[k][c] = B[k][c]) into acc[ct] for column tile ct.
__device__ __forceinline__ void mfma_64(const double (*As)[kNB + 1], const double (*Bs)[kNB + 1],
                                        v4d *acc) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
#pragma unroll
    for (int kk = 0; kk < kNB; kk += 4) {
      const double av = As[16 * w + lr][kk + lk];
      const double bv = Bs[kk + lk][16 * ct + lr];
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[ct], 0, 0, 0);
    }
  }
}

__global__ __launch_bounds__(256) void k_trtri_diag(int32_t ld, const double *L, double *Li,
                                                    bool unit) {
  __shared__ double l[kNB][kNB + 1];
  __shared__ double x[kNB][kNB + 1];
  const int tid = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * kNB;
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int i = q / kNB, j = q % kNB;
    l[i][j] = (j < i || (j == i && !unit)) ? L[(k0 + i) * ld + k0 + j] : (j == i ? 1.0 : 0.0);
    x[i][j] = 0.0;
  }
  __syncthreads();
  if (tid < kNB) {  // column c of the block's inverse by forward substitution
    const int c = tid;
    x[c][c] = 1.0 / l[c][c];
    for (int i = c + 1; i < kNB; ++i) {
      double t = 0.0;
      for (int k = c; k < i; ++k) t += l[i][k] * x[k][c];
      x[i][c] = -t / l[i][i];
    }
  }
  __syncthreads();
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int i = q / kNB, j = q % kNB;
    Li[(k0 + i) * ld + k0 + j] = x[i][j];
  }
}

// X[ib][kb] = Li[ib][ib] B[ib][kb] for kb = blockIdx.x < ib.
__global__ __launch_bounds__(256) void k_trinv_finalize(int32_t ld, int32_t ib, double *Li) {
  __shared__ double As[kNB][kNB + 1];
  __shared__ double Bs[kNB][kNB + 1];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)ib * kNB, c0 = (int64_t)blockIdx.x * kNB;
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int r = q / kNB, k = q % kNB;
    As[r][k] = Li[(r0 + r) * ld + r0 + k];  // Li[ib][ib] (zero above its diagonal)
    Bs[r][k] = Li[(r0 + r) * ld + c0 + k];  // B[ib][kb]
  }
  __syncthreads();
  v4d acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = v4d{0.0, 0.0, 0.0, 0.0};
  mfma_64(As, Bs, acc);
  const int w = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      Li[(r0 + 16 * w + 4 * v + lk) * ld + c0 + 16 * ct + lr] = acc[ct][v];
}

// B[i][kb] -= L[i][ib] X[ib][kb] for every tile i > ib, kb <= ib (block t: i = ib+1+t/(ib+1),
// kb = t mod (ib+1)); each tile has one writer per launch.
__global__ __launch_bounds__(256) void k_trinv_update(int32_t ld, int32_t ib, const double *L,
                                                      double *Li) {
  __shared__ double As[kNB][kNB + 1];
  __shared__ double Bs[kNB][kNB + 1];
  const int tid = threadIdx.x;
  const int32_t i = ib + 1 + (int32_t)(blockIdx.x / (unsigned)(ib + 1));
  const int32_t kb = (int32_t)(blockIdx.x % (unsigned)(ib + 1));
  const int64_t r0 = (int64_t)i * kNB, j0 = (int64_t)ib * kNB, c0 = (int64_t)kb * kNB;
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int r = q / kNB, k = q % kNB;
    As[r][k] = L[(r0 + r) * ld + j0 + k];   // L[i][ib]
    Bs[r][k] = Li[(j0 + r) * ld + c0 + k];  // X[ib][kb]
  }
  __syncthreads();
  v4d acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = v4d{0.0, 0.0, 0.0, 0.0};
  mfma_64(As, Bs, acc);
  const int w = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      Li[(r0 + 16 * w + 4 * v + lk) * ld + c0 + 16 * ct + lr] -= acc[ct][v];
}

// Li = L^{-1} (Li zero outside the diagonal blocks, which k_trtri_diag has filled).
static void trinv_blocks(int32_t ld, int32_t nbk, const double *L, double *Li, hipStream_t s) {
  for (int32_t ib = 0; ib < nbk; ++ib) {
    if (ib > 0) k_trinv_finalize<<<(unsigned)ib, 256, 0, s>>>(ld, ib, Li);
    const int64_t tiles = (int64_t)(nbk - ib - 1) * (ib + 1);
    if (tiles > 0) k_trinv_update<<<(unsigned)tiles, 256, 0, s>>>(ld, ib, L, Li);
  }
  SA_LAUNCH_CHECK();
}

// C = X^T Y for lower-triangular X and Y (ld x ld, zero above the diagonal; Cholesky:
// X = Y = L^{-1}; LU: X = (U^T)^{-1}, Y = L^{-1}), n x n row-major output.  Tile (ib, jb)
// of 64 x 64 sums X[kb][ib]^T Y[kb][jb] over kb >= max(ib, jb) (the other tiles are zero),
// both tiles staged in LDS (X transposed on the way in) and multiplied on the matrix cores.
// sym: X = Y, so only tiles ib >= jb are computed and the off-diagonal ones are also written
// transposed.
// Block t enumerates the tile pairs row-major (the lower triangle when sym).
__global__ __launch_bounds__(256) void k_gram_tiles(int32_t n, int32_t ld, int32_t nbk,
                                                    const double *X, const double *Y,
                                                    double *C, bool sym) {
  __shared__ double As[kNB][kNB + 1];
  __shared__ double Bs[kNB][kNB + 1];
  const int64_t t = blockIdx.x;
  int32_t ib, jb;
  if (sym) {
    int32_t a = (int32_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)a * (a + 1) / 2 > t) --a;
    while ((int64_t)(a + 1) * (a + 2) / 2 <= t) ++a;
    ib = a;
    jb = (int32_t)(t - (int64_t)a * (a + 1) / 2);
  } else {
    ib = (int32_t)(t / nbk);
    jb = (int32_t)(t % nbk);
  }
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)ib * kNB, j0 = (int64_t)jb * kNB;
  v4d acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int32_t kb = ib > jb ? ib : jb; kb < nbk; ++kb) {
    const int64_t k0 = (int64_t)kb * kNB;
    for (int q = tid; q < kNB * kNB; q += 256) {
      const int k = q / kNB, c = q % kNB;
      As[c][k] = X[(k0 + k) * ld + i0 + c];  // A[r][k] = X[k][r]
      Bs[k][c] = Y[(k0 + k) * ld + j0 + c];
    }
    __syncthreads();
    mfma_64(As, Bs, acc);
    __syncthreads();
  }
  const int w = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = i0 + 16 * w + 4 * v + lk, col = j0 + 16 * ct + lr;
      if (row < n && col < n) {
        C[row * n + col] = acc[ct][v];
        // a diagonal tile holds both (r, c) and (c, r): each is written once, by its own lane
        if (sym && ib != jb) C[col * n + row] = acc[ct][v];
      }
    }
}

static void gram(int32_t n, int32_t ld, int32_t nbk, const double *X, const double *Y,
                 double *C, bool sym, hipStream_t s) {
  const int64_t tiles = sym ? (int64_t)nbk * (nbk + 1) / 2 : (int64_t)nbk * nbk;
  k_gram_tiles<<<(unsigned)tiles, 256, 0, s>>>(n, ld, nbk, X, Y, C, sym);
  SA_LAUNCH_CHECK();
}

// ---- blocked right-looking LU without pivoting, 64 x 64 blocks --------------------------------
// D holds the whole matrix (identity pad).  Step kb factors the diagonal block (unit L below,
// U on and above), solves the row panel U12 = L11^{-1} A12 and the column panel
// L21 = A21 U11^{-1}, and updates the whole trailing matrix A22 -= L21 U12 on the matrix
// cores.  err bit 64 on a zero or non-finite pivot.
__global__ __launch_bounds__(256) void k_getrf_diag(int32_t ld, int32_t k0, double *D,
                                                    int32_t *err) {
  __shared__ double a[kNB][kNB + 1];
  const int tid = threadIdx.x;
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int i = q / kNB, j = q % kNB;
    a[i][j] = D[(int64_t)(k0 + i) * ld + k0 + j];
  }
  __syncthreads();
  for (int j = 0; j < kNB; ++j) {
    const double piv = a[j][j];
    if (tid == 0 && (!(piv != 0.0) || !isfinite(piv))) atomicOr(err, 64);
    for (int i = j + 1 + tid; i < kNB; i += 256) a[i][j] /= piv;
    __syncthreads();
    for (int q = tid; q < kNB * kNB; q += 256) {
      const int i = q / kNB, k = q % kNB;
      if (i > j && k > j) a[i][k] -= a[i][j] * a[j][k];
    }
    __syncthreads();
  }
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int i = q / kNB, j = q % kNB;
    D[(int64_t)(k0 + i) * ld + k0 + j] = a[i][j];
  }
}

// Row panel right of the diagonal block: column c of U12 solves L11 x = a by forward
// substitution with the unit diagonal (one thread per column, the 64 unknowns in registers).
__global__ __launch_bounds__(256) void k_trsm_row_panel(int32_t ld, int32_t k0, double *D) {
  __shared__ double lk[kNB][kNB + 1];
  const int tid = threadIdx.x;
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int i = q / kNB, j = q % kNB;
    lk[i][j] = (j < i) ? D[(int64_t)(k0 + i) * ld + k0 + j] : 0.0;
  }
  __syncthreads();
  const int64_t c = (int64_t)k0 + kNB + (int64_t)blockIdx.x * 256 + tid;
  if (c >= ld) return;
  double x[kNB];
#pragma unroll
  for (int j = 0; j < kNB; ++j) x[j] = D[((int64_t)k0 + j) * ld + c];
#pragma unroll
  for (int j = 0; j < kNB; ++j) {
    double t = x[j];
#pragma unroll
    for (int m = 0; m < j; ++m) t -= lk[j][m] * x[m];
    x[j] = t;
  }
#pragma unroll
  for (int j = 0; j < kNB; ++j) D[((int64_t)k0 + j) * ld + c] = x[j];
}

// Column panel below the diagonal block: row i of L21 solves x U11 = a (one thread per row).
__global__ __launch_bounds__(256) void k_trsm_col_panel(int32_t ld, int32_t k0, double *D) {
  __shared__ double uk[kNB][kNB + 1];
  const int tid = threadIdx.x;
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int i = q / kNB, j = q % kNB;
    uk[i][j] = (j >= i) ? D[(int64_t)(k0 + i) * ld + k0 + j] : 0.0;
  }
  __syncthreads();
  const int64_t i = (int64_t)k0 + kNB + (int64_t)blockIdx.x * 256 + tid;
  if (i >= ld) return;
  double *row = D + i * ld + k0;
  double x[kNB];
#pragma unroll
  for (int j = 0; j < kNB; ++j) x[j] = row[j];
#pragma unroll
  for (int j = 0; j < kNB; ++j) {
    double t = x[j];
#pragma unroll
    for (int m = 0; m < j; ++m) t -= x[m] * uk[m][j];
    x[j] = t / uk[j][j];
  }
#pragma unroll
  for (int j = 0; j < kNB; ++j) row[j] = x[j];
}

// Trailing update after step kb: D[ib][jb] -= L[ib][kb] U[kb][jb] for every block pair
// kb < ib, jb < nbk (workgroup t: ib = kb+1 + t/m, jb = kb+1 + t%m, m = nbk-kb-1).
__global__ __launch_bounds__(256) void k_gemm_update(int32_t ld, int32_t kb, int32_t nbk,
                                                     double *D) {
  __shared__ double As[kNB][kNB + 1];
  __shared__ double Bs[kNB][kNB + 1];
  const int32_t m = nbk - kb - 1;
  const int32_t ib = kb + 1 + (int32_t)(blockIdx.x / m), jb = kb + 1 + (int32_t)(blockIdx.x % m);
  const int64_t r0 = (int64_t)ib * kNB, c0 = (int64_t)jb * kNB, k0 = (int64_t)kb * kNB;
  const int tid = threadIdx.x;
  for (int q = tid; q < kNB * kNB; q += 256) {
    const int r = q / kNB, k = q % kNB;
    As[r][k] = D[(r0 + r) * ld + k0 + k];  // L21 block (row r, column k)
    Bs[r][k] = D[(k0 + r) * ld + c0 + k];  // U12 block (row r, column k)
  }
  __syncthreads();
  v4d acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = v4d{0.0, 0.0, 0.0, 0.0};
  mfma_64(As, Bs, acc);
  const int w = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      D[(r0 + 16 * w + 4 * v + lk) * ld + c0 + 16 * ct + lr] -= acc[ct][v];
}

// Lower forms of the two factors: Lb = unit lower part of D, Ut = U^T (lower).
__global__ void k_split_lu(int32_t ld, const double *D, double *Lb, double *Ut) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)ld * ld) return;
  const int64_t i = q / ld, j = q % ld;
  Lb[q] = (j < i) ? D[q] : (j == i ? 1.0 : 0.0);
  Ut[q] = (j <= i) ? D[j * ld + i] : 0.0;
}

// Symmetry of the coarsest operator before a Cholesky solve (which reads only the lower
// triangle): mx[0] = max |a_ij|, mx[1] = max |a_ij - a_ji| as the bit patterns of
// non-negative doubles (ordered like the values); err bit 256 when mx[1] > 1e-10 mx[0].
__global__ void k_sym_max(int32_t ld, const double *D, unsigned long long *mx) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)ld * ld) return;
  const int64_t i = q / ld, j = q % ld;
  const double a = fabs(D[q]), d = fabs(D[q] - D[j * ld + i]);
  if (a > 0.0) atomicMax(&mx[0], (unsigned long long)__double_as_longlong(a));
  if (d > 0.0) atomicMax(&mx[1], (unsigned long long)__double_as_longlong(d));
}
__global__ void k_sym_flag(const unsigned long long *mx, int32_t *err) {
  const double amax = __longlong_as_double((long long)mx[0]);
  const double asym = __longlong_as_double((long long)mx[1]);
  if (!(asym <= 1e-10 * amax)) atomicOr(err, 256);
}

// LU path of coarse_inverse: D (ld x ld, padded) is factored in place; Li (ld x ld) is
// scratch.  Ainv = W^T L^{-1} with W = (U^T)^{-1}.
static void lu_inverse(int32_t ld, int32_t nbk, int32_t n, double *D, double *Li, double *Ainv,
                       int32_t *err, hipStream_t s) {
  for (int32_t kb = 0; kb < nbk; ++kb) {
    const int32_t k0 = kb * kNB;
    k_getrf_diag<<<1, 256, 0, s>>>(ld, k0, D, err);
    const int32_t rest = ld - k0 - kNB;
    if (rest > 0) {
      k_trsm_row_panel<<<(unsigned)ceil_div(rest, 256), 256, 0, s>>>(ld, k0, D);
      k_trsm_col_panel<<<(unsigned)ceil_div(rest, 256), 256, 0, s>>>(ld, k0, D);
      const int64_t m = nbk - kb - 1;
      k_gemm_update<<<(unsigned)(m * m), 256, 0, s>>>(ld, kb, nbk, D);
    }
    SA_LAUNCH_CHECK();
  }
  const int64_t cnt = (int64_t)ld * ld;
  double *Lb = (double *)dev_alloc(sizeof(double) * (size_t)cnt, s);
  double *Ut = (double *)dev_alloc(sizeof(double) * (size_t)cnt, s);
  k_split_lu<<<grid_for(cnt), kBlock, 0, s>>>(ld, D, Lb, Ut);
  SA_LAUNCH_CHECK();
  // Li = Lb^{-1}; then W = Ut^{-1} into D (the factor is no longer needed)
  fill_f64(Li, 0.0, cnt, s);
  k_trtri_diag<<<(unsigned)nbk, 256, 0, s>>>(ld, Lb, Li, true);
  trinv_blocks(ld, nbk, Lb, Li, s);
  fill_f64(D, 0.0, cnt, s);
  k_trtri_diag<<<(unsigned)nbk, 256, 0, s>>>(ld, Ut, D, false);
  trinv_blocks(ld, nbk, Ut, D, s);
  SA_LAUNCH_CHECK();
  gram(n, ld, nbk, D, Li, Ainv, false, s);
  dev_free(Lb, s);
  dev_free(Ut, s);
}

void coarse_inverse(const Csr &A, double *Ainv, int32_t *err, bool lu, hipStream_t s) {
  const int32_t n = A.n;
  if (n <= 0) return;
  const int32_t ld = (int32_t)ceil_div(n, kNB) * kNB;
  const int32_t nbk = ld / kNB;
  const int64_t cnt = (int64_t)ld * ld;
  double *D = (double *)dev_alloc(sizeof(double) * (size_t)cnt, s);
  double *Li = (double *)dev_alloc(sizeof(double) * (size_t)cnt, s);
  fill_f64(D, 0.0, cnt, s);
  fill_f64(Li, 0.0, cnt, s);
  k_dense_scatter<<<grid_for(n), kBlock, 0, s>>>(n, ld, A.rp, A.col, A.val, D);
  SA_LAUNCH_CHECK();
  if (ld > n) {
    k_pad_identity<<<grid_for(ld - n), kBlock, 0, s>>>(n, ld, D);
    SA_LAUNCH_CHECK();
  }
  if (lu) {
    lu_inverse(ld, nbk, n, D, Li, Ainv, err, s);
    dev_free(D, s);
    dev_free(Li, s);
    return;
  }
  {
    unsigned long long *mx = (unsigned long long *)dev_alloc(2 * sizeof(unsigned long long), s);
    SA_HIP(hipMemsetAsync(mx, 0, 2 * sizeof(unsigned long long), s));
    k_sym_max<<<grid_for(cnt), kBlock, 0, s>>>(ld, D, mx);
    k_sym_flag<<<1, 1, 0, s>>>(mx, err);
    SA_LAUNCH_CHECK();
    dev_free(mx, s);
  }
  for (int32_t kb = 0; kb < nbk; ++kb) {
    const int32_t k0 = kb * kNB;
    k_potrf_diag<<<1, 256, 0, s>>>(ld, k0, D, err);
    const int32_t below = ld - k0 - kNB;
    if (below > 0) {
      k_trsm_panel<<<(unsigned)ceil_div(below, 256), 256, 0, s>>>(ld, k0, D);
      const int64_t m = nbk - kb - 1;
      k_syrk_mfma<<<(unsigned)(m * (m + 1) / 2), 256, 0, s>>>(ld, kb, nbk, D);
    }
    SA_LAUNCH_CHECK();
  }
  k_trtri_diag<<<(unsigned)nbk, 256, 0, s>>>(ld, D, Li, false);
  trinv_blocks(ld, nbk, D, Li, s);
  SA_LAUNCH_CHECK();
  gram(n, ld, nbk, Li, Li, Ainv, true, s);
  dev_free(D, s);
  dev_free(Li, s);
}

}  // namespace sa
