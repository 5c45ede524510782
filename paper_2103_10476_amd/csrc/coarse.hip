// Coarsest level (Sec. 3.1: a direct solve once the hierarchy reaches <= 1000 unknowns):
// dense Cholesky A_L = L L^T in one workgroup, L^{-1} by forward substitution (one column per
// thread), and A_L^{-1} = L^{-T} L^{-1} on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
// The V-cycle then applies A_L^{-1} as a dense GEMV.  The factor's rounding order differs
// from a sequential Cholesky, so this is the one setup result that matches a CPU reference
// to rounding (~1e-16 relative) rather than bit for bit.
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

// Right-looking Cholesky on the lower triangle of D (row-major, leading dimension ld).
__global__ __launch_bounds__(1024) void k_cholesky(int32_t n, int32_t ld, double *D,
                                                   int32_t *err) {
  __shared__ double s_ljj;
  const int tid = threadIdx.x;
  for (int32_t j = 0; j < n; ++j) {
    if (tid == 0) {
      const double d = D[(int64_t)j * ld + j];
      if (!(d > 0.0)) atomicOr(err, 64);
      s_ljj = sqrt(d);
      D[(int64_t)j * ld + j] = s_ljj;
    }
    __syncthreads();
    const double ljj = s_ljj;
    for (int32_t i = j + 1 + tid; i < n; i += blockDim.x) D[(int64_t)i * ld + j] /= ljj;
    __syncthreads();
    // trailing update of the lower triangle: D[i][k] -= D[i][j] * D[k][j], j < k <= i
    const int32_t m = n - j - 1;
    const int64_t tri = (int64_t)m * (m + 1) / 2;
    for (int64_t t = tid; t < tri; t += blockDim.x) {
      // t -> (a, b) with 0 <= b <= a < m, row-major over the triangle
      int32_t a = (int32_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
      while ((int64_t)a * (a + 1) / 2 > t) --a;
      while ((int64_t)(a + 1) * (a + 2) / 2 <= t) ++a;
      const int32_t b = (int32_t)(t - (int64_t)a * (a + 1) / 2);
      const int32_t i = j + 1 + a, k = j + 1 + b;
      D[(int64_t)i * ld + k] -= D[(int64_t)i * ld + j] * D[(int64_t)k * ld + j];
    }
    __syncthreads();
  }
}

// Column c of L^{-1} (lower triangular), written into Li (row-major, leading dim ld).
__global__ void k_trinv(int32_t n, int32_t ld, const double *L, double *Li) {
  const int64_t c64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c64 >= n) return;
  const int32_t c = (int32_t)c64;
  Li[(int64_t)c * ld + c] = 1.0 / L[(int64_t)c * ld + c];
  for (int32_t i = c + 1; i < n; ++i) {
    double s = 0.0;
    for (int32_t k = c; k < i; ++k) s += L[(int64_t)i * ld + k] * Li[(int64_t)k * ld + c];
    Li[(int64_t)i * ld + c] = -s / L[(int64_t)i * ld + i];
  }
}

// C = Li^T Li on 16x16 tiles, one wavefront per tile, K in steps of 4.  Operand layout of
// v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16]; it receives
// D[4v + l/16][l%16] in result register v = 0..3 (checked against a dense inverse on the
// GPU).  Li is zero-padded to ld (a multiple of 16).
__global__ __launch_bounds__(64) void k_gram_mfma(int32_t n, int32_t ld, const double *Li,
                                                  double *C) {
  const int lane = threadIdx.x;
  const int32_t i = blockIdx.x * 16 + (lane & 15);
  const int32_t j = blockIdx.y * 16 + (lane & 15);
  const int32_t kk = lane >> 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int32_t k0 = 0; k0 < ld; k0 += 4) {
    const double a = Li[(int64_t)(k0 + kk) * ld + i];  // A[i][k] = Li[k][i]
    const double b = Li[(int64_t)(k0 + kk) * ld + j];  // B[k][j] = Li[k][j]
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  const int32_t col = blockIdx.y * 16 + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int32_t row = blockIdx.x * 16 + 4 * v + (lane >> 4);
    if (row < n && col < n) C[(int64_t)row * n + col] = acc[v];
  }
}

void coarse_inverse(const Csr &A, double *Ainv, int32_t *err, hipStream_t s) {
  const int32_t n = A.n;
  if (n <= 0) return;
  const int32_t ld = (int32_t)ceil_div(n, 16) * 16;
  const size_t sz = sizeof(double) * (size_t)ld * ld;
  double *D = (double *)dev_alloc(sz, s);
  double *Li = (double *)dev_alloc(sz, s);
  SA_HIP(hipMemsetAsync(D, 0, sz, s));
  SA_HIP(hipMemsetAsync(Li, 0, sz, s));
  k_dense_scatter<<<grid_for(n), kBlock, 0, s>>>(n, ld, A.rp, A.col, A.val, D);
  SA_LAUNCH_CHECK();
  k_cholesky<<<1, 1024, 0, s>>>(n, ld, D, err);
  SA_LAUNCH_CHECK();
  k_trinv<<<grid_for(n, 64), 64, 0, s>>>(n, ld, D, Li);
  SA_LAUNCH_CHECK();
  dim3 g(ld / 16, ld / 16);
  k_gram_mfma<<<g, 64, 0, s>>>(n, ld, Li, Ainv);
  SA_LAUNCH_CHECK();
  dev_free(D, s);
  dev_free(Li, s);
}

}  // namespace sa
