// Solve-phase kernels: CSR SpMV with fused smoother/transfer epilogues, the canonical inner
// product, vector updates and the PCG scalar steps.
//
// SpMV layout: a block of 256 threads owns a run of at most 256 consecutive rows, chosen by
// the row plan so that every block carries about the same number of entries plus a per-row
// cost.  The block streams the rows' entries through LDS in coalesced chunks, forming each
// product val*x[col] once; then every thread adds the products of its own row (at most 64
// entries, or any length in the plain order) in ascending column order, and longer rows are
// otherwise summed by a wavefront as 64 interleaved in-order partial sums added in order (the
// row-sum orders defined with spmv_block).  Results are bit-identical to that row-by-row
// definition, while the global
// loads stay fully coalesced (HBM-bound: ~12 B/entry for FP64, ~8 B/entry for FP32).
// Operators with short rows use a sliced-ELL copy instead (k_spmv_sell).
#include "solve_device.hpp"

namespace sa {

template <class T, class Epi, bool Split>
__global__ __launch_bounds__(kBlock) void k_spmv(const int32_t *__restrict__ bstart,
                                                 const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col,
                                                 const T *__restrict__ val,
                                                 const T *__restrict__ x, Epi epi) {
  __shared__ SpmvShared<T> sh;
  spmv_block<T, Epi, Split>(xcd_block(blockIdx.x, gridDim.x), bstart, rp, col, val, x, epi,
                            sh);
}

// Sliced-ELL SpMV: one wavefront per 64-row slice, lane l on row 64 s + l.  The k-th entries
// of the slice's rows are contiguous, so every value and index load is a full 64-lane run;
// entries are taken 8 at a time (indices and values, then the x gathers, then the in-order
// adds); rows are at most 64 entries, summed in ascending column order from 0 like the CSR
// kernel's short rows.  The workgroup's 4 slices are consecutive and XCD-grouped like the
// CSR row blocks.
template <class T, class Epi>
__global__ __launch_bounds__(kBlock) void k_spmv_sell(int32_t n, int32_t nslice,
                                                      const int32_t *__restrict__ sptr,
                                                      const int32_t *__restrict__ scol,
                                                      const T *__restrict__ sval,
                                                      const T *__restrict__ x, Epi epi) {
  const int32_t sl =
      xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (int32_t)(threadIdx.x >> 6);
  if (sl >= nslice) return;  // wave-uniform
  const int32_t lane = threadIdx.x & 63;
  const int32_t row = sl * 64 + lane;
  const int32_t p0 = sptr[sl];
  const int32_t w = (sptr[sl + 1] - p0) >> 6;
  typename Epi::Pre pre{};
  if (row < n) pre = epi.load(row);
  const int32_t *cb = scol + p0 + lane;
  const T *vb = sval + p0 + lane;
  T s = T(0);
  for (int32_t k = 0; k < w; k += 8) {
    int32_t c[8];
    T v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int32_t kk = min(k + q, w - 1);  // in bounds even if loaded eagerly
      c[q] = (k + q < w) ? cb[kk * 64] : -1;
      v[q] = vb[kk * 64];
    }
    T xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xv[q] = c[q] >= 0 ? x[c[q]] : T(0);
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (c[q] >= 0) s += v[q] * xv[q];
  }
  if (row < n) epi.store(row, s, pre);
}

// Slice widths (times 64): a wavefront's maximum row length.  Launched over nslice*64
// threads, whole wavefronts.
__global__ void k_sell_width(int32_t n, int32_t nslice, const int32_t *rp, int32_t *w64) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t len = i < n ? rp[i + 1] - rp[i] : 0;
  for (int off = 32; off >= 1; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
  if ((threadIdx.x & 63) == 0 && (i >> 6) < nslice) w64[i >> 6] = 64 * len;
}
// Thread per (padded) row: its entries into the slice, then padding.
template <class T>
__global__ void k_sell_fill(int32_t n, int32_t nslice, const int32_t *rp, const int32_t *col,
                            const double *val, const int32_t *ptr, int32_t *scol, T *sval) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nslice * 64) return;
  const int32_t sl = (int32_t)(i >> 6), l = (int32_t)(i & 63);
  const int32_t p = ptr[sl], w = (ptr[sl + 1] - p) >> 6;
  int32_t b = 0, len = 0;
  if (i < n) {
    b = rp[i];
    len = rp[i + 1] - b;
  }
  for (int32_t k = 0; k < w; ++k) {
    const int32_t o = p + k * 64 + l;
    if (k < len) {
      if (scol) scol[o] = col[b + k];
      sval[o] = (T)val[b + k];
    } else {
      if (scol) scol[o] = -1;
      sval[o] = T(0);
    }
  }
}

bool sell_build(const Csr &A, Sell &S, bool f32, Arena &ar, hipStream_t s) {
  S = Sell{};
  if (A.n <= 0 || A.nnz > 12 * (int64_t)A.n) return false;
  const int32_t nslice = (int32_t)ceil_div(A.n, 64);
  const int32_t maxlen = max_row_length(A.n, A.rp, s);
  // a thread sums its row in order: the layout only serves rows of the plain order
  if (maxlen > kLongRow) return false;
  if ((int64_t)nslice * 64 * maxlen >= ((int64_t)1 << 31)) return false;  // int32 offsets
  Arena tmp;
  tmp.stream = s;
  int32_t *w64 = tmp.alloc<int32_t>(nslice + 1);
  k_sell_width<<<grid_for((int64_t)nslice * 64), kBlock, 0, s>>>(A.n, nslice, A.rp, w64);
  SA_LAUNCH_CHECK();
  int32_t *ptr = tmp.alloc<int32_t>(nslice + 1);
  exclusive_scan_i32(w64, ptr, nslice, s);
  const int32_t total = read1(ptr + nslice, s);
  if ((int64_t)total * 4 > A.nnz * 5) return false;  // padding above a quarter
  S.nslice = nslice;
  S.ptr = ar.alloc<int32_t>(nslice + 1);
  SA_HIP(hipMemcpyAsync(S.ptr, ptr, sizeof(int32_t) * (nslice + 1), hipMemcpyDeviceToDevice, s));
  S.col = ar.alloc<int32_t>(total);
  S.val = ar.alloc<double>(total);
  if (f32) S.valf = ar.alloc<float>(total);
  const unsigned g = grid_for((int64_t)nslice * 64);
  k_sell_fill<double><<<g, kBlock, 0, s>>>(A.n, nslice, A.rp, A.col, A.val, S.ptr, S.col, S.val);
  if (f32)
    k_sell_fill<float><<<g, kBlock, 0, s>>>(A.n, nslice, A.rp, A.col, A.val, S.ptr, nullptr,
                                            S.valf);
  SA_LAUNCH_CHECK();
  return true;
}

void sell_values(const Csr &A, const Sell &S, hipStream_t s) {
  if (!S.ptr) return;
  const unsigned g = grid_for((int64_t)S.nslice * 64);
  k_sell_fill<double><<<g, kBlock, 0, s>>>(A.n, S.nslice, A.rp, A.col, A.val, S.ptr, nullptr,
                                           S.val);
  if (S.valf)
    k_sell_fill<float><<<g, kBlock, 0, s>>>(A.n, S.nslice, A.rp, A.col, A.val, S.ptr, nullptr,
                                            S.valf);
  SA_LAUNCH_CHECK();
}

// Row partition: block b owns rows plan[2b] .. plan[2b+2]-1, whose entries start at
// plan[2b+1]; the pairs are stored side by side so a block reads its row and entry ranges
// with one load.
__global__ void k_spmv_plan(int32_t n, const int32_t *rp, int32_t nblk, int32_t *plan) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nblk) return;
  int32_t lo = n;
  if (b < nblk) {
    const int64_t target = b * kPlanWindow;
    int32_t hi = n;  // first r in [0, n] with rp[r] + 8 r >= target
    lo = 0;
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if ((int64_t)rp[mid] + (int64_t)kPlanRowCost * mid >= target) hi = mid;
      else lo = mid + 1;
    }
  }
  plan[2 * b] = lo;
  plan[2 * b + 1] = rp[lo];
}

void spmv_plan(Csr &A, Arena &ar, hipStream_t s) {
  const int64_t cost = A.nnz + (int64_t)kPlanRowCost * A.n;
  A.nblk = (int32_t)ceil_div(cost + 1, kPlanWindow);
  A.bstart = ar.alloc<int32_t>(2 * ((int64_t)A.nblk + 1));
  k_spmv_plan<<<grid_for(A.nblk + 1), kBlock, 0, s>>>(A.n, A.rp, A.nblk, A.bstart);
  SA_LAUNCH_CHECK();
}

template <class T, class Epi>
static void launch_spmv(const SpmvArgs<T> &a, const Epi &epi, hipStream_t s) {
  if (a.n <= 0) return;
  if (a.sval)
    k_spmv_sell<T, Epi><<<(unsigned)ceil_div(a.nslice, kBlock / 64), kBlock, 0, s>>>(
        a.n, a.nslice, a.sptr, a.scol, a.sval, a.x, epi);
  else if (a.plain)
    k_spmv<T, Epi, false><<<(unsigned)a.nblk, kBlock, 0, s>>>(a.bstart, a.rp, a.col, a.val, a.x,
                                                              epi);
  else
    k_spmv<T, Epi, true><<<(unsigned)a.nblk, kBlock, 0, s>>>(a.bstart, a.rp, a.col, a.val, a.x,
                                                             epi);
  SA_LAUNCH_CHECK();
}

template <class T>
void spmv_store(const SpmvArgs<T> &a, T *y, hipStream_t s) {
  launch_spmv(a, EpStore<T>{y}, s);
}
template <class T>
void spmv_scale(const SpmvArgs<T> &a, const T *d, T *y, hipStream_t s) {
  launch_spmv(a, EpScale<T>{d, y}, s);
}
template <class T>
void spmv_scale_max(const SpmvArgs<T> &a, const T *d, T *y, unsigned long long *part,
                    hipStream_t s) {
  SpmvArgs<T> c = a;
  c.sval = nullptr;  // the CSR kernels carry the maximum
  launch_spmv(c, EpScaleMax<T>{d, y, part}, s);
}
template <class T>
void spmv_resid(const SpmvArgs<T> &a, const T *f, T *r, hipStream_t s) {
  launch_spmv(a, EpResid<T>{f, r}, s);
}
template <class T>
void spmv_add(const SpmvArgs<T> &a, T *u, hipStream_t s) {
  launch_spmv(a, EpAdd<T>{u}, s);
}
template <class T>
void spmv_cheb_start(const SpmvArgs<T> &a, const T *f, const T *invD, T theta, T *r, T *d,
                     hipStream_t s) {
  launch_spmv(a, EpChebStart<T>{f, invD, theta, r, d}, s);
}
template <class T>
void spmv_cheb_step(const SpmvArgs<T> &a, const T *rin, T *rout, const T *invD, T c1, T c2,
                    T *u, bool uzero, T *dout, bool last, hipStream_t s) {
  launch_spmv(a, EpChebStep<T>{a.x, rin, invD, rout, u, dout, c1, c2, uzero, last}, s);
}
template <class T>
void spmv_jacobi(const SpmvArgs<T> &a, const T *f, const T *invD, T w, T *u2, hipStream_t s) {
  launch_spmv(a, EpJacobi<T>{a.x, f, invD, w, u2}, s);
}

#define SA_INST_SPMV(T)                                                                     \
  template void spmv_store<T>(const SpmvArgs<T> &, T *, hipStream_t);                       \
  template void spmv_scale<T>(const SpmvArgs<T> &, const T *, T *, hipStream_t);            \
  template void spmv_scale_max<T>(const SpmvArgs<T> &, const T *, T *, unsigned long long *, \
                                  hipStream_t);                                             \
  template void spmv_resid<T>(const SpmvArgs<T> &, const T *, T *, hipStream_t);            \
  template void spmv_add<T>(const SpmvArgs<T> &, T *, hipStream_t);                         \
  template void spmv_cheb_start<T>(const SpmvArgs<T> &, const T *, const T *, T, T *, T *,   \
                                   hipStream_t);                                            \
  template void spmv_cheb_step<T>(const SpmvArgs<T> &, const T *, T *, const T *, T, T, T *, \
                                  bool, T *, bool, hipStream_t);                            \
  template void spmv_jacobi<T>(const SpmvArgs<T> &, const T *, const T *, T, T *, hipStream_t);
SA_INST_SPMV(double)
SA_INST_SPMV(float)

// ---- vector kernels ---------------------------------------------------------------------
template <class T>
__global__ void k_cheb_first(int32_t n, const T *f, const T *invD, T theta, T *d, T *u,
                             bool write_u) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cheb_first_at<T>(i, f, invD, theta, d, u, write_u);
}
template <class T>
void cheb_first(int32_t n, const T *f, const T *invD, T theta, T *d, T *u, bool write_u,
                hipStream_t s) {
  if (n <= 0) return;
  k_cheb_first<T><<<grid_for(n), kBlock, 0, s>>>(n, f, invD, theta, d, u, write_u);
  SA_LAUNCH_CHECK();
}
template <class T>
__global__ void k_vec_add(int32_t n, T *u, const T *d) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) vec_add_at<T>(i, u, d);
}
template <class T>
void vec_add(int32_t n, T *u, const T *d, hipStream_t s) {
  if (n <= 0) return;
  k_vec_add<T><<<grid_for(n), kBlock, 0, s>>>(n, u, d);
  SA_LAUNCH_CHECK();
}
template <class T>
__global__ void k_jacobi_first(int32_t n, const T *f, const T *invD, T w, T *u) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) jacobi_first_at<T>(i, f, invD, w, u);
}
template <class T>
void jacobi_first(int32_t n, const T *f, const T *invD, T w, T *u, hipStream_t s) {
  if (n <= 0) return;
  k_jacobi_first<T><<<grid_for(n), kBlock, 0, s>>>(n, f, invD, w, u);
  SA_LAUNCH_CHECK();
}
#define SA_INST_VEC(T)                                                                     \
  template void cheb_first<T>(int32_t, const T *, const T *, T, T *, T *, bool, hipStream_t); \
  template void vec_add<T>(int32_t, T *, const T *, hipStream_t);                          \
  template void jacobi_first<T>(int32_t, const T *, const T *, T, T *, hipStream_t);
SA_INST_VEC(double)
SA_INST_VEC(float)

__global__ void k_cast_df(const double *a, float *b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
__global__ void k_cast_fd(const float *a, double *b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}
void cast_f64_to_f32(const double *a, float *b, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast_df<<<grid_for(n), kBlock, 0, s>>>(a, b, n);
  SA_LAUNCH_CHECK();
}
void cast_f32_to_f64(const float *a, double *b, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast_fd<<<grid_for(n), kBlock, 0, s>>>(a, b, n);
  SA_LAUNCH_CHECK();
}

// ---- canonical inner product ------------------------------------------------------------
// Blocks of 4096 terms; lane t of 256 sums terms t + 256 m (m = 0..15) sequentially from 0,
// then s[t] += s[t + w] for w = 128 ... 1; block results are reduced by the same rule.
__global__ __launch_bounds__(kBlock) void k_dot_stage(const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      int64_t n, double *__restrict__ part) {
  __shared__ double sh[kBlock];
  dot_block(blockIdx.x, x, y, n, part + blockIdx.x, sh);
}

int64_t dot_ws_size(int64_t n) {
  int64_t tot = 8;
  int64_t m = n;
  do {
    m = ceil_div(m, 4096);
    if (m < 1) m = 1;
    tot += m;
  } while (m > 1);
  return tot;
}

void dot_f64(const double *x, const double *y, int64_t n, double *res, double *ws,
             hipStream_t s) {
  // First stage multiplies; later stages sum partials.  The final stage writes *res.
  int64_t m = n;
  const double *in = x;
  const double *iny = y;
  double *out = ws;
  for (;;) {
    int64_t nb = ceil_div(m, 4096);
    if (nb < 1) nb = 1;
    double *dst = (nb == 1) ? res : out;
    k_dot_stage<<<(unsigned)nb, kBlock, 0, s>>>(in, iny, m, dst);
    SA_LAUNCH_CHECK();
    if (nb == 1) break;
    in = out;
    iny = nullptr;
    out += nb;
    m = nb;
  }
}

// ---- dense GEMV for the coarsest level (one wavefront per row) -------------------------
__global__ __launch_bounds__(kBlock) void k_gemv(int32_t n, const double *__restrict__ M,
                                                 const double *__restrict__ x,
                                                 double *__restrict__ y) {
  const int64_t row = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (row < n) gemv_row(row, n, M, x, y);
}
void gemv_f64(int32_t n, const double *M, const double *x, double *y, hipStream_t s) {
  if (n <= 0) return;
  k_gemv<<<(unsigned)ceil_div(n, kBlock / 64), kBlock, 0, s>>>(n, M, x, y);
  SA_LAUNCH_CHECK();
}

// ---- PCG updates ----------------------------------------------------------------------------
__global__ void k_update_xr(int32_t n, double *x, double *r, const double *p, const double *q,
                            const PcgScalars *S) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) update_xr_at(i, x, r, p, q, S->alpha);
}
void pcg_update_xr(int32_t n, double *x, double *r, const double *p, const double *q,
                   const PcgScalars *S, hipStream_t s) {
  k_update_xr<<<grid_for(n), kBlock, 0, s>>>(n, x, r, p, q, S);
  SA_LAUNCH_CHECK();
}
__global__ void k_update_p(int32_t n, double *p, const double *z, const PcgScalars *S) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) update_p_at(i, p, z, S->beta);
}
void pcg_update_p(int32_t n, double *p, const double *z, const PcgScalars *S, hipStream_t s) {
  k_update_p<<<grid_for(n), kBlock, 0, s>>>(n, p, z, S);
  SA_LAUNCH_CHECK();
}
__global__ void k_vec_sub(int32_t n, const double *z, const double *zo, double *w) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) vec_sub_at(i, z, zo, w);
}
void vec_sub(int32_t n, const double *z, const double *zold, double *w, hipStream_t s) {
  k_vec_sub<<<grid_for(n), kBlock, 0, s>>>(n, z, zold, w);
  SA_LAUNCH_CHECK();
}
__global__ void k_pcg_alpha(PcgScalars *S) { pcg_alpha_on(S); }
void pcg_alpha(PcgScalars *S, hipStream_t s) {
  k_pcg_alpha<<<1, 1, 0, s>>>(S);
  SA_LAUNCH_CHECK();
}
__global__ void k_pcg_beta(PcgScalars *S, bool pr) { pcg_beta_on(S, pr); }
void pcg_beta(PcgScalars *S, bool pr, hipStream_t s) {
  k_pcg_beta<<<1, 1, 0, s>>>(S, pr);
  SA_LAUNCH_CHECK();
}
__global__ void k_pcg_init(PcgScalars *S) { pcg_init_on(S); }
void pcg_init_rho(PcgScalars *S, hipStream_t s) {
  k_pcg_init<<<1, 1, 0, s>>>(S);
  SA_LAUNCH_CHECK();
}

}  // namespace sa
