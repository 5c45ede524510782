// Fills and exclusive prefix sums.
#include "common.hpp"

namespace sa {

template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

template <class T>
static void fill(T *p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = grid_for(n);
  if (g > 65536) g = 65536;
  k_fill<T><<<g, kBlock, 0, s>>>(p, v, n);
  SA_LAUNCH_CHECK();
}

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) { fill(p, v, n, s); }
void fill_f64(double *p, double v, int64_t n, hipStream_t s) { fill(p, v, n, s); }
void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s) { fill(p, v, n, s); }

// ---- exclusive scan -----------------------------------------------------------------
// Three phases: per-block totals (each block covers kScanTile elements), a recursive scan
// of the block totals, then a per-block scan seeded with the block's offset.
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

template <class T>
__device__ T block_exclusive(T v, T *sh, T &total) {
  // Hillis-Steele inclusive scan over the 256 thread sums in LDS.
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    T add = (t >= off) ? sh[t - off] : T(0);
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  total = sh[kBlock - 1];
  T excl = sh[t] - v;
  __syncthreads();
  return excl;
}

template <class T>
__global__ void k_scan_totals(const T *in, int64_t n, T *totals) {
  __shared__ T sh[kBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += in[base + k];
  T tot;
  block_exclusive<T>(s, sh, tot);
  if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

template <class T>
__global__ void k_scan_apply(const T *in, T *out, int64_t n, const T *offsets) {
  __shared__ T sh[kBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T vals[kScanItems];
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    vals[k] = (base + k < n) ? in[base + k] : T(0);
    s += vals[k];
  }
  T tot;
  T run = block_exclusive<T>(s, sh, tot) + offsets[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += vals[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) out[n] = run;
}

// n <= kScanTile: the whole scan in one block (out may equal in: every thread reads its items
// before the block scan's barriers, and writes after them).
template <class T>
__global__ void k_scan_single(const T *in, T *out, int64_t n) {
  __shared__ T sh[kBlock];
  const int64_t base = (int64_t)threadIdx.x * kScanItems;
  T vals[kScanItems];
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    vals[k] = (base + k < n) ? in[base + k] : T(0);
    s += vals[k];
  }
  T tot;
  T run = block_exclusive<T>(s, sh, tot);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += vals[k];
  }
  if (threadIdx.x == 0) out[n] = tot;
}

template <class T>
static void scan_impl(const T *in, T *out, int64_t n, hipStream_t s) {
  if (n <= 0) {
    fill(out, T(0), 1, s);
    return;
  }
  if (n <= kScanTile) {
    k_scan_single<T><<<1, kBlock, 0, s>>>(in, out, n);
    SA_LAUNCH_CHECK();
    return;
  }
  int64_t nb = ceil_div(n, kScanTile);
  T *tot = (T *)dev_alloc(sizeof(T) * (nb + 1), s);
  k_scan_totals<T><<<(unsigned)nb, kBlock, 0, s>>>(in, n, tot);
  SA_LAUNCH_CHECK();
  scan_impl<T>(tot, tot, nb, s);  // in place: tot has nb+1 slots (nb >= 2 here)
  k_scan_apply<T><<<(unsigned)nb, kBlock, 0, s>>>(in, out, n, tot);
  SA_LAUNCH_CHECK();
  dev_free(tot, s);
}

void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
  scan_impl<int32_t>(in, out, n, s);
}
void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
  scan_impl<int64_t>(in, out, n, s);
}

}  // namespace sa
