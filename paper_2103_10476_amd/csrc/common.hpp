// Internal definitions shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/saamg.h"

namespace sa {

// Failure inside the library: carries a status code; converted to the return value at the
// C boundary.
struct Error : std::runtime_error {
  sa_status code;
  Error(sa_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define SA_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::sa::Error(e_ == hipErrorOutOfMemory ? SA_ERR_OOM : SA_ERR_HIP,                \
                        std::string(#call) + ": " + hipGetErrorString(e_));                \
  } while (0)

#define SA_LAUNCH_CHECK() SA_HIP(hipGetLastError())

constexpr int kBlock = 256;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Workgroups are handed to the 8 XCDs round-robin (workgroup b runs on XCD b mod 8), and
// each XCD has its own L2.  Renumbering so that XCD x takes one contiguous run of row blocks
// keeps the x entries a block gathers from neighbouring rows (stencil planes) in that XCD's
// L2 instead of fetching them once per XCD.  A bijection on [0, nb).
__device__ __forceinline__ int32_t xcd_block(uint32_t b, uint32_t nb) {
  constexpr uint32_t kXcd = 8;
  const uint32_t q = nb / kXcd, r = nb % kXcd;
  const uint32_t x = b % kXcd, k = b / kXcd;
  return (int32_t)(x * q + (x < r ? x : r) + k);
}

inline unsigned grid_for(int64_t n, int block = kBlock) {
  int64_t g = ceil_div(n, block);
  return (unsigned)(g < 1 ? 1 : g);
}

// Stream-ordered device allocation from the library's caching allocator (alloc.hip): a
// block released on stream s is reused only for later work on s.
void *dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void *p, hipStream_t s);
// Returns every cached (free) block to the driver; synchronises the device.
void dev_release_cached();
// Returns the cached blocks of stream s (before s is destroyed).
void dev_release_stream(hipStream_t s);
// Bytes held by live allocations and by cached free blocks.
void dev_cache_stats(size_t *in_use, size_t *cached);
// Per-request accounting: while a Meter is installed on a thread, the device bytes (size
// classes) allocated by that thread are charged to it until freed, from any thread.  The
// Meter must outlive every block charged to it.
struct Meter {
  int64_t live = 0, peak = 0;
  Meter *parent = nullptr;  // also charged (e.g. a server's total)
};
void meter_begin(Meter *m);
void meter_end();
void meter_read(const Meter *m, int64_t *live, int64_t *peak);  // consistent snapshot
// Blocking device-to-host copy staged through a per-thread pinned buffer.
void readback(void *host, const void *dev, size_t bytes, hipStream_t s);
// A per-thread pinned host buffer of at least `bytes`, separate from the readback staging:
// kernels write it through its device mapping while the calling thread polls it.
void *pinned_status(size_t bytes);

// A typed device buffer owned by an Arena or held as a temporary.
template <class T>
struct DBuf {
  T *p = nullptr;
  int64_t n = 0;
};

// Owns a set of device allocations; frees them in its destructor (stream ordered).
struct Arena {
  hipStream_t stream = nullptr;
  std::vector<void *> ptrs;
  int64_t bytes = 0;
  template <class T>
  T *alloc(int64_t count) {
    size_t b = (size_t)(count > 0 ? count : 1) * sizeof(T);
    T *p = (T *)dev_alloc(b, stream);
    ptrs.push_back(p);
    bytes += (int64_t)b;
    return p;
  }
  void release() {
    for (void *p : ptrs) dev_free(p, stream);
    ptrs.clear();
    bytes = 0;
  }
  ~Arena() {
    try {
      release();
    } catch (...) {
    }
  }
};

// Device CSR view.  bstart/nblk: the SpMV row partition (see spmv_plan).
struct Csr {
  int32_t n = 0, ncols = 0;
  int64_t nnz = 0;
  int32_t *rp = nullptr;
  int32_t *col = nullptr;
  double *val = nullptr;
  int32_t *bstart = nullptr;  // SpMV plan: nblk+1 pairs (first row, first entry)
  int32_t nblk = 0;
  int32_t maxrow = -1;        // longest row when known (the pattern's, kept by value updates)
};

// Sliced-ELL copy of a CSR operator for the solve-phase SpMV.  Rows in slices of 64 (one per
// wavefront); slice s is stored column-major from ptr[s] with width w_s = (ptr[s+1]-ptr[s])/64,
// entry k of row 64 s + l at ptr[s] + 64 k + l, so the k-th entries of a slice's rows are
// contiguous.  Rows keep their entry order (ascending columns); the w_s - len tail of a row
// is padding with col -1 and value 0.
struct Sell {
  int32_t nslice = 0;
  int32_t *ptr = nullptr;  // nslice+1 entry offsets (multiples of 64)
  int32_t *col = nullptr;
  double *val = nullptr;
  float *valf = nullptr;   // FP32 values (FP32 V-cycle only)
};

struct CsrF {  // float copy of the values for the FP32 V-cycle
  int32_t n = 0, ncols = 0;
  int64_t nnz = 0;
  const int32_t *rp = nullptr;
  const int32_t *col = nullptr;
  float *val = nullptr;
};

// Blocking readback of one value.
template <class T>
T read1(const T *dptr, hipStream_t s) {
  T v;
  readback(&v, dptr, sizeof(T), s);
  return v;
}

// ---- primitives (scan.hip) ------------------------------------------------------------
// out[0..n] = exclusive prefix sums of in[0..n-1], out[n] = total (out may alias in only
// when in has n+1 slots).  Deterministic (integer).
void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s);
void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void fill_f64(double *p, double v, int64_t n, hipStream_t s);
void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);

// ---- vector kernels and the canonical inner product (blas.hip) --------------------------
// dot: canonical tree (blocks of 4096, 256 lanes x 16 sequential, then pairwise halving),
// result written to *res (device).  ws must hold ceil(n/4096) + ceil(n/4096^2) + 8 doubles.
void dot_f64(const double *x, const double *y, int64_t n, double *res, double *ws,
             hipStream_t s);
int64_t dot_ws_size(int64_t n);

}  // namespace sa
